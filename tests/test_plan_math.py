"""Host-side plan arithmetic of the library (csrc/plan_math.cpp), built with
g++ on its own and driven by a small test program: the multiply-shift
division used by the kernels' index math, the FFT radix plans, the
vertical and horizontal tables against the oracle's definitions, and the
variable-density solver's face weights and batch prediction."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import oracle.variable
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2009_12849_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "plan_math.h"
#include "monc_types.h"
using namespace monc;

static unsigned fast_div(unsigned x, unsigned mul, int shift) {  // device formula, on the host
  const unsigned long long t = ((unsigned long long)x * mul) >> 32;
  return (unsigned)((t + x) >> shift);
}

int main(int argc, char** argv) {
  // 1. division: every divisor up to 9000 and the row lengths the library uses,
  //    dividends at the edges and spread over [0, 2^31)
  unsigned long long bad = 0, checked = 0;
  unsigned s = 12345u;
  for (unsigned d = 1; d <= 9000; ++d) {
    unsigned mul; int sh;
    div_magic(d, mul, sh);
    const unsigned xs[] = {0u, 1u, d - 1, d, d + 1, 2 * d - 1, 2 * d, 0x7fffffffu, 0x7fffffffu - d, 0x7ffffffeu};
    for (unsigned x : xs) { ++checked; if (x <= 0x7fffffffu && fast_div(x, mul, sh) != x / d) ++bad; }
    for (int r = 0; r < 64; ++r) {
      s = s * 1664525u + 1013904223u;
      const unsigned x = s & 0x7fffffffu;
      ++checked;
      if (fast_div(x, mul, sh) != x / d) ++bad;
    }
  }
  // block strides ny * B of the spectral layout (B = 1..8) for 3-smooth ny up to 8192
  for (unsigned ny = 1; ny <= 8192; ++ny) {
    unsigned r = ny;
    while (r % 2 == 0) r /= 2;
    while (r % 3 == 0) r /= 3;
    if (r != 1) continue;
    for (unsigned bw = 1; bw <= 8; bw *= 2) {
      const unsigned d = ny * bw;
      if (d <= 9000) continue;
      unsigned mul; int sh;
      div_magic(d, mul, sh);
      const unsigned edge[4] = {d - 1, d, 2 * d - 1, 0x7fffffffu};
      for (int t = 0; t < 256; ++t) {
        s = s * 1664525u + 1013904223u;
        const unsigned x = (t < 4) ? edge[t] : (s & 0x7fffffffu);
        ++checked;
        if (fast_div(x, mul, sh) != x / d) ++bad;
      }
    }
  }
  std::printf("div %llu %llu\n", checked, bad);
  // 2. radix plans
  const int ns[] = {1, 2, 3, 4, 6, 8, 9, 12, 16, 27, 48, 96, 243, 256, 768, 1024, 1536, 2048, 4096, 6561, 8192, 5, 7, 10, 14, 9000};
  for (int n : ns) {
    FftPlan fp{};
    const bool ok = radix_plan(n, fp);
    std::printf("radix %d %d %d", n, ok ? 1 : 0, ok ? fp.npass : 0);
    if (ok) for (int p = 0; p < fp.npass; ++p) std::printf(" %d", fp.rad[p]);
    std::printf("\n");
  }
  // 3. LDS layouts shared by the kernels and the host
  for (int s = 2; s <= kTriSmax; ++s)
    std::printf("tri %d %d %d\n", s, tri_lane_slots(s, true), tri_lane_slots(s, false));
  for (int n = 16; n <= 4096; ++n) {
    int r = n;
    while (r % 2 == 0) r /= 2;
    while (r % 3 == 0) r /= 3;
    if (r != 1) continue;
    for (int cb = 8; cb <= 16; cb += 8) {
      const int len = xlds_len(n, cb);
      std::vector<int> seen(len, 0);
      int bad = 0;
      for (int i = 0; i < n; ++i) {
        const int j = xlds_index(i, n, cb);
        if (j < 0 || j >= len || seen[j]++) ++bad;
      }
      std::printf("xlds %d %d %d %d %d\n", n, cb, len, xsw_on(n, cb) ? 1 : 0, bad);
    }
  }
  // 4. tables from dz, rho0 on stdin
  int nz; std::scanf("%d", &nz);
  std::vector<double> dz(nz), rho(nz);
  for (int k = 0; k < nz; ++k) std::scanf("%lf", &dz[k]);
  for (int k = 0; k < nz; ++k) std::scanf("%lf", &rho[k]);
  VerticalTables t = vertical_tables(nz, dz.data(), rho.data());
  std::printf("rH %.17g\n", t.rH);
  for (int k = 0; k < nz; ++k) std::printf("vt %.17g %.17g %.17g\n", t.ta[k], t.tc[k], t.rhow[k]);
  for (double v : modified_wavenumbers(48, 25, 25.0)) std::printf("lx %.17g\n", v);
  std::vector<double> tw = twiddles(12);
  for (size_t i = 0; i < tw.size(); i += 2) std::printf("tw %.17g %.17g\n", tw[i], tw[i + 1]);
  // 5. the variable-density solver's face weights and batch prediction
  std::vector<double> za, zb;
  face_weights(nz, dz.data(), za, zb);
  for (int k = 0; k < nz; ++k) std::printf("fw %.17g %.17g\n", za[k], zb[k]);
  const double kb[][4] = {{1e-3, 1.0, 3, 1e-10}, {1e-3, 1e-3, 2, 1e-10}, {0.0, 1.0, 3, 1e-10},
                          {1e-2, 1.0, 2, 0.0}, {0.5, 1.0, 1, 1e-10}, {1e-9, 1e-8, 1, 1e-10}};
  for (const auto& c : kb) std::printf("kb %d\n", krylov_batch(c[0], c[1], (int)c[2], c[3], 32));
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("plan_math")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    subprocess.run([gxx, "-O2", "-std=c++17", f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}",
                    str(src), os.path.join(CSRC, "plan_math.cpp"), "-o", str(exe)], check=True)
    g = synth.make_grid("2048x2048x160")
    stdin = f"{g.nz}\n" + " ".join(repr(float(x)) for x in g.dz) + "\n" + " ".join(repr(float(x)) for x in g.rho0) + "\n"
    out = subprocess.run([str(exe)], input=stdin, capture_output=True, text=True, check=True).stdout
    return g, out.splitlines()


def test_multiply_shift_division(driver):
    _, lines = driver
    (checked, bad), = [tuple(map(int, l.split()[1:])) for l in lines if l.startswith("div ")]
    assert checked > 500000 and bad == 0


def test_radix_plans(driver):
    _, lines = driver
    for l in (l for l in lines if l.startswith("radix ")):
        f = list(map(int, l.split()[1:]))
        n, ok, npass, rads = f[0], f[1], f[2], f[3:]
        smooth = n >= 1 and all(p in (2, 3) for p in _prime_factors(n))
        assert ok == (1 if smooth else 0), n
        if ok:
            assert len(rads) == npass and int(np.prod(rads)) == n, (n, rads)
            assert all(r in (2, 3, 4, 8) for r in rads), (n, rads)
            # radix 8 first, at most one radix 4 or 2, then the 3s
            twos = [r for r in rads if r in (2, 4, 8)]
            assert rads[:len(twos)] == twos and sum(r in (2, 4) for r in twos) <= 1


def _prime_factors(n):
    out, p = [], 2
    while n > 1 and p * p <= n:
        while n % p == 0:
            out.append(p)
            n //= p
        p += 1
    if n > 1:
        out.append(n)
    return out


def test_tridiagonal_lds_chunks(driver):
    """A lane's LDS chunk (16-byte slots, an odd count) holds its S rows in the
    storage precision, and with FP32 storage also the S-2 parked FP64
    right-hand sides that go over them."""
    _, lines = driver
    rows = [tuple(map(int, l.split()[1:])) for l in lines if l.startswith("tri ")]
    assert len(rows) == 15
    for s, f32, f64 in rows:
        assert f32 % 2 == 1 and f64 % 2 == 1, (s, f32, f64)
        assert 16 * f32 >= 8 * s and 16 * f32 >= 16 * (s - 2), (s, f32)
        assert 16 * f64 >= 16 * s, (s, f64)
        assert f32 <= f64


def test_x_transform_lds_index_is_a_bijection(driver):
    """Every compile-time x length: the LDS index map (XOR-permuted bank rows
    for radix-16 transforms, padding otherwise) is one-to-one into the
    buffer the host sizes, in both precisions."""
    _, lines = driver
    rows = [tuple(map(int, l.split()[1:])) for l in lines if l.startswith("xlds ")]
    assert len(rows) > 40
    for n, cb, length, sw, bad in rows:
        assert bad == 0, (n, cb)
        assert length == n if sw else length > n, (n, cb, length)
    assert any(r[3] for r in rows) and not all(r[3] for r in rows)


def test_vertical_tables_match_oracle(driver):
    g, lines = driver
    a, c = oracle.tridiag_coefficients(g.dz, g.rho0)
    vt = np.array([list(map(float, l.split()[1:])) for l in lines if l.startswith("vt ")])
    assert vt.shape == (g.nz, 3)
    # same formulas, evaluated in a different order: a few ulps
    np.testing.assert_allclose(vt[:, 0], a, rtol=1e-15, atol=0)
    np.testing.assert_allclose(vt[:, 1], c, rtol=1e-15, atol=0)
    rH = float(next(l for l in lines if l.startswith("rH ")).split()[1])
    assert abs(rH * np.sum(g.dz) - 1.0) < 1e-15


def test_horizontal_tables(driver):
    _, lines = driver
    lx = np.array([float(l.split()[1]) for l in lines if l.startswith("lx ")])
    ref, _ = oracle.modified_wavenumbers(48, 1, 25.0, 1.0)
    np.testing.assert_allclose(lx, ref, rtol=1e-15, atol=1e-18)
    tw = np.array([list(map(float, l.split()[1:])) for l in lines if l.startswith("tw ")])
    ref = np.exp(-2j * np.pi * np.arange(12) / 12)
    # the angle 2 pi t / n is rounded before the sine and cosine: a few ulps
    np.testing.assert_allclose(tw[:, 0] + 1j * tw[:, 1], ref, rtol=0, atol=2e-15)


def test_face_weights_match_oracle(driver):
    """za_k q_k + zb_k q_{k+1} is the oracle's face value of a column q
    (oracle.face_densities, the linear interpolation in z)."""
    g, lines = driver
    fw = np.array([list(map(float, l.split()[1:])) for l in lines if l.startswith("fw ")])
    assert fw.shape == (g.nz, 2)
    assert fw[-1, 0] == 0.0 and fw[-1, 1] == 0.0
    q = np.asarray(g.rho0, dtype=np.float64)
    col = q[:, None, None] * np.ones((1, 1, 1))
    _, _, rz = oracle.variable.face_densities(col, g.dz)
    mine = fw[:-1, 0] * q[:-1] + fw[:-1, 1] * q[1:]
    np.testing.assert_allclose(mine, rz[:, 0, 0], rtol=1e-15, atol=0)


def test_krylov_batch_prediction(driver):
    """Rate 0.1 per iteration from 1e-3 to 1e-10: 7 more; no decrease or no
    residual: 1; tol 0: the cap; a slow rate: capped at 32; one iteration to
    go: 1."""
    _, lines = driver
    got = [int(l.split()[1]) for l in lines if l.startswith("kb ")]
    assert got == [7, 1, 1, 32, 32, 1]
