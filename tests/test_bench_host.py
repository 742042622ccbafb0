"""Host logic of bench.py: kernel-name classification, counter arithmetic and
the counter summary (CPU only; a synthetic counter file stands in for
rocprofv3's output)."""
import csv

import numpy as np
import pytest

import bench


@pytest.mark.parametrize("name,expect", [
    ("void monc::k_xfwd_ct<float, 1, 2048>(monc::LaunchArgs)", ("mixed", "resid_fftx")),
    ("void monc::k_xfwd_ct<double, 0, 2048>(monc::LaunchArgs)", ("fp64", "div_fftx")),
    ("void monc::k_xfwd_gen<float, 0>(monc::LaunchArgs)", ("mixed", "div_fftx")),
    ("void monc::k_ffty_ct<double, true, 2048>(monc::LaunchArgs)", ("fp64", "ffty_inv")),
    ("void monc::k_ffty_ct<float, false, 1024>(monc::LaunchArgs)", ("mixed", "ffty_fwd")),
    ("void monc::k_ffty_pp<true, 2048>(monc::LaunchArgs)", ("mixed", "ffty_inv")),
    ("void monc::k_ffty_pp<false, 4096>(monc::LaunchArgs)", ("mixed", "ffty_fwd")),
    ("void monc::k_tridiag<float, 10, 256>(monc::LaunchArgs)", ("mixed", "tridiag")),
    ("void monc::k_xinv_ct<float, 1, 2048>(monc::LaunchArgs)", ("mixed", "ifftx_corr")),
    ("void monc::k_xinv_ct<float, 0, 2048>(monc::LaunchArgs)", ("mixed", "ifftx")),
    ("void monc::k_grad<double, 2, false>(monc::LaunchArgs)", ("fp64", "grad")),
    ("void monc::k_grad<float, 4, false>(monc::LaunchArgs)", ("mixed", "grad_final")),
    ("(anonymous namespace)::k_probe_copy(float vector[4] const*, float vector[4]*, long long)", ("probe", "copy")),
    ("void at::native::elementwise_kernel<128, 4>(int, Foo)", None),
])
def test_classify_kernel(name, expect):
    assert bench.classify_kernel(name) == expect


def test_counter_bytes():
    c = {"TCC_EA0_RDREQ_32B_sum": 3, "TCC_EA0_RDREQ_64B_sum": 5, "TCC_EA0_RDREQ_128B_sum": 7}
    assert bench.read_bytes(c) == 32 * 3 + 64 * 5 + 128 * 7
    assert bench.write_bytes({"TCC_EA0_WRREQ_sum": 10, "TCC_EA0_WRREQ_64B_sum": 4}) == 64 * 4 + 32 * 6


def _write_csv(path, rows):
    with open(path, "w", newline="") as fh:
        wr = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        wr.writeheader()
        for r in rows:
            wr.writerow(r)


def test_summary_calibrates_on_the_probe_copy(tmp_path):
    known = bench.CALIB_MIB * (1 << 20)
    copy = "(anonymous namespace)::k_probe_copy(float vector[4] const*, float vector[4]*, long long)"
    grad = "void monc::k_grad<float, 4, false>(monc::LaunchArgs)"
    # raw counters read the copy 1.25x high (all 128-byte requests) and its
    # writes exactly; the gradient reads 2 A and writes A
    A = 1 << 30
    rd = [dict(Dispatch_Id=1, Kernel_Name=copy, Counter_Name="TCC_EA0_RDREQ_128B_sum",
               Counter_Value=1.25 * known / 128),
          dict(Dispatch_Id=2, Kernel_Name=grad, Counter_Name="TCC_EA0_RDREQ_128B_sum", Counter_Value=2.5 * A / 128)]
    wr = [dict(Dispatch_Id=1, Kernel_Name=copy, Counter_Name="TCC_EA0_WRREQ_sum", Counter_Value=known / 64),
          dict(Dispatch_Id=1, Kernel_Name=copy, Counter_Name="TCC_EA0_WRREQ_64B_sum", Counter_Value=known / 64),
          dict(Dispatch_Id=2, Kernel_Name=grad, Counter_Name="TCC_EA0_WRREQ_sum", Counter_Value=A / 64),
          dict(Dispatch_Id=2, Kernel_Name=grad, Counter_Name="TCC_EA0_WRREQ_64B_sum", Counter_Value=A / 64)]
    _write_csv(tmp_path / "rd.csv", rd)
    _write_csv(tmp_path / "wr.csv", wr)
    text = bench.summarize_counters(str(tmp_path / "rd.csv"), str(tmp_path / "wr.csv"), "256x256x128", "cmd")
    vals = {}
    for line in text.splitlines():
        line = line.split("#", 1)[0].strip()
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    assert np.isclose(float(vals["calibration.read_factor"]), 0.8)
    assert np.isclose(float(vals["calibration.write_factor"]), 1.0)
    assert np.isclose(float(vals["mixed.grad_final.read_bytes_per_launch"]), 2 * A, rtol=1e-6)
    assert np.isclose(float(vals["mixed.grad_final.bytes_per_launch"]), 3 * A, rtol=1e-6)
    assert vals["kernels_sha256_16"] == bench.kernel_source_hash()


def test_summary_dram_cross_check(tmp_path):
    # third pass: requests addressed to local memory, scaled by the copy's
    # bytes per request (64 here); the gradient's come to 2 A read, A written
    known = bench.CALIB_MIB * (1 << 20)
    copy = "(anonymous namespace)::k_probe_copy(float vector[4] const*, float vector[4]*, long long)"
    grad = "void monc::k_grad<float, 4, false>(monc::LaunchArgs)"
    A = 1 << 30
    rd = [dict(Dispatch_Id=1, Kernel_Name=copy, Counter_Name="TCC_EA0_RDREQ_128B_sum", Counter_Value=known / 128),
          dict(Dispatch_Id=2, Kernel_Name=grad, Counter_Name="TCC_EA0_RDREQ_128B_sum", Counter_Value=2 * A / 128)]
    wr = [dict(Dispatch_Id=1, Kernel_Name=copy, Counter_Name="TCC_EA0_WRREQ_sum", Counter_Value=known / 64),
          dict(Dispatch_Id=1, Kernel_Name=copy, Counter_Name="TCC_EA0_WRREQ_64B_sum", Counter_Value=known / 64),
          dict(Dispatch_Id=2, Kernel_Name=grad, Counter_Name="TCC_EA0_WRREQ_sum", Counter_Value=A / 64),
          dict(Dispatch_Id=2, Kernel_Name=grad, Counter_Name="TCC_EA0_WRREQ_64B_sum", Counter_Value=A / 64)]
    dr = [dict(Dispatch_Id=1, Kernel_Name=copy, Counter_Name="TCC_EA0_RDREQ_DRAM_sum", Counter_Value=known / 64),
          dict(Dispatch_Id=1, Kernel_Name=copy, Counter_Name="TCC_EA0_WRREQ_DRAM_sum", Counter_Value=known / 64),
          dict(Dispatch_Id=2, Kernel_Name=grad, Counter_Name="TCC_EA0_RDREQ_DRAM_sum", Counter_Value=2 * A / 64),
          dict(Dispatch_Id=2, Kernel_Name=grad, Counter_Name="TCC_EA0_WRREQ_DRAM_sum", Counter_Value=A / 64)]
    for name, rows in (("rd", rd), ("wr", wr), ("dr", dr)):
        _write_csv(tmp_path / f"{name}.csv", rows)
    text = bench.summarize_counters(str(tmp_path / "rd.csv"), str(tmp_path / "wr.csv"), "256x256x128", "cmd",
                                    str(tmp_path / "dr.csv"))
    line = [ln for ln in text.splitlines() if ln.startswith("dram.mixed.grad_final.bytes_per_launch")][0]
    assert np.isclose(float(line.split(":", 1)[1].split("#", 1)[0]), 3 * A, rtol=1e-6)


def test_kernel_hash_ignores_comments_not_code():
    # a counter summary stays valid across comment edits and goes stale on
    # any change of the code, string literals included
    base = 'int f(int a) { return a + 1; } // one\nconst char* s = "x // y";\n'
    same = '/* doc */\nint f(int a)  {\n  return a + 1;  // two\n}\nconst char* s = "x // y";'
    code = 'int f(int a) { return a + 2; }\nconst char* s = "x // y";\n'
    lit = 'int f(int a) { return a + 1; }\nconst char* s = "x // z";\n'
    assert bench.strip_comments(base) == bench.strip_comments(same)
    assert bench.strip_comments(base) != bench.strip_comments(code)
    assert bench.strip_comments(base) != bench.strip_comments(lit)
    assert bench.strip_comments("char c = '\"'; /* a */ int b;") == "char c = '\"'; int b;"
