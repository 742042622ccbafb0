// Host-side plan arithmetic (see plan_math.h).
#include "plan_math.h"

#include <cmath>
#include <cstdio>

#include "../../include/monc.h"

namespace monc {

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

static bool only_2_3(int n) {
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

int check_plan_args(int nx, int ny, int nz, double dx, double dy, const double* dz, const double* rho0,
                    int dtype, std::string& err) {
  char buf[256];
  if (nx < 1 || ny < 1 || nz < 1) {
    std::snprintf(buf, sizeof buf, "grid size must be >= 1 (got nx=%d ny=%d nz=%d)", nx, ny, nz);
    err = buf;
    return MONC_EINVAL;
  }
  if (nx > MONC_MAX_N || ny > MONC_MAX_N || nz > MONC_MAX_NZ) {
    std::snprintf(buf, sizeof buf, "grid size above the limits (nx, ny <= %d, nz <= %d): nx=%d ny=%d nz=%d",
                  MONC_MAX_N, MONC_MAX_NZ, nx, ny, nz);
    err = buf;
    return MONC_EUNSUPPORTED;
  }
  if (!only_2_3(nx) || !only_2_3(ny)) {
    std::snprintf(buf, sizeof buf, "nx and ny must have no prime factor above 3 (got nx=%d ny=%d)", nx, ny);
    err = buf;
    return MONC_EUNSUPPORTED;
  }
  if (!finite_pos(dx) || !finite_pos(dy)) {
    std::snprintf(buf, sizeof buf, "dx and dy must be finite and > 0 (got dx=%g dy=%g)", dx, dy);
    err = buf;
    return MONC_EINVAL;
  }
  if (dz == nullptr || rho0 == nullptr) {
    err = "dz and rho0 must be non-null host arrays of nz values";
    return MONC_EINVAL;
  }
  for (int k = 0; k < nz; ++k) {
    if (!finite_pos(dz[k])) {
      std::snprintf(buf, sizeof buf, "dz[%d] must be finite and > 0 (got %g)", k, dz[k]);
      err = buf;
      return MONC_EINVAL;
    }
    if (!finite_pos(rho0[k])) {
      std::snprintf(buf, sizeof buf, "rho0[%d] must be finite and > 0 (got %g)", k, rho0[k]);
      err = buf;
      return MONC_EINVAL;
    }
  }
  if (dtype != MONC_FP64 && dtype != MONC_MIXED) {
    std::snprintf(buf, sizeof buf, "dtype must be MONC_FP64 (0) or MONC_MIXED (1) (got %d)", dtype);
    err = buf;
    return MONC_EINVAL;
  }
  return MONC_OK;
}

bool radix_plan(int n, FftPlan& fp) {
  fp.n = n;
  fp.npass = 0;
  int a = 0, b = 0, m = n;
  while (m % 2 == 0) { m /= 2; ++a; }
  while (m % 3 == 0) { m /= 3; ++b; }
  if (m != 1) return false;
  auto push = [&](int r) {
    if (fp.npass >= kMaxPass) return false;
    fp.rad[fp.npass++] = r;
    return true;
  };
  while (a >= 3) { if (!push(8)) return false; a -= 3; }
  if (a == 2 && !push(4)) return false;
  if (a == 1 && !push(2)) return false;
  for (int i = 0; i < b; ++i) if (!push(3)) return false;
  return true;
}

bool fft_threads(FftPlan& fp, int elems) {
  if (elems < 1) elems = 1;
  int nt = (fp.n + elems - 1) / elems;
  if (nt < 1) nt = 1;
  for (;;) {
    bool ok = true;
    for (int p = 0; p < fp.npass; ++p) {
      const int R = fp.rad[p];
      const int bm = (kGenericElems + R - 1) / R;  // butterflies a thread can hold
      const int nb = fp.n / R;
      if ((nb + nt - 1) / nt > bm) ok = false;
    }
    if (ok) break;
    ++nt;
  }
  if (nt > 1024) return false;
  fp.nt = nt;
  return true;
}

VerticalTables vertical_tables(int nz, const double* dz, const double* rho0) {
  VerticalTables t;
  t.rho0.assign(rho0, rho0 + nz);
  t.dz.assign(dz, dz + nz);
  t.rhow.assign(nz, 0.0);
  t.rdz.assign(nz, 0.0);
  t.rdzc.assign(nz, 0.0);
  t.ta.assign(nz, 0.0);
  t.tc.assign(nz, 0.0);
  double H = 0.0;
  for (int k = 0; k < nz; ++k) {
    H += dz[k];
    t.rdz[k] = 1.0 / dz[k];
  }
  t.rH = 1.0 / H;
  for (int k = 0; k + 1 < nz; ++k) {
    const double dzc = 0.5 * (dz[k] + dz[k + 1]);
    // face zw_{k+1} lies dz_k/2 above centre k and dz_{k+1}/2 below centre k+1
    t.rhow[k] = (dz[k + 1] * rho0[k] + dz[k] * rho0[k + 1]) / (dz[k] + dz[k + 1]);
    t.rdzc[k] = 1.0 / dzc;
  }
  for (int k = 0; k < nz; ++k) {
    if (k >= 1) t.ta[k] = t.rhow[k - 1] * t.rdzc[k - 1] / dz[k];
    if (k + 1 < nz) t.tc[k] = t.rhow[k] * t.rdzc[k] / dz[k];
  }
  return t;
}

std::vector<double> modified_wavenumbers(int n, int count, double h) {
  std::vector<double> lam(count);
  const double pi = 3.14159265358979323846;
  for (int m = 0; m < count; ++m) {
    const double s = std::sin(pi * (double)m / (double)n);
    lam[m] = 4.0 / (h * h) * s * s;
  }
  return lam;
}

std::vector<double> twiddles(int n) {
  std::vector<double> tw(2 * (size_t)n);
  const double pi = 3.14159265358979323846;
  for (int t = 0; t < n; ++t) {
    const double ang = 2.0 * pi * (double)t / (double)n;
    tw[2 * (size_t)t] = std::cos(ang);
    tw[2 * (size_t)t + 1] = -std::sin(ang);
  }
  // exact values at the quarter points
  if (n % 4 == 0) {
    tw[2 * (size_t)(n / 4)] = 0.0;
    tw[2 * (size_t)(n / 4) + 1] = -1.0;
    tw[2 * (size_t)(3 * n / 4)] = 0.0;
    tw[2 * (size_t)(3 * n / 4) + 1] = 1.0;
  }
  if (n % 2 == 0) {
    tw[2 * (size_t)(n / 2)] = -1.0;
    tw[2 * (size_t)(n / 2) + 1] = 0.0;
  }
  return tw;
}

void div_magic(unsigned d, unsigned& mul, int& shift) {
  int l = 0;
  while ((1ull << l) < d) ++l;
  shift = l;
  mul = (unsigned)((((1ull << l) - d) << 32) / d + 1);
}

void face_weights(int nz, const double* dz, std::vector<double>& za, std::vector<double>& zb) {
  za.assign(nz > 0 ? nz : 0, 0.0);
  zb.assign(nz > 0 ? nz : 0, 0.0);
  for (int k = 0; k + 1 < nz; ++k) {
    const double s = dz[k] + dz[k + 1];
    za[k] = dz[k + 1] / s;
    zb[k] = dz[k] / s;
  }
}

int krylov_batch(double rel, double rel_prev, int done, double tol, int cap) {
  if (cap < 1) cap = 1;
  if (!(done >= 1) || !(rel > 0.0) || !(rel_prev > 0.0)) return 1;
  const double rate = std::pow(rel / rel_prev, 1.0 / done);
  if (!(rate > 0.0 && rate < 1.0)) return 1;
  if (!(tol > 0.0)) return cap;
  // (a count that is whole up to rounding is not rounded up)
  const double want = std::ceil(std::log(tol / rel) / std::log(rate) - 1e-9);
  if (!(want >= 1.0)) return 1;
  return want >= (double)cap ? cap : (int)want;
}

}  // namespace monc
