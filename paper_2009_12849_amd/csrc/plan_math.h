// Host-side plan arithmetic: argument checks, vertical metrics, horizontal
// eigenvalues, FFT radix plans and twiddle tables. Pure C++ (no HIP calls),
// so every check runs before the device is touched.
#pragma once
#include <string>
#include <vector>

#include "monc_types.h"

namespace monc {

// Returns 0 if the arguments describe a valid plan, else a MONC_E* code and a
// message in `err`.
int check_plan_args(int nx, int ny, int nz, double dx, double dy, const double* dz, const double* rho0,
                    int dtype, std::string& err);

// n = 2^a 3^b -> radix sequence (8s first, then one 4 or 2, then 3s).
// Returns false if n has another prime factor or needs too many passes.
bool radix_plan(int n, FftPlan& fp);

// Threads per transform for `elems` elements per thread; checks that every
// pass fits the per-thread butterfly budget of the runtime-length kernels
// (kGenericElems elements).
bool fft_threads(FftPlan& fp, int elems);

struct VerticalTables {
  std::vector<double> rho0, rhow, rdz, rdzc, dz, ta, tc;
  double rH = 0.0;
};

// Face density rhow_k on the top face of cell k (linear interpolation in z
// between the centres), reciprocal spacings, and the tridiagonal
// off-diagonals a_k = rhow_{k-1}/(dz_k dzc_{k-1}), c_k = rhow_k/(dz_k dzc_k).
VerticalTables vertical_tables(int nz, const double* dz, const double* rho0);

// Multiplier and shift for x / d by multiplication, 0 <= x < 2^31, d >= 1:
// shift = ceil(log2 d), mul = floor(2^32 (2^shift - d) / d) + 1, and then
// x / d = (umulhi(x, mul) + x) >> shift.
void div_magic(unsigned d, unsigned& mul, int& shift);

// lam(m) = (4/h^2) sin^2(pi m / n), m = 0 .. count-1.
std::vector<double> modified_wavenumbers(int n, int count, double h);

// exp(-2 pi i t / n), t = 0 .. n-1, as interleaved (re, im).
std::vector<double> twiddles(int n);

// Weights of the linear interpolation in z of a cell-centred quantity q to
// the top face of cell k: q_face = za_k q_k + zb_k q_{k+1} with
// za_k = dz_{k+1}/(dz_k + dz_{k+1}), zb_k = dz_k/(dz_k + dz_{k+1}); both 0 on
// the lid (k = nz-1), which has no face above.
void face_weights(int nz, const double* dz, std::vector<double>& za, std::vector<double>& zb);

// Iterations the Krylov solver queues before it next reads its status: the
// count that the convergence rate over the last `done` iterations (relative
// residual rel_prev before them, rel after) predicts to reach tol, at least 1
// and at most cap; 1 when no rate can be measured (no decrease, or rel = 0),
// cap when tol = 0.
int krylov_batch(double rel, double rel_prev, int done, double tol, int cap);

}  // namespace monc
