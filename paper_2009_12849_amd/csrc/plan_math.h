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

}  // namespace monc
