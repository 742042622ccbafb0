// Launchers of the projection kernels (kernels.hip).
#pragma once
#include <stddef.h>

#include "monc_types.h"

namespace monc {

// Raise the dynamic-LDS limit of every kernel to the CU's 160 KB.
void init_kernel_attributes();

// Transform lengths with a compile-time FFT kernel (others take the
// runtime-length kernels); such kernels use n/8 threads per transform (1 if
// n < 8; along y n/16 from n = 2048 on) and need blockDim = (transforms or
// columns per workgroup) * that.
bool ct_supported(int n);
// lengths with the persistent FP32 y-FFT kernel (32 elements per thread)
bool pp_supported(int n);
inline int ct_threads_host(int n) { return ct_threads_x_n(n); }
inline int ct_threads_y_host(int n, int ept) { return ct_threads_y_n(n, ept); }

// ct_n: the compile-time length, or 0 for the runtime-length kernel.
// mode 0: divergence of (u, v, w); mode 1 (float only): the FP64 residual
// D(u) - D(G p1) with the first-pass pressure p1 in io.s2; mode 2: the FP64
// field at io.u (nz, ny, nx), rounded to the storage type.
void launch_xfwd(const LaunchArgs& a, int grid, int block, size_t lds, bool fp64, int mode, int ct_n, void* stream);
// ept: elements per thread of the compile-time kernel (8 or 16; 32 = the
// persistent FP32 kernel, whose grid covers the CUs once)
void launch_ffty(const LaunchArgs& a, int grid, int block, size_t lds, bool fp64, bool inverse, int ct_n, int ept,
                 void* stream);
// rows: rows per lane, one of kTriRows (the member's tris)
void launch_tridiag(const LaunchArgs& a, int grid, int block, size_t lds, bool fp64, int rows, bool pairs, void* stream);
// the result goes to io.p (mode 0), io.s1 (mode 1, float only: the
// correction delta) or io.s2 (mode 2, float only: the first-pass pressure)
void launch_xinv(const LaunchArgs& a, int grid, int block, size_t lds, bool fp64, int mode, int ct_n, void* stream);
// fp64: pressure from io.p (FP64); else (mixed path) p1 + delta summed in
// FP64 from io.s2 + io.s1, and written rounded to io.p. vec: points per
// thread (2 needs an even nx, 4 a multiple of 4; else 1)
// red: also the per-level horizontal mean and max of u, v, w, p into io.stats
// (after launch_stats_init on the same stream)
void launch_grad(const LaunchArgs& a, int grid, bool fp64, int vec, bool red, void* stream);
void launch_stats_init(double* stats, int nz, void* stream);

}  // namespace monc
