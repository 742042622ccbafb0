// Kernels of the variable-density projection: preconditioned conjugate
// gradients for D_rho(G p) = D_rho(u*) with a density rho(x, y, z), the
// non-separable problem on which the FFT solve is only an approximate
// inverse (the paper's Sec. 4 sets the FFT solver beside a Krylov solver;
// Sec. 5 proposes a preconditioner built from the problem's structure and a
// mixed-precision solver with a double-precision restart).
//
// All vectors are FP64 (nz, ny, nx) fields; the preconditioned residual z is
// in the plan's storage type (ZT). Face densities come from rho on the fly:
//   rx = (rho_i + rho_{i+1})/2, ry = (rho_j + rho_{j+1})/2 (periodic),
//   rz_k = za_k rho_k + zb_k rho_{k+1}, za_k = dz_{k+1}/(dz_k + dz_{k+1}),
//   zb_k = dz_k/(dz_k + dz_{k+1}) (0 on the lid).
// A workgroup of kVarBlock threads takes kVarSpan consecutive points of one
// level (blockIdx.y = level), kVarPts per thread at stride kVarBlock, so
// accesses stay coalesced and the level's vertical metrics are uniform.
// Inner products are weighted by dz_k (the weight that makes D_rho G
// self-adjoint); each workgroup writes its partial sum and a one-workgroup
// kernel adds the partials in a fixed order, so results are deterministic.
#include <hip/hip_runtime.h>

#include "krylov.h"

namespace monc {

namespace {

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// sum over the workgroup (kVarBlock threads), valid in thread 0
__device__ __forceinline__ double block_sum(double x) {
  __shared__ double part[kVarBlock / 64];
  x = wave_sum(x);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
#pragma unroll
    for (int w = 0; w < kVarBlock / 64; ++w) s += part[w];
  return s;
}

struct Pt {
  long long o;   // offset of the point
  long long ow, oe, os, on;  // x and y neighbours (periodic)
  bool live;
};

__device__ __forceinline__ Pt point(const VarGrid& g, int t) {
  Pt p;
  const int nh = g.nx * g.ny;
  const int idx = blockIdx.x * kVarSpan + t * kVarBlock + threadIdx.x;
  p.live = idx < nh;
  const int id = p.live ? idx : 0;
  const int j = id / g.nx, i = id - j * g.nx;
  const long long row = (long long)blockIdx.y * nh + (long long)j * g.nx;
  p.o = row + i;
  p.ow = row + (i == 0 ? g.nx - 1 : i - 1);
  p.oe = row + (i == g.nx - 1 ? 0 : i + 1);
  p.os = (long long)blockIdx.y * nh + (long long)(j == 0 ? g.ny - 1 : j - 1) * g.nx + i;
  p.on = (long long)blockIdx.y * nh + (long long)(j == g.ny - 1 ? 0 : j + 1) * g.nx + i;
  return p;
}

__device__ __forceinline__ long long part_index() { return (long long)blockIdx.y * gridDim.x + blockIdx.x; }

}  // namespace

// r = D_rho(u*), p = 0, partial sums of dz r^2
__global__ void __launch_bounds__(kVarBlock) k_var_div(VarGrid g, const double* __restrict__ u,
                                                     const double* __restrict__ v, const double* __restrict__ w,
                                                     double* __restrict__ r, double* __restrict__ p,
                                                     double* __restrict__ part) {
  const int k = blockIdx.y;
  const long long pl = (long long)g.nx * g.ny;
  const bool top = k < g.nz - 1, bot = k > 0;
  const double rdz = g.rdz[k], dz = g.dz[k];
  const double za = g.za[k], zb = g.zb[k];
  const double zam = bot ? g.za[k - 1] : 0.0, zbm = bot ? g.zb[k - 1] : 0.0;
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < kVarPts; ++t) {
    const Pt q = point(g, t);
    if (!q.live) continue;
    const double rc = g.rho[q.o];
    const double rxe = 0.5 * (rc + g.rho[q.oe]), rxw = 0.5 * (g.rho[q.ow] + rc);
    const double ryn = 0.5 * (rc + g.rho[q.on]), rys = 0.5 * (g.rho[q.os] + rc);
    double div = (rxe * u[q.o] - rxw * u[q.ow]) * g.rdx + (ryn * v[q.o] - rys * v[q.os]) * g.rdy;
    double ft = 0.0, fb = 0.0;
    if (top) ft = (za * rc + zb * g.rho[q.o + pl]) * w[q.o];
    if (bot) fb = (zam * g.rho[q.o - pl] + zbm * rc) * w[q.o - pl];
    div += (ft - fb) * rdz;
    r[q.o] = div;
    p[q.o] = 0.0;
    acc += dz * div * div;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[part_index()] = s;
}

// q = D_rho(G d), partial sums of dz d q
__global__ void __launch_bounds__(kVarBlock) k_var_apply(VarGrid g, const double* __restrict__ d,
                                                       double* __restrict__ q, double* __restrict__ part) {
  const int k = blockIdx.y;
  const long long pl = (long long)g.nx * g.ny;
  const bool top = k < g.nz - 1, bot = k > 0;
  const double rdz = g.rdz[k], dz = g.dz[k];
  const double ct = top ? g.rdzc[k] * rdz : 0.0, cb = bot ? g.rdzc[k - 1] * rdz : 0.0;
  const double za = g.za[k], zb = g.zb[k];
  const double zam = bot ? g.za[k - 1] : 0.0, zbm = bot ? g.zb[k - 1] : 0.0;
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < kVarPts; ++t) {
    const Pt x = point(g, t);
    if (!x.live) continue;
    const double rc = g.rho[x.o], dc = d[x.o];
    const double rxe = 0.5 * (rc + g.rho[x.oe]), rxw = 0.5 * (g.rho[x.ow] + rc);
    const double ryn = 0.5 * (rc + g.rho[x.on]), rys = 0.5 * (g.rho[x.os] + rc);
    double a = (rxe * (d[x.oe] - dc) - rxw * (dc - d[x.ow])) * g.rdx2 +
               (ryn * (d[x.on] - dc) - rys * (dc - d[x.os])) * g.rdy2;
    if (top) a += (za * rc + zb * g.rho[x.o + pl]) * (d[x.o + pl] - dc) * ct;
    if (bot) a -= (zam * g.rho[x.o - pl] + zbm * rc) * (dc - d[x.o - pl]) * cb;
    q[x.o] = a;
    acc += dz * dc * a;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[part_index()] = s;
}

// alpha = rz/dq; p += alpha d; r -= alpha q; partial sums of dz r^2
__global__ void __launch_bounds__(kVarBlock) k_var_update(VarGrid g, const double* __restrict__ scal, int it,
                                                        double* __restrict__ p, double* __restrict__ r,
                                                        const double* __restrict__ d, const double* __restrict__ q,
                                                        double* __restrict__ part) {
  const double rz = scal[var_slot(it, kVarRZ)], dq = scal[var_slot(it, kVarDQ)];
  const double alpha = dq != 0.0 ? rz / dq : 0.0;
  const double dz = g.dz[blockIdx.y];
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < kVarPts; ++t) {
    const Pt x = point(g, t);
    if (!x.live) continue;
    p[x.o] += alpha * d[x.o];
    const double rn = r[x.o] - alpha * q[x.o];
    r[x.o] = rn;
    acc += dz * rn * rn;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[part_index()] = s;
}

// partial sums of dz r z and dz z q (the second for the flexible update)
template <typename ZT>
__global__ void __launch_bounds__(kVarBlock) k_var_dots(VarGrid g, const double* __restrict__ r,
                                                      const ZT* __restrict__ z, const double* __restrict__ q,
                                                      double* __restrict__ part0, double* __restrict__ part1) {
  const double dz = g.dz[blockIdx.y];
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int t = 0; t < kVarPts; ++t) {
    const Pt x = point(g, t);
    if (!x.live) continue;
    const double zc = (double)z[x.o];
    a0 += dz * r[x.o] * zc;
    a1 += dz * zc * q[x.o];
  }
  const double s0 = block_sum(a0);
  __syncthreads();  // block_sum's LDS is reused
  const double s1 = block_sum(a1);
  if (threadIdx.x == 0) {
    part0[part_index()] = s0;
    part1[part_index()] = s1;
  }
}

// d = z + beta d, beta = -alpha_{it-1} <z_it, q_{it-1}> / rz_{it-1} (0 at it = 0)
template <typename ZT>
__global__ void __launch_bounds__(kVarBlock) k_var_dir(VarGrid g, const double* __restrict__ scal, int it,
                                                     const ZT* __restrict__ z, double* __restrict__ d) {
  double beta = 0.0;
  if (it > 0) {
    const double rzp = scal[var_slot(it - 1, kVarRZ)], dqp = scal[var_slot(it - 1, kVarDQ)];
    const double alpha = dqp != 0.0 ? rzp / dqp : 0.0;
    beta = rzp != 0.0 ? -alpha * scal[var_slot(it, kVarZQ)] / rzp : 0.0;
  }
#pragma unroll
  for (int t = 0; t < kVarPts; ++t) {
    const Pt x = point(g, t);
    if (!x.live) continue;
    d[x.o] = (double)z[x.o] + (it > 0 ? beta * d[x.o] : 0.0);
  }
}

// partial sums of dz p (the gauge)
__global__ void __launch_bounds__(kVarBlock) k_var_wsum(VarGrid g, const double* __restrict__ p,
                                                      double* __restrict__ part) {
  const double dz = g.dz[blockIdx.y];
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < kVarPts; ++t) {
    const Pt x = point(g, t);
    if (x.live) acc += dz * p[x.o];
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[part_index()] = s;
}

// p -= scal[slot] * rw: with rw = 1 / (nx ny sum dz) the dz-weighted mean
__global__ void __launch_bounds__(kVarBlock) k_var_shift(VarGrid g, const double* __restrict__ scal, int slot,
                                                       double rw, double* __restrict__ p) {
  const double m = scal[slot] * rw;
#pragma unroll
  for (int t = 0; t < kVarPts; ++t) {
    const Pt x = point(g, t);
    if (x.live) p[x.o] -= m;
  }
}

// scal[slot] = sum of part[0 .. n) in a fixed order (one workgroup)
__global__ void __launch_bounds__(kVarBlock) k_var_finish(const double* __restrict__ part, long long n,
                                                        double* __restrict__ scal, int slot) {
  double acc = 0.0;
  for (long long i = threadIdx.x; i < n; i += kVarBlock) acc += part[i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) scal[slot] = s;
}

__global__ void k_var_zero(double* __restrict__ x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
static dim3 var_grid(const VarGrid& g) { return dim3((unsigned)var_blocks_per_level(g.nx, g.ny), (unsigned)g.nz); }

void launch_var_div(const VarGrid& g, const double* u, const double* v, const double* w, double* r, double* p,
                    double* part, void* stream) {
  hipLaunchKernelGGL(k_var_div, var_grid(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, u, v, w, r, p, part);
}

void launch_var_apply(const VarGrid& g, const double* d, double* q, double* part, void* stream) {
  hipLaunchKernelGGL(k_var_apply, var_grid(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, d, q, part);
}

void launch_var_update(const VarGrid& g, const double* scal, int it, double* p, double* r, const double* d,
                       const double* q, double* part, void* stream) {
  hipLaunchKernelGGL(k_var_update, var_grid(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, scal, it, p, r, d, q,
                     part);
}

void launch_var_dots(const VarGrid& g, const double* r, const void* z, bool z64, const double* q, double* part0,
                     double* part1, void* stream) {
  if (z64)
    hipLaunchKernelGGL(k_var_dots<double>, var_grid(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, r,
                       static_cast<const double*>(z), q, part0, part1);
  else
    hipLaunchKernelGGL(k_var_dots<float>, var_grid(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, r,
                       static_cast<const float*>(z), q, part0, part1);
}

void launch_var_dir(const VarGrid& g, const double* scal, int it, const void* z, bool z64, double* d, void* stream) {
  if (z64)
    hipLaunchKernelGGL(k_var_dir<double>, var_grid(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, scal, it,
                       static_cast<const double*>(z), d);
  else
    hipLaunchKernelGGL(k_var_dir<float>, var_grid(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, scal, it,
                       static_cast<const float*>(z), d);
}

void launch_var_wsum(const VarGrid& g, const double* p, double* part, void* stream) {
  hipLaunchKernelGGL(k_var_wsum, var_grid(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, p, part);
}

void launch_var_shift(const VarGrid& g, const double* scal, int slot, double rw, double* p, void* stream) {
  hipLaunchKernelGGL(k_var_shift, var_grid(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, scal, slot, rw, p);
}

void launch_var_finish(const double* part, long long n, double* scal, int slot, void* stream) {
  hipLaunchKernelGGL(k_var_finish, dim3(1), dim3(kVarBlock), 0, (hipStream_t)stream, part, n, scal, slot);
}

void launch_var_zero(double* x, int n, void* stream) {
  if (n > 0) hipLaunchKernelGGL(k_var_zero, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, x, n);
}

}  // namespace monc
