// Kernels of the variable-density projection: preconditioned conjugate
// gradients for D_rho(G p) = D_rho(u*) with a density rho(x, y, z), the
// non-separable problem on which the FFT solve is only an approximate
// inverse (the paper's Sec. 4 sets the FFT solver beside a Krylov solver;
// Sec. 5 proposes a preconditioner built from the problem's structure and a
// mixed-precision solver with a double-precision restart).
//
// Preconditioner: M^-1 = Lbar^-1, Lbar the separable operator with the
// plan's rho0(z), solved spectrally. Both D_rho G and Lbar are
// -D (face density) G, so their energies p^T A p differ only in the face
// density that weighs each face's |G p|^2: the preconditioned operator's
// condition is at most max(rho_face / rho0) / min(rho_face / rho0) on every
// grid (12 iterations at +-30 % density to a relative residual of 1e-10,
// from 16 x 32 to 256^2 points a level). A symmetric density scaling
// S Lbar^-1 S, S = diag(sqrt(rho0 / rho)), saved a few iterations on square
// domains but loses that bound: G(S p) carries p G(S), which dominates for
// the lowest modes of a long domain (16 x 1024 x 6, dy = 57 m: no
// convergence in 200 iterations), so it is not used.
//
// All vectors are FP64 (nz, ny, nx) fields; the preconditioned residual z is
// in the plan's storage type (ZT). Face densities come from rho on the fly:
//   rx = (rho_i + rho_{i+1})/2, ry = (rho_j + rho_{j+1})/2 (periodic),
//   rz_k = za_k rho_k + zb_k rho_{k+1}, za_k = dz_{k+1}/(dz_k + dz_{k+1}),
//   zb_k = dz_k/(dz_k + dz_{k+1}) (0 on the lid).
// A workgroup of kVarBlock threads takes a 2-D tile of kVarSpan points of a
// level, min(nx, 256) wide (kVarPts per thread at stride kVarBlock in the
// tile, coalesced along rows). The stencil
// kernels (divergence, operator) walk them up a group of kVarLevels levels
// (blockIdx.y), keeping the column's values of the levels below and above in
// registers, so only the x and y neighbours come through the caches; the
// pointwise kernels take one level per workgroup (more, shorter workgroups
// stream faster). For even nx the operator works on pairs of adjacent x
// points with 16-byte loads (k_var_apply2).
// Inner products are weighted by dz_k (the weight that makes D_rho G
// self-adjoint); each workgroup writes its partial sum and a one-workgroup
// kernel adds the partials in a fixed order, so results are deterministic.
// Loads are unconditional (a point past the level reads point 0, a missing
// level reads its own) and the results selected, so that all loads of a
// thread's points issue together.
#include <hip/hip_runtime.h>

#include "krylov.h"

namespace monc {

namespace {

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// sum over a workgroup of NT threads, valid in thread 0
template <int NT>
__device__ __forceinline__ double block_sum(double x) {
  __shared__ double part[NT / 64];
  x = wave_sum(x);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += part[w];
  return s;
}

// One thread's points: kVarPts points of a level at stride kVarBlock
// (horizontal offsets inside a level and their x and y neighbours, periodic),
// revisited on each level of the workgroup's group of kVarLevels levels.
struct Col {
  int h[kVarPts], hw[kVarPts], he[kVarPts], hs[kVarPts], hn[kVarPts];
  bool live[kVarPts];
};

// The workgroup's (point chunk, level group)
struct Blk {
  int x, y;
};
__device__ __forceinline__ Blk var_block() { return Blk{(int)blockIdx.x, (int)blockIdx.y}; }

__device__ __forceinline__ Col columns(const VarGrid& g, const Blk& bk) {
  Col c;
  const int tw = var_tile_w(g.nx), th = var_tile_h(g.nx), ntx = var_tiles_x(g.nx);
  const int tile_y = bk.x / ntx, tile_x = bk.x - tile_y * ntx;
#pragma unroll
  for (int t = 0; t < kVarPts; ++t) {
    const int sl = t * kVarBlock + threadIdx.x;          // slot in the tile
    const int rr = sl / tw, ic = tile_x * tw + (sl - rr * tw), jr = tile_y * th + rr;
    c.live[t] = rr < th && ic < g.nx && jr < g.ny;
    // outside the grid: point 0, nothing stored
    const int j = c.live[t] ? jr : 0, i = c.live[t] ? ic : 0;
    const int row = j * g.nx;
    c.h[t] = row + i;
    c.hw[t] = row + (i == 0 ? g.nx - 1 : i - 1);
    c.he[t] = row + (i == g.nx - 1 ? 0 : i + 1);
    c.hs[t] = (j == 0 ? g.ny - 1 : j - 1) * g.nx + i;
    c.hn[t] = (j == g.ny - 1 ? 0 : j + 1) * g.nx + i;
  }
  return c;
}

// levels [level_begin, level_end) of a workgroup whose group holds LV levels
template <int LV>
__device__ __forceinline__ int level_begin(const Blk& bk) { return bk.y * LV; }
template <int LV>
__device__ __forceinline__ int level_end(const VarGrid& g, const Blk& bk) { return min(g.nz, (bk.y + 1) * LV); }

__device__ __forceinline__ long long part_index() { return (long long)blockIdx.y * gridDim.x + blockIdx.x; }

__device__ __forceinline__ bool var_done(const double* scal) { return scal[kVarDone] != 0.0; }

// vertical metrics of level k
struct Lev {
  bool top, bot;      // a face above / below inside the domain
  double dz, rdz, ct, cb, za, zb, zam, zbm;
};

__device__ __forceinline__ Lev level(const VarGrid& g, int k) {
  Lev L;
  L.top = k < g.nz - 1;
  L.bot = k > 0;
  L.dz = g.dz[k];
  L.rdz = g.rdz[k];
  L.ct = L.top ? g.rdzc[k] * L.rdz : 0.0;
  L.cb = L.bot ? g.rdzc[k - 1] * L.rdz : 0.0;
  L.za = g.za[k];       // 0 on the lid
  L.zb = g.zb[k];
  L.zam = L.bot ? g.za[k - 1] : 0.0;
  L.zbm = L.bot ? g.zb[k - 1] : 0.0;
  return L;
}

}  // namespace

// r = D_rho(u*) and p = 0; partial sums of dz r^2. Each thread walks up its group of
// levels keeping rho and w of the level below in registers.
__global__ void __launch_bounds__(kVarBlock) k_var_div(VarGrid g, const double* __restrict__ u,
                                                     const double* __restrict__ v, const double* __restrict__ w,
                                                     double* __restrict__ r, double* __restrict__ p,
                                                     double* __restrict__ part) {
  const Blk bk = var_block();
  const Col c = columns(g, bk);
  const long long nh = (long long)g.nx * g.ny;
  const int k0 = level_begin<kVarLevels>(bk), k1 = level_end<kVarLevels>(g, bk);
  double rdn[kVarPts], wdn[kVarPts], rc[kVarPts];
  {
    const long long b0 = (long long)k0 * nh, bd = k0 > 0 ? b0 - nh : b0;
#pragma unroll
    for (int t = 0; t < kVarPts; ++t) {
      rdn[t] = g.rho[bd + c.h[t]];
      wdn[t] = w[bd + c.h[t]];
      rc[t] = g.rho[b0 + c.h[t]];
    }
  }
  double acc = 0.0;
  for (int k = k0; k < k1; ++k) {
    const Lev L = level(g, k);
    const long long b = (long long)k * nh, bu = L.top ? b + nh : b;
#pragma unroll
    for (int t = 0; t < kVarPts; ++t) {
      const double ru = g.rho[bu + c.h[t]], wc = w[b + c.h[t]];
      const double rxe = 0.5 * (rc[t] + g.rho[b + c.he[t]]), rxw = 0.5 * (g.rho[b + c.hw[t]] + rc[t]);
      const double ryn = 0.5 * (rc[t] + g.rho[b + c.hn[t]]), rys = 0.5 * (g.rho[b + c.hs[t]] + rc[t]);
      // top and bottom face fluxes, selected away on the lids (whatever w holds there)
      const double ft = L.top ? (L.za * rc[t] + L.zb * ru) * wc : 0.0;
      const double fb = L.bot ? (L.zam * rdn[t] + L.zbm * rc[t]) * wdn[t] : 0.0;
      const double div = (rxe * u[b + c.h[t]] - rxw * u[b + c.hw[t]]) * g.rdx +
                         (ryn * v[b + c.h[t]] - rys * v[b + c.hs[t]]) * g.rdy + (ft - fb) * L.rdz;
      if (c.live[t]) {
        r[b + c.h[t]] = div;
        p[b + c.h[t]] = 0.0;
        acc += L.dz * div * div;
      }
      rdn[t] = rc[t];
      rc[t] = ru;
      wdn[t] = wc;
    }
  }
  const double s = block_sum<kVarBlock>(acc);
  if (threadIdx.x == 0) part[part_index()] = s;
}

// q = D_rho(G d), partial sums of dz d q; d and rho of the levels below and
// above stay in registers as the thread walks up
__global__ void __launch_bounds__(kVarBlock) k_var_apply(VarGrid g, const double* __restrict__ scal,
                                                       const double* __restrict__ d, double* __restrict__ q,
                                                       double* __restrict__ part) {
  if (var_done(scal)) return;
  const Blk bk = var_block();
  const Col c = columns(g, bk);
  const long long nh = (long long)g.nx * g.ny;
  const int k0 = level_begin<kVarLevels>(bk), k1 = level_end<kVarLevels>(g, bk);
  double ddn[kVarPts], rdn[kVarPts], dc[kVarPts], rc[kVarPts];
  {
    const long long b0 = (long long)k0 * nh, bd = k0 > 0 ? b0 - nh : b0;
#pragma unroll
    for (int t = 0; t < kVarPts; ++t) {
      ddn[t] = d[bd + c.h[t]];
      rdn[t] = g.rho[bd + c.h[t]];
      dc[t] = d[b0 + c.h[t]];
      rc[t] = g.rho[b0 + c.h[t]];
    }
  }
  double acc = 0.0;
  for (int k = k0; k < k1; ++k) {
    const Lev L = level(g, k);
    const long long b = (long long)k * nh, bu = L.top ? b + nh : b;
#pragma unroll
    for (int t = 0; t < kVarPts; ++t) {
      const double du = d[bu + c.h[t]], ru = g.rho[bu + c.h[t]];
      const double rxe = 0.5 * (rc[t] + g.rho[b + c.he[t]]), rxw = 0.5 * (g.rho[b + c.hw[t]] + rc[t]);
      const double ryn = 0.5 * (rc[t] + g.rho[b + c.hn[t]]), rys = 0.5 * (g.rho[b + c.hs[t]] + rc[t]);
      const double rzt = L.za * rc[t] + L.zb * ru;          // 0 on the lid
      const double rzb = L.zam * rdn[t] + L.zbm * rc[t];    // 0 at k = 0
      const double a = (rxe * (d[b + c.he[t]] - dc[t]) - rxw * (dc[t] - d[b + c.hw[t]])) * g.rdx2 +
                       (ryn * (d[b + c.hn[t]] - dc[t]) - rys * (dc[t] - d[b + c.hs[t]])) * g.rdy2 +
                       rzt * (du - dc[t]) * L.ct - rzb * (dc[t] - ddn[t]) * L.cb;
      if (c.live[t]) {
        q[b + c.h[t]] = a;
        acc += L.dz * dc[t] * a;
      }
      ddn[t] = dc[t];
      dc[t] = du;
      rdn[t] = rc[t];
      rc[t] = ru;
    }
  }
  const double s = block_sum<kVarBlock>(acc);
  if (threadIdx.x == 0) part[part_index()] = s;
}

// The operator for even nx on pairs of adjacent x points with 16-byte
// loads: a workgroup's tile (var_tile_h rows of var_tile_w / 2 pairs) holds
// kVarSpan/2 pairs, two per thread at stride kVarBlock; a pair's x
// neighbours outside it are two 8-byte loads. 10 load instructions per pair
// instead of 16 for two points.
typedef double d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ d2v ld2(const double* p) { return *reinterpret_cast<const d2v*>(p); }

__global__ void __launch_bounds__(kVarBlock) k_var_apply2(VarGrid g, const double* __restrict__ scal,
                                                        const double* __restrict__ d, double* __restrict__ q,
                                                        double* __restrict__ part) {
  if (var_done(scal)) return;
  constexpr int NP = kVarPts / 2;   // pairs per thread
  const Blk bk = var_block();
  const int hx = g.nx / 2;
  const int txp = var_tile_w(g.nx) / 2, tyr = var_tile_h(g.nx), ntx = var_tiles_x(g.nx);
  const int tile_y = bk.x / ntx, tile_x = bk.x - tile_y * ntx;
  int h[NP], hw[NP], he[NP], hs[NP], hn[NP];
  bool live[NP];
#pragma unroll
  for (int t = 0; t < NP; ++t) {
    const int sl = t * kVarBlock + threadIdx.x;          // slot in the tile
    const int rr = sl / txp, pc = tile_x * txp + (sl - rr * txp), jr = tile_y * tyr + rr;
    live[t] = rr < tyr && pc < hx && jr < g.ny;
    const int j = live[t] ? jr : 0, i0 = live[t] ? 2 * pc : 0;   // outside the grid: pair 0, nothing stored
    const int row = j * g.nx;
    h[t] = row + i0;
    hw[t] = row + (i0 == 0 ? g.nx - 1 : i0 - 1);
    he[t] = row + (i0 + 2 == g.nx ? 0 : i0 + 2);
    hs[t] = (j == 0 ? g.ny - 1 : j - 1) * g.nx + i0;
    hn[t] = (j == g.ny - 1 ? 0 : j + 1) * g.nx + i0;
  }
  const long long nh = (long long)g.nx * g.ny;
  const int k0 = level_begin<kVarLevels>(bk), k1 = level_end<kVarLevels>(g, bk);
  d2v ddn[NP], rdn[NP], dc[NP], rc[NP];
  {
    const long long b0 = (long long)k0 * nh, bd = k0 > 0 ? b0 - nh : b0;
#pragma unroll
    for (int t = 0; t < NP; ++t) {
      ddn[t] = ld2(d + bd + h[t]);
      rdn[t] = ld2(g.rho + bd + h[t]);
      dc[t] = ld2(d + b0 + h[t]);
      rc[t] = ld2(g.rho + b0 + h[t]);
    }
  }
  double acc = 0.0;
  for (int k = k0; k < k1; ++k) {
    const Lev L = level(g, k);
    const long long b = (long long)k * nh, bu = L.top ? b + nh : b;
#pragma unroll
    for (int t = 0; t < NP; ++t) {
      const d2v du = ld2(d + bu + h[t]), ru = ld2(g.rho + bu + h[t]);
      const d2v dn = ld2(d + b + hn[t]), ds = ld2(d + b + hs[t]);
      const d2v rn = ld2(g.rho + b + hn[t]), rs = ld2(g.rho + b + hs[t]);
      const double dw = d[b + hw[t]], de = d[b + he[t]];
      const double rw = g.rho[b + hw[t]], re = g.rho[b + he[t]];
      d2v a;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const double dce = dc[t][e], rce = rc[t][e];
        const double dE = e ? de : dc[t][1], dW = e ? dc[t][0] : dw;
        const double rE = e ? re : rc[t][1], rW = e ? rc[t][0] : rw;
        const double rxe = 0.5 * (rce + rE), rxw = 0.5 * (rW + rce);
        const double ryn = 0.5 * (rce + rn[e]), rys = 0.5 * (rs[e] + rce);
        const double rzt = L.za * rce + L.zb * ru[e];          // 0 on the lid
        const double rzb = L.zam * rdn[t][e] + L.zbm * rce;    // 0 at k = 0
        a[e] = (rxe * (dE - dce) - rxw * (dce - dW)) * g.rdx2 + (ryn * (dn[e] - dce) - rys * (dce - ds[e])) * g.rdy2 +
               rzt * (du[e] - dce) * L.ct - rzb * (dce - ddn[t][e]) * L.cb;
      }
      if (live[t]) {
        *reinterpret_cast<d2v*>(q + b + h[t]) = a;
        acc += L.dz * (dc[t][0] * a[0] + dc[t][1] * a[1]);
      }
      ddn[t] = dc[t];
      dc[t] = du;
      rdn[t] = rc[t];
      rc[t] = ru;
    }
  }
  const double sm = block_sum<kVarBlock>(acc);
  if (threadIdx.x == 0) part[part_index()] = sm;
}

// alpha = rz/dq; p += alpha d; r -= alpha q; partial sums of dz r^2
__global__ void __launch_bounds__(kVarBlock) k_var_update(VarGrid g, const double* __restrict__ scal, int it,
                                                        double* __restrict__ p, double* __restrict__ r,
                                                        const double* __restrict__ d, const double* __restrict__ q,
                                                        double* __restrict__ part) {
  if (var_done(scal)) return;
  const double rz = scal[var_slot(it, kVarRZ)], dq = scal[var_slot(it, kVarDQ)];
  const double alpha = dq != 0.0 ? rz / dq : 0.0;
  const Blk bk = var_block();
  const Col c = columns(g, bk);
  const long long nh = (long long)g.nx * g.ny;
  double acc = 0.0;
  for (int k = level_begin<1>(bk), k1 = level_end<1>(g, bk); k < k1; ++k) {
    const long long b = (long long)k * nh;
    const double dz = g.dz[k];
#pragma unroll
    for (int t = 0; t < kVarPts; ++t) {
      const long long o = b + c.h[t];
      const double pn = p[o] + alpha * d[o];
      const double rn = r[o] - alpha * q[o];
      if (c.live[t]) {
        p[o] = pn;
        r[o] = rn;
        acc += dz * rn * rn;
      }
    }
  }
  const double s = block_sum<kVarBlock>(acc);
  if (threadIdx.x == 0) part[part_index()] = s;
}

// partial sums of dz r z (<r, z>) and, for the flexible update (FLEX),
// dz z q (<z, q>)
template <typename ZT, bool FLEX>
__global__ void __launch_bounds__(kVarBlock) k_var_dots(VarGrid g, const double* __restrict__ scal,
                                                      const double* __restrict__ r, const ZT* __restrict__ z,
                                                      const double* __restrict__ q, double* __restrict__ part0,
                                                      double* __restrict__ part1) {
  if (var_done(scal)) return;
  const Blk bk = var_block();
  const Col c = columns(g, bk);
  const long long nh = (long long)g.nx * g.ny;
  double a0 = 0.0, a1 = 0.0;
  for (int k = level_begin<1>(bk), k1 = level_end<1>(g, bk); k < k1; ++k) {
    const long long b = (long long)k * nh;
    const double dz = g.dz[k];
#pragma unroll
    for (int t = 0; t < kVarPts; ++t) {
      const long long o = b + c.h[t];
      const double zc = (double)z[o], rc = r[o];
      if (c.live[t]) a0 += dz * rc * zc;
      if constexpr (FLEX) {
        const double qc = q[o];
        if (c.live[t]) a1 += dz * zc * qc;
      }
    }
  }
  const double s0 = block_sum<kVarBlock>(a0);
  if (threadIdx.x == 0) part0[part_index()] = s0;
  if constexpr (FLEX) {
    __syncthreads();  // block_sum's LDS is reused
    const double s1 = block_sum<kVarBlock>(a1);
    if (threadIdx.x == 0) part1[part_index()] = s1;
  }
}

// d = z + beta d (beta = 0 at it = 0); flexible (Polak-Ribiere):
// beta = <z_it, r_it - r_{it-1}> / rz_{it-1} = -alpha_{it-1} <z_it, q_{it-1}> / rz_{it-1};
// otherwise (Fletcher-Reeves) beta = rz_it / rz_{it-1}
template <typename ZT, bool FLEX>
__global__ void __launch_bounds__(kVarBlock) k_var_dir(VarGrid g, const double* __restrict__ scal, int it,
                                                     const ZT* __restrict__ z, double* __restrict__ d) {
  if (var_done(scal)) return;
  double beta = 0.0;
  if (it > 0) {
    const double rzp = scal[var_slot(it - 1, kVarRZ)];
    if constexpr (FLEX) {
      const double dqp = scal[var_slot(it - 1, kVarDQ)];
      const double alpha = dqp != 0.0 ? rzp / dqp : 0.0;
      beta = rzp != 0.0 ? -alpha * scal[var_slot(it, kVarZQ)] / rzp : 0.0;
    } else {
      beta = rzp != 0.0 ? scal[var_slot(it, kVarRZ)] / rzp : 0.0;
    }
  }
  const Blk bk = var_block();
  const Col c = columns(g, bk);
  const long long nh = (long long)g.nx * g.ny;
  for (int k = level_begin<1>(bk), k1 = level_end<1>(g, bk); k < k1; ++k) {
    const long long b = (long long)k * nh;
#pragma unroll
    for (int t = 0; t < kVarPts; ++t) {
      const long long o = b + c.h[t];
      const double zc = (double)z[o];
      // d is not yet defined at it = 0
      const double dn = it > 0 ? zc + beta * d[o] : zc;
      if (c.live[t]) d[o] = dn;
    }
  }
}

// partial sums of dz p (the gauge)
__global__ void __launch_bounds__(kVarBlock) k_var_wsum(VarGrid g, const double* __restrict__ p,
                                                      double* __restrict__ part) {
  const Blk bk = var_block();
  const Col c = columns(g, bk);
  const long long nh = (long long)g.nx * g.ny;
  double acc = 0.0;
  for (int k = level_begin<1>(bk), k1 = level_end<1>(g, bk); k < k1; ++k) {
    const long long b = (long long)k * nh;
    const double dz = g.dz[k];
#pragma unroll
    for (int t = 0; t < kVarPts; ++t) {
      const double pc = p[b + c.h[t]];
      if (c.live[t]) acc += dz * pc;
    }
  }
  const double s = block_sum<kVarBlock>(acc);
  if (threadIdx.x == 0) part[part_index()] = s;
}

// p -= scal[slot] * rw: with rw = 1 / (nx ny sum dz) the dz-weighted mean
__global__ void __launch_bounds__(kVarBlock) k_var_shift(VarGrid g, const double* __restrict__ scal, int slot,
                                                       double rw, double* __restrict__ p) {
  const double m = scal[slot] * rw;
  const Blk bk = var_block();
  const Col c = columns(g, bk);
  const long long nh = (long long)g.nx * g.ny;
  for (int k = level_begin<1>(bk), k1 = level_end<1>(g, bk); k < k1; ++k) {
    const long long b = (long long)k * nh;
#pragma unroll
    for (int t = 0; t < kVarPts; ++t) {
      const double pn = p[b + c.h[t]] - m;
      if (c.live[t]) p[b + c.h[t]] = pn;
    }
  }
}

// sum of part[0 .. n) in a fixed order (one workgroup of kVarFinishBlock threads)
__device__ __forceinline__ double finish_sum(const double* __restrict__ part, long long n) {
  double acc = 0.0;
  for (long long i = threadIdx.x; i < n; i += 4 * kVarFinishBlock) {
    double a[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const long long ie = i + (long long)e * kVarFinishBlock;
      a[e] = ie < n ? part[ie] : 0.0;
    }
    acc += (a[0] + a[1]) + (a[2] + a[3]);
  }
  return block_sum<kVarFinishBlock>(acc);
}

__global__ void __launch_bounds__(kVarFinishBlock) k_var_finish(const double* __restrict__ part0,
                                                              const double* __restrict__ part1, long long n,
                                                              double* __restrict__ scal, int slot0, int slot1,
                                                              int gated) {
  if (gated && var_done(scal)) return;
  const double s0 = finish_sum(part0, n);
  if (threadIdx.x == 0) scal[slot0] = s0;
  if (part1) {
    __syncthreads();  // block_sum's LDS is reused
    const double s1 = finish_sum(part1, n);
    if (threadIdx.x == 0) scal[slot1] = s1;
  }
}

__global__ void __launch_bounds__(kVarFinishBlock) k_var_finish_rr(const double* __restrict__ part, long long n,
                                                                 double* __restrict__ scal, int it, double tol2) {
  if (var_done(scal)) return;
  const double rr = finish_sum(part, n);
  if (threadIdx.x == 0) {
    scal[var_slot(it, kVarRR)] = rr;
    scal[kVarLast] = (double)it;
    scal[kVarLastRR] = rr;
    if (!isfinite(rr)) scal[kVarDone] = 2.0;
    else if (rr <= tol2 * scal[var_slot(0, kVarRR)]) scal[kVarDone] = 1.0;
  }
}

__global__ void k_var_zero(double* __restrict__ x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
// the stencil kernels' grid (level groups of kVarLevels) and the pointwise
// kernels' grid (one level per workgroup)
static dim3 var_grid_stencil(const VarGrid& g) {
  return dim3((unsigned)var_blocks_per_level(g.nx, g.ny), (unsigned)var_level_groups(g.nz));
}
static dim3 var_grid(const VarGrid& g) { return dim3((unsigned)var_blocks_per_level(g.nx, g.ny), (unsigned)g.nz); }

void launch_var_div(const VarGrid& g, const double* u, const double* v, const double* w, double* r, double* p,
                    double* part, void* stream) {
  hipLaunchKernelGGL(k_var_div, var_grid_stencil(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, u, v, w, r, p, part);
}

void launch_var_apply(const VarGrid& g, const double* scal, const double* d, double* q, double* part, void* stream) {
  if (g.nx % 2 == 0)
    hipLaunchKernelGGL(k_var_apply2, var_grid_stencil(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, scal, d, q,
                       part);
  else
    hipLaunchKernelGGL(k_var_apply, var_grid_stencil(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, scal, d, q, part);
}

void launch_var_update(const VarGrid& g, const double* scal, int it, double* p, double* r, const double* d,
                       const double* q, double* part, void* stream) {
  hipLaunchKernelGGL(k_var_update, var_grid(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, scal, it, p, r, d, q,
                     part);
}

// the FP64 preconditioner takes the Fletcher-Reeves update, the FP32 one the
// flexible update
void launch_var_dots(const VarGrid& g, const double* scal, const double* r, const void* z, bool z64, const double* q,
                     double* part0, double* part1, void* stream) {
  if (z64)
    hipLaunchKernelGGL((k_var_dots<double, false>), var_grid(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, scal, r,
                       static_cast<const double*>(z), q, part0, part1);
  else
    hipLaunchKernelGGL((k_var_dots<float, true>), var_grid(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, scal, r,
                       static_cast<const float*>(z), q, part0, part1);
}

void launch_var_dir(const VarGrid& g, const double* scal, int it, const void* z, bool z64, double* d, void* stream) {
  if (z64)
    hipLaunchKernelGGL((k_var_dir<double, false>), var_grid(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, scal,
                       it, static_cast<const double*>(z), d);
  else
    hipLaunchKernelGGL((k_var_dir<float, true>), var_grid(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, scal, it,
                       static_cast<const float*>(z), d);
}

void launch_var_wsum(const VarGrid& g, const double* p, double* part, void* stream) {
  hipLaunchKernelGGL(k_var_wsum, var_grid(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, p, part);
}

void launch_var_shift(const VarGrid& g, const double* scal, int slot, double rw, double* p, void* stream) {
  hipLaunchKernelGGL(k_var_shift, var_grid(g), dim3(kVarBlock), 0, (hipStream_t)stream, g, scal, slot, rw, p);
}

void launch_var_finish(const double* part0, const double* part1, long long n, double* scal, int slot0, int slot1,
                       bool gated, void* stream) {
  hipLaunchKernelGGL(k_var_finish, dim3(1), dim3(kVarFinishBlock), 0, (hipStream_t)stream, part0, part1, n, scal,
                     slot0, slot1, gated ? 1 : 0);
}

void launch_var_finish_rr(const double* part, long long n, double* scal, int it, double tol2, void* stream) {
  hipLaunchKernelGGL(k_var_finish_rr, dim3(1), dim3(kVarFinishBlock), 0, (hipStream_t)stream, part, n, scal, it,
                     tol2);
}

void launch_var_zero(double* x, int n, void* stream) {
  if (n > 0) hipLaunchKernelGGL(k_var_zero, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, x, n);
}

}  // namespace monc
