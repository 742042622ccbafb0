// HIP kernels of the pressure projection for gfx950 (wave64, LDS-staged).
//
// Phases of one projection (the FFT pressure solver of the paper's Sec. 4:
// forward FFT, vertical ODE per wavenumber in Fourier space, backward FFT):
//   xfwd     divergence D(u*) (or the FP64 residual D(u*) - D(G p1) of the
//            mixed path) computed straight into the first radix pass of the
//            x-direction real FFT; two real rows ride in one complex
//            transform and are separated afterwards
//   ffty     y-direction complex FFT of every (level, m) column
//   tridiag  FP64 tridiagonal solve in z of every (m, n) column, partitioned
//            over lanes, (0,0) column with the gauge
//   xinv     x-direction complex-to-real FFT, writes p (or p1 + delta)
//   grad     pressure-gradient correction u -= G p, w lid = 0
//
// The FFT phases exist twice: with the transform length fixed at compile
// time (CtFft, for the lengths listed in kernels.h) and with a runtime length
// (fft_lds) for every other 2^a 3^b length.
//
// Every kernel serves a group of members: blockIdx.x is mapped to a member
// through LaunchArgs::block_start, and each member's sizes and tables come
// from its MemberDesc.
#include <hip/hip_runtime.h>

#include "fft_core.h"
#include "kernels.h"

namespace monc {

__device__ __forceinline__ int find_member(const LaunchArgs& a, int b) {
  int m = 0;
  while (m + 1 < a.nmem && b >= a.block_start[m + 1]) ++m;
  return m;
}

// Load through a global-address-space pointer (table pointers held in a
// descriptor are generic, which would otherwise become flat loads).
template <typename T>
__device__ __forceinline__ T ldg(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}

// x / d for 0 <= x < 2^31 with a precomputed multiplier: q = (umulhi(x, mul)
// + x) >> shift, where shift = ceil(log2 d) and mul = floor(2^32 (2^shift -
// d) / d) + 1 (division by invariant integers by multiplication, the variant
// with the extra addition, valid for every 31-bit dividend).
__device__ __forceinline__ unsigned fast_div(int x, unsigned mul, int shift) {
  const unsigned long long t = __umulhi((unsigned)x, mul);
  return (unsigned)((t + (unsigned)x) >> shift);
}

// Workgroups go to the 8 XCDs round-robin (XCD = blockIdx mod 8), each XCD
// with its own L2. Remap a member's local block index so that every XCD
// works through one contiguous range of tiles: neighbouring rows and levels,
// which the stencils read twice, then meet in the same L2. Applies when the
// member's first block sits on XCD 0; the tail beyond a multiple of 8 keeps
// its index.
__device__ __forceinline__ int xcd_local_block(const LaunchArgs& a, int mi) {
  const int start = a.block_start[mi];
  const int lb = blockIdx.x - start;
  if (start & 7) return lb;
  const int full = (a.block_start[mi + 1] - start) & ~7;
  if (lb >= full) return lb;
  return (lb & 7) * (full >> 3) + (lb >> 3);
}

// A descriptor with a skip flag drives the Krylov solver's preconditioner:
// once the solver has converged the flag is set and the solve's remaining
// launches return at once (whole workgroups, before any barrier).
__device__ __forceinline__ bool skipped(const MemberDesc& d) { return d.skip && *d.skip != 0.0; }

// ---------------------------------------------------------------------------
// per-row context of the stencils: offsets of the neighbouring rows and the
// vertical metrics of the row's level
// ---------------------------------------------------------------------------
struct RowCtx {
  long long off;    // row (k, j)
  long long soff;   // row (k, j-1)
  long long noff;   // row (k, j+1)
  long long plane;  // ny * nx
  int k;
  bool top;         // k < nz-1: a w face above
  bool bot;         // k > 0: a w face below
  double rho0, rhow, rhowm, rdz, rdzc, rdzcm;
  float rho0f, rhowf, rhowmf, rdzf;
};

__device__ __forceinline__ RowCtx make_row(const MemberDesc& d, long long row, bool valid) {
  RowCtx c;
  const int ny = d.ny, nz = d.nz;
  const long long r = valid ? row : 0;
  // rows (ny nz of them) and their level and row index fit 32 bits
  const int k = (int)r / ny;
  const int j = (int)r - k * ny;
  c.k = k;
  c.off = r * d.nx;
  c.soff = ((long long)k * ny + (j == 0 ? ny - 1 : j - 1)) * d.nx;
  c.noff = ((long long)k * ny + (j == ny - 1 ? 0 : j + 1)) * d.nx;
  c.plane = (long long)ny * d.nx;
  c.top = k < nz - 1;
  c.bot = k > 0;
  const int km = c.bot ? k - 1 : k;
  c.rho0 = ldg(d.rho0 + k);
  c.rdz = ldg(d.rdz + k);
  c.rhow = ldg(d.rhow + k);    // 0 on the lid row
  c.rdzc = ldg(d.rdzc + k);    // 0 on the lid row
  c.rhowm = c.bot ? ldg(d.rhow + km) : 0.0;
  c.rdzcm = c.bot ? ldg(d.rdzc + km) : 0.0;
  c.rho0f = ldg(d.rho0f + k);
  c.rdzf = ldg(d.rdzf + k);
  c.rhowf = ldg(d.rhowf + k);
  c.rhowmf = c.bot ? ldg(d.rhowf + km) : 0.0f;
  return c;
}

// Values known to be equal on every lane of a wave, moved to scalar
// registers (readfirstlane): a row context is per transform, and when a
// transform's thread count is a multiple of 64 it spans whole waves, so
// vector registers would hold the same value 64 times.
__device__ __forceinline__ int wuni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ long long wuni(long long x) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)x);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)x >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double wuni(double x) { return __longlong_as_double(wuni(__double_as_longlong(x))); }
__device__ __forceinline__ float wuni(float x) { return __int_as_float(wuni(__float_as_int(x))); }
__device__ __forceinline__ RowCtx wuni(const RowCtx& c) {
  RowCtx r;
  r.off = wuni(c.off);
  r.soff = wuni(c.soff);
  r.noff = wuni(c.noff);
  r.plane = wuni(c.plane);
  r.k = wuni(c.k);
  r.top = wuni((int)c.top) != 0;
  r.bot = wuni((int)c.bot) != 0;
  r.rho0 = wuni(c.rho0);
  r.rhow = wuni(c.rhow);
  r.rhowm = wuni(c.rhowm);
  r.rdz = wuni(c.rdz);
  r.rdzc = wuni(c.rdzc);
  r.rdzcm = wuni(c.rdzcm);
  r.rho0f = wuni(c.rho0f);
  r.rhowf = wuni(c.rhowf);
  r.rhowmf = wuni(c.rhowmf);
  r.rdzf = wuni(c.rdzf);
  return r;
}

template <typename T>
__device__ __forceinline__ T div_at(const MemberDesc& d, const RowCtx& c, const T* __restrict__ u,
                                    const T* __restrict__ v, const T* __restrict__ w, int i);

template <>
__device__ __forceinline__ double div_at<double>(const MemberDesc& d, const RowCtx& c, const double* __restrict__ u,
                                                 const double* __restrict__ v, const double* __restrict__ w, int i) {
  const int im = (i == 0) ? d.nx - 1 : i - 1;
  const double hor = (u[c.off + i] - u[c.off + im]) * d.rdx + (v[c.off + i] - v[c.soff + i]) * d.rdy;
  const double ft = c.top ? c.rhow * w[c.off + i] : 0.0;
  const double fb = c.bot ? c.rhowm * w[c.off - c.plane + i] : 0.0;
  return c.rho0 * hor + (ft - fb) * c.rdz;
}

template <>
__device__ __forceinline__ float div_at<float>(const MemberDesc& d, const RowCtx& c, const float* __restrict__ u,
                                               const float* __restrict__ v, const float* __restrict__ w, int i) {
  const int im = (i == 0) ? d.nx - 1 : i - 1;
  const float hor = (u[c.off + i] - u[c.off + im]) * d.rdxf + (v[c.off + i] - v[c.soff + i]) * d.rdyf;
  const float ft = c.top ? c.rhowf * w[c.off + i] : 0.0f;
  const float fb = c.bot ? c.rhowmf * w[c.off - c.plane + i] : 0.0f;
  return c.rho0f * hor + (ft - fb) * c.rdzf;
}

// Global-address-space views of a generic pointer (the scratch fields and
// the output pressure come from a by-value argument struct, so the compiler
// cannot infer their address space and would emit flat accesses).
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// FP64 operator L p1 = D(G p1) at one point from the float first-pass
// pressure p1 and its six neighbours (pE, pW along x, pN, pS along y, pU, pD
// along z; pU, pD ignored on the lid and bottom rows).
__device__ __forceinline__ double lap_at(const MemberDesc& d, const RowCtx& c, double p0, double pE, double pW,
                                         double pN, double pS, double pU, double pD) {
  const double gxe = (pE - p0) * d.rdx, gxw = (p0 - pW) * d.rdx;
  const double gyn = (pN - p0) * d.rdy, gys = (p0 - pS) * d.rdy;
  const double ft = c.top ? c.rhow * ((pU - p0) * c.rdzc) : 0.0;
  const double fb = c.bot ? c.rhowm * ((p0 - pD) * c.rdzcm) : 0.0;
  return c.rho0 * ((gxe - gxw) * d.rdx + (gyn - gys) * d.rdy) + (ft - fb) * c.rdz;
}

// FP64 divergence D(u*) of float fields at one point
__device__ __forceinline__ double div64_at(const MemberDesc& d, const RowCtx& c, const float* __restrict__ u,
                                           const float* __restrict__ v, const float* __restrict__ w, int i) {
  const int im = (i == 0) ? d.nx - 1 : i - 1;
  const double hor = ((double)u[c.off + i] - (double)u[c.off + im]) * d.rdx +
                     ((double)v[c.off + i] - (double)v[c.soff + i]) * d.rdy;
  const double ft = c.top ? c.rhow * (double)w[c.off + i] : 0.0;
  const double fb = c.bot ? c.rhowm * (double)w[c.off - c.plane + i] : 0.0;
  return c.rho0 * hor + (ft - fb) * c.rdz;
}

// FP64 residual r = D(u*) - L p1 of the mixed path at one point, from the
// float inputs u*, v*, w* and the first-pass pressure p1 (io.s2).
__device__ __forceinline__ double resid_at(const MemberDesc& d, const RowCtx& c, const IoPtrs& io, int i) {
  const float* __restrict__ p = io.s2;
  const int nx = d.nx;
  const int im = (i == 0) ? nx - 1 : i - 1;
  const int ip = (i == nx - 1) ? 0 : i + 1;
  const double pc = p[c.off + i];
  const double pu = c.top ? (double)p[c.off + c.plane + i] : pc;
  const double pd = c.bot ? (double)p[c.off - c.plane + i] : pc;
  const double b = div64_at(d, c, reinterpret_cast<const float*>(io.u), reinterpret_cast<const float*>(io.v),
                            reinterpret_cast<const float*>(io.w), i);
  return b - lap_at(d, c, pc, p[c.off + ip], p[c.off + im], p[c.noff + i], p[c.soff + i], pu, pd);
}

// Sources of the x-forward transform: MODE 0 the divergence D(u*), MODE 1
// the mixed path's FP64 residual D(u*) - L p1, MODE 2 a given FP64 field
// (io.u) rounded to T, i.e. the spectral solve applied to an arbitrary
// right-hand side (the preconditioner of the variable-density Krylov
// solver).
template <typename T, int MODE>
__device__ __forceinline__ T source_at(const MemberDesc& d, const RowCtx& c, const IoPtrs& io, int i) {
  if constexpr (MODE == 0) {
    return div_at<T>(d, c, reinterpret_cast<const T*>(io.u), reinterpret_cast<const T*>(io.v),
                     reinterpret_cast<const T*>(io.w), i);
  } else if constexpr (MODE == 2) {
    return (T)reinterpret_cast<const double*>(io.u)[c.off + i];
  } else {
    return (T)resid_at(d, c, io, i);
  }
}

// ---------------------------------------------------------------------------
// Vector forms of the stencils: V = 16 bytes / sizeof(T) consecutive points
// of one row from 16-byte loads (rows start 16-byte aligned: nx is a
// multiple of V for every compile-time length). The x-neighbours outside
// the vector come from scalar loads (cache hits).
// ---------------------------------------------------------------------------
template <typename T> struct Vec {
  static constexpr int n = 16 / sizeof(T);
  typedef T type __attribute__((ext_vector_type(16 / sizeof(T))));
};

template <typename T>
__device__ __forceinline__ typename Vec<T>::type ldv(const T* p) {
  return *reinterpret_cast<const typename Vec<T>::type*>(p);
}

template <typename T>
__device__ __forceinline__ void stv(T* p, typename Vec<T>::type x) {
  *reinterpret_cast<typename Vec<T>::type*>(p) = x;
}

// divergence D(u) at points i0 .. i0+V-1 of a row, arithmetic in T
template <typename T>
__device__ __forceinline__ void div_vec(const MemberDesc& d, const RowCtx& c, const IoPtrs& io, int i0, T* out) {
  constexpr int V = Vec<T>::n;
  using vt = typename Vec<T>::type;
  const T* __restrict__ u = reinterpret_cast<const T*>(io.u);
  const T* __restrict__ v = reinterpret_cast<const T*>(io.v);
  const T* __restrict__ w = reinterpret_cast<const T*>(io.w);
  const bool f64 = sizeof(T) == 8;
  const T rdx = f64 ? (T)d.rdx : (T)d.rdxf, rdy = f64 ? (T)d.rdy : (T)d.rdyf;
  const T rho0 = f64 ? (T)c.rho0 : (T)c.rho0f, rdz = f64 ? (T)c.rdz : (T)c.rdzf;
  const T rhow = f64 ? (T)c.rhow : (T)c.rhowf, rhowm = f64 ? (T)c.rhowm : (T)c.rhowmf;
  const vt uc = ldv(u + c.off + i0);
  const T um = u[c.off + (i0 == 0 ? d.nx - 1 : i0 - 1)];
  const vt vc = ldv(v + c.off + i0), vs = ldv(v + c.soff + i0);
  vt wc = (vt)(T)0, wb = (vt)(T)0;
  if constexpr (sizeof(T) == 8) {
    // FP64: both w loads unconditional (level k clamped on the bottom row) so
    // they issue with the others; the lid and bottom faces are selected away
    const vt wcl = ldv(w + c.off + i0), wbl = ldv(w + c.off - (c.bot ? c.plane : 0) + i0);
#pragma unroll
    for (int e = 0; e < V; ++e) {
      wc[e] = c.top ? wcl[e] : (T)0;
      wb[e] = c.bot ? wbl[e] : (T)0;
    }
  } else {
    // FP32: the branches keep fewer loads in flight and fewer registers live,
    // which measures faster here
    if (c.top) wc = ldv(w + c.off + i0);
    if (c.bot) wb = ldv(w + c.off - c.plane + i0);
  }
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const T uw = e ? uc[e - 1] : um;
    out[e] = rho0 * ((uc[e] - uw) * rdx + (vc[e] - vs[e]) * rdy) + (rhow * wc[e] - rhowm * wb[e]) * rdz;
  }
}

// Both rows of a pair (k, j) and (k, j+1) of one level: row j's v is row j+1's
// southern neighbour, so 11 loads serve the two rows instead of 12. The
// arithmetic is div_vec's, term for term.
template <typename T>
__device__ __forceinline__ void div_pair_vec(const MemberDesc& d, const RowCtx& c0, const RowCtx& c1,
                                             const IoPtrs& io, int i0, T* out0, T* out1) {
  constexpr int V = Vec<T>::n;
  using vt = typename Vec<T>::type;
  const T* __restrict__ u = reinterpret_cast<const T*>(io.u);
  const T* __restrict__ v = reinterpret_cast<const T*>(io.v);
  const T* __restrict__ w = reinterpret_cast<const T*>(io.w);
  const bool f64 = sizeof(T) == 8;
  const T rdx = f64 ? (T)d.rdx : (T)d.rdxf, rdy = f64 ? (T)d.rdy : (T)d.rdyf;
  // one level: both rows share the vertical coefficients and lid flags
  const T rho0 = f64 ? (T)c0.rho0 : (T)c0.rho0f, rdz = f64 ? (T)c0.rdz : (T)c0.rdzf;
  const T rhow = f64 ? (T)c0.rhow : (T)c0.rhowf, rhowm = f64 ? (T)c0.rhowm : (T)c0.rhowmf;
  const int iw = (i0 == 0) ? d.nx - 1 : i0 - 1;
  const vt u0 = ldv(u + c0.off + i0), u1 = ldv(u + c1.off + i0);
  const T um0 = u[c0.off + iw], um1 = u[c1.off + iw];
  const vt vs = ldv(v + c0.soff + i0), v0 = ldv(v + c0.off + i0), v1 = ldv(v + c1.off + i0);
  vt wc0 = (vt)(T)0, wb0 = (vt)(T)0, wc1 = (vt)(T)0, wb1 = (vt)(T)0;
  if constexpr (sizeof(T) == 8) {
    const long long bo = c0.bot ? c0.plane : 0;
    const vt a0 = ldv(w + c0.off + i0), a1 = ldv(w + c1.off + i0);
    const vt b0 = ldv(w + c0.off - bo + i0), b1 = ldv(w + c1.off - bo + i0);
#pragma unroll
    for (int e = 0; e < V; ++e) {
      wc0[e] = c0.top ? a0[e] : (T)0;
      wc1[e] = c0.top ? a1[e] : (T)0;
      wb0[e] = c0.bot ? b0[e] : (T)0;
      wb1[e] = c0.bot ? b1[e] : (T)0;
    }
  } else {
    if (c0.top) {
      wc0 = ldv(w + c0.off + i0);
      wc1 = ldv(w + c1.off + i0);
    }
    if (c0.bot) {
      wb0 = ldv(w + c0.off - c0.plane + i0);
      wb1 = ldv(w + c1.off - c0.plane + i0);
    }
  }
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const T uw0 = e ? u0[e - 1] : um0, uw1 = e ? u1[e - 1] : um1;
    out0[e] = rho0 * ((u0[e] - uw0) * rdx + (v0[e] - vs[e]) * rdy) + (rhow * wc0[e] - rhowm * wb0[e]) * rdz;
    out1[e] = rho0 * ((u1[e] - uw1) * rdx + (v1[e] - v0[e]) * rdy) + (rhow * wc1[e] - rhowm * wb1[e]) * rdz;
  }
}

typedef float f4v __attribute__((ext_vector_type(4)));
template <int W> using fwv = float __attribute__((ext_vector_type(W)));

template <int W>
__device__ __forceinline__ fwv<W> ldw(const float* p) {
  return *reinterpret_cast<const fwv<W>*>(p);
}

// FP64 residual D(u*) - L p1 at points i0 .. i0+W-1 of a row from the loaded
// neighbourhood (float data; pc: p1 of the row, pn/ps: rows j +- 1, pu/pd:
// levels k +- 1, pe/pw: x-neighbours outside the vector, um: u west of the
// vector; pu/pd, wc/wb ignored on the lid and bottom rows).
// The same terms as div64_at - lap_at with the row's coefficients multiplied
// out once (rho0/dx, rho0/dx^2, ...) and every pressure difference taken
// before it is scaled: one FP64 fused multiply-add per term. The callers pass
// wc = 0 and pu = pc on the lid row, wb = 0 and pd = pc on the bottom row,
// where the row's rhow (lid) and rhowm (bottom) are 0 as well. A point's
// value does not depend on W.
template <int W>
__device__ __forceinline__ void resid_core(const MemberDesc& d, const RowCtx& c, fwv<W> pc, fwv<W> pn, fwv<W> ps,
                                           fwv<W> pu, fwv<W> pd, float pw, float pe, fwv<W> uc, float um,
                                           fwv<W> vc, fwv<W> vs, fwv<W> wc, fwv<W> wb, float* out) {
  const double bx = c.rho0 * d.rdx, by = c.rho0 * d.rdy;      // D(u*) horizontal
  const double wt = c.rdz * c.rhow, wm = c.rdz * c.rhowm;     // D(u*) vertical
  const double ax = bx * d.rdx, ay = by * d.rdy;              // L p1 horizontal
  const double cu = wt * c.rdzc, cd = wm * c.rdzcm;           // L p1 vertical
#pragma unroll
  for (int e = 0; e < W; ++e) {
    const double uW = (e > 0) ? (double)uc[e > 0 ? e - 1 : 0] : (double)um;
    const double p0 = pc[e];
    const double pE = (e < W - 1) ? (double)pc[e < W - 1 ? e + 1 : 0] : (double)pe;
    const double pW = (e > 0) ? (double)pc[e > 0 ? e - 1 : 0] : (double)pw;
    const double dxx = (pE - p0) - (p0 - pW), dyy = ((double)pn[e] - p0) - (p0 - (double)ps[e]);
    double r = bx * ((double)uc[e] - uW);
    r = fma(by, (double)vc[e] - (double)vs[e], r);
    r = fma(wt, (double)wc[e], r);
    r = fma(-wm, (double)wb[e], r);
    r = fma(-ax, dxx, r);
    r = fma(-ay, dyy, r);
    r = fma(-cu, (double)pu[e] - p0, r);
    r = fma(cd, p0 - (double)pd[e], r);
    out[e] = (float)r;
  }
}

template <int W>
__device__ __forceinline__ void resid_vec(const MemberDesc& d, const RowCtx& c, const IoPtrs& io, int i0,
                                          float* out) {
  const float* __restrict__ u = reinterpret_cast<const float*>(io.u);
  const float* __restrict__ v = reinterpret_cast<const float*>(io.v);
  const float* __restrict__ w = reinterpret_cast<const float*>(io.w);
  const float* __restrict__ p = io.s2;
  const int nx = d.nx;
  const int iw = (i0 == 0) ? nx - 1 : i0 - 1, ie = (i0 + W == nx) ? 0 : i0 + W;
  const fwv<W> pc = ldw<W>(p + c.off + i0);
  const float pw = p[c.off + iw], pe = p[c.off + ie];
  const fwv<W> pn = ldw<W>(p + c.noff + i0), ps = ldw<W>(p + c.soff + i0);
  const fwv<W> uc = ldw<W>(u + c.off + i0);
  const float um = u[c.off + iw];
  const fwv<W> vc = ldw<W>(v + c.off + i0), vs = ldw<W>(v + c.soff + i0);
  fwv<W> pu = pc, pd = pc, wc = (fwv<W>)0.0f, wb = (fwv<W>)0.0f;
  if (c.top) {
    pu = ldw<W>(p + c.off + c.plane + i0);
    wc = ldw<W>(w + c.off + i0);
  }
  if (c.bot) {
    pd = ldw<W>(p + c.off - c.plane + i0);
    wb = ldw<W>(w + c.off - c.plane + i0);
  }
  resid_core<W>(d, c, pc, pn, ps, pu, pd, pw, pe, uc, um, vc, vs, wc, wb, out);
}

// Both rows of a pair (k, j) and (k, j+1) of one level: they share p1 rows j
// and j+1 and v row j, so 17 vector loads serve the two rows instead of 20.
template <int W>
__device__ __forceinline__ void resid_pair_vec(const MemberDesc& d, const RowCtx& c0, const RowCtx& c1,
                                               const IoPtrs& io, int i0, float* out0, float* out1) {
  const float* __restrict__ u = reinterpret_cast<const float*>(io.u);
  const float* __restrict__ v = reinterpret_cast<const float*>(io.v);
  const float* __restrict__ w = reinterpret_cast<const float*>(io.w);
  const float* __restrict__ p = io.s2;
  const int nx = d.nx;
  const int iw = (i0 == 0) ? nx - 1 : i0 - 1, ie = (i0 + W == nx) ? 0 : i0 + W;
  const fwv<W> ps = ldw<W>(p + c0.soff + i0), p0 = ldw<W>(p + c0.off + i0), p1 = ldw<W>(p + c1.off + i0);
  const fwv<W> p2 = ldw<W>(p + c1.noff + i0);
  const float pw0 = p[c0.off + iw], pe0 = p[c0.off + ie], pw1 = p[c1.off + iw], pe1 = p[c1.off + ie];
  const fwv<W> u0 = ldw<W>(u + c0.off + i0), u1 = ldw<W>(u + c1.off + i0);
  const float um0 = u[c0.off + iw], um1 = u[c1.off + iw];
  const fwv<W> vs = ldw<W>(v + c0.soff + i0), v0 = ldw<W>(v + c0.off + i0), v1 = ldw<W>(v + c1.off + i0);
  fwv<W> pu0 = p0, pd0 = p0, pu1 = p1, pd1 = p1;
  fwv<W> wc0 = (fwv<W>)0.0f, wb0 = (fwv<W>)0.0f, wc1 = (fwv<W>)0.0f, wb1 = (fwv<W>)0.0f;
  if (c0.top) {  // one level: c0.top == c1.top, c0.bot == c1.bot
    pu0 = ldw<W>(p + c0.off + c0.plane + i0);
    pu1 = ldw<W>(p + c1.off + c1.plane + i0);
    wc0 = ldw<W>(w + c0.off + i0);
    wc1 = ldw<W>(w + c1.off + i0);
  }
  if (c0.bot) {
    pd0 = ldw<W>(p + c0.off - c0.plane + i0);
    pd1 = ldw<W>(p + c1.off - c1.plane + i0);
    wb0 = ldw<W>(w + c0.off - c0.plane + i0);
    wb1 = ldw<W>(w + c1.off - c1.plane + i0);
  }
  resid_core<W>(d, c0, p0, p1, ps, pu0, pd0, pw0, pe0, u0, um0, v0, vs, wc0, wb0, out0);
  resid_core<W>(d, c1, p1, p2, p0, pu1, pd1, pw1, pe1, u1, um1, v1, v0, wc1, wb1, out1);
}

template <typename T, int MODE>
__device__ __forceinline__ void source_vec(const MemberDesc& d, const RowCtx& c, const IoPtrs& io, int i0, T* out) {
  if constexpr (MODE == 0) {
    div_vec<T>(d, c, io, i0, out);
  } else if constexpr (MODE == 2) {
    const double* __restrict__ r = reinterpret_cast<const double*>(io.u) + c.off + i0;
#pragma unroll
    for (int e = 0; e < Vec<T>::n; e += 2) {
      const Vec<double>::type x = ldv(r + e);
      out[e] = (T)x[0];
      out[e + 1] = (T)x[1];
    }
  } else {
    resid_vec<4>(d, c, io, i0, reinterpret_cast<float*>(out));
  }
}

// Separate two real rows packed as z = a + i b:
// A[m] = (Z[m] + conj Z[N-m])/2, B[m] = (Z[m] - conj Z[N-m])/(2i).
// (row 0 gives A[m], row 1 gives B[m]; zr = Z[N-m])
template <typename T>
__device__ __forceinline__ cx<T> split_bin(cx<T> z, cx<T> zr, int row) {
  const T h = (T)0.5;
  return row ? cx<T>{h * (z.y + zr.y), h * (zr.x - z.x)} : cx<T>{h * (z.x + zr.x), h * (z.y - zr.y)};
}

// Spectral layout (column blocks of sbw bins, see MemberDesc): the value of
// row r = k*ny + j at bin m sits at spec_row(r) + spec_col(m). Levels are
// `plane` apart (padded so that the plane stride is an odd multiple of 256
// bytes); inside a block the rows are sbw apart, so a y-FFT tile of sbw
// columns is one contiguous run and a row pair writes 2 sbw adjacent values.
__device__ __forceinline__ long long spec_row(const MemberDesc& d, long long r) {
  const int k = (int)r / d.ny;
  return (long long)k * d.plane + (long long)((int)r - k * d.ny) * d.sbw;
}
__device__ __forceinline__ long long spec_col(const MemberDesc& d, int m) {
  return (long long)(m >> d.lbw) * d.bst + (m & (d.sbw - 1));
}
// A row pair's spectral values in slot order: slots walk the column blocks,
// and inside a block first row 0's sbw bins, then row 1's. When the two rows
// are adjacent (same level) that is their memory order, so consecutive lanes
// touch consecutive addresses and a store or load covers 2 sbw values at a
// time. Slot s holds bin m of row `row` at offset `off` from the row start.
struct PairSlot {
  int row, m;
  long long off;
};
__device__ __forceinline__ PairSlot pair_slot(const MemberDesc& d, int s) {
  const int blk = s >> (d.lbw + 1), w = s & (2 * d.sbw - 1);
  return PairSlot{w >> d.lbw, (blk << d.lbw) | (w & (d.sbw - 1)), (long long)blk * d.bst + (w & (d.sbw - 1))};
}
// slots covering bins 0 .. nxh-1 (whole blocks)
__device__ __forceinline__ int pair_slots(const MemberDesc& d) { return ((d.nxh + d.sbw - 1) >> d.lbw) << (d.lbw + 1); }

// (n, m) of the value at offset x (< ny * nxp) inside a level
__device__ __forceinline__ void spec_nm(const MemberDesc& d, int x, int& n, int& m) {
  const int b = (int)fast_div(x, d.bst_mul, d.bst_shift);
  const int rem = x - b * d.bst;
  n = rem >> d.lbw;
  m = (b << d.lbw) | (rem & (d.sbw - 1));
}

// Row pairs of the stencil kernels in (level, pair) tiles: consecutive
// pair slots walk d.ptj pairs of d.ptk consecutive levels before moving on, so
// the rows a stencil re-reads (levels k +- 1, rows j +- 1) are read by
// workgroups that run at about the same time on the same XCD and meet in its
// L2. ptk = 1 or odd ny (pairs straddle levels) keeps the linear order.
// Bijection of [0, nz * per) that walks tiles of TJ consecutive items of TK
// consecutive levels (per items per level), ragged tiles at the edges;
// identity for TK <= 1 and beyond the grid.
// (32-bit arithmetic: nz * per, a count of rows or row pairs, fits 32 bits)
__device__ __forceinline__ long long tiled_index(long long p, long long per, int nz, int TK, int TJ) {
  if (TK <= 1 || p >= (long long)nz * per) return p;
  const int pi = (int)p, pe = (int)per;
  const int blk = TK * pe;
  const int kb = pi / blk;
  const int rem = pi - kb * blk;
  const int tk = min(TK, nz - kb * TK);          // levels in this block
  const int jt = rem / (tk * TJ);
  const int tj = min(TJ, pe - jt * TJ);
  const int in = rem - jt * tk * TJ;
  const int k = kb * TK + in / tj;
  const int jp = jt * TJ + in % tj;
  return (long long)k * pe + jp;
}

__device__ __forceinline__ long long tiled_pair(const MemberDesc& d, long long p) {
  if (d.ny & 1) return p;
  return tiled_index(p, d.ny / 2, d.nz, d.ptk, d.ptj);
}

// ---------------------------------------------------------------------------
// x-direction forward real FFT, compile-time length N (NT = ct_threads(N)
// threads per transform: N/16 from 512 points, N/8 below; blockDim =
// transforms per workgroup * NT)
// ---------------------------------------------------------------------------
// The residual variant at lengths whose transforms share a wave and whose
// stencil does not walk whole rows per wave (lengths that are not a multiple
// of 64, such as 16-48, 96, 144, 288, or whose whole-wave workgroups would
// pass 512 threads: 576, 1152, 2304) keeps its row contexts in vector
// registers: about 172 registers, 2 waves per SIMD. A budget for 3 spills 2-6
// registers and measured about 1 % faster where it applied before the
// whole-row stencil; a budget for 5 waves at the longer lengths spills 16 and
// loses 6 %.
template <typename T, int MODE, int N>
__global__ void __launch_bounds__(512)
    __attribute__((amdgpu_waves_per_eu(MODE == 1 && ct_threads(N) % 64 != 0 && !xres_wave_rows(N) ? 3 : 1, 8)))
    k_xfwd_ct(LaunchArgs a) {
  constexpr int NT = ct_threads(N);
  using F = CtFft<T, N, NT, false>;
  extern __shared__ unsigned char smem_raw[];
  const int mi = find_member(a, blockIdx.x);
  const MemberDesc& d = *a.mem[mi];
  if (skipped(d)) return;
  const IoPtrs io = a.io[mi];
  // workgroups in launch order for the residual (1-7 % faster than grouped
  // by XCD: 2048^2 x 160, 1024^2 x 256, 4096^2 x 64 and the ensemble), by XCD
  // for the divergence (FP32 2 % faster that way at 2048^2 x 160; FP64 4 %
  // slower there but 7 % faster at 4096^2 x 64) and the given-field mode
  constexpr bool PLAIN = MODE == 1;
  const int lb = PLAIN ? (int)blockIdx.x - a.block_start[mi] : xcd_local_block(a, mi);
  const int ipw = blockDim.x / NT;
  // scalar row contexts for the residual only, and only where a transform
  // spans whole waves (NT a multiple of 64: then no wave holds lanes of two
  // transforms): its registers fall from 174 to 126 and its occupancy rises
  // from 2 to 4 waves per SIMD, and it gains; the divergence variants measure
  // slower with scalar contexts
  constexpr bool UNI = NT % 64 == 0 && MODE == 1;
  const int inst = UNI ? wuni((int)(threadIdx.x / NT)) : (int)(threadIdx.x / NT);
  const int q = threadIdx.x - inst * NT;
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw) + inst * xlds_len(N, 2 * sizeof(T));
  const long long pair = tiled_pair(d, (long long)lb * ipw + inst);
  const long long r0 = 2 * pair, r1 = 2 * pair + 1;
  const bool v0 = r0 < d.nrow, v1 = r1 < d.nrow;
  RowCtx c0 = make_row(d, r0, v0), c1 = make_row(d, r1, v1);
  if constexpr (UNI) {
    c0 = wuni(c0);
    c1 = wuni(c1);
  }
  // 1. vector phase: the stencil on 16-byte chunks of both rows, packed as
  //    z = row0 + i row1 into LDS in natural order: chunk i0 of the rows with
  //    contexts (c0, c1) and validity (v0, v1) into transform slot L
  constexpr int V = Vec<T>::n;
  auto stencil = [&](const RowCtx& c0, const RowCtx& c1, bool v0, bool v1, int i0, cx<T>* L) {
    T s0[V], s1[V];
    // a full pair within one level (even ny): the two rows share loads
    const bool pair = !(d.ny & 1) && v1;
    if constexpr (sizeof(T) == 8) {
      if (MODE == 0 && pair) {
        div_pair_vec<T>(d, c0, c1, io, i0, s0, s1);
      } else {
        // both rows unconditionally (an invalid row's context points at row
        // 0), so all loads of the chunk issue together; invalid rows zeroed
        source_vec<T, MODE>(d, c0, io, i0, s0);
        source_vec<T, MODE>(d, c1, io, i0, s1);
#pragma unroll
        for (int e = 0; e < V; ++e) {
          s0[e] = v0 ? s0[e] : (T)0;
          s1[e] = v1 ? s1[e] : (T)0;
        }
      }
    } else {
      if (pair && MODE == 0) {
        div_pair_vec<T>(d, c0, c1, io, i0, s0, s1);
      } else if (pair && MODE == 1) {
        resid_pair_vec<4>(d, c0, c1, io, i0, s0, s1);
      } else {
        if (v0) source_vec<T, MODE>(d, c0, io, i0, s0);
        else
          for (int e = 0; e < V; ++e) s0[e] = (T)0;
        if (v1) source_vec<T, MODE>(d, c1, io, i0, s1);
        else
          for (int e = 0; e < V; ++e) s1[e] = (T)0;
      }
    }
#pragma unroll
    for (int e = 0; e < V; ++e) L[xpad<T, N>(i0 + e)] = cx<T>{s0[e], s1[e]};
  };
  if constexpr (MODE == 1 && xres_wave_rows(N)) {
    // residual with transforms narrower than a wave: each wave takes one
    // transform's run of 64 chunks of W points at a time (the host launches
    // whole waves), so the row contexts are wave-uniform, in scalar
    // registers, as in the case above; this halves the registers and doubles
    // the waves. Every point's value is the per-thread mapping's.
    constexpr int W = xres_chunk(N);
    constexpr int C = N / (64 * W);  // wave runs per transform
    const int nw = blockDim.x / 64, wv = wuni((int)(threadIdx.x / 64)), ln = threadIdx.x & 63;
    cx<T>* lds0 = reinterpret_cast<cx<T>*>(smem_raw);
    for (int it = wv; it < ipw * C; it += nw) {
      const int ins = it / C, ch = it - ins * C;
      const long long pr = tiled_pair(d, (long long)lb * ipw + ins);
      const bool w0 = 2 * pr < d.nrow, w1 = 2 * pr + 1 < d.nrow;
      const RowCtx e0 = wuni(make_row(d, 2 * pr, w0)), e1 = wuni(make_row(d, 2 * pr + 1, w1));
      const int i0 = (ch * 64 + ln) * W;
      float s0[W], s1[W];
      if (!(d.ny & 1) && w1) {
        resid_pair_vec<W>(d, e0, e1, io, i0, s0, s1);
      } else {
        if (w0) resid_vec<W>(d, e0, io, i0, s0);
        else
          for (int e = 0; e < W; ++e) s0[e] = 0.0f;
        if (w1) resid_vec<W>(d, e1, io, i0, s1);
        else
          for (int e = 0; e < W; ++e) s1[e] = 0.0f;
      }
      cx<T>* L = lds0 + ins * xlds_len(N, 2 * sizeof(T));
#pragma unroll
      for (int e = 0; e < W; ++e) L[xpad<T, N>(i0 + e)] = cx<T>{s0[e], s1[e]};
    }
  } else {
#pragma unroll
    for (int t = 0; t < N / (V * NT); ++t) stencil(c0, c1, v0, v1, (q + t * NT) * V, lds);
  }
  __syncthreads();
  cx<T> v[F::VMAX];
#pragma unroll
  for (int t = 0; t < F::BT0; ++t) {
    const int b = q + t * NT;
    if (F::valid_first(b)) {
#pragma unroll
      for (int r = 0; r < F::R0; ++r) v[t * F::R0 + r] = lds[xpad<T, N>(b + r * F::NB0)];
    }
  }
  __syncthreads();
  auto li = [](int i) { return xpad<T, N>(i); };
  F::run(v, lds, li, q, reinterpret_cast<const cx<T>*>(d.twx));
#pragma unroll
  for (int t = 0; t < F::BTL; ++t) {
    const int b = q + t * NT;
    if (F::valid_last(b)) {
#pragma unroll
      for (int r = 0; r < F::RL; ++r) lds[xpad<T, N>(F::out_index(q, t, r))] = v[t * F::RL + r];
    }
  }
  __syncthreads();
  cx<T>* S = reinterpret_cast<cx<T>*>(io.spec);
  const long long so0 = spec_row(d, v0 ? r0 : 0), so1 = spec_row(d, v1 ? r1 : 0);
  const int ns = pair_slots(d);
  if (sizeof(T) == 4 && d.sbw >= 2) {
    // FP32 with column blocks at least 2 wide: a lane takes two adjacent
    // slots (bins m, m+1 of one row, adjacent in memory, 16-byte aligned:
    // m, the block and row offsets and the plane are even) and stores them
    // with one 16-byte access; a block's last valid bin may be alone. Half
    // the store instructions of one slot per lane, which measured as the
    // costliest phase of these kernels.
    for (int s2 = q; s2 < ns / 2; s2 += NT) {
      const PairSlot ps = pair_slot(d, 2 * s2);
      if (ps.m < d.nxh && (ps.row ? v1 : v0)) {
        const cx<T> b0 = split_bin<T>(lds[xpad<T, N>(ps.m)], lds[xpad<T, N>(ps.m == 0 ? 0 : N - ps.m)], ps.row);
        cx<T>* dst = S + (ps.row ? so1 : so0) + ps.off;
        if (ps.m + 1 < d.nxh) {
          const cx<T> b1 = split_bin<T>(lds[xpad<T, N>(ps.m + 1)], lds[xpad<T, N>(N - ps.m - 1)], ps.row);
          typedef T t4 __attribute__((ext_vector_type(4)));
          t4 v;
          v[0] = b0.x;
          v[1] = b0.y;
          v[2] = b1.x;
          v[3] = b1.y;
          *reinterpret_cast<t4*>(dst) = v;
        } else {
          *dst = b0;
        }
      }
    }
  } else {
    for (int s = q; s < ns; s += NT) {
      const PairSlot ps = pair_slot(d, s);
      if (ps.m < d.nxh && (ps.row ? v1 : v0)) {
        const cx<T> z = lds[xpad<T, N>(ps.m)];
        const cx<T> zr = lds[xpad<T, N>(ps.m == 0 ? 0 : N - ps.m)];
        S[(ps.row ? so1 : so0) + ps.off] = split_bin<T>(z, zr, ps.row);
      }
    }
  }
}

// runtime length (fallback)
template <typename T, int MODE>
__global__ void __launch_bounds__(1024) k_xfwd_gen(LaunchArgs a) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
  const int mi = find_member(a, blockIdx.x);
  const MemberDesc& d = *a.mem[mi];
  if (skipped(d)) return;
  const IoPtrs io = a.io[mi];
  const int lb = xcd_local_block(a, mi);
  const int N = d.nx, nt = d.fx.nt;
  const int ipw = blockDim.x / nt;
  const int inst = threadIdx.x / nt;
  const bool active = inst < ipw;
  const int q = active ? (int)(threadIdx.x - inst * nt) : kBig;
  cx<T>* buf = smem + (active ? inst : 0) * N;
  const long long pair = tiled_pair(d, (long long)lb * ipw + inst);
  const long long r0 = 2 * pair, r1 = 2 * pair + 1;
  const bool v0 = active && r0 < d.nrow, v1 = active && r1 < d.nrow;
  const RowCtx c0 = make_row(d, r0, v0), c1 = make_row(d, r1, v1);
  if (active) {
    for (int i = q; i < N; i += nt) {
      const T s0 = v0 ? source_at<T, MODE>(d, c0, io, i) : (T)0;
      const T s1 = v1 ? source_at<T, MODE>(d, c1, io, i) : (T)0;
      buf[i] = cx<T>{s0, s1};
    }
  }
  __syncthreads();
  fft_lds<T, false>(buf, 1, d.fx, reinterpret_cast<const cx<T>*>(d.twx), q);
  if (active) {
    cx<T>* S = reinterpret_cast<cx<T>*>(io.spec);
    const long long so0 = spec_row(d, v0 ? r0 : 0), so1 = spec_row(d, v1 ? r1 : 0);
    for (int m = q; m < d.nxh; m += nt) {
      const cx<T> z = buf[m], zr = buf[m == 0 ? 0 : N - m];
      const long long cm = spec_col(d, m);
      if (v0) S[so0 + cm] = split_bin<T>(z, zr, 0);
      if (v1) S[so1 + cm] = split_bin<T>(z, zr, 1);
    }
  }
}

// ---------------------------------------------------------------------------
// y-direction complex FFT, in place on the spectral buffer. A workgroup takes
// one level and MT = blockDim / NT consecutive m columns; LDS holds them as
// [j][c] so that consecutive lanes touch consecutive columns (128-byte rows).
// ---------------------------------------------------------------------------
template <typename T, bool INV, int N, int EPT>
__global__ void __launch_bounds__(1024) k_ffty_ct(LaunchArgs a) {
  constexpr int NT = ct_threads_y(N, EPT);
  using F = CtFft<T, N, NT, INV>;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int mi = find_member(a, blockIdx.x);
  const MemberDesc& d = *a.mem[mi];
  if (skipped(d)) return;
  const IoPtrs io = a.io[mi];
  const int lb = xcd_local_block(a, mi);
  const int mt = blockDim.x / NT;
  const int tiles = (d.nxh + mt - 1) / mt;
  const int k = lb / tiles;
  const int c = threadIdx.x % mt;
  const int q = threadIdx.x / mt;
  const int m = (lb - k * tiles) * mt + c;
  const bool valid = m < d.nxh;
  cx<T>* S = reinterpret_cast<cx<T>*>(io.spec) + (long long)k * d.plane + spec_col(d, valid ? m : 0);
  const int rs = d.sbw;  // row stride inside a column block
  cx<T> v[F::VMAX];
  // FP32: unconditional loads (an invalid column reads column 0), zeroed
  // after; FP64 keeps the guarded loads, which measure faster there
#pragma unroll
  for (int t = 0; t < F::BT0; ++t) {
    const int b = q + t * NT;
    if (F::valid_first(b)) {
#pragma unroll
      for (int r = 0; r < F::R0; ++r) {
        if constexpr (sizeof(T) == 4) {
          const cx<T> x = S[(b + r * F::NB0) * rs];
          v[t * F::R0 + r] = valid ? x : cx<T>{0, 0};
        } else {
          v[t * F::R0 + r] = valid ? S[(b + r * F::NB0) * rs] : cx<T>{0, 0};
        }
      }
    }
  }
  auto li = [mt, c](int i) { return i * mt + c; };
  F::run(v, lds, li, q, reinterpret_cast<const cx<T>*>(d.twy));
  if (valid) {
#pragma unroll
    for (int t = 0; t < F::BTL; ++t) {
      const int b = q + t * NT;
      if (F::valid_last(b)) {
#pragma unroll
        for (int r = 0; r < F::RL; ++r) S[F::out_index(q, t, r) * rs] = v[t * F::RL + r];
      }
    }
  }
}

// y-direction complex FFT, persistent form (FP32, 32 elements per thread, so
// that the 8 columns of a 2048-point tile take 512 threads and the prefetch
// below fits the register budget of two waves per SIMD). The grid covers the
// CUs once; workgroup w walks the launch's tiles w, w + gridDim.x, ... and
// issues the loads of its next tile before transforming the current one, so
// that the transform, its LDS exchanges and its stores overlap the next
// tile's loads (a workgroup holds a CU's LDS alone, so nothing else would
// cover them). Twiddles come from an LDS copy of the table: a global load
// issued during the transform would wait behind the prefetched tile.
template <bool INV, int N>
__global__ void __launch_bounds__(512) k_ffty_pp(LaunchArgs a) {
  using T = float;
  constexpr int NT = ct_threads_y(N, 32);
  constexpr int MT = pp_columns(N);  // columns per tile
  using F = CtFft<T, N, NT, INV>;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* twl = lds + N * MT;
  const int total = a.block_start[a.nmem];
  if ((int)blockIdx.x >= total) return;
  // every member of a launch has the same length N, hence the same table
  {
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.mem[0]->twy);
    for (int i = threadIdx.x; i < N; i += blockDim.x) twl[i] = load_tw(tw + i);
  }
  // Tile tb of the launch: a workgroup-uniform base (the tile's first column
  // in its level) and this lane's 32-bit element offset from it, so that every
  // access is a scalar base plus one vector offset. A column past nxh takes
  // the level's last column (transformed, never stored).
  struct Tile {
    cx<T>* base;
    unsigned off;
    int rs;
    bool valid, live;
  };
  auto tile = [&](int tb, int c) {
    const int mi = find_member(a, tb);
    const MemberDesc& d = *a.mem[mi];
    const int lb = tb - a.block_start[mi];
    const int tiles = (d.nxh + MT - 1) / MT;
    const int k = lb / tiles;
    const int m0 = (lb - k * tiles) * MT;
    const int m = m0 + c;
    Tile t;
    t.valid = m < d.nxh;
    t.live = !skipped(d);
    t.rs = wuni(d.sbw);
    const long long b0 = (long long)k * d.plane + spec_col(d, m0);
    t.base = reinterpret_cast<cx<T>*>(a.io[mi].spec) + b0;
    t.off = (unsigned)(spec_col(d, t.valid ? m : d.nxh - 1) - spec_col(d, m0));
    return t;
  };
  // element i of the lane's column (global-address-space accesses through
  // the two-float vector type)
  typedef T pair __attribute__((ext_vector_type(2)));
  auto ld = [](const Tile& t, int i) -> cx<T> {
    const pair x = ((const __attribute__((address_space(1))) pair*)t.base)[t.off + (unsigned)(i * t.rs)];
    return cx<T>{x.x, x.y};
  };
  auto st = [](const Tile& t, int i, cx<T> x) {
    ((__attribute__((address_space(1))) pair*)t.base)[t.off + (unsigned)(i * t.rs)] = pair{x.x, x.y};
  };
  cx<T> v[F::VMAX], nx[F::VMAX];
  // The lane's column and row index are re-read through an empty asm at every
  // tile: the LDS and twiddle addresses derived from them are then computed
  // where they are used instead of being hoisted out of the loop, where they
  // would hold registers the prefetched tile needs.
  auto lane = [](int& c, int& q) {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    c = t % MT;
    q = t / MT;
  };
  int cur = blockIdx.x, c, q;
  lane(c, q);
  Tile tc = tile(cur, c);
  auto load = [&](const Tile& t, int q, cx<T>* dst) {
#pragma unroll
    for (int u = 0; u < F::BT0; ++u) {
      const int b = q + u * NT;
      if (F::valid_first(b)) {
#pragma unroll
        for (int r = 0; r < F::R0; ++r) dst[u * F::R0 + r] = ld(t, b + r * F::NB0);
      }
    }
  };
  if (tc.live) load(tc, q, v);
  __syncthreads();  // the twiddle table
  while (true) {
    const int nxt = cur + gridDim.x;
    Tile tn;
    tn.live = false;
    lane(c, q);
    if (nxt < total) {
      tn = tile(nxt, c);
      if (tn.live) load(tn, q, nx);
    }
    if (tc.live) {  // uniform over the workgroup (one member per tile)
      lane(c, q);
      F::run_tw(v, lds, [c](int i) { return i * MT + c; }, q, [twl](int i) { return twl[i]; });
      if (tc.valid) {
#pragma unroll
        for (int u = 0; u < F::BTL; ++u) {
          const int b = q + u * NT;
          if (F::valid_last(b)) {
#pragma unroll
            for (int r = 0; r < F::RL; ++r) st(tc, F::out_index(q, u, r), v[u * F::RL + r]);
          }
        }
      }
    }
    if (nxt >= total) break;
    cur = nxt;
    tc = tn;
#pragma unroll
    for (int i = 0; i < F::VMAX; ++i) v[i] = nx[i];
  }
}

template <typename T, bool INV>
__global__ void __launch_bounds__(1024) k_ffty_gen(LaunchArgs a) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int mi = find_member(a, blockIdx.x);
  const MemberDesc& d = *a.mem[mi];
  if (skipped(d)) return;
  const IoPtrs io = a.io[mi];
  const int lb = xcd_local_block(a, mi);
  const int mt = d.ymt, ny = d.ny, nt = d.fy.nt;
  const int tiles = (d.nxh + mt - 1) / mt;
  const int k = lb / tiles;
  const int m0 = (lb - k * tiles) * mt;
  const int c = threadIdx.x % mt;
  int q = threadIdx.x / mt;
  if (q >= nt) q = kBig;
  cx<T>* S = reinterpret_cast<cx<T>*>(io.spec) + (long long)k * d.plane;
  const int tot = ny * mt;
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int j = idx / mt, cc = idx - j * mt, m = m0 + cc;
    buf[idx] = (m < d.nxh) ? S[(long long)j * d.sbw + spec_col(d, m)] : cx<T>{0, 0};
  }
  __syncthreads();
  fft_lds<T, INV>(buf + c, mt, d.fy, reinterpret_cast<const cx<T>*>(d.twy), q);
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int j = idx / mt, cc = idx - j * mt, m = m0 + cc;
    if (m < d.nxh) S[(long long)j * d.sbw + spec_col(d, m)] = buf[idx];
  }
}

// ---------------------------------------------------------------------------
// x-direction inverse (complex-to-real) FFT of row pairs, written to
// MODE 0: io.p (storage type T), the pressure;
// MODE 1 (mixed, T = float): io.s1, the refinement's correction delta;
// MODE 2 (mixed, T = float): io.s2, the first-pass pressure p1.
// Z[m] = X_a[m] + i X_b[m], Z[N-m] = conj X_a[m] + i conj X_b[m]; the
// imaginary parts of the self-conjugate bins (m = 0, m = N/2) are dropped.
// ---------------------------------------------------------------------------
template <typename T, class Idx>
__device__ __forceinline__ void pack_bins(cx<T>* buf, const Idx& idx, cx<T> xa, cx<T> xb, int N, int m) {
  const bool selfconj = (m == 0) || (2 * m == N);
  if (selfconj) {
    xa.y = 0;
    xb.y = 0;
  }
  buf[idx(m)] = cx<T>{xa.x - xb.y, xa.y + xb.x};
  if (!selfconj) buf[idx(N - m)] = cx<T>{xa.x + xb.y, xb.x - xa.y};
}

template <typename T, class Idx>
__device__ __forceinline__ void pack_rows(cx<T>* buf, const Idx& idx, const cx<T>* __restrict__ S, long long o0,
                                          long long o1, bool v0, bool v1, int N, int m, long long cm) {
  cx<T> xa = v0 ? S[o0 + cm] : cx<T>{0, 0};
  cx<T> xb = v1 ? S[o1 + cm] : cx<T>{0, 0};
  const bool selfconj = (m == 0) || (2 * m == N);
  if (selfconj) {
    xa.y = 0;
    xb.y = 0;
  }
  buf[idx(m)] = cx<T>{xa.x - xb.y, xa.y + xb.x};
  if (!selfconj) buf[idx(N - m)] = cx<T>{xa.x + xb.y, xb.x - xa.y};
}

template <typename T, int MODE>
__device__ __forceinline__ __attribute__((address_space(1))) T* xinv_dest(const IoPtrs& io) {
  if constexpr (MODE == 0) return gptr(reinterpret_cast<T*>(io.p));
  else if constexpr (MODE == 1) return gptr(reinterpret_cast<T*>(io.s1));
  else return gptr(reinterpret_cast<T*>(io.s2));
}

template <typename T, int MODE>
__device__ __forceinline__ void store_rows(const MemberDesc& d, const IoPtrs& io, long long r0, long long r1, bool v0,
                                           bool v1, int i, cx<T> z) {
  const int N = d.nx;
  auto p = xinv_dest<T, MODE>(io);
  if (v0) p[r0 * N + i] = z.x;
  if (v1) p[r1 * N + i] = z.y;
}

template <typename T, int MODE, int N>
__global__ void __launch_bounds__(512) k_xinv_ct(LaunchArgs a) {
  constexpr int NT = ct_threads(N);
  using F = CtFft<T, N, NT, true>;
  extern __shared__ unsigned char smem_raw[];
  const int mi = find_member(a, blockIdx.x);
  const MemberDesc& d = *a.mem[mi];
  if (skipped(d)) return;
  const IoPtrs io = a.io[mi];
  const int lb = blockIdx.x - a.block_start[mi];
  const int ipw = blockDim.x / NT;
  const int inst = threadIdx.x / NT;
  const int q = threadIdx.x - inst * NT;
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw) + inst * xlds_len(N, 2 * sizeof(T));
  const long long pair = (long long)lb * ipw + inst;
  const long long r0 = 2 * pair, r1 = 2 * pair + 1;
  const bool v0 = r0 < d.nrow, v1 = r1 < d.nrow;
  const cx<T>* S = reinterpret_cast<const cx<T>*>(io.spec);
  auto li = [](int i) { return xpad<T, N>(i); };
  if (sizeof(T) == 4 && d.sbw >= 2) {
    // FP32 with column blocks at least 2 wide: bins m, m+1 (m even) of a row
    // are adjacent and 16-byte aligned in memory, so a lane loads both with
    // one access (half the load instructions). Pairs m = 0, 2, .. up to nx/2
    // over NT threads; the slot after bin nx/2 (a padding slot of the row's
    // last block: nx/2 + 1 is odd, the padded row length a multiple of 8) is
    // read and dropped. Loads first and unconditional, as below.
    typedef T t4 __attribute__((ext_vector_type(4)));
    constexpr int NP = N / 4 + 1;  // pairs (m even, m <= N/2)
    constexpr int RND2 = (NP + NT - 1) / NT;
    const long long so0 = spec_row(d, v0 ? r0 : 0), so1 = spec_row(d, v1 ? r1 : 0);
    t4 ya[RND2], yb[RND2];
#pragma unroll
    for (int t = 0; t < RND2; ++t) {
      const int m = 2 * (q + t * NT);
      const bool in = m <= N / 2;
      const long long cm = spec_col(d, in ? m : 0);
      const t4 a = *reinterpret_cast<const t4*>(S + so0 + cm), b = *reinterpret_cast<const t4*>(S + so1 + cm);
      ya[t] = (in && v0) ? a : (t4)(T)0;
      yb[t] = (in && v1) ? b : (t4)(T)0;
    }
#pragma unroll
    for (int t = 0; t < RND2; ++t) {
      const int m = 2 * (q + t * NT);
      if (m <= N / 2) {
        pack_bins<T>(lds, li, cx<T>{ya[t][0], ya[t][1]}, cx<T>{yb[t][0], yb[t][1]}, N, m);
        if (m + 1 <= N / 2) pack_bins<T>(lds, li, cx<T>{ya[t][2], ya[t][3]}, cx<T>{yb[t][2], yb[t][3]}, N, m + 1);
      }
    }
  } else {
    // nx/2 + 1 bins over NT threads: N/(2 NT) + 1 rounds, loads issued first
    // and unconditional (clamped bin; a missing row reads row 0), selected after
    constexpr int RND = N / (2 * NT) + 1;
    const long long so0 = spec_row(d, v0 ? r0 : 0), so1 = spec_row(d, v1 ? r1 : 0);
    cx<T> xa[RND], xb[RND];
#pragma unroll
    for (int t = 0; t < RND; ++t) {
      const int m = q + t * NT;
      const bool in = m <= N / 2;
      const long long cm = spec_col(d, in ? m : N / 2);
      const cx<T> a = S[so0 + cm], b = S[so1 + cm];
      xa[t] = (in && v0) ? a : cx<T>{0, 0};
      xb[t] = (in && v1) ? b : cx<T>{0, 0};
    }
#pragma unroll
    for (int t = 0; t < RND; ++t) {
      const int m = q + t * NT;
      if (m <= N / 2) pack_bins<T>(lds, li, xa[t], xb[t], N, m);
    }
  }
  __syncthreads();
  cx<T> v[F::VMAX];
#pragma unroll
  for (int t = 0; t < F::BT0; ++t) {
    const int b = q + t * NT;
    if (F::valid_first(b)) {
#pragma unroll
      for (int r = 0; r < F::R0; ++r) v[t * F::R0 + r] = lds[xpad<T, N>(b + r * F::NB0)];
    }
  }
  __syncthreads();
  F::run(v, lds, li, q, reinterpret_cast<const cx<T>*>(d.twx));
#pragma unroll
  for (int t = 0; t < F::BTL; ++t) {
    const int b = q + t * NT;
    if (F::valid_last(b)) {
#pragma unroll
      for (int r = 0; r < F::RL; ++r) lds[xpad<T, N>(F::out_index(q, t, r))] = v[t * F::RL + r];
    }
  }
  __syncthreads();
  // vector phase: 16-byte chunks of both rows
  constexpr int V = Vec<T>::n;
  using vt = typename Vec<T>::type;
  auto p = reinterpret_cast<__attribute__((address_space(1))) vt*>(xinv_dest<T, MODE>(io));
#pragma unroll
  for (int t = 0; t < N / (V * NT); ++t) {
    const int i0 = (q + t * NT) * V;
    vt a0, a1;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const cx<T> z = lds[xpad<T, N>(i0 + e)];
      a0[e] = z.x;
      a1[e] = z.y;
    }
    if (v0) p[(r0 * N + i0) / V] = a0;
    if (v1) p[(r1 * N + i0) / V] = a1;
  }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(1024) k_xinv_gen(LaunchArgs a) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
  const int mi = find_member(a, blockIdx.x);
  const MemberDesc& d = *a.mem[mi];
  if (skipped(d)) return;
  const IoPtrs io = a.io[mi];
  const int lb = blockIdx.x - a.block_start[mi];
  const int N = d.nx, nt = d.fx.nt;
  const int ipw = blockDim.x / nt;
  const int inst = threadIdx.x / nt;
  const bool active = inst < ipw;
  const int q = active ? (int)(threadIdx.x - inst * nt) : kBig;
  cx<T>* buf = smem + (active ? inst : 0) * N;
  const long long pair = (long long)lb * ipw + inst;
  const long long r0 = 2 * pair, r1 = 2 * pair + 1;
  const bool v0 = active && r0 < d.nrow, v1 = active && r1 < d.nrow;
  const cx<T>* S = reinterpret_cast<const cx<T>*>(io.spec);
  auto ident = [](int i) { return i; };
  const long long so0 = spec_row(d, v0 ? r0 : 0), so1 = spec_row(d, v1 ? r1 : 0);
  if (active)
    for (int m = q; m < d.nxh; m += nt) pack_rows<T>(buf, ident, S, so0, so1, v0, v1, N, m, spec_col(d, m));
  __syncthreads();
  fft_lds<T, true>(buf, 1, d.fx, reinterpret_cast<const cx<T>*>(d.twx), q);
  if (active)
    for (int i = q; i < N; i += nt) store_rows<T, MODE>(d, io, r0, r1, v0, v1, i, buf[i]);
}

// ---------------------------------------------------------------------------
// FP64 tridiagonal solve per wavenumber column (partitioned elimination).
//
// Column (m, n): rows a_k P_{k-1} + (-a_k - c_k - rho0_k lam) P_k + c_k P_{k+1}
// = B_k, lam = lamx[m] + lamy[n], solved in FP64 whatever the storage type.
// P lanes of one wave share a column; lane q owns rows q*S .. q*S+S-1 (rows
// >= nz read P_k - P_{k-1} = 0: decoupled from the system by the lid).
//  1. each lane eliminates inside its chunk so that every row depends only on
//     the chunk's first unknown F_q and last unknown L_q;
//  2. the interface rows of L_q are substituted into those of F_q, leaving a
//     tridiagonal system in F_0..F_{P-1}, one row per lane;
//  3. that system is solved by parallel cyclic reduction over the P lanes
//     (wave shuffles, log2 P steps);
//  4. L_q follows from F_q, F_{q+1}; every lane substitutes back.
// The result is scaled by 1/(nx ny) (the inverse-FFT factor). The singular
// (0,0) column: its right-hand side loses its dz-weighted mean, the top
// unknown is pinned to 0, and the solution is shifted to the gauge
// sum_k dz_k P_k = 0.
// ---------------------------------------------------------------------------
struct Row5 {
  double a, b, c, x, y;  // sub, diag, sup, rhs (re, im)
};

__device__ __forceinline__ double shfl_d(double v, int src) { return __shfl(v, src); }

__device__ __forceinline__ Row5 shfl_row(const Row5& r, int src) {
  return Row5{shfl_d(r.a, src), shfl_d(r.b, src), shfl_d(r.c, src), shfl_d(r.x, src), shfl_d(r.y, src)};
}

// 1/x in FP64: the hardware reciprocal refined by one Newton step (error
// about one ulp; the solve does not need the correctly rounded quotient)
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  return r;
}

// Value of lane q - H (FROM_BELOW) or q + H of the same 16-lane row, moved
// with DPP (row_shr / row_shl) on the vector ALU instead of the LDS
// crossbar; a lane whose source lies outside its row reads 0. With P = 16
// lanes per column, a row is a column; every use multiplies such a value by
// a coupling that is already zero at the column's ends.
template <int H, bool FROM_BELOW>
__device__ __forceinline__ double dpp_shift(double v) {
  constexpr int ctrl = FROM_BELOW ? 0x110 + H : 0x100 + H;
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int l2 = __builtin_amdgcn_mov_dpp(lo, ctrl, 0xF, 0xF, true);
  const int h2 = __builtin_amdgcn_mov_dpp(hi, ctrl, 0xF, 0xF, true);
  return __hiloint2double(h2, l2);
}

// One cyclic-reduction step at distance H on unit-diagonal rows (a, c, x, y).
template <int H>
__device__ __forceinline__ void pcr_step16(double& a, double& c, double& x, double& y) {
  const double la = dpp_shift<H, true>(a), lc = dpp_shift<H, true>(c);
  const double lx = dpp_shift<H, true>(x), ly = dpp_shift<H, true>(y);
  const double ha = dpp_shift<H, false>(a), hc = dpp_shift<H, false>(c);
  const double hx = dpp_shift<H, false>(x), hy = dpp_shift<H, false>(y);
  const double ib = rcp64(1.0 - lc * a - ha * c);
  const double na = -la * a, nc = -hc * c;
  const double nx = x - lx * a - hx * c, ny = y - ly * a - hy * c;
  a = na * ib;
  c = nc * ib;
  x = nx * ib;
  y = ny * ib;
}

// sum over the P lanes of a column (aligned power-of-two lane group)
__device__ __forceinline__ double2 column_sum(double2 v, int P) {
  for (int o = P / 2; o > 0; o /= 2) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  return v;
}

// One tile of columns; SING: the tile holds the (0,0) column (tile 0), so
// the mean removal, the pinned top row and the gauge are compiled in.
template <typename TS, int S, bool SING, bool PAIRS>
__device__ __forceinline__ void tri_tile(const MemberDesc& d, const IoPtrs& io, int lb, double2* stage) {
  const int P = d.triP, CW = d.tricw, nz = d.nz, nxh = d.nxh, nxp = d.nxp;
  const int lp = __builtin_ctz(P), lcw = __builtin_ctz(CW);  // both powers of two
  constexpr bool F32 = sizeof(TS) == 4;      // FP32 storage: rows staged as FP32
  constexpr int SP = tri_lane_slots(S, F32); // padded chunk length in LDS (16-byte slots)
  // slot of the parked right-hand side of row r (1 <= r <= S-2)
  constexpr int PK0 = F32 ? 1 : 0;
  const int lrow = P * SP + 1;               // odd stride: columns start in different banks
  // columns run linearly over the padded level plane in memory order (offset
  // x inside a level holds column (n, m) = spec_nm(x)), so a tile is one
  // aligned contiguous run of each level; padding columns (m >= nxh) ride
  // along as dummy systems with a zero right-hand side and are neither read
  // nor written
  const int ncolp = d.ny * nxp;
  const int col0 = lb * CW;
  using CS = cx<TS>;
  CS* Sg = reinterpret_cast<CS*>(io.spec);
  const long long plane = d.plane;

  // 1. coalesced load of CW columns x nz levels into LDS. blockDim = CW P:
  //    thread (cc, kq) = (tid mod CW, tid / CW) stages rows kq S .. kq S + S-1
  //    of column cc, i.e. exactly the rows that lane kq of that column will
  //    eliminate; a wave's load touches CW consecutive columns of each of its
  //    levels. The loads are unconditional (clamped address, zero selected
  //    afterwards) so that all of them are in flight before the first wait.
  //    The PAIRS instance (FP32 storage, even S, tiles of at least 8
  //    columns): thread (cp, kr) = (tid mod CW/2, tid / (CW/2)) stages levels
  //    kr S/2 .. kr S/2 + S/2-1 of the column pair 2cp, 2cp+1 instead, with
  //    16-byte accesses: the same runs in half the memory instructions. A pair
  //    never straddles the end of the plane (col0, ncolp and the plane are
  //    even), so its address is in bounds whenever either column is valid.
  const int tid = threadIdx.x;
  const int cc = tid & (CW - 1), kq = tid >> lcw;
  const int ks = kq * S;
  double2* sst = stage + cc * lrow + kq * SP;
  const int scol_g = col0 + cc;
  int sn, sm;
  spec_nm(d, scol_g, sn, sm);
  const bool sok = scol_g < ncolp && sm < nxh;
  static_assert(!PAIRS || (F32 && S % 2 == 0), "column pairs need FP32 storage and an even row count");
  constexpr int S2 = PAIRS ? S / 2 : 1;
  constexpr bool pairs = PAIRS;
  const int cp = pairs ? tid & ((CW >> 1) - 1) : 0, kr = pairs ? tid >> (lcw - 1) : 0;
  const int gA = col0 + 2 * cp, ks2 = kr * S2;
  int nA, mA, nB, mB;
  spec_nm(d, gA, nA, mA);
  spec_nm(d, gA + 1, nB, mB);
  const bool okA = pairs && gA < ncolp && mA < nxh, okB = pairs && gA + 1 < ncolp && mB < nxh;
  const long long plane4 = plane / 2;  // a level in 16-byte units (FP32 pairs)
  // the pair's chunk slots: column 2cp + h, lane chunk kr / 2, rows (kr mod 2) S/2 ..
  auto pslot = [&](int h) {
    return reinterpret_cast<float2*>(stage + (2 * cp + h) * lrow + (kr >> 1) * SP) + (kr & 1) * S2;
  };
  CS ld[S];
  float4 ld4[S2];
  if constexpr (pairs) {
    // levels ks2 .. ks2+S2-1, clamped to nz-1 (those rows are zeroed below)
    const float4* src = reinterpret_cast<const float4*>(Sg + ((okA || okB) ? gA : 0) + (long long)min(ks2, nz - 1) * plane);
#pragma unroll
    for (int j = 0; j < S2; ++j) {
      ld4[j] = src[0];
      if (j + 1 < S2) src += (ks2 + j + 1 < nz) ? plane4 : 0;
    }
  } else {
    // levels ks .. ks+S-1, clamped to nz-1 (those rows are zeroed below)
    const CS* src = Sg + (sok ? scol_g : 0) + (long long)min(ks, nz - 1) * plane;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      ld[j] = src[0];
      if (j + 1 < S) src += (ks + j + 1 < nz) ? plane : 0;
    }
  }

  const int c = tid >> lp, q = tid & (P - 1);
  const int col = col0 + c;
  int ncol, mcol;
  spec_nm(d, col, ncol, mcol);
  const bool valid = col < ncolp && mcol < nxh;
  const bool singular = SING && valid && (col == 0);
  double2* scol = stage + c * lrow;
  const int k0 = q * S;

  // coefficients of the lane's rows (the tables run past nz with rows that
  // are decoupled from the system): loads issued while the column data is
  // still arriving
  const double lamv = ldg(d.lamy + min(ncol, d.ny - 1)) + ldg(d.lamx + min(mcol, nxh - 1));
  double A[S], B[S], C[S], R0[S];
#pragma unroll
  for (int r = 0; r < S; ++r) {
    A[r] = ldg(d.tra + k0 + r);
    C[r] = ldg(d.trc + k0 + r);
    R0[r] = ldg(d.trr + k0 + r);
  }
  // column data into LDS (zero outside the grid)
  if constexpr (pairs) {
    float2* la = pslot(0);
    float2* lb = pslot(1);
#pragma unroll
    for (int j = 0; j < S2; ++j) {
      const bool in = ks2 + j < nz;  // every slot exists; rows >= nz are never read
      la[j] = okA && in ? make_float2(ld4[j].x, ld4[j].y) : make_float2(0.0f, 0.0f);
      lb[j] = okB && in ? make_float2(ld4[j].z, ld4[j].w) : make_float2(0.0f, 0.0f);
    }
  } else {
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const bool in = sok && ks + j < nz;  // every slot exists; rows >= nz are never read
      if constexpr (F32)
        reinterpret_cast<float2*>(sst)[j] = in ? make_float2(ld[j].x, ld[j].y) : make_float2(0.0f, 0.0f);
      else
        sst[j] = make_double2(in ? (double)ld[j].x : 0.0, in ? (double)ld[j].y : 0.0);
    }
  }
  // padding columns (m >= nxh) solve a well-conditioned dummy system with a
  // zero right-hand side and are never stored
  const double lam = valid ? lamv : 1.0;
#pragma unroll
  for (int r = 0; r < S; ++r) B[r] = -(A[r] + C[r]) - R0[r] * lam;
  if (singular) {  // (0,0) column: its top row is pinned (identity)
#pragma unroll
    for (int r = 0; r < S; ++r)
      if (k0 + r == nz - 1) {
        A[r] = 0.0;
        B[r] = 1.0;
        C[r] = 0.0;
      }
  }
  __syncthreads();

  // staged data: zero for rows >= nz and for padding columns
  double2 D[S];
#pragma unroll
  for (int r = 0; r < S; ++r) {
    if constexpr (F32) {
      const float2 t = reinterpret_cast<const float2*>(scol + q * SP)[r];
      D[r] = make_double2(t.x, t.y);
    } else {
      D[r] = scol[q * SP + r];
    }
  }
  asm volatile("" ::: "memory");  // the slots are reused as FP64 below
  // (0,0) column (one per member, lanes of one wave): remove the dz-weighted
  // mean of the right-hand side, then pin the top row (identity, rhs 0)
  if (singular) {
    double2 sum = make_double2(0.0, 0.0);
#pragma unroll
    for (int r = 0; r < S; ++r) {
      const double dzr = (k0 + r < nz) ? ldg(d.dz + (k0 + r)) : 0.0;
      sum.x += dzr * D[r].x;
      sum.y += dzr * D[r].y;
    }
    sum = column_sum(sum, P);
#pragma unroll
    for (int r = 0; r < S; ++r) {
      const int k = k0 + r;
      if (k < nz - 1) {
        D[r].x -= sum.x * d.rH;
        D[r].y -= sum.y * d.rH;
      } else {
        D[r] = make_double2(0.0, 0.0);
      }
    }
  }

  // Deflation of the near-null direction (FP64 storage). The dz-weighted sum
  // of a column's rows cancels its vertical fluxes, which leaves
  // sum_k dz_k B_k = -lam sum_k dz_k rho0_k P_k: the component of P along
  // the constants, c = -sum dz B / (lam sum dz rho0), is known in closed
  // form. With P = c + Q the elimination solves T Q = B - rho0 sum dz B /
  // sum dz rho0 for the part orthogonal to it, so round-off amplified by the
  // near-singularity of the low-wavenumber columns (lam -> 0) acts on Q, not
  // on the large c ~ 1/lam. The (0,0) column (lam = 0) keeps its own gauge
  // treatment; padding columns have B = 0, so c = 0.
  // Only waves holding a column with lam < lamdef (condition number above
  // ~1e4: the lowest wavenumbers, a few columns in a million) do it; the
  // branch is uniform over the wave, so the lane reduction sees every lane.
  double2 cdef = make_double2(0.0, 0.0);
  if constexpr (!F32) {
    if (__any(lam < d.lamdef)) {
    double2 sb = make_double2(0.0, 0.0);
#pragma unroll
    for (int r = 0; r < S; ++r) {
      const double dzr = (k0 + r < nz) ? ldg(d.dz + (k0 + r)) : 0.0;
      sb.x += dzr * D[r].x;
      sb.y += dzr * D[r].y;
    }
    sb = column_sum(sb, P);  // every lane of the column takes part
    if (!singular) {
      const double gx = sb.x * d.rSr, gy = sb.y * d.rSr;
#pragma unroll
      for (int r = 0; r < S; ++r) {  // R0 = rho0 on real rows, 0 past nz
        D[r].x -= R0[r] * gx;
        D[r].y -= R0[r] * gy;
      }
      const double il = 1.0 / lam;
      cdef = make_double2(-gx * il, -gy * il);
    }
    }
  }

  // 1. chunk elimination: x_r + al_r x_0 + ga_r x_{r+1} = de_r (r >= 1), then
  //    backward to x_r = e_r - f_r x_0 - g_r x_{S-1}, kept in (de, al, ga)
  double al[S], ga[S];
  double2 de[S];
#pragma unroll
  for (int r = 1; r < S; ++r) {
    if (r == 1) {
      const double inv = rcp64(B[1]);
      al[1] = A[1] * inv;
      ga[1] = C[1] * inv;
      de[1] = make_double2(D[1].x * inv, D[1].y * inv);
    } else {
      const double inv = rcp64(B[r] - A[r] * ga[r - 1]);
      al[r] = -A[r] * al[r - 1] * inv;
      ga[r] = C[r] * inv;
      de[r] = make_double2((D[r].x - A[r] * de[r - 1].x) * inv, (D[r].y - A[r] * de[r - 1].y) * inv);
    }
  }
  // interface row of L_q:  al L_q... written as  aL F_q + L_q + cL F_{q+1} = dL
  const double aL = al[S - 1], cL = ga[S - 1];
  const double2 dL = de[S - 1];
  de[S - 1] = make_double2(0.0, 0.0);
  al[S - 1] = 0.0;
  ga[S - 1] = -1.0;
#pragma unroll
  for (int r = S - 2; r >= 1; --r) {
    const double g = ga[r];
    de[r] = make_double2(de[r].x - g * de[r + 1].x, de[r].y - g * de[r + 1].y);
    al[r] = al[r] - g * al[r + 1];
    ga[r] = -g * ga[r + 1];
  }
  // interface row of F_q:  A0 L_{q-1} + (B0 - C0 f1) F_q - C0 g1 L_q = D0 - C0 e1
  const double aF = A[0], bF = B[0] - C[0] * al[1], cF = -C[0] * ga[1];
  const double2 dF = make_double2(D[0].x - C[0] * de[1].x, D[0].y - C[0] * de[1].y);
  // park e_r in the lane's own LDS slots (their right-hand sides are
  // consumed) while the interface system is solved: fewer live registers
#pragma unroll
  for (int r = 1; r < S - 1; ++r) scol[q * SP + r - PK0] = de[r];
  asm volatile("" ::: "memory");

  // 2. substitute L_{q-1} (from lane q-1) and L_q into the F_q row
  const int lane = __lane_id();
  const int up = (q > 0) ? lane - 1 : lane, dn = (q < P - 1) ? lane + 1 : lane;
  const bool row16 = P == 16;  // a column is one DPP row: shifts on the vector ALU
  const double aLm = row16 ? dpp_shift<1, true>(aL) : shfl_d(aL, up);
  const double cLm = row16 ? dpp_shift<1, true>(cL) : shfl_d(cL, up);
  const double dLmx = row16 ? dpp_shift<1, true>(dL.x) : shfl_d(dL.x, up);
  const double dLmy = row16 ? dpp_shift<1, true>(dL.y) : shfl_d(dL.y, up);
  Row5 row;
  {
    const double am = (q > 0) ? aF : 0.0;  // coupling to L_{q-1}
    row.a = -am * aLm;
    row.b = bF - am * cLm - cF * aL;
    row.c = -cF * cL;
    row.x = dF.x - am * dLmx - cF * dL.x;
    row.y = dF.y - am * dLmy - cF * dL.y;
  }

  // 3. parallel cyclic reduction over the P lanes of the column, on rows
  //    scaled to a unit diagonal (four values travel per neighbour, one
  //    reciprocal per step). A lane without a partner at distance h already
  //    has a zero coupling on that side (the first lane's a and the last
  //    lane's c are zero, and each step keeps them zero out to distance 2h),
  //    so whatever it reads there (its own row through an LDS permute, 0
  //    through DPP) is multiplied by zero.
  {
    const double ib = rcp64(row.b);
    row.a *= ib;
    row.c *= ib;
    row.x *= ib;
    row.y *= ib;
  }
  if (row16) {
    pcr_step16<1>(row.a, row.c, row.x, row.y);
    pcr_step16<2>(row.a, row.c, row.x, row.y);
    pcr_step16<4>(row.a, row.c, row.x, row.y);
    pcr_step16<8>(row.a, row.c, row.x, row.y);
  } else
  for (int h = 1; h < P; h *= 2) {
    const int sl = (q >= h) ? lane - h : lane, sr = (q + h < P) ? lane + h : lane;
    const double la = shfl_d(row.a, sl), lc = shfl_d(row.c, sl), lx = shfl_d(row.x, sl), ly = shfl_d(row.y, sl);
    const double ha = shfl_d(row.a, sr), hc = shfl_d(row.c, sr), hx = shfl_d(row.x, sr), hy = shfl_d(row.y, sr);
    const double nb = 1.0 - lc * row.a - ha * row.c;
    const double ib = rcp64(nb);
    const double na = -la * row.a, nc = -hc * row.c;
    const double nx = row.x - lx * row.a - hx * row.c;
    const double ny = row.y - ly * row.a - hy * row.c;
    row.a = na * ib;
    row.c = nc * ib;
    row.x = nx * ib;
    row.y = ny * ib;
  }
  const double2 F = make_double2(row.x, row.y);

  // 4. L_q = dL - aL F_q - cL F_{q+1}, then the chunk's interior rows
  const double Fnx = row16 ? dpp_shift<1, false>(F.x) : shfl_d(F.x, dn);
  const double Fny = row16 ? dpp_shift<1, false>(F.y) : shfl_d(F.y, dn);
  const double2 Fn = (q < P - 1) ? make_double2(Fnx, Fny) : make_double2(0.0, 0.0);
  const double2 L = make_double2(dL.x - aL * F.x - cL * Fn.x, dL.y - aL * F.y - cL * Fn.y);
  double2 X[S];
#pragma unroll
  for (int r = 0; r < S; ++r) {
    if (r == 0) X[r] = F;
    else if (r == S - 1) X[r] = L;
    else {
      const double2 e = scol[q * SP + r - PK0];
      X[r] = make_double2(e.x - al[r] * F.x - ga[r] * L.x, e.y - al[r] * F.y - ga[r] * L.y);
    }
  }
  // the deflated constant back (0 for the (0,0) and padding columns)
  if constexpr (!F32) {
#pragma unroll
    for (int r = 0; r < S; ++r) {
      X[r].x += cdef.x;
      X[r].y += cdef.y;
    }
  }
  // (0,0) column: gauge sum_k dz_k P_k = 0
  if (singular) {
    double2 sum = make_double2(0.0, 0.0);
#pragma unroll
    for (int r = 0; r < S; ++r) {
      const double dzr = (k0 + r < nz) ? ldg(d.dz + (k0 + r)) : 0.0;
      sum.x += dzr * X[r].x;
      sum.y += dzr * X[r].y;
    }
    sum = column_sum(sum, P);
#pragma unroll
    for (int r = 0; r < S; ++r) {
      X[r].x -= sum.x * d.rH;
      X[r].y -= sum.y * d.rH;
    }
  }
  // the solution back into the chunk (rows >= nz are never stored); FP32
  // storage writes it scaled by 1/(nx ny) and rounded, over the parked values
  asm volatile("" ::: "memory");
  if constexpr (F32) {
    const double sc = d.inv_nxny;
    float2* out = reinterpret_cast<float2*>(scol + q * SP);
#pragma unroll
    for (int r = 0; r < S; ++r) out[r] = make_float2((float)(X[r].x * sc), (float)(X[r].y * sc));
  } else {
#pragma unroll
    for (int r = 0; r < S; ++r) scol[q * SP + r] = X[r];
  }
  __syncthreads();

  // coalesced store (the staging thread's rows), scaled by 1/(nx ny)
  if constexpr (pairs) {
    const float2* la = pslot(0);
    const float2* lb = pslot(1);
    float2 xa[S2], xb[S2];
#pragma unroll
    for (int j = 0; j < S2; ++j) {
      xa[j] = la[j];
      xb[j] = lb[j];
    }
    CS* dA = Sg + gA + (long long)ks2 * plane;
    float4* d4 = reinterpret_cast<float4*>(dA);
#pragma unroll
    for (int j = 0; j < S2; ++j) {
      if (ks2 + j < nz) {
        if (okA && okB) d4[j * plane4] = make_float4(xa[j].x, xa[j].y, xb[j].x, xb[j].y);
        else if (okA) dA[j * plane] = CS{xa[j].x, xa[j].y};
        else if (okB) dA[j * plane + 1] = CS{xb[j].x, xb[j].y};
      }
    }
  } else if (sok) {
    CS* dst = Sg + scol_g + (long long)ks * plane;
    if constexpr (F32) {
      float2 x[S];
#pragma unroll
      for (int j = 0; j < S; ++j) x[j] = reinterpret_cast<const float2*>(sst)[j];
#pragma unroll
      for (int j = 0; j < S; ++j)
        if (ks + j < nz) dst[j * plane] = CS{x[j].x, x[j].y};
    } else {
      const double sc = d.inv_nxny;
      double2 x[S];
#pragma unroll
      for (int j = 0; j < S; ++j) x[j] = sst[j];
#pragma unroll
      for (int j = 0; j < S; ++j)
        if (ks + j < nz) dst[j * plane] = CS{(TS)(x[j].x * sc), (TS)(x[j].y * sc)};
    }
  }
}

// FP32 storage up to 10 rows per lane: a register budget for 4 waves per
// SIMD (the LDS chunks then fit 4 such workgroups per CU); the solve is
// latency-bound and gains more from the extra wave than it loses to a
// 16-byte spill at 10 rows
template <typename TS, int S, int MAXT, bool PAIRS>
__global__ void __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(S <= 10 && sizeof(TS) == 4 ? 4 : 1, 8)))
k_tridiag(LaunchArgs a) {
  extern __shared__ unsigned char smem_raw[];
  double2* stage = reinterpret_cast<double2*>(smem_raw);
  const int mi = find_member(a, blockIdx.x);
  const MemberDesc& d = *a.mem[mi];
  if (skipped(d)) return;
  const IoPtrs io = a.io[mi];
  // a spectrum larger than the 256 MB Infinity Cache: tiles in launch order,
  // not grouped by XCD. A column is read once, so there is no L2 reuse to
  // group for, and the workgroups in flight then cover one contiguous run of
  // columns of every level instead of eight runs an eighth of a plane apart
  // (2048^2 x 160, 1024^2 x 256, 4096^2 x 64: 2-7 % faster). Smaller members
  // keep the XCD grouping, which measured 3 % faster on an ensemble of them.
  const bool big = (double)d.plane * d.nz * sizeof(cx<TS>) > 256.0 * (1 << 20);
  const int lb = big ? (int)blockIdx.x - a.block_start[mi] : xcd_local_block(a, mi);
  if (lb == 0)
    tri_tile<TS, S, true, PAIRS>(d, io, lb, stage);
  else
    tri_tile<TS, S, false, PAIRS>(d, io, lb, stage);
}

// ---------------------------------------------------------------------------
// Pressure-gradient correction u -= G p, evaluated in FP64 from an FP64
// pressure (p itself on the FP64 path; on the mixed path p1 + delta, summed
// in FP64 from the two float scratch fields, and written rounded to float as
// the output p); the fields are T. A thread owns VEC consecutive points of one row of one
// level (vector loads and stores need nx % VEC == 0); w[nz-1] = 0.
// ---------------------------------------------------------------------------
// Per-level horizontal reductions of the projection's outputs (the
// diagnostics an I/O server takes of a prognostic field, Sec. 3): stats[(2 f
// + s) nz + k] for field f = u, v, w, p and statistic s = mean, max over the
// nx ny points of level k. p is the pressure the velocities were corrected
// with (p1 + delta in FP64 on the mixed path). The gradient kernel folds them
// in: each workgroup reduces its points and adds one partial per statistic
// with a device-wide atomic, so the accumulation order (and the last bits of
// the means) can vary from run to run.
__global__ void __launch_bounds__(256) k_stats_init(double* stats, int nz) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < 8 * nz) stats[t] = ((t / nz) & 1) ? -__builtin_inf() : 0.0;
}

// st[0..3]: sums of u, v, w, p over the caller's points, st[4..7]: maxima;
// added into level k's statistics (sums scaled by rh = 1/(nx ny)) with the
// hardware FP64 atomic add and max (the buffer is device memory)
__device__ __forceinline__ void stats_commit(double* stats, int nz, int k, const double* st, double rh) {
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    __hip_atomic_fetch_add(stats + (2 * f) * nz + k, st[f] * rh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_max(stats + (2 * f + 1) * nz + k, st[4 + f], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Workgroup reduction of the statistics (`whole`: every point of the
// workgroup is in level k), else one partial per thread.
__device__ __forceinline__ void stats_reduce(double* stats, int nz, int k, double* st, double rh, bool whole,
                                             bool live) {
  if (!whole) {
    if (live) stats_commit(stats, nz, k, st, rh);
    return;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      st[f] += __shfl_xor(st[f], o);
      st[4 + f] = fmax(st[4 + f], __shfl_xor(st[4 + f], o));
    }
  }
  __shared__ double part[16][8];  // one row per wave (blockDim <= 1024)
  const int wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int f = 0; f < 8; ++f) part[wv][f] = st[f];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < nw; ++i) {
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        st[f] += part[i][f];
        st[4 + f] = fmax(st[4 + f], part[i][4 + f]);
      }
    }
    stats_commit(stats, nz, k, st, rh);
  }
}

template <typename T, int VEC, bool RED>
__global__ void __launch_bounds__(256) k_grad(LaunchArgs a) {
  typedef T tv __attribute__((ext_vector_type(VEC)));
  typedef double dv __attribute__((ext_vector_type(VEC)));
  const int mi = find_member(a, blockIdx.x);
  const MemberDesc& d = *a.mem[mi];
  const IoPtrs io = a.io[mi];
  const int lb = xcd_local_block(a, mi);
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const long long nh = (long long)nx * ny;
  // blocks walk (level, row) tiles like the stencil kernels when a row is a
  // whole number of blocks: p one level up is then read by a block of the
  // same tile, close in time, and hits the XCD's L2
  long long blk = lb;
  const int bpr = d.nx / (int)(blockDim.x * VEC);  // blocks per row
  const bool rowblk = bpr >= 1 && bpr * (int)blockDim.x * VEC == d.nx;  // a block lies in one row
  if (d.ptk > 1 && rowblk) {
    const long long row = tiled_index(lb / bpr, d.ny, d.nz, d.ptk, 8);
    blk = row * bpr + lb % bpr;
  }
  const long long g0 = (blk * blockDim.x + threadIdx.x) * VEC;  // first point
  // a block inside one row: its row (level k, row j) and liveness follow from
  // the block index, workgroup-uniform, so the divisions and the level's
  // coefficient load run on the scalar unit
  const int row = rowblk ? (int)(blk / bpr) : 0;
  const bool live = rowblk ? row < ny * nz : g0 < nh * nz;
  if (!RED && !live) return;
  // with the reductions every thread reaches the workgroup reduction: one
  // past the grid reads point 0, stores nothing and contributes nothing
  const long long g = live ? g0 : 0;
  int k, j, i;
  if (rowblk) {
    const int rw = live ? row : 0;
    k = rw / ny;
    j = rw - k * ny;
    i = live ? (int)(blk - (long long)row * bpr) * (int)blockDim.x * VEC + (int)threadIdx.x * VEC : 0;
  } else {
    k = (int)(g / nh);
    const int h = (int)(g - (long long)k * nh);  // nx ny fits 32 bits
    j = h / nx;
    i = h - j * nx;
  }
  const long long base = (long long)k * nh;
  const long long he = base + (long long)j * nx + ((i + VEC == nx) ? 0 : i + VEC);  // east of the last point
  const long long hn = base + (long long)((j == ny - 1) ? 0 : j + 1) * nx + i;
  T* __restrict__ u = reinterpret_cast<T*>(io.u);
  T* __restrict__ v = reinterpret_cast<T*>(io.v);
  T* __restrict__ w = reinterpret_cast<T*>(io.w);
  const bool top = k == nz - 1;
  // p in FP64: the FP64 path's p, or on the mixed path p1 + delta from the
  // first-pass pressure (io.s2) and the correction (io.s1), summed in FP64.
  // Loads go through global-address-space pointers (the pointers come from a
  // by-value argument struct).
  auto ldp = [&](long long o) -> dv {
    if constexpr (sizeof(T) == 8) {
      return ldg(reinterpret_cast<const dv*>(reinterpret_cast<const double*>(io.p) + o));
    } else {
      const tv hi = ldg(reinterpret_cast<const tv*>(io.s2 + o));
      const tv lo = ldg(reinterpret_cast<const tv*>(io.s1 + o));
      dv r;
#pragma unroll
      for (int e = 0; e < VEC; ++e) r[e] = (double)hi[e] + (double)lo[e];
      return r;
    }
  };
  auto ldp1 = [&](long long o) -> double {
    if constexpr (sizeof(T) == 8) return ldg(reinterpret_cast<const double*>(io.p) + o);
    else return (double)ldg(io.s2 + o) + (double)ldg(io.s1 + o);
  };
  const dv pc = ldp(g);
  const dv pn = ldp(hn);
  const double pel = ldp1(he);
  // p one level up is read unconditionally (clamped on the lid row, where w
  // is set to 0 below) so that all loads issue together
  const dv pu = ldp(top ? g : g + nh);
  // u, v, w are read and written once per point: nontemporal accesses (the
  // pressure fields, re-read as neighbours by other workgroups, keep the
  // normal cache policy)
  tv uu = __builtin_nontemporal_load(reinterpret_cast<const tv*>(u + g));
  tv vv = __builtin_nontemporal_load(reinterpret_cast<const tv*>(v + g));
  tv ww = __builtin_nontemporal_load(reinterpret_cast<const tv*>(w + g));
  const double rz = ldg(d.rdzc + k);  // 0 on the lid row
  const double rdx = d.rdx, rdy = d.rdy;
#pragma unroll
  for (int e = 0; e < VEC; ++e) {
    const double pe = (e + 1 < VEC) ? pc[(e + 1) % VEC] : pel;
    uu[e] = (T)((double)uu[e] - (pe - pc[e]) * rdx);
    vv[e] = (T)((double)vv[e] - (pn[e] - pc[e]) * rdy);
    ww[e] = top ? (T)0 : (T)((double)ww[e] - (pu[e] - pc[e]) * rz);
  }
  if (live) {
    __builtin_nontemporal_store(uu, reinterpret_cast<tv*>(u + g));
    __builtin_nontemporal_store(vv, reinterpret_cast<tv*>(v + g));
    __builtin_nontemporal_store(ww, reinterpret_cast<tv*>(w + g));
    if constexpr (sizeof(T) == 4) {
      // the mixed path's pressure output: p1 + delta rounded to float
      tv po;
#pragma unroll
      for (int e = 0; e < VEC; ++e) po[e] = (T)pc[e];
      __builtin_nontemporal_store(po, reinterpret_cast<tv*>(reinterpret_cast<T*>(io.p) + g));
    }
  }
  if constexpr (RED) {
    double st[8];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      st[f] = 0.0;
      st[4 + f] = -__builtin_inf();
    }
    if (live) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const double x[4] = {(double)uu[e], (double)vv[e], (double)ww[e], pc[e]};
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          st[f] += x[f];
          st[4 + f] = fmax(st[4 + f], x[f]);
        }
      }
    }
    // a workgroup whose points lie in one level reduces them first
    const long long gb = blk * blockDim.x * VEC;
    const long long gl = min(gb + (long long)blockDim.x * VEC, nh * nz) - 1;
    stats_reduce(io.stats, nz, k, st, 1.0 / (double)nh, gb / nh == gl / nh, live);
  }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <typename K>
static void set_lds_limit(K kern) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
}

#define MONC_TRI_ROWS(X) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(10) X(12) X(16)
#define MONC_CT_SIZES(X) X(16) X(32) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(1536) X(2048) X(4096)
// lengths with the persistent FP32 y kernel (32 elements per thread)
#define MONC_PP_SIZES(X) X(1024) X(1536) X(2048) X(4096)

bool ct_supported(int n) {
  switch (n) {
#define MONC_CASE(N) case N:
    MONC_CT_SIZES(MONC_CASE)
#undef MONC_CASE
    return true;
    default:
      return false;
  }
}

bool pp_supported(int n) {
  switch (n) {
#define MONC_CASE(N) case N:
    MONC_PP_SIZES(MONC_CASE)
#undef MONC_CASE
    return true;
    default:
      return false;
  }
}

void init_kernel_attributes() {
  set_lds_limit(k_xfwd_gen<double, 0>);
  set_lds_limit(k_xfwd_gen<float, 0>);
  set_lds_limit(k_xfwd_gen<float, 1>);
  set_lds_limit(k_xfwd_gen<double, 2>);
  set_lds_limit(k_xfwd_gen<float, 2>);
  set_lds_limit(k_ffty_gen<double, false>);
  set_lds_limit(k_ffty_gen<double, true>);
  set_lds_limit(k_ffty_gen<float, false>);
  set_lds_limit(k_ffty_gen<float, true>);
  set_lds_limit(k_xinv_gen<double, 0>);
  set_lds_limit(k_xinv_gen<float, 0>);
  set_lds_limit(k_xinv_gen<float, 1>);
  set_lds_limit(k_xinv_gen<float, 2>);
#define MONC_TRI_ATTR(S)                   \
  set_lds_limit(k_tridiag<double, S, 256, false>); \
  set_lds_limit(k_tridiag<float, S, 256, false>);  \
  set_lds_limit(k_tridiag<double, S, 512, false>); \
  set_lds_limit(k_tridiag<float, S, 512, false>);  \
  if constexpr (S % 2 == 0) {                      \
    set_lds_limit(k_tridiag<float, S, 256, S % 2 == 0>); \
    set_lds_limit(k_tridiag<float, S, 512, S % 2 == 0>); \
  }
  MONC_TRI_ROWS(MONC_TRI_ATTR)
#undef MONC_TRI_ATTR
#define MONC_ATTR(N)                          \
  set_lds_limit(k_xfwd_ct<double, 0, N>);     \
  set_lds_limit(k_xfwd_ct<float, 0, N>);      \
  set_lds_limit(k_xfwd_ct<float, 1, N>);      \
  set_lds_limit(k_xfwd_ct<double, 2, N>);     \
  set_lds_limit(k_xfwd_ct<float, 2, N>);      \
  set_lds_limit(k_ffty_ct<double, false, N, 8>); \
  set_lds_limit(k_ffty_ct<double, true, N, 8>);  \
  set_lds_limit(k_ffty_ct<float, false, N, 8>);  \
  set_lds_limit(k_ffty_ct<float, true, N, 8>);   \
  set_lds_limit(k_ffty_ct<double, false, N, 16>); \
  set_lds_limit(k_ffty_ct<double, true, N, 16>);  \
  set_lds_limit(k_ffty_ct<float, false, N, 16>);  \
  set_lds_limit(k_ffty_ct<float, true, N, 16>);   \
  set_lds_limit(k_xinv_ct<double, 0, N>);     \
  set_lds_limit(k_xinv_ct<float, 0, N>);      \
  set_lds_limit(k_xinv_ct<float, 1, N>);      \
  set_lds_limit(k_xinv_ct<float, 2, N>);
  MONC_CT_SIZES(MONC_ATTR)
#undef MONC_ATTR
#define MONC_PP_ATTR(N)                  \
  set_lds_limit(k_ffty_pp<false, N>);    \
  set_lds_limit(k_ffty_pp<true, N>);
  MONC_PP_SIZES(MONC_PP_ATTR)
#undef MONC_PP_ATTR
}

#define MONC_GO(kern) hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, (hipStream_t)stream, a)

void launch_xfwd(const LaunchArgs& a, int grid, int block, size_t lds, bool fp64, int mode, int ct_n, void* stream) {
  switch (ct_n) {
#define MONC_CASE(N)                                        \
  case N:                                                   \
    if (fp64 && mode == 2) MONC_GO((k_xfwd_ct<double, 2, N>)); \
    else if (fp64) MONC_GO((k_xfwd_ct<double, 0, N>));      \
    else if (mode == 0) MONC_GO((k_xfwd_ct<float, 0, N>));  \
    else if (mode == 1) MONC_GO((k_xfwd_ct<float, 1, N>));  \
    else MONC_GO((k_xfwd_ct<float, 2, N>));                 \
    return;
    MONC_CT_SIZES(MONC_CASE)
#undef MONC_CASE
    default:
      if (fp64 && mode == 2) MONC_GO((k_xfwd_gen<double, 2>));
      else if (fp64) MONC_GO((k_xfwd_gen<double, 0>));
      else if (mode == 0) MONC_GO((k_xfwd_gen<float, 0>));
      else if (mode == 1) MONC_GO((k_xfwd_gen<float, 1>));
      else MONC_GO((k_xfwd_gen<float, 2>));
  }
}

void launch_ffty(const LaunchArgs& a, int grid, int block, size_t lds, bool fp64, bool inverse, int ct_n, int ept,
                 void* stream) {
  if (ept == 32 && !fp64) {
    switch (ct_n) {
#define MONC_CASE(N)                                  \
  case N:                                             \
    if (inverse) MONC_GO((k_ffty_pp<true, N>));       \
    else MONC_GO((k_ffty_pp<false, N>));              \
    return;
      MONC_PP_SIZES(MONC_CASE)
#undef MONC_CASE
      default: break;  // rejected by the plan's tile check
    }
    return;
  }
  switch (ct_n) {
#define MONC_CASE(N)                                                                  \
  case N:                                                                             \
    if (ept == 16) {                                                                  \
      if (fp64) {                                                                     \
        if (inverse) MONC_GO((k_ffty_ct<double, true, N, 16>));                       \
        else MONC_GO((k_ffty_ct<double, false, N, 16>));                              \
      } else {                                                                        \
        if (inverse) MONC_GO((k_ffty_ct<float, true, N, 16>));                        \
        else MONC_GO((k_ffty_ct<float, false, N, 16>));                               \
      }                                                                               \
    } else {                                                                          \
      if (fp64) {                                                                     \
        if (inverse) MONC_GO((k_ffty_ct<double, true, N, 8>));                        \
        else MONC_GO((k_ffty_ct<double, false, N, 8>));                               \
      } else {                                                                        \
        if (inverse) MONC_GO((k_ffty_ct<float, true, N, 8>));                         \
        else MONC_GO((k_ffty_ct<float, false, N, 8>));                                \
      }                                                                               \
    }                                                                                 \
    return;
    MONC_CT_SIZES(MONC_CASE)
#undef MONC_CASE
    default:
      if (fp64) {
        if (inverse) MONC_GO((k_ffty_gen<double, true>));
        else MONC_GO((k_ffty_gen<double, false>));
      } else {
        if (inverse) MONC_GO((k_ffty_gen<float, true>));
        else MONC_GO((k_ffty_gen<float, false>));
      }
  }
}

void launch_xinv(const LaunchArgs& a, int grid, int block, size_t lds, bool fp64, int mode, int ct_n, void* stream) {
  switch (ct_n) {
#define MONC_CASE(N)                                        \
  case N:                                                   \
    if (fp64) MONC_GO((k_xinv_ct<double, 0, N>));           \
    else if (mode == 0) MONC_GO((k_xinv_ct<float, 0, N>));  \
    else if (mode == 1) MONC_GO((k_xinv_ct<float, 1, N>));  \
    else MONC_GO((k_xinv_ct<float, 2, N>));                 \
    return;
    MONC_CT_SIZES(MONC_CASE)
#undef MONC_CASE
    default:
      if (fp64) MONC_GO((k_xinv_gen<double, 0>));
      else if (mode == 0) MONC_GO((k_xinv_gen<float, 0>));
      else if (mode == 1) MONC_GO((k_xinv_gen<float, 1>));
      else MONC_GO((k_xinv_gen<float, 2>));
  }
}

// FP32 tridiagonal instance: column pairs (even S only) or single columns
template <int S, int MAXT>
static void launch_tri_f32(const LaunchArgs& a, int grid, int block, size_t lds, bool pairs, void* stream) {
  if constexpr (S % 2 == 0) {
    if (pairs) {
      MONC_GO((k_tridiag<float, S, MAXT, S % 2 == 0>));
      return;
    }
  }
  MONC_GO((k_tridiag<float, S, MAXT, false>));
}

void launch_tridiag(const LaunchArgs& a, int grid, int block, size_t lds, bool fp64, int rows, bool pairs,
                    void* stream) {
  switch (rows) {
#define MONC_CASE(S)                                         \
  case S:                                                    \
    if (block <= 256) {                                      \
      if (fp64) MONC_GO((k_tridiag<double, S, 256, false>)); \
      else launch_tri_f32<S, 256>(a, grid, block, lds, pairs, stream); \
    } else {                                                 \
      if (fp64) MONC_GO((k_tridiag<double, S, 512, false>)); \
      else launch_tri_f32<S, 512>(a, grid, block, lds, pairs, stream); \
    }                                                        \
    return;
    MONC_TRI_ROWS(MONC_CASE)
#undef MONC_CASE
  }
}

void launch_grad(const LaunchArgs& a, int grid, bool fp64, int vec, bool red, void* stream) {
  const dim3 g(grid), b(256);
  hipStream_t st = (hipStream_t)stream;
#define MONC_GRAD(V)                                                                       \
  if (red) {                                                                               \
    if (fp64) hipLaunchKernelGGL((k_grad<double, V, true>), g, b, 0, st, a);               \
    else hipLaunchKernelGGL((k_grad<float, V, true>), g, b, 0, st, a);                     \
  } else {                                                                                 \
    if (fp64) hipLaunchKernelGGL((k_grad<double, V, false>), g, b, 0, st, a);              \
    else hipLaunchKernelGGL((k_grad<float, V, false>), g, b, 0, st, a);                    \
  }
  if (vec == 4) {
    MONC_GRAD(4)
  } else if (vec == 2) {
    MONC_GRAD(2)
  } else {
    MONC_GRAD(1)
  }
#undef MONC_GRAD
}

void launch_stats_init(double* stats, int nz, void* stream) {
  hipLaunchKernelGGL(k_stats_init, dim3((8 * nz + 255) / 256), dim3(256), 0, (hipStream_t)stream, stats, nz);
}

}  // namespace monc
