// Shared host/device descriptors of the projection library.
//
// A launch covers one phase (e.g. "y-direction FFT") for a group of members
// (one member for monc_project, every member of a batch for
// monc_project_batched). Static per-member data (sizes, metric tables,
// twiddles, FFT plans, tile parameters, workspace) lives in a device array of
// MemberDesc; the per-call field pointers and the block ranges of the members
// travel by value in LaunchArgs (about 3.6 KB, under the 4 KB kernel-argument
// limit).
#pragma once
#include <stdint.h>

namespace monc {

constexpr int kMaxPass = 16;            // radix passes of one FFT (3^8 needs 8)
constexpr int kMaxLaunchMembers = 48;   // members per grouped launch (LaunchArgs under 4 KB)
constexpr int kTriSmax = 16;            // rows per lane in the tridiagonal solver
constexpr int kTriPmax = 64;            // lanes per column (one wave)
constexpr int kBig = 1 << 30;           // "inactive" lane index
constexpr int kGenericElems = 8;        // max elements per thread of the runtime-length FFT
constexpr int kSpecBlockMax = 8;        // widest spectral column block (nxp is a multiple of it)
// LDS slots (16 bytes each) per lane chunk of the tridiagonal solver, an odd
// count so that the chunks of consecutive lanes start in different bank
// groups. FP64 storage stages its S rows as FP64; FP32 storage keeps them as
// FP32 (8 bytes a row) and parks the S-2 eliminated FP64 right-hand sides
// over them, so the chunk holds the larger of the two.
constexpr int tri_lane_slots(int s, bool f32) {
  return f32 ? ((s + 1) / 2 > s - 2 ? (s + 1) / 2 : (s - 2 > 1 ? s - 2 : 1)) | 1 : s | 1;
}

// The tridiagonal kernel with FP32 storage, an even row count and tiles of at
// least 8 columns moves column pairs with 16-byte accesses (its own kernel
// instance): half the memory instructions for the same runs; narrower tiles
// measured slower that way.
constexpr bool tri_pairs(int s, int cw, bool f32) { return f32 && s % 2 == 0 && cw >= 8; }
// Threads per compile-time transform (shared by the kernels and the host's
// launch shapes), and so the radix plan (16 elements per thread take radix-16
// passes): along x sixteen elements each from length 512 on, eight below;
// along y sixteen from length 2048 on, so that a 1024-thread workgroup still
// holds several columns of the longest transforms, eight below.
constexpr int ct_threads_x_n(int n) { return n >= 512 ? n / 16 : (n >= 8 ? n / 8 : 1); }
// Fewest transforms of nt threads that fill whole waves (64 lanes).
constexpr int wave_transforms(int nt) {
  int m = 1;
  while (m * nt % 64 != 0) m *= 2;
  return m;
}
// The residual's stencil phase at lengths whose transforms do not fill whole
// waves, are a multiple of 64 points and fit whole waves in 512 threads (64,
// 128, 192, 256, 384, 512, 768, 1536) walks whole rows per wave (64 lanes x
// xres_chunk points: 4 where the length allows, else 2, else 1), so that each
// wave handles one transform's rows at a time and its row contexts are
// wave-uniform; its workgroups then hold whole waves.
constexpr bool xres_wave_rows(int n) {
  return ct_threads_x_n(n) % 64 != 0 && n % 64 == 0 && wave_transforms(ct_threads_x_n(n)) * ct_threads_x_n(n) <= 512;
}
constexpr int xres_chunk(int n) { return n % 256 == 0 ? 4 : (n % 128 == 0 ? 2 : 1); }
// Along y the elements per thread (8: radix-8 passes, 16: radix-16 passes)
// are a tile parameter: default sixteen from length 2048 on, eight below.
constexpr int ct_yept_default(int n) { return n >= 2048 ? 16 : 8; }
constexpr int ct_threads_y_n(int n, int ept) { return n >= ept ? n / ept : 1; }
// columns per tile of the persistent FP32 y kernel (32 elements per thread,
// at most 512 threads)
constexpr int pp_columns(int n) { return n >= 32 ? 512 / (n / 32) : 1; }

// x-FFT LDS layout (shared by the kernels and the host's LDS sizes). For
// transforms with radix-16 passes (16 elements per thread), a bank row (256
// bytes: 2^bits complex values) is permuted by XOR of the value's index with
// the row number, which spreads the stride-16 writes over all banks at no LDS
// cost; other lengths (radix 8 and below, where it measured slower, or not
// whole bank rows) get one pad slot after every 2^shift values (128 bytes).
constexpr int kXswBits32 = 5;    // FP32 complex (8 B): 32 values per bank row
constexpr int kXswBits64 = 4;    // FP64 complex (16 B): 16 values per bank row
constexpr int kXpadShift32 = 4;
constexpr int kXpadShift64 = 3;
constexpr int xsw_bits(int cb) { return cb == 16 ? kXswBits64 : kXswBits32; }
constexpr bool xsw_on(int n, int cb) { return ct_threads_x_n(n) * 16 == n && n % (1 << xsw_bits(cb)) == 0; }
// LDS slots of one x transform of length n (complex values of cb bytes)
constexpr int xlds_len(int n, int cb) {
  return xsw_on(n, cb) ? n : n + (n >> (cb == 16 ? kXpadShift64 : kXpadShift32)) + 1;
}
// LDS slot of element i of an x transform of length n (a bijection of
// [0, n) into [0, xlds_len(n, cb)))
constexpr int xlds_index(int i, int n, int cb) {
  return xsw_on(n, cb) ? i ^ ((i >> xsw_bits(cb)) & ((1 << xsw_bits(cb)) - 1))
                       : i + (i >> (cb == 16 ? kXpadShift64 : kXpadShift32));
}

struct FftPlan {
  int n;                  // transform length (2^a 3^b)
  int npass;              // number of Stockham passes
  int nt;                 // threads cooperating on one transform
  int rad[kMaxPass];      // radix of each pass (2, 3, 4 or 8)
};

struct MemberDesc {
  int nx, ny, nz;
  int nxh;                // nx/2 + 1 spectral values per row
  int nxp;                // padded count of m slots per spectral row (multiple of kSpecBlockMax)
  int dtype;              // 0 = FP64, 1 = mixed
  long long nrow;         // nz * ny real rows
  long long plane;        // complex values per level: ny * nxp, padded
  double rdx, rdy;        // 1/dx, 1/dy
  double inv_nxny;        // 1/(nx ny), the inverse-FFT normalisation
  double rH;              // 1 / sum(dz)
  double rSr;             // 1 / sum(dz rho0), the near-null deflation of the column solves
  double lamdef;          // columns with a smaller horizontal eigenvalue are deflated
  float rdxf, rdyf;       // FP32 copies for the FP32 stencil
  // FP64 vertical tables, all of length nz
  const double* rho0;     // reference density at centres
  const double* rhow;     // density on the top face of cell k (0 at k = nz-1)
  const double* rdz;      // 1/dz_k
  const double* rdzc;     // 1/dzc_k (0 at k = nz-1)
  const double* dz;       // dz_k (gauge weights)
  const double* ta;       // tridiagonal sub-diagonal a_k (a_0 = 0)
  const double* tc;       // tridiagonal super-diagonal c_k (c_{nz-1} = 0)
  // The tridiagonal solver's rows, kTriPmax past nz: row k of the column with
  // eigenvalue lam reads tra_k P_{k-1} - (tra_k + trc_k + trr_k lam) P_k +
  // trc_k P_{k+1}. Rows past nz read P_k - P_{k-1} = 0 (tra 1, trc 0, trr 0):
  // nonsingular for every lam, and the lid (c_{nz-1} = 0) keeps them out of
  // the real rows, so a lane's rows need no range checks.
  const double* tra;
  const double* trc;
  const double* trr;
  // FP32 copies for the FP32 stencil
  const float* rho0f;
  const float* rhowf;
  const float* rdzf;
  // horizontal eigenvalues
  const double* lamx;     // [nxh]
  const double* lamy;     // [ny]
  // twiddles exp(-2 pi i t / n), complex in the storage precision
  const void* twx;        // [nx]
  const void* twy;        // [ny]
  FftPlan fx, fy;
  int ymt;                // y-FFT columns per workgroup
  int triP;               // tridiagonal lanes per column (power of 2)
  int tris;               // rows per lane (>= 2)
  int tricw;              // columns per workgroup (blockDim / triP)
  int ptk;                // levels per (level, row pair) tile of the stencil kernels (1 = row order)
  int ptj;                // row pairs per such tile of the x-forward kernels (8 to 64)
  int xpw;                // x-direction transforms (row pairs) per workgroup of the compile-time kernels
  int yept;               // elements per thread of the compile-time y-FFT kernels (8 or 16)
  // Spectral layout: a level's half spectrum sits in column blocks of sbw
  // consecutive m (the y-FFT tile width), each block row-major over n:
  // element (k, n, m) at k*plane + (m >> lbw)*bst + n*sbw + (m & (sbw-1)).
  int sbw;                // block width, a power of 2 <= kSpecBlockMax (divides nxp)
  int lbw;                // log2 sbw
  int bst;                // elements per block of a level: ny * sbw
  unsigned bst_mul;       // x / bst = (umulhi(x, bst_mul) + x) >> bst_shift for 31-bit x
  int bst_shift;
  void* spec;             // spectral workspace, nz levels of `plane` complex values
  // null, or (the preconditioner's copy of the descriptor) the Krylov
  // solver's converged flag: while *skip != 0 the FFT and tridiagonal
  // kernels do nothing
  const double* skip;
};

struct IoPtrs {
  void* u = nullptr;
  void* v = nullptr;
  void* w = nullptr;
  void* p = nullptr;
  void* spec = nullptr;     // spectral buffer used by this launch
  double* stats = nullptr;  // per-level horizontal mean and max of u, v, w, p, or null
  // mixed path, two float fields (nz, ny, nx) of scratch: s2 holds the
  // first-pass pressure p1, s1 the refinement's correction delta
  float* s1 = nullptr;
  float* s2 = nullptr;
};

struct LaunchArgs {
  int nmem;
  int block_start[kMaxLaunchMembers + 1];
  const MemberDesc* mem[kMaxLaunchMembers];  // device descriptors
  IoPtrs io[kMaxLaunchMembers];
};
static_assert(sizeof(LaunchArgs) <= 4096, "kernel arguments are limited to 4 KB");

}  // namespace monc
