// Launchers of the variable-density Krylov kernels (krylov.hip): plain
// device pointers to FP64 (nz, ny, nx) fields.
#pragma once

namespace monc {

constexpr int kVarBlock = 256;                  // threads per workgroup
constexpr int kVarPts = 4;                      // points per thread
constexpr int kVarSpan = kVarBlock * kVarPts;   // points of one level per workgroup
constexpr int kVarLevels = 4;                   // levels per stencil workgroup (walked upwards)
constexpr int kVarFinishBlock = 1024;           // threads of the partial-sum reduction

// Scalars in scal[]: a status row, then per iteration it the dz-weighted
// <r_it, z_it>, <d_it, q_it>, <r_it, r_it> and <z_it, q_{it-1}>.
// Status: the gauge sum of p; the done flag (0 running, 1 converged,
// 2 non-finite residual); the last iteration whose <r, r> was formed, and
// that <r, r>. Once the flag is set every later kernel of the solve returns
// at once, so the host can queue several iterations between reads.
enum { kVarRZ = 0, kVarDQ = 1, kVarRR = 2, kVarZQ = 3, kVarSlots = 4 };
enum { kVarGauge = 0, kVarDone = 1, kVarLast = 2, kVarLastRR = 3 };
inline __host__ __device__ int var_slot(int it, int s) { return kVarSlots * (it + 1) + s; }

// A workgroup covers a 2-D tile of a level: var_tile_w(nx) = min(nx, 256)
// points wide and kVarSpan / var_tile_w rows high, so that the rows a
// stencil reads above and below its own are few against the rows it
// computes (a run of kVarSpan points would be a single row at nx = 1024).
inline __host__ __device__ int var_tile_w(int nx) { return nx < 256 ? nx : 256; }
inline __host__ __device__ int var_tile_h(int nx) { return kVarSpan / var_tile_w(nx); }
inline __host__ __device__ int var_tiles_x(int nx) { return (nx + var_tile_w(nx) - 1) / var_tile_w(nx); }
inline __host__ __device__ int var_tiles_y(int nx, int ny) { return (ny + var_tile_h(nx) - 1) / var_tile_h(nx); }
inline __host__ __device__ long long var_blocks_per_level(int nx, int ny) {
  return (long long)var_tiles_x(nx) * var_tiles_y(nx, ny);
}
inline __host__ __device__ int var_level_groups(int nz) { return (nz + kVarLevels - 1) / kVarLevels; }
inline long long var_stencil_parts(int nx, int ny, int nz) { return var_blocks_per_level(nx, ny) * var_level_groups(nz); }

inline long long var_point_parts(int nx, int ny, int nz) { return var_blocks_per_level(nx, ny) * nz; }

struct VarGrid {
  int nx, ny, nz;
  double rdx, rdy;          // 1/dx, 1/dy
  double rdx2, rdy2;        // 1/dx^2, 1/dy^2
  const double* rho;        // density at the cell centres, (nz, ny, nx)
  const double* dz;         // [nz] layer thicknesses (inner-product weights)
  const double* rdz;        // [nz] 1/dz_k
  const double* rdzc;       // [nz] 1/dzc_k (0 at nz-1)
  const double* za;         // [nz] dz_{k+1}/(dz_k + dz_{k+1}) (0 at nz-1)
  const double* zb;         // [nz] dz_k/(dz_k + dz_{k+1}) (0 at nz-1)
};

// part: one partial sum per workgroup: var_stencil_parts entries after the
// divergence and the operator, var_point_parts after the other kernels.
// Kernels taking scal (except the divergence) do nothing once the done
// flag is set.
void launch_var_div(const VarGrid& g, const double* u, const double* v, const double* w, double* r, double* p,
                    double* part, void* stream);
void launch_var_apply(const VarGrid& g, const double* scal, const double* d, double* q, double* part, void* stream);
void launch_var_update(const VarGrid& g, const double* scal, int it, double* p, double* r, const double* d,
                       const double* q, double* part, void* stream);
// z: FP64 (z64) or FP32 field
void launch_var_dots(const VarGrid& g, const double* scal, const double* r, const void* z, bool z64, const double* q,
                     double* part0, double* part1, void* stream);
void launch_var_dir(const VarGrid& g, const double* scal, int it, const void* z, bool z64, double* d, void* stream);
// the dz-weighted sum of p, and p -= scal[slot] * rw
void launch_var_wsum(const VarGrid& g, const double* p, double* part, void* stream);
void launch_var_shift(const VarGrid& g, const double* scal, int slot, double rw, double* p, void* stream);
// scal[slot0] = sum part0 (and scal[slot1] = sum part1 when part1 is given);
// gated: skip once done
void launch_var_finish(const double* part0, const double* part1, long long n, double* scal, int slot0, int slot1,
                       bool gated, void* stream);
// <r, r> of iteration it into its slot and the status row; sets the done
// flag when it is <= tol2 <r_0, r_0> or not finite
void launch_var_finish_rr(const double* part, long long n, double* scal, int it, double tol2, void* stream);
void launch_var_zero(double* x, int n, void* stream);

}  // namespace monc
