/*
 * monc.h -- C ABI of the MI355X (gfx950) anelastic pressure projection.
 *
 * The operation is the pressure solve of a cloud-resolving model's dynamical
 * core: the paper ("A highly scalable Met Office NERC Cloud model", Sec. 4,
 * "Performance and scaling", the paragraph on the FFT pressure solver)
 * describes it as a forward FFT over the periodic horizontal, a vertical ODE
 * per horizontal wavenumber solved in Fourier space, and a backward FFT; the
 * single-precision solver variant is discussed in the same section and a
 * mixed-precision solver with a double-precision restart and self-tuning in
 * Sec. 5 ("Conclusions and further work").
 *
 * Discrete problem solved (Arakawa C-grid, second-order finite volume):
 *   arrays are C-order (nz, ny, nx), x fastest, periodic in x and y;
 *   p[k,j,i] at the cell centre, u at the east face x=(i+1)dx, v at the north
 *   face y=(j+1)dy, w[k] at the top face of cell k (w[nz-1] is the rigid lid,
 *   and the bottom lid w=0 at z=0 is implicit);
 *   dz[k] is the thickness of layer k, dzc_k = (dz_k + dz_{k+1})/2, rho0[k]
 *   the reference density at cell centres, interpolated linearly in z to the
 *   faces (rhow_k);
 *   D(u) = rho0_k[(u_i-u_{i-1})/dx + (v_j-v_{j-1})/dy]
 *          + (rhow_k w_k - rhow_{k-1} w_{k-1})/dz_k        (zero flux at lids)
 *   G(p) = ((p_{i+1}-p_i)/dx, (p_{j+1}-p_j)/dy, (p_{k+1}-p_k)/dzc_k)
 *   find p with D(G p) = D(u*) and sum_k dz_k sum_ij p = 0 (gauge), then
 *   u = u* - G p (dt folded into p) and w[nz-1] = 0.
 * Horizontally this is diagonal in the discrete Fourier basis with the
 * modified wavenumbers (4/dx^2)sin^2(pi m/nx) + (4/dy^2)sin^2(pi n/ny); per
 * wavenumber it leaves one real tridiagonal system in z (complex right-hand
 * side), solved in FP64 on every path.
 *
 * Thread safety: all functions may be called from several host threads; a
 * plan (and a batch) must not be used by two calls that overlap in time
 * (one workspace per plan). Every enqueueing call is asynchronous on the
 * given stream and never synchronises the host, except monc_project_var,
 * which reads its solver's status from the device.
 */
#ifndef MONC_H
#define MONC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct monc_plan monc_plan;   /* opaque; owns its device workspace */

/* precision of a plan */
enum {
  MONC_FP64 = 0,   /* double storage and arithmetic everywhere */
  MONC_MIXED = 1   /* float storage; FP32 stencils and FFTs; FP64 tridiagonal
                      and mean mode; one FP64 iterative-refinement step */
};

/* status codes */
enum {
  MONC_OK = 0,
  MONC_EINVAL = -1,        /* bad argument (null/misaligned/aliased pointer,
                              bad size, mixed dtypes in a batch, ...)        */
  MONC_EUNSUPPORTED = -2,  /* valid but unsupported (e.g. a size above the
                              kernel limits)                                 */
  MONC_ENOMEM = -3,        /* device allocation failed                       */
  MONC_EHIP = -4           /* a HIP runtime call or launch failed            */
};

/* Limits of the library: nx, ny in [1, 8192] with no prime factor above 3
 * (FFT radices 2, 3, 4, 8); nz in [1, 1024]; batches of 1..256 members. */
#define MONC_MAX_N 8192
#define MONC_MAX_NZ 1024
#define MONC_MAX_BATCH 256
/* Most independent graph branches a batch schedule deals its groups to. */
#define MONC_MAX_BRANCHES 4

/*
 * Create a plan on the current HIP device.
 *   nx, ny, nz : grid size;
 *   dx, dy     : horizontal spacings [m], finite and > 0;
 *   dz[nz]     : layer thicknesses [m], finite and > 0 (host pointer);
 *   rho0[nz]   : reference density at layer centres, finite and > 0 (host);
 *   dtype      : MONC_FP64 or MONC_MIXED.
 * dz and rho0 are copied; the caller keeps ownership. All argument checks
 * run on the host before any HIP call. Returns NULL on failure and sets the
 * message read by monc_last_error().
 */
monc_plan* monc_plan_create(int nx, int ny, int nz, double dx, double dy,
                            const double* dz, const double* rho0, int dtype);

/* Release a plan and its device memory (NULL is ignored). The caller must
 * make sure no enqueued work still uses the plan. */
void monc_plan_destroy(monc_plan* plan);

/*
 * Project one field in place.
 *   u, v, w : device arrays (nz, ny, nx) of double (MONC_FP64) or float
 *             (MONC_MIXED), updated in place; w[nz-1] is ignored on input and
 *             written as 0;
 *   p       : device array (nz, ny, nx), output only, gauge sum dz*p = 0;
 *   stream  : a hipStream_t (NULL = the default stream).
 * All four pointers must be non-null, 16-byte aligned and non-overlapping.
 * The mixed path (Sec. 4's single-precision solver with Sec. 5's
 * double-precision restart, as one refinement step): a first solve with the
 * FP32 divergence, FP32 transforms and the FP64 tridiagonal gives p1; the
 * residual D(u*) - D(G p1) is formed in FP64 from the float inputs and
 * solved the same way for a correction delta; p1 + delta is summed in FP64. It returns p = p1 + delta rounded to float, and u = u* - G(p1 +
 * delta) evaluated in FP64 before rounding, so differencing the returned
 * float p does not reproduce u to full accuracy. Scratch: two float fields
 * of the plan's size, allocated with the plan.
 * Returns MONC_OK, MONC_EINVAL or MONC_EHIP.
 */
int monc_project(monc_plan* plan, void* u, void* v, void* w, void* p, void* stream);

/*
 * monc_project without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc. Same arguments, results (bit for bit) and errors as
 * monc_project, plus MONC_EUNSUPPORTED for a plan whose workspace does not fit
 * the limit below. The workspace (the spectral buffer, and on MIXED plans
 * the two float scratch fields) comes from a static device array of 128 MiB
 * per GPU (enough for a 256x256x128 grid on either path), held until the
 * process ends; the plan's own workspace is left untouched. No part of it
 * needs clearing: every call writes what it reads. All calls on one GPU
 * share that array, so calls that overlap in time on one GPU race (serialise
 * them, e.g. on one stream). Its device address is resolved when a plan is
 * created on the device (else at the first call). No profiling events.
 */
int monc_project_noalloc(monc_plan* plan, void* u, void* v, void* w, void* p, void* stream);

/*
 * Project `count` independent members in one go. plans[i] is member i's
 * plan; u[i], v[i], w[i], p[i] are its arrays as in monc_project. All plans
 * must share one dtype and one device. The whole batch is validated before
 * anything is enqueued (all or nothing). The first call for a given set of
 * plans and pointers builds a schedule (grouped per-phase launches covering
 * every member, in the member order and grouping that monc_autotune chose
 * for this set of grids, else largest first in one group) and captures it in
 * a HIP graph; later calls with the same plans and pointers replay the
 * graph, others re-capture. The batch is the ensemble workload of the
 * paper's self-tuning proposal (Sec. 5): many independent solves scheduled
 * together on one device.
 */
int monc_project_batched(monc_plan* const* plans, int count,
                         void* const* u, void* const* v, void* const* w,
                         void* const* p, void* stream);

/*
 * monc_project plus per-level horizontal reductions of its outputs, the
 * diagnostic an I/O server takes of a prognostic field (Sec. 3 of the paper:
 * the server's "horizontal reduction" actions), folded into the
 * pressure-gradient kernel so that the fields are not read again.
 * stats: device array of 8*nz doubles (caller-owned, 8-byte aligned, not
 * overlapping the fields); on completion stats[(2f + s)*nz + k] holds, for
 * field f = 0..3 (u, v, w after the projection, p) and statistic s = 0 (mean)
 * or 1 (max), that statistic over the nx*ny points of level k. p is the
 * pressure the velocities were corrected with: the output p on the FP64
 * path, p1 + delta in FP64 on the mixed path (whose stored p is its FP32
 * rounding). Means are accumulated with device-wide atomics, so their last
 * bits can differ between runs; maxima are exact. Otherwise as monc_project.
 * Returns MONC_OK, MONC_EINVAL or MONC_EHIP.
 */
int monc_project_reduce(monc_plan* plan, void* u, void* v, void* w, void* p, double* stats, void* stream);

/* Projection with a density rho(x, y, z) that also varies horizontally: the
 * non-separable problem, on which the FFT solve above is no longer exact.
 * The paper's Sec. 4 sets the FFT solver beside an iterative Krylov solver
 * (preconditioned BiCGStab); Sec. 5 proposes preconditioners built from the
 * problem's structure and a mixed-precision solver with a double-precision
 * restart. Here the plan's own spectral solve is the preconditioner of a
 * conjugate-gradient solve in FP64:
 *   D_rho(u) = [rx_i u_i - rx_{i-1} u_{i-1}]/dx + [ry_j v_j - ry_{j-1} v_{j-1}]/dy
 *              + (rz_k w_k - rz_{k-1} w_{k-1})/dz_k           (zero flux at lids)
 *   rx = (rho_i + rho_{i+1})/2, ry = (rho_j + rho_{j+1})/2 (periodic),
 *   rz_k = (dz_{k+1} rho_k + dz_k rho_{k+1})/(dz_k + dz_{k+1});
 *   find p with D_rho(G p) = D_rho(u*) and sum_k dz_k sum_ij p = 0, then
 *   u = u* - G p and w[nz-1] = 0.
 * With rho[k,j,i] = rho0[k] this is monc_project's problem.
 * Method: CG in the dz-weighted inner product (in which D_rho G is
 * self-adjoint), z = M^-1 r the plan's spectral solve with its rho0 (the
 * horizontal mean of rho per level is the natural choice): FP64 for an FP64
 * plan; for a MIXED plan FP32 transforms with the FP64 tridiagonal solve and
 * no refinement step. The residual and the iterates stay FP64; with the
 * FP32 preconditioner the direction update is the flexible (Polak-Ribiere)
 * one, which tolerates its inexactness, with the FP64 one the classic
 * Fletcher-Reeves update (one inner product fewer per iteration).
 * Arguments: rho, u, v, w, p are FP64 device arrays (nz, ny, nx), 16-byte
 * aligned and pairwise disjoint, whatever the plan's precision; rho (> 0
 * everywhere) is read only, u, v, w are updated in place, p is written.
 * tol >= 0: stop once ||r|| <= tol ||D_rho(u*)|| (dz-weighted 2-norms of
 * the residual r = D_rho(u*) - D_rho(G p)); maxit in [1, 10000]: the most
 * iterations. *iters and *relres (either may be NULL) receive the iterations
 * taken and the final ||r||/||D_rho(u*)||; reaching maxit is not an error,
 * the caller compares *relres with tol. Work vectors (four fields) are
 * allocated on the plan by the first call and freed with it.
 * Unlike the other entry points this one synchronises the stream: the
 * residual-norm reduction decides convergence on the device (later kernels
 * of the solve then do nothing), and the host reads the solver's status once
 * per batch of queued iterations (two or three reads for a typical solve).
 * The per-iteration scalars and the preconditioner's copy of the plan's
 * descriptor live in the plan's work vectors, so calls on one plan must not
 * overlap (as for every entry point).
 * Returns MONC_OK, MONC_EINVAL (bad argument, non-finite input, breakdown),
 * MONC_ENOMEM or MONC_EHIP.
 */
int monc_project_var(monc_plan* plan, const double* rho, double* u, double* v, double* w, double* p, double tol,
                     int maxit, int* iters, double* relres, void* stream);

/* Message of the last failure on the calling thread ("" if none). */
const char* monc_last_error(void);

/* ---------------------------------------------------------------------
 * Introspection, tuning, profiling and stage-wise access (used by tests
 * and the benchmark; not needed for ordinary use).
 * ------------------------------------------------------------------- */

/* Geometry of the spectral workspace. Value (k, n, m) of the half spectrum
 * (m = 0..nx/2) sits at element
 *   k * (*plane_len) + (m / B) * ny * B + n * B + (m % B),   B = *col_block:
 * each level holds its columns in blocks of B consecutive m (B a power of
 * two, 1..8, the width of the plan's y-FFT tiles), each block stored row by
 * row, so that a y-FFT tile reads one contiguous run. *row_len >= nx/2+1 is
 * the padded count of m slots (a multiple of 8) and *plane_len >= ny *
 * (*row_len). The layout can change when the plan's tile parameters change
 * (monc_plan_set_params, monc_autotune); query it after those calls.
 * *elem_bytes is 16 (FP64) or 8 (MIXED). Any output pointer may be NULL.
 * Returns the number of complex elements (nz * plane_len), or 0 for a NULL
 * plan. */
size_t monc_spectral_layout(const monc_plan* plan, int* row_len, int* col_block, long long* plane_len,
                            int* elem_bytes);

/* Stage-wise execution on caller buffers (all device pointers, sizes as in
 * monc_project; `spec` holds monc_spectral_layout() complex elements):
 *   MONC_STAGE_FORWARD  bufs = {u, v, w, spec}: spec = unnormalised real 2-D
 *                       FFT per level of D(u) (m = 0..nx/2 of each row);
 *   MONC_STAGE_SOLVE    bufs = {spec}: in place, each wavenumber column
 *                       replaced by its tridiagonal solution times 1/(nx ny)
 *                       (the (0,0) column with the gauge);
 *   MONC_STAGE_INVERSE  bufs = {spec, p}: p = inverse real 2-D FFT without
 *                       extra scaling (imaginary parts of self-conjugate bins
 *                       ignored); spec is overwritten;
 *   MONC_STAGE_GRADIENT bufs = {p, u, v, w}: u -= G p (in place), w lid = 0;
 *   MONC_STAGE_RESIDUAL bufs = {u, v, w, p, spec} (MIXED only): spec = FFT of
 *                       the FP64 residual D(u) - D(G p) rounded to float
 *                       (the refinement's right-hand side).
 * Returns MONC_OK, MONC_EINVAL or MONC_EHIP. */
enum {
  MONC_STAGE_FORWARD = 1,
  MONC_STAGE_SOLVE = 2,
  MONC_STAGE_INVERSE = 3,
  MONC_STAGE_GRADIENT = 4,
  MONC_STAGE_RESIDUAL = 5
};
int monc_debug_stage(monc_plan* plan, int stage, void* const* bufs, int nbufs, void* stream);

/* Kernel identifiers used by the profiler. */
enum {
  MONC_K_DIV_FFTX = 0,    /* divergence fused with the x-direction r2c FFT  */
  MONC_K_FFTY_FWD = 1,    /* y-direction c2c forward FFT                    */
  MONC_K_TRIDIAG = 2,     /* FP64 tridiagonal solve per wavenumber column   */
  MONC_K_FFTY_INV = 3,    /* y-direction c2c inverse FFT                    */
  MONC_K_IFFTX = 4,       /* x-direction c2r inverse FFT (writes p)         */
  MONC_K_GRAD = 5,        /* pressure-gradient correction (FP64 path)       */
  MONC_K_RESID_FFTX = 6,  /* FP64 residual fused with the x r2c FFT (MIXED) */
  MONC_K_GRAD_FINAL = 7,  /* p1 + delta and FP64 gradient correction (MIXED)*/
  MONC_K_COUNT = 8
};
const char* monc_kernel_name(int kernel_id);

/* Per-kernel timing with HIP events recorded on the launch stream around
 * every launch of the kernels in `mask` (bit i = kernel id i); 0 disables.
 * Applies to monc_project/monc_project_batched calls on this plan (for a
 * batch, the first member's plan controls it). */
int monc_profile_enable(monc_plan* plan, unsigned mask);
/* Wait for the recorded events, add their durations per kernel into
 * ms[MONC_K_COUNT] and launches[MONC_K_COUNT], and clear the record. */
int monc_profile_read(monc_plan* plan, double* ms, int* launches);

/* Self-tuning (the paper's Sec. 5 proposes performance tuning done
 * dynamically by the model): time candidate schedules on this device and
 * keep the fastest. For every distinct grid among plans[0..count-1], the tile
 * parameters (FFT elements per thread, y-FFT columns per workgroup,
 * tridiagonal lanes per column and columns per workgroup, x transforms per
 * workgroup, the radix plan of the compile-time y-FFT) are tuned on the
 * grid's first plan, one parameter after the
 * other, and copied to its other plans. For count > 1 the batch schedule
 * of monc_project_batched over these plans is then tuned as a whole: each
 * member order (largest or smallest first), grouping (all members per
 * phase, or groups of at most 1024, 512, 256, 128 or 64 MB of working set,
 * each running its whole phase sequence) and number of graph branches the
 * groups are dealt to (1, 2 or 4) is captured and its graph replayed on
 * scratch fields.
 * Results are stored in the plans / the schedule table and in the JSON cache
 * named by the MONC_TUNE_CACHE environment variable (if set), which plans and
 * batches of the same grids read back. Allocates scratch fields, synchronises
 * the stream. Returns MONC_OK or an error (MONC_EINVAL for a bad batch as in
 * monc_project_batched, MONC_ENOMEM). */
int monc_autotune(monc_plan* const* plans, int count, void* stream);

/* The batch schedule monc_project_batched uses for these plans (tuned, read
 * from the cache, or the default): out[0] = member order (0 largest first,
 * 1 smallest first), out[1] = working-set budget per group in MB (0 = one
 * group, every phase over all members), out[2] = number of groups, out[3] =
 * graph branches (1..MONC_MAX_BRANCHES): with a budget, group g runs on
 * branch g mod branches, and the branches are independent chains of the
 * captured graph that the device runs concurrently. out holds 4 ints. */
int monc_batch_schedule(monc_plan* const* plans, int count, int* out);
/* Set that schedule by hand (order 0 or 1, budget_mb >= 0, branches in
 * [1, MONC_MAX_BRANCHES]; branches only matter with budget_mb > 0); the next
 * monc_project_batched call over these plans captures it. */
int monc_batch_set_schedule(monc_plan* const* plans, int count, int order, int budget_mb, int branches);

/* Streaming-bandwidth probes: one launch of the plainest kernel that moves
 * a known number of bytes, to measure the bandwidth a streaming kernel
 * reaches on the device (the practical ceiling next to the vendor's HBM
 * peak) and to calibrate hardware traffic counters. kind and buffers (device
 * pointers, 16-byte aligned, `bytes` each unless stated, a multiple of 16):
 *   MONC_PROBE_READ    reads a; b is a 16-byte sink that is never written
 *                      in practice (read bytes: `bytes`);
 *   MONC_PROBE_WRITE   writes zeros to a (written: `bytes`);
 *   MONC_PROBE_COPY    copies a to b (read and written: `bytes` each);
 *   MONC_PROBE_UPDATE  b, c, d -= a elementwise as floats, in place (read
 *                      4 x `bytes`, written 3 x `bytes`).
 * Asynchronous on `stream`. Returns MONC_OK, MONC_EINVAL (bad kind, size or
 * pointer), MONC_EUNSUPPORTED (too large for one launch) or MONC_EHIP. */
enum { MONC_PROBE_READ = 0, MONC_PROBE_WRITE = 1, MONC_PROBE_COPY = 2, MONC_PROBE_UPDATE = 3 };
int monc_stream_probe(int kind, void* a, void* b, void* c, void* d, size_t bytes, void* stream);

/* Number of tile parameters. */
#define MONC_NPARAMS 7

/* Current tile parameters of a plan, out[MONC_NPARAMS]:
 *   out[0] = x-FFT elements per thread (runtime-length FFTs only),
 *   out[1] = y-FFT elements per thread (runtime-length FFTs only),
 *   out[2] = y-FFT columns per workgroup,
 *   out[3] = tridiagonal lanes per column (power of 2, <= 64),
 *   out[4] = tridiagonal columns per workgroup (power of 2, times out[3]
 *            at most 1024 threads),
 *   out[5] = x-direction transforms (row pairs) per workgroup of the
 *            compile-time x-FFT kernels (at most 512 threads and 160 KB of
 *            LDS per workgroup; default 256 threads' worth; the mixed
 *            path's residual kernel, at lengths whose transforms are
 *            narrower than a wave, rounds it to whole waves),
 *   out[6] = elements per thread of the compile-time y-FFT kernels, i.e.
 *            their radix plan: 8 (radix-8 passes) or 16 (radix-16 passes);
 *            default 16 from ny = 2048 on, else 8. On MONC_MIXED plans with
 *            ny = 1024, 1536, 2048 or 4096 also 32: a persistent kernel
 *            (one workgroup per CU, 512 columns' worth of threads, each
 *            workgroup loading its next tile while transforming the
 *            current one) whose tile width is fixed by ny; out[2] then
 *            only sets the spectral column blocks. Other values or plans:
 *            MONC_EINVAL. */
int monc_plan_params(const monc_plan* plan, int* out);
/* Set them from in[MONC_NPARAMS] (values are checked; 0 keeps the current
 * value). Synchronises the device. */
int monc_plan_set_params(monc_plan* plan, const int* in);

#ifdef __cplusplus
}
#endif
#endif /* MONC_H */
