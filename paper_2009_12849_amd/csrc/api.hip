// C ABI of the projection library: plans, the single and batched projection,
// stage-wise access, per-kernel profiling and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/monc.h"
#include "kernels.h"
#include "krylov.h"
#include "monc_types.h"
#include "plan_math.h"

using namespace monc;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(MONC_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// profiler: HIP event pairs around the launches of selected kernels
// ---------------------------------------------------------------------------
struct Profiler {
  unsigned mask = 0;
  struct Rec {
    int id;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  std::mutex mu;

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ~Profiler() {
    for (auto& r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
static std::atomic<unsigned long long> g_plan_ids{1};
static std::once_flag g_attr_once;

struct monc_plan {
  unsigned long long id = 0;
  unsigned long long version = 0;  // bumped when tile parameters change
  int nx = 0, ny = 0, nz = 0, dtype = 0, device = 0;
  double dx = 0, dy = 0;
  std::vector<double> dz, rho0;
  int ex = 8, ey = 8, ymt = 0, triP = 0, tricw = 0, xpw = 0, yept = 0;  // tile parameters (0 = automatic)
  MemberDesc h{};                          // host copy with device pointers
  MemberDesc* d_desc = nullptr;            // device copy
  void* d_tables = nullptr;
  void* d_spec = nullptr;
  float* d_s1 = nullptr;     // mixed path scratch: divergence, then the correction
  float* d_s2 = nullptr;     // mixed path scratch: first-pass pressure
  size_t spec_elems = 0;
  void* d_var = nullptr;     // work vectors of monc_project_var (allocated at its first call)
  MemberDesc h_pre{};        // the preconditioner's descriptor: h plus the solver's done flag
  Profiler prof;
};

static size_t elem_bytes(int dtype) { return dtype == MONC_FP64 ? 8 : 4; }
static size_t cplx_bytes(int dtype) { return 2 * elem_bytes(dtype); }

static int pow2_floor(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}

// Rows per lane of the tridiagonal kernel for nz rows on P lanes: the
// smallest compiled row count (2..8, 10, 12, 16) that covers them, 0 if none.
static int tri_rows(int nz, int P) {
  const int s = std::max(2, (nz + P - 1) / P);
  if (s <= 8) return s;
  if (s <= 10) return 10;
  if (s <= 12) return 12;
  if (s <= kTriSmax) return kTriSmax;
  return 0;
}

// Derive FFT plans and tile parameters from (ex, ey, ymt, triP, tricw, xpw,
// yept); 0 = default.
static int configure_tiles(monc_plan* pl, int ex, int ey, int ymt, int triP, int tricw, int xpw, int yept) {
  MemberDesc& h = pl->h;
  FftPlan fx{}, fy{};
  if (!radix_plan(pl->nx, fx) || !radix_plan(pl->ny, fy))
    return fail(MONC_EUNSUPPORTED, "no radix plan for nx=%d ny=%d", pl->nx, pl->ny);
  if (ex <= 0) ex = pl->ex;
  if (ey <= 0) ey = pl->ey;
  if (ex > kGenericElems || ey > kGenericElems)
    return fail(MONC_EINVAL, "elements per thread must be <= %d (got %d, %d)", kGenericElems, ex, ey);
  if (!fft_threads(fx, ex) || !fft_threads(fy, ey))
    return fail(MONC_EUNSUPPORTED, "FFT of nx=%d or ny=%d needs more than 1024 threads", pl->nx, pl->ny);
  const size_t cb = cplx_bytes(pl->dtype);
  // elements per thread of the compile-time y-FFT (its radix plan): 8 or 16,
  // or 32 = the persistent FP32 kernel (mixed plans, lengths of
  // pp_supported)
  if (yept <= 0) yept = pl->yept;
  if (yept != 0 && yept != 8 && yept != 16 && yept != 32)
    return fail(MONC_EINVAL, "y-FFT elements per thread must be 8, 16 or 32 (got %d)", yept);
  if (yept == 32 && (pl->dtype == MONC_FP64 || !pp_supported(pl->ny)))
    return fail(MONC_EINVAL, "32 y-FFT elements per thread (the persistent kernel) need a mixed plan and ny of "
                             "1024, 1536, 2048 or 4096 (got ny=%d)", pl->ny);
  const int yeff = yept > 0 ? yept : ct_yept_default(pl->ny);
  // y-FFT columns per workgroup (also the width of the spectral column
  // blocks, up to 8): 128 bytes of a row by default, bounded by the
  // workgroup size (1024) and 128 KB of LDS
  const int nty = ct_supported(pl->ny) ? ct_threads_y_host(pl->ny, yeff) : fy.nt;
  if (nty > 1024)
    return fail(MONC_EUNSUPPORTED, "a %d-point y-FFT with %d elements per thread needs more than 1024 threads", pl->ny,
                yeff);
  const int mt_cap = std::max(1, std::min(1024 / nty, (int)(131072 / (pl->ny * cb))));
  if (ymt <= 0) ymt = pl->ymt > 0 ? pl->ymt : (int)(128 / cb);
  if (ymt > 64) return fail(MONC_EINVAL, "y-FFT columns per workgroup must be <= 64 (got %d)", ymt);
  ymt = std::max(1, std::min(ymt, mt_cap));
  const int nxh = pl->nx / 2 + 1;
  ymt = std::min(ymt, pow2_floor(nxh) * 2);
  // tridiagonal lanes per column: default = fewest lanes with <= 6 rows each
  if (triP <= 0) triP = pl->triP;
  if (triP <= 0) {
    triP = 1;
    while ((pl->nz + triP - 1) / triP > 6 && triP < kTriPmax) triP *= 2;
  }
  if (triP & (triP - 1) || triP > kTriPmax)
    return fail(MONC_EINVAL, "tridiagonal lanes per column must be a power of 2 <= %d (got %d)", kTriPmax, triP);
  const int s = tri_rows(pl->nz, triP);
  if (s == 0)
    return fail(MONC_EINVAL, "%d lanes leave %d rows per lane (max %d)", triP, (pl->nz + triP - 1) / triP, kTriSmax);
  // tridiagonal tile: columns per workgroup (0 = automatic: 256 threads, four
  // waves, so that five workgroups fit a CU at ~100 registers per lane)
  if (tricw <= 0) tricw = pl->tricw;
  const int cw = tricw > 0 ? tricw : std::max(1, 256 / triP);
  if (cw & (cw - 1) || cw * triP > 512)
    return fail(MONC_EINVAL, "tridiagonal columns per workgroup must be a power of 2 with %d lanes <= 512 threads (got %d)",
                triP, cw);
  // x transforms per workgroup of the compile-time x kernels (default: 256
  // threads); at most 512 threads and 160 KB of LDS
  if (xpw <= 0) xpw = pl->xpw;
  int xeff = 1;
  if (ct_supported(pl->nx)) {
    const int nt = ct_threads_host(pl->nx);
    const size_t per = (size_t)xlds_len(pl->nx, (int)cb) * cb;
    xeff = xpw > 0 ? xpw : std::max(1, 256 / nt);
    if (xeff * nt > 512 || xeff * per > 160 * 1024)
      return fail(MONC_EINVAL, "%d x transforms of %d points per workgroup exceed 512 threads or 160 KB of LDS", xeff,
                  pl->nx);
  }
  pl->ex = ex;
  pl->ey = ey;
  pl->ymt = ymt;
  pl->xpw = xpw;
  h.xpw = xeff;
  pl->yept = yept;
  h.yept = yeff;
  // spectral column blocks as wide as a y-FFT tile (up to kSpecBlockMax), so
  // that the tile is one contiguous run of each level
  h.sbw = std::min(kSpecBlockMax, pow2_floor(ymt));
  h.lbw = 0;
  while ((1 << h.lbw) < h.sbw) ++h.lbw;
  h.bst = pl->ny * h.sbw;
  div_magic((unsigned)h.bst, h.bst_mul, h.bst_shift);
  pl->triP = triP;
  pl->tricw = tricw;
  h.fx = fx;
  h.fy = fy;
  h.ymt = ymt;
  h.triP = triP;
  h.tris = s;
  h.tricw = cw;
  return MONC_OK;
}

static int upload_desc(monc_plan* pl) {
  HIP_TRY(hipMemcpy(pl->d_desc, &pl->h, sizeof(MemberDesc), hipMemcpyHostToDevice));
  return MONC_OK;
}

// ---------------------------------------------------------------------------
// tuning cache (flat JSON object: "arch:nx,ny,nz:dtype" -> [ex, ey, ymt, triP, tricw, xpw, yept];
// entries without the last value read it as 0, the default)
// ---------------------------------------------------------------------------
static std::mutex g_cache_mu;

static std::string cache_key(const monc_plan* pl) {
  char buf[128];
  std::snprintf(buf, sizeof buf, "gfx950:%d,%d,%d:%s", pl->nx, pl->ny, pl->nz,
                pl->dtype == MONC_FP64 ? "fp64" : "mixed");
  return buf;
}

static std::map<std::string, std::vector<int>> read_cache(const char* path) {
  std::map<std::string, std::vector<int>> out;
  FILE* f = std::fopen(path, "r");
  if (!f) return out;
  std::string s;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
  std::fclose(f);
  size_t pos = 0;
  while ((pos = s.find('"', pos)) != std::string::npos) {
    const size_t end = s.find('"', pos + 1);
    if (end == std::string::npos) break;
    std::string key = s.substr(pos + 1, end - pos - 1);
    const size_t lb = s.find('[', end), rb = s.find(']', end);
    if (lb == std::string::npos || rb == std::string::npos || rb < lb) break;
    std::vector<int> vals;
    const char* p = s.c_str() + lb + 1;
    while (p < s.c_str() + rb) {
      char* q = nullptr;
      long v = std::strtol(p, &q, 10);
      if (q == p) { ++p; continue; }
      vals.push_back((int)v);
      p = q;
    }
    out[key] = vals;
    pos = rb + 1;
  }
  return out;
}

static void write_cache(const char* path, const std::map<std::string, std::vector<int>>& m) {
  std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  size_t i = 0;
  for (auto& kv : m) {
    std::fprintf(f, "  \"%s\": [", kv.first.c_str());
    for (size_t j = 0; j < kv.second.size(); ++j) std::fprintf(f, "%s%d", j ? ", " : "", kv.second[j]);
    std::fprintf(f, "]%s\n", ++i < m.size() ? "," : "");
  }
  std::fprintf(f, "}\n");
  std::fclose(f);
  std::rename(tmp.c_str(), path);
}

// ---------------------------------------------------------------------------
// static workspace of the allocation-free entry point (monc_project_noalloc)
// ---------------------------------------------------------------------------
// One array per GPU, held until the process ends. In host code the name
// `scratch` only stands for the symbol: its device address (different on
// every device) comes from hipGetSymbolAddress, resolved once per device with
// that device current and kept in g_scratch_ptr.
static constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the static workspace on the current device.
static int static_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(MONC_EHIP, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return fail(MONC_EUNSUPPORTED, "device %d is beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(MONC_EHIP, "hipGetSymbolAddress of the static workspace failed on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MONC_OK;
}

// ---------------------------------------------------------------------------
// plan creation
// ---------------------------------------------------------------------------
extern "C" monc_plan* monc_plan_create(int nx, int ny, int nz, double dx, double dy, const double* dz,
                                       const double* rho0, int dtype) {
  std::string err;
  const int rc = check_plan_args(nx, ny, nz, dx, dy, dz, rho0, dtype, err);
  if (rc != MONC_OK) {
    g_err = err;
    return nullptr;
  }
  auto pl = std::make_unique<monc_plan>();
  pl->id = g_plan_ids.fetch_add(1);
  pl->nx = nx;
  pl->ny = ny;
  pl->nz = nz;
  pl->dx = dx;
  pl->dy = dy;
  pl->dtype = dtype;
  pl->dz.assign(dz, dz + nz);
  pl->rho0.assign(rho0, rho0 + nz);
  MemberDesc& h = pl->h;
  h.nx = nx;
  h.ny = ny;
  h.nz = nz;
  h.nxh = nx / 2 + 1;
  h.nxp = (h.nxh + kSpecBlockMax - 1) / kSpecBlockMax * kSpecBlockMax;
  h.dtype = dtype;
  h.nrow = (long long)nz * ny;
  // spectral level stride: an odd multiple of 256 bytes, so that the
  // tridiagonal solver's walk down a column does not revisit one HBM channel
  h.plane = (long long)ny * h.nxp;
  {
    const long long cbytes = (long long)cplx_bytes(dtype);
    if (((h.plane * cbytes) / 256) % 2 == 0) h.plane += 256 / cbytes;
  }
  h.rdx = 1.0 / dx;
  h.rdy = 1.0 / dy;
  h.inv_nxny = 1.0 / ((double)nx * (double)ny);
  // stencil kernels walk (8 level x J row pair) tiles once a level of one
  // field outgrows an XCD's L2 share (4 MB); smaller grids stay in row order.
  // The x-forward kernels take J row pairs of about 512 KB per level and
  // field (8 to 64 pairs: 64 at 1024 FP32 points a row, 32 at 2048 FP32 or
  // 1024 FP64, 16 at 2048 FP64 or 4096 FP32, 8 at 4096 FP64), the gradient
  // J = 8 rows: each workgroup writes its spectral bins as short runs spread
  // over the level, which a tile whose J pairs run at about the same time
  // turns into longer runs, while the neighbour rows its stencil re-reads
  // must still meet in L2. At 2048^2 x 160 (mixed) 32 pairs against 8: the
  // divergence 2.47 -> 2.31 ms and the residual 3.45 -> 3.30 ms; 64 pairs
  // were as fast but re-read 15-20 % more from HBM (traffic over
  // algorithmic bytes 1.21 / 1.60 against 1.07 / 1.34).
  h.ptk = ((double)nx * ny * elem_bytes(dtype) >= 4.0 * (1 << 20)) ? 8 : 1;
  {
    const double pair_bytes = 2.0 * nx * elem_bytes(dtype);
    int j = 8;
    while (j < 64 && 2 * j * pair_bytes <= (double)(1 << 19)) j *= 2;
    h.ptj = j;
  }
  h.rdxf = (float)h.rdx;
  h.rdyf = (float)h.rdy;
  // tile parameters (cached tuning first)
  int ex = 0, ey = 0, ymt = 0, triP = 0, tricw = 0, xpw = 0, yept = 0;
  if (const char* path = std::getenv("MONC_TUNE_CACHE")) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto m = read_cache(path);
    auto it = m.find(cache_key(pl.get()));
    if (it != m.end() && (it->second.size() == MONC_NPARAMS || it->second.size() == MONC_NPARAMS - 1)) {
      ex = it->second[0];
      ey = it->second[1];
      ymt = it->second[2];
      triP = it->second[3];
      tricw = it->second[4];
      xpw = it->second[5];
      yept = it->second.size() > 6 ? it->second[6] : 0;
    }
  }
  if (configure_tiles(pl.get(), ex, ey, ymt, triP, tricw, xpw, yept) != MONC_OK &&
      configure_tiles(pl.get(), 8, 8, 0, 0, 0, 0, 0) != MONC_OK)
    return nullptr;

  // host tables
  VerticalTables vt = vertical_tables(nz, dz, rho0);
  h.rH = vt.rH;
  {
    double sr = 0.0, cmax = 0.0;
    for (int k = 0; k < nz; ++k) {
      sr += dz[k] * rho0[k];
      cmax = std::max(cmax, (vt.ta[k] + vt.tc[k]) / rho0[k]);
    }
    h.rSr = 1.0 / sr;
    // a column with lam >= 1e-4 max_k (a_k + c_k)/rho0_k has a condition
    // number below ~1e4 and gains nothing from the deflation
    h.lamdef = 1e-4 * cmax;
  }
  std::vector<double> lamx = modified_wavenumbers(nx, h.nxh, dx);
  std::vector<double> lamy = modified_wavenumbers(ny, ny, dy);
  std::vector<double> twx = twiddles(nx), twy = twiddles(ny);

  // one device blob for the tables: 7 FP64 vertical, 3 FP32 vertical,
  // lamx, lamy, twiddles in the storage precision
  const size_t eb = elem_bytes(dtype);
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  size_t off = 0;
  const size_t o_v64 = off; off += al(7 * (size_t)nz * 8);
  const size_t o_v32 = off; off += al(3 * (size_t)nz * 4);
  const size_t o_lx = off; off += al((size_t)h.nxh * 8);
  const size_t o_ly = off; off += al((size_t)ny * 8);
  const size_t o_tx = off; off += al((size_t)nx * 2 * eb);
  const size_t o_ty = off; off += al((size_t)ny * 2 * eb);
  const size_t o_tr = off; off += al(3 * (size_t)(nz + kTriPmax) * 8);
  const size_t tables_bytes = off;
  std::vector<unsigned char> blob(tables_bytes, 0);
  double* v64 = reinterpret_cast<double*>(blob.data() + o_v64);
  const std::vector<double>* cols[7] = {&vt.rho0, &vt.rhow, &vt.rdz, &vt.rdzc, &vt.dz, &vt.ta, &vt.tc};
  for (int t = 0; t < 7; ++t) std::memcpy(v64 + (size_t)t * nz, cols[t]->data(), (size_t)nz * 8);
  float* v32 = reinterpret_cast<float*>(blob.data() + o_v32);
  for (int k = 0; k < nz; ++k) {
    v32[k] = (float)vt.rho0[k];
    v32[nz + k] = (float)vt.rhow[k];
    v32[2 * nz + k] = (float)vt.rdz[k];
  }
  std::memcpy(blob.data() + o_lx, lamx.data(), lamx.size() * 8);
  std::memcpy(blob.data() + o_ly, lamy.data(), lamy.size() * 8);
  auto put_tw = [&](size_t o, const std::vector<double>& tw) {
    if (dtype == MONC_FP64) {
      std::memcpy(blob.data() + o, tw.data(), tw.size() * 8);
    } else {
      float* f = reinterpret_cast<float*>(blob.data() + o);
      for (size_t i = 0; i < tw.size(); ++i) f[i] = (float)tw[i];
    }
  };
  put_tw(o_tx, twx);
  put_tw(o_ty, twy);
  {
    const size_t nt = (size_t)nz + kTriPmax;
    double* tr = reinterpret_cast<double*>(blob.data() + o_tr);
    for (size_t k = 0; k < nt; ++k) {
      const bool in = k < (size_t)nz;
      tr[k] = in ? vt.ta[k] : 1.0;
      tr[nt + k] = in ? vt.tc[k] : 0.0;
      tr[2 * nt + k] = in ? vt.rho0[k] : 0.0;
    }
  }

  // device side
  std::call_once(g_attr_once, [] { init_kernel_attributes(); });
  if (hipGetDevice(&pl->device) != hipSuccess) {
    fail(MONC_EHIP, "hipGetDevice failed (no usable HIP device)");
    return nullptr;
  }
  {
    // set-up of the allocation-free entry point on this device (its first
    // call retries and reports a failure)
    void* unused = nullptr;
    (void)static_scratch(&unused);
  }
  pl->spec_elems = (size_t)nz * h.plane;
  auto release = [&]() {
    if (pl->d_tables) (void)hipFree(pl->d_tables);
    if (pl->d_spec) (void)hipFree(pl->d_spec);
    if (pl->d_s1) (void)hipFree(pl->d_s1);
    if (pl->d_s2) (void)hipFree(pl->d_s2);
    if (pl->d_desc) (void)hipFree(pl->d_desc);
  };
  if (hipMalloc(&pl->d_tables, tables_bytes) != hipSuccess ||
      hipMalloc(&pl->d_spec, pl->spec_elems * cplx_bytes(dtype)) != hipSuccess ||
      hipMalloc((void**)&pl->d_desc, sizeof(MemberDesc)) != hipSuccess ||
      (dtype == MONC_MIXED &&
       (hipMalloc((void**)&pl->d_s1, (size_t)nx * ny * nz * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&pl->d_s2, (size_t)nx * ny * nz * sizeof(float)) != hipSuccess))) {
    (void)hipGetLastError();
    release();
    fail(MONC_ENOMEM, "device allocation failed for a %dx%dx%d plan", nx, ny, nz);
    return nullptr;
  }
  if (hipMemcpy(pl->d_tables, blob.data(), tables_bytes, hipMemcpyHostToDevice) != hipSuccess) {
    release();
    fail(MONC_EHIP, "table upload failed");
    return nullptr;
  }
  unsigned char* base = reinterpret_cast<unsigned char*>(pl->d_tables);
  const double* d64 = reinterpret_cast<const double*>(base + o_v64);
  h.rho0 = d64;
  h.rhow = d64 + nz;
  h.rdz = d64 + 2 * (size_t)nz;
  h.rdzc = d64 + 3 * (size_t)nz;
  h.dz = d64 + 4 * (size_t)nz;
  h.ta = d64 + 5 * (size_t)nz;
  h.tc = d64 + 6 * (size_t)nz;
  h.tra = reinterpret_cast<const double*>(base + o_tr);
  h.trc = h.tra + nz + kTriPmax;
  h.trr = h.trc + nz + kTriPmax;
  const float* d32 = reinterpret_cast<const float*>(base + o_v32);
  h.rho0f = d32;
  h.rhowf = d32 + nz;
  h.rdzf = d32 + 2 * (size_t)nz;
  h.lamx = reinterpret_cast<const double*>(base + o_lx);
  h.lamy = reinterpret_cast<const double*>(base + o_ly);
  h.twx = base + o_tx;
  h.twy = base + o_ty;
  h.spec = pl->d_spec;
  if (upload_desc(pl.get()) != MONC_OK) {
    release();
    return nullptr;
  }
  g_err.clear();
  return pl.release();
}

static void drop_batch_cache_for(unsigned long long plan_id);

extern "C" void monc_plan_destroy(monc_plan* pl) {
  if (!pl) return;
  drop_batch_cache_for(pl->id);
  if (pl->d_tables) (void)hipFree(pl->d_tables);
  if (pl->d_spec) (void)hipFree(pl->d_spec);
  if (pl->d_s1) (void)hipFree(pl->d_s1);
  if (pl->d_s2) (void)hipFree(pl->d_s2);
  if (pl->d_desc) (void)hipFree(pl->d_desc);
  if (pl->d_var) (void)hipFree(pl->d_var);
  delete pl;
}

extern "C" const char* monc_last_error(void) { return g_err.c_str(); }

extern "C" size_t monc_spectral_layout(const monc_plan* pl, int* row_len, int* col_block, long long* plane_len,
                                       int* eb) {
  if (!pl) return 0;
  if (row_len) *row_len = pl->h.nxp;
  if (col_block) *col_block = pl->h.sbw;
  if (plane_len) *plane_len = pl->h.plane;
  if (eb) *eb = (int)cplx_bytes(pl->dtype);
  return pl->spec_elems;
}

extern "C" const char* monc_kernel_name(int id) {
  static const char* names[MONC_K_COUNT] = {"div_fftx", "ffty_fwd",  "tridiag",    "ffty_inv",
                                            "ifftx",    "grad",      "resid_fftx", "grad_final"};
  if (id < 0 || id >= MONC_K_COUNT) return "";
  return names[id];
}

// ---------------------------------------------------------------------------
// grouped launches
// ---------------------------------------------------------------------------
struct GroupMember {
  const MemberDesc* h;  // host copy
  const MemberDesc* d;  // device copy
  IoPtrs io;
};

struct Group {
  std::vector<GroupMember> mem;
  bool fp64 = true;
};

enum Phase {
  PH_XFWD, PH_XPRE, PH_RESID, PH_YFWD, PH_TRI, PH_YINV, PH_XINV, PH_XINV_P1, PH_XINV_CORR, PH_GRAD, PH_GRAD_MIXED
};

static int phase_kernel_id(Phase ph) {
  switch (ph) {
    case PH_XFWD: case PH_XPRE: return MONC_K_DIV_FFTX;
    case PH_RESID: return MONC_K_RESID_FFTX;
    case PH_YFWD: return MONC_K_FFTY_FWD;
    case PH_TRI: return MONC_K_TRIDIAG;
    case PH_YINV: return MONC_K_FFTY_INV;
    case PH_XINV: case PH_XINV_P1: case PH_XINV_CORR: return MONC_K_IFFTX;
    case PH_GRAD: return MONC_K_GRAD;
    case PH_GRAD_MIXED: return MONC_K_GRAD_FINAL;
  }
  return 0;
}

static bool is_xphase(Phase ph) {
  return ph == PH_XFWD || ph == PH_XPRE || ph == PH_RESID || ph == PH_XINV || ph == PH_XINV_P1 || ph == PH_XINV_CORR;
}
static bool is_yphase(Phase ph) { return ph == PH_YFWD || ph == PH_YINV; }

// Launch shape of one member in one phase. Members whose shapes agree share
// a launch; `variant` identifies the kernel instance (compile-time length or
// the runtime-length kernel) and `block` its workgroup size.
struct Shape {
  int variant = 0;   // compile-time length, or 0 for the runtime-length kernel
  int sub = 0;       // kernel instance within the variant (tridiagonal: column pairs)
  int block = 256;
  size_t lds = 0;
  long long blocks = 0;       // tiles of the phase
  bool persistent = false;    // the grid covers the CUs once and walks the tiles
};


// compute units of the current device (queried once per device)
static int cu_count() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int n = cache[dev].load();
  if (n <= 0) {
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cache[dev].store(n);
  }
  return n;
}

static Shape member_shape(const MemberDesc& d, Phase ph, bool fp64) {
  const size_t cb = fp64 ? 16 : 8;
  Shape s;
  if (is_xphase(ph)) {
    const long long pairs = (d.nrow + 1) / 2;
    if (ct_supported(d.nx)) {
      const int nt = ct_threads_host(d.nx);
      int ipw = d.xpw > 0 ? d.xpw : std::max(1, 256 / nt);
      // the residual kernel at these lengths walks whole rows per wave: its
      // workgroups hold whole waves, the nearest multiple of m transforms
      // (up, unless that passes 512 threads; m nt <= 512, and at most 16
      // transforms of 256 to 1536 points stay within the LDS limit)
      if (ph == PH_RESID && xres_wave_rows(d.nx)) {
        const int m = wave_transforms(nt);
        ipw = (ipw + m - 1) / m * m;
        if (ipw * nt > 512) ipw -= m;
      }
      s.variant = d.nx;
      s.block = ipw * nt;
      s.lds = (size_t)ipw * xlds_len(d.nx, (int)cb) * cb;
      s.blocks = (pairs + ipw - 1) / ipw;
    } else {
      s.block = std::max(256, (d.fx.nt + 63) / 64 * 64);
      const int ipw = s.block / d.fx.nt;
      s.lds = (size_t)ipw * d.nx * cb;
      s.blocks = (pairs + ipw - 1) / ipw;
    }
  } else if (is_yphase(ph)) {
    if (ct_supported(d.ny) && d.yept == 32) {
      // the persistent kernel: a fixed number of columns per tile (ymt then
      // only sets the spectral column blocks)
      const int nt = ct_threads_y_host(d.ny, 32);
      const int mt = pp_columns(d.ny);
      s.variant = d.ny;
      s.block = mt * nt;
      s.lds = (size_t)d.ny * (mt + 1) * cb;  // the tile and the twiddle table
      s.blocks = (long long)d.nz * ((d.nxh + mt - 1) / mt);
      s.persistent = true;
    } else if (ct_supported(d.ny)) {
      const int nt = ct_threads_y_host(d.ny, d.yept);
      const int mt = std::max(1, std::min(d.ymt, 1024 / nt));
      s.variant = d.ny;
      s.block = mt * nt;
      s.lds = (size_t)d.ny * mt * cb;
      s.blocks = (long long)d.nz * ((d.nxh + mt - 1) / mt);
    } else {
      s.block = std::max(64, (d.ymt * d.fy.nt + 63) / 64 * 64);
      s.lds = (size_t)d.ny * d.ymt * cb;
      s.blocks = (long long)d.nz * ((d.nxh + d.ymt - 1) / d.ymt);
    }
  } else if (ph == PH_TRI) {
    s.variant = d.tris;
    s.sub = tri_pairs(d.tris, d.tricw, !fp64) ? 1 : 0;
    s.block = d.tricw * d.triP;
    s.lds = (size_t)d.tricw * (d.triP * tri_lane_slots(d.tris, !fp64) + 1) * 16;  // matches the kernel's column stride
    s.blocks = ((long long)d.ny * d.nxp + d.tricw - 1) / d.tricw;  // over the padded plane
  } else {
    // points per thread: 16-byte field accesses on the mixed path (4 floats),
    // 2 doubles on the FP64 path; fewer when nx does not divide
    const int want = (ph == PH_GRAD_MIXED) ? 4 : 2;
    const int vec = (d.nx % want == 0) ? want : (d.nx % 2 == 0) ? 2 : 1;
    const long long nvec = (long long)d.nx * d.ny * d.nz / vec;
    s.variant = vec;
    s.blocks = (nvec + 255) / 256;
  }
  return s;
}

static int launch_one(const Group& g, const std::vector<int>& idx, Phase ph, const Shape& sh, void* stream,
                      Profiler* prof) {
  LaunchArgs a;
  std::memset(&a, 0, sizeof a);
  a.nmem = (int)idx.size();
  long long blocks = 0;
  size_t lds = 0;
  int block = sh.block;
  for (size_t t = 0; t < idx.size(); ++t) {
    const GroupMember& m = g.mem[idx[t]];
    const Shape s = member_shape(*m.h, ph, g.fp64);
    a.mem[t] = m.d;
    a.io[t] = m.io;
    a.block_start[t] = (int)blocks;
    blocks += s.blocks;
    lds = std::max(lds, s.lds);
    block = std::max(block, s.block);
    if (blocks > (1LL << 31) - 1) return fail(MONC_EUNSUPPORTED, "grid too large");
  }
  a.block_start[idx.size()] = (int)blocks;
  if (block > 1024) return fail(MONC_EUNSUPPORTED, "launch needs %d threads per workgroup", block);
  if (lds > 160 * 1024) return fail(MONC_EUNSUPPORTED, "phase needs %zu bytes of LDS", lds);
  if (blocks == 0) return MONC_OK;
  // a persistent kernel takes one workgroup per CU slot its LDS leaves
  const long long slots = (long long)cu_count() * (long long)std::max<size_t>(1, (160 * 1024) / std::max<size_t>(lds, 1));
  const int grid = sh.persistent ? (int)std::min(blocks, slots) : (int)blocks;
  const int kid = phase_kernel_id(ph);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timed = prof && (prof->mask >> kid & 1u);
  if (timed) {
    std::lock_guard<std::mutex> lk(prof->mu);
    e0 = prof->get();
    e1 = prof->get();
    if (e0) (void)hipEventRecord(e0, (hipStream_t)stream);
  }
  const int v = sh.variant;
  switch (ph) {
    case PH_XFWD: launch_xfwd(a, grid, block, lds, g.fp64, 0, v, stream); break;
    case PH_XPRE: launch_xfwd(a, grid, block, lds, g.fp64, 2, v, stream); break;
    case PH_RESID: launch_xfwd(a, grid, block, lds, false, 1, v, stream); break;
    case PH_YFWD: launch_ffty(a, grid, block, lds, g.fp64, false, v, g.mem[idx[0]].h->yept, stream); break;
    case PH_YINV: launch_ffty(a, grid, block, lds, g.fp64, true, v, g.mem[idx[0]].h->yept, stream); break;
    case PH_TRI: launch_tridiag(a, grid, block, lds, g.fp64, v, sh.sub != 0, stream); break;
    case PH_XINV: launch_xinv(a, grid, block, lds, g.fp64, 0, v, stream); break;
    case PH_XINV_P1: launch_xinv(a, grid, block, lds, false, 2, v, stream); break;
    case PH_XINV_CORR: launch_xinv(a, grid, block, lds, false, 1, v, stream); break;
    case PH_GRAD:
    case PH_GRAD_MIXED: {
      // per-level reductions of the outputs when the caller asked for them
      bool red = false;
      for (size_t t = 0; t < idx.size(); ++t)
        if (a.io[t].stats) {
          launch_stats_init(a.io[t].stats, g.mem[idx[t]].h->nz, stream);
          red = true;
        }
      launch_grad(a, grid, ph == PH_GRAD && g.fp64, v, red, stream);
      break;
    }
  }
  hipError_t le = hipGetLastError();
  if (timed) {
    std::lock_guard<std::mutex> lk(prof->mu);
    if (e1) (void)hipEventRecord(e1, (hipStream_t)stream);
    if (e0 && e1) prof->recs.push_back({kid, e0, e1});
  }
  if (le != hipSuccess) return fail(MONC_EHIP, "launch of %s failed: %s", monc_kernel_name(kid), hipGetErrorString(le));
  return MONC_OK;
}

// One phase for every member of the group: members are partitioned by kernel
// instance and workgroup size, and each partition (up to kMaxLaunchMembers
// members) is one launch.
static int launch_phase(const Group& g, Phase ph, void* stream, Profiler* prof) {
  std::vector<std::pair<std::array<int, 3>, std::vector<int>>> parts;
  std::vector<Shape> shapes;
  for (int i = 0; i < (int)g.mem.size(); ++i) {
    const Shape s = member_shape(*g.mem[i].h, ph, g.fp64);
    // the compile-time kernels need blockDim to match each member exactly,
    // and the y kernels the member's elements per thread
    const std::array<int, 3> key{s.variant, s.variant ? s.block : 0,
                                 !s.variant ? 0 : is_yphase(ph) ? g.mem[i].h->yept : s.sub};
    size_t pi = 0;
    while (pi < parts.size() && (parts[pi].first != key || parts[pi].second.size() >= (size_t)kMaxLaunchMembers)) ++pi;
    if (pi == parts.size()) {
      parts.push_back({key, {}});
      shapes.push_back(s);
    }
    parts[pi].second.push_back(i);
  }
  for (size_t pi = 0; pi < parts.size(); ++pi) {
    const int rc = launch_one(g, parts[pi].second, ph, shapes[pi], stream, prof);
    if (rc != MONC_OK) return rc;
  }
  return MONC_OK;
}

static int run_phases(const std::vector<Group>& groups, const std::vector<Phase>& phases, void* stream,
                      Profiler* prof) {
  for (Phase ph : phases)
    for (const auto& g : groups) {
      const int rc = launch_phase(g, ph, stream, prof);
      if (rc != MONC_OK) return rc;
    }
  return MONC_OK;
}

static const std::vector<Phase>& full_sequence(bool fp64) {
  static const std::vector<Phase> f64 = {PH_XFWD, PH_YFWD, PH_TRI, PH_YINV, PH_XINV, PH_GRAD};
  // mixed: the first solve leaves p1 in s2; the residual D(u*) - L p1
  // (FP64) is solved for the correction delta (into s1); the gradient kernel
  // forms p1 + delta in FP64, corrects u, v, w with it and writes p
  static const std::vector<Phase> mixed = {PH_XFWD, PH_YFWD, PH_TRI, PH_YINV, PH_XINV_P1, PH_RESID,
                                           PH_YFWD, PH_TRI,  PH_YINV, PH_XINV_CORR, PH_GRAD_MIXED};
  return fp64 ? f64 : mixed;
}

// The launch pointers of one member: caller fields, the plan's spectral
// workspace and (mixed plans) its two scratch fields.
static IoPtrs plan_io(const monc_plan* pl, void* u, void* v, void* w, void* p) {
  IoPtrs io;
  io.u = u;
  io.v = v;
  io.w = w;
  io.p = p;
  io.spec = pl->d_spec;
  io.s1 = pl->d_s1;
  io.s2 = pl->d_s2;
  return io;
}

// ---------------------------------------------------------------------------
// pointer checks
// ---------------------------------------------------------------------------
static int check_fields(const monc_plan* pl, void* const* ptrs, int n, const char* what) {
  const size_t bytes = (size_t)pl->nx * pl->ny * pl->nz * elem_bytes(pl->dtype);
  for (int i = 0; i < n; ++i) {
    if (!ptrs[i]) return fail(MONC_EINVAL, "%s: pointer %d is null", what, i);
    if (reinterpret_cast<uintptr_t>(ptrs[i]) % 16 != 0)
      return fail(MONC_EINVAL, "%s: pointer %d is not 16-byte aligned", what, i);
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const uintptr_t a = reinterpret_cast<uintptr_t>(ptrs[i]), b = reinterpret_cast<uintptr_t>(ptrs[j]);
      if (a < b + bytes && b < a + bytes) return fail(MONC_EINVAL, "%s: arrays %d and %d overlap", what, i, j);
    }
  return MONC_OK;
}

static int check_device(const monc_plan* pl) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(MONC_EHIP, "hipGetDevice failed");
  if (dev != pl->device)
    return fail(MONC_EINVAL, "plan was created on device %d but device %d is current", pl->device, dev);
  return MONC_OK;
}

// ---------------------------------------------------------------------------
// single projection
// ---------------------------------------------------------------------------
extern "C" int monc_project(monc_plan* pl, void* u, void* v, void* w, void* p, void* stream) {
  if (!pl) return fail(MONC_EINVAL, "plan is null");
  void* ptrs[4] = {u, v, w, p};
  int rc = check_fields(pl, ptrs, 4, "monc_project");
  if (rc != MONC_OK) return rc;
  rc = check_device(pl);
  if (rc != MONC_OK) return rc;
  Group g;
  g.fp64 = pl->dtype == MONC_FP64;
  g.mem.push_back({&pl->h, pl->d_desc, plan_io(pl, u, v, w, p)});
  std::vector<Group> groups{g};
  return run_phases(groups, full_sequence(g.fp64), stream, pl->prof.mask ? &pl->prof : nullptr);
}

extern "C" int monc_project_reduce(monc_plan* pl, void* u, void* v, void* w, void* p, double* stats,
                                   void* stream) {
  if (!pl) return fail(MONC_EINVAL, "plan is null");
  if (!stats || reinterpret_cast<uintptr_t>(stats) % 8 != 0) return fail(MONC_EINVAL, "stats is null or misaligned");
  void* ptrs[4] = {u, v, w, p};
  int rc = check_fields(pl, ptrs, 4, "monc_project_reduce");
  if (rc != MONC_OK) return rc;
  {
    const uintptr_t s0 = reinterpret_cast<uintptr_t>(stats), s1 = s0 + 8 * sizeof(double) * pl->nz;
    const size_t bytes = (size_t)pl->nx * pl->ny * pl->nz * elem_bytes(pl->dtype);
    for (int i = 0; i < 4; ++i) {
      const uintptr_t a = reinterpret_cast<uintptr_t>(ptrs[i]);
      if (a < s1 && s0 < a + bytes) return fail(MONC_EINVAL, "monc_project_reduce: stats overlaps array %d", i);
    }
  }
  rc = check_device(pl);
  if (rc != MONC_OK) return rc;
  Group g;
  g.fp64 = pl->dtype == MONC_FP64;
  IoPtrs io = plan_io(pl, u, v, w, p);
  io.stats = stats;
  g.mem.push_back({&pl->h, pl->d_desc, io});
  std::vector<Group> groups{g};
  return run_phases(groups, full_sequence(g.fp64), stream, pl->prof.mask ? &pl->prof : nullptr);
}

// ---------------------------------------------------------------------------
// allocation-free projection
// ---------------------------------------------------------------------------
static size_t align256(size_t x);

extern "C" int monc_project_noalloc(monc_plan* pl, void* u, void* v, void* w, void* p, void* stream) {
  if (!pl) return fail(MONC_EINVAL, "plan is null");
  void* ptrs[4] = {u, v, w, p};
  int rc = check_fields(pl, ptrs, 4, "monc_project_noalloc");
  if (rc != MONC_OK) return rc;
  rc = check_device(pl);
  if (rc != MONC_OK) return rc;
  const bool fp64 = pl->dtype == MONC_FP64;
  const size_t spec = align256(pl->spec_elems * cplx_bytes(pl->dtype));
  const size_t field = align256((size_t)pl->nx * pl->ny * pl->nz * sizeof(float));
  const size_t need = spec + (fp64 ? 0 : 2 * field);
  if (need > kStaticScratchBytes)
    return fail(MONC_EUNSUPPORTED,
                "monc_project_noalloc: a %dx%dx%d %s plan needs %zu bytes of workspace, above the static %zu",
                pl->nx, pl->ny, pl->nz, fp64 ? "FP64" : "MIXED", need, kStaticScratchBytes);
  void* base = nullptr;
  rc = static_scratch(&base);
  if (rc != MONC_OK) return rc;
  // the plan's own workspace is not touched: every kernel takes its
  // workspace pointers from the launch arguments
  unsigned char* b = static_cast<unsigned char*>(base);
  IoPtrs io = plan_io(pl, u, v, w, p);
  io.spec = b;
  io.s1 = fp64 ? nullptr : reinterpret_cast<float*>(b + spec);
  io.s2 = fp64 ? nullptr : reinterpret_cast<float*>(b + spec + field);
  Group g;
  g.fp64 = fp64;
  g.mem.push_back({&pl->h, pl->d_desc, io});
  std::vector<Group> groups{g};
  return run_phases(groups, full_sequence(fp64), stream, nullptr);  // no profiling events
}

// ---------------------------------------------------------------------------
// variable-density projection: preconditioned conjugate gradients
// ---------------------------------------------------------------------------
static constexpr int kVarMaxIt = 10000;

// Work vectors of one plan, carved from one allocation: r, d, q (FP64
// fields), z (storage type), two partial-sum arrays, the scalars (status
// row and one row per iteration), the vertical interpolation weights za, zb,
// the preconditioner's device descriptor and its scaling field s (FP32).
struct VarWs {
  double *r, *d, *q, *part0, *part1, *scal, *za, *zb;
  void* z;
  MemberDesc* desc;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int var_workspace(monc_plan* pl, VarWs* ws) {
  const size_t n = (size_t)pl->nx * pl->ny * pl->nz;
  const size_t nparts = (size_t)var_point_parts(pl->nx, pl->ny, pl->nz);  // the larger count
  constexpr int kParts = 10;
  const size_t sizes[kParts] = {n * 8, n * 8, n * 8, n * elem_bytes(pl->dtype), nparts * 8, nparts * 8,
                                (size_t)(kVarMaxIt + 2) * kVarSlots * 8, (size_t)pl->nz * 8, (size_t)pl->nz * 8,
                                sizeof(MemberDesc)};
  size_t off[kParts], total = 0;
  for (int i = 0; i < kParts; ++i) {
    off[i] = total;
    total += align256(sizes[i]);
  }
  if (!pl->d_var) {
    if (hipMalloc(&pl->d_var, total) != hipSuccess) {
      pl->d_var = nullptr;
      (void)hipGetLastError();
      return fail(MONC_ENOMEM, "monc_project_var: cannot allocate %zu bytes of work vectors", total);
    }
    std::vector<double> za, zb;
    face_weights(pl->nz, pl->dz.data(), za, zb);
    char* b = static_cast<char*>(pl->d_var);
    if (hipMemcpy(b + off[7], za.data(), pl->nz * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b + off[8], zb.data(), pl->nz * 8, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(pl->d_var);
      pl->d_var = nullptr;
      return fail(MONC_EHIP, "monc_project_var: upload of the interpolation weights failed");
    }
  }
  char* b = static_cast<char*>(pl->d_var);
  ws->r = reinterpret_cast<double*>(b + off[0]);
  ws->d = reinterpret_cast<double*>(b + off[1]);
  ws->q = reinterpret_cast<double*>(b + off[2]);
  ws->z = b + off[3];
  ws->part0 = reinterpret_cast<double*>(b + off[4]);
  ws->part1 = reinterpret_cast<double*>(b + off[5]);
  ws->scal = reinterpret_cast<double*>(b + off[6]);
  ws->za = reinterpret_cast<double*>(b + off[7]);
  ws->zb = reinterpret_cast<double*>(b + off[8]);
  ws->desc = reinterpret_cast<MemberDesc*>(b + off[9]);
  return MONC_OK;
}

static int read_scalars(const double* dev, double* host, int n, void* stream) {
  if (hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess ||
      hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    return fail(MONC_EHIP, "monc_project_var: reading the solver's status failed: %s",
                hipGetErrorString(hipGetLastError()));
  return MONC_OK;
}

static int var_launched(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MONC_EHIP, "monc_project_var: launch of %s failed: %s", what, hipGetErrorString(e));
  return MONC_OK;
}

extern "C" int monc_project_var(monc_plan* pl, const double* rho, double* u, double* v, double* w, double* p,
                                double tol, int maxit, int* iters, double* relres, void* stream) {
  if (!pl) return fail(MONC_EINVAL, "plan is null");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(MONC_EINVAL, "monc_project_var: tol must be finite and >= 0");
  if (maxit < 1 || maxit > kVarMaxIt)
    return fail(MONC_EINVAL, "monc_project_var: maxit must be in [1, %d], got %d", kVarMaxIt, maxit);
  {
    void* ptrs[5] = {const_cast<double*>(rho), u, v, w, p};
    const size_t bytes = (size_t)pl->nx * pl->ny * pl->nz * sizeof(double);
    for (int i = 0; i < 5; ++i) {
      if (!ptrs[i]) return fail(MONC_EINVAL, "monc_project_var: pointer %d is null", i);
      if (reinterpret_cast<uintptr_t>(ptrs[i]) % 16 != 0)
        return fail(MONC_EINVAL, "monc_project_var: pointer %d is not 16-byte aligned", i);
    }
    for (int i = 0; i < 5; ++i)
      for (int j = i + 1; j < 5; ++j) {
        const uintptr_t a = reinterpret_cast<uintptr_t>(ptrs[i]), b = reinterpret_cast<uintptr_t>(ptrs[j]);
        if (a < b + bytes && b < a + bytes) return fail(MONC_EINVAL, "monc_project_var: arrays %d and %d overlap", i, j);
      }
  }
  int rc = check_device(pl);
  if (rc != MONC_OK) return rc;
  VarWs ws;
  rc = var_workspace(pl, &ws);
  if (rc != MONC_OK) return rc;
  const MemberDesc& h = pl->h;
  VarGrid g;
  g.nx = pl->nx;
  g.ny = pl->ny;
  g.nz = pl->nz;
  g.rdx = 1.0 / pl->dx;
  g.rdy = 1.0 / pl->dy;
  g.rdx2 = g.rdx * g.rdx;
  g.rdy2 = g.rdy * g.rdy;
  g.rho = rho;
  g.dz = h.dz;
  g.rdz = h.rdz;
  g.rdzc = h.rdzc;
  g.za = ws.za;
  g.zb = ws.zb;
  const long long np_st = var_stencil_parts(pl->nx, pl->ny, pl->nz);  // partials of the stencil kernels
  const long long np_pt = var_point_parts(pl->nx, pl->ny, pl->nz);    // partials of the pointwise kernels
  const bool z64 = pl->dtype == MONC_FP64;
  Profiler* prof = pl->prof.mask ? &pl->prof : nullptr;

  // preconditioner z = M^-1 r: the plan's spectral solve with r as its
  // source, through a copy of the plan's descriptor that carries the
  // solver's done flag (queued iterations past convergence then cost only
  // their launches)
  pl->h_pre = pl->h;
  pl->h_pre.skip = ws.scal + kVarDone;
  if (hipMemcpyAsync(ws.desc, &pl->h_pre, sizeof(MemberDesc), hipMemcpyHostToDevice, (hipStream_t)stream) !=
      hipSuccess)
    return fail(MONC_EHIP, "monc_project_var: descriptor upload failed");
  Group pre;
  pre.fp64 = z64;
  IoPtrs pio;
  pio.u = ws.r;
  pio.p = ws.z;
  pio.spec = pl->d_spec;
  pre.mem.push_back({&pl->h_pre, ws.desc, pio});
  static const std::vector<Phase> pre_seq = {PH_XPRE, PH_YFWD, PH_TRI, PH_YINV, PH_XINV};
  const std::vector<Group> pre_groups{pre};
  // z_it = M^-1 r_it, <r_it, z_it>, <z_it, q_{it-1}>, then d_it
  auto direction = [&](int i) {
    int e = run_phases(pre_groups, pre_seq, stream, prof);
    if (e != MONC_OK) return e;
    launch_var_dots(g, ws.scal, ws.r, ws.z, z64, ws.q, ws.part0, ws.part1, stream);
    if ((e = var_launched("the inner products")) != MONC_OK) return e;
    // <z, q> only for the flexible update (FP32 preconditioner)
    launch_var_finish(ws.part0, (i > 0 && !z64) ? ws.part1 : nullptr, np_pt, ws.scal, var_slot(i, kVarRZ),
                      var_slot(i, kVarZQ), true, stream);
    if ((e = var_launched("the partial-sum reduction")) != MONC_OK) return e;
    launch_var_dir(g, ws.scal, i, ws.z, z64, ws.d, stream);
    return var_launched("the direction update");
  };
  // q = L d_it, alpha, p_{it+1}, r_{it+1} and its norm (sets the done flag)
  const double tol2 = tol * tol;
  auto step = [&](int i) {
    launch_var_apply(g, ws.scal, ws.d, ws.q, ws.part0, stream);
    int e = var_launched("the operator");
    if (e != MONC_OK) return e;
    launch_var_finish(ws.part0, nullptr, np_st, ws.scal, var_slot(i, kVarDQ), 0, true, stream);
    if ((e = var_launched("the partial-sum reduction")) != MONC_OK) return e;
    launch_var_update(g, ws.scal, i, p, ws.r, ws.d, ws.q, ws.part0, stream);
    if ((e = var_launched("the solution update")) != MONC_OK) return e;
    launch_var_finish_rr(ws.part0, np_pt, ws.scal, i + 1, tol2, stream);
    return var_launched("the residual norm");
  };

  launch_var_zero(ws.scal, (maxit + 2) * kVarSlots, stream);
  launch_var_div(g, u, v, w, ws.r, p, ws.part0, stream);
  if ((rc = var_launched("the divergence")) != MONC_OK) return rc;
  // <r_0, r_0>, through the residual-norm reduction of iteration 0: it sets
  // the done flag when the input is already divergence-free (or tol >= 1) and
  // flags a non-finite input, so the host needs no read before the first
  // batch; a done flag makes the queued work of that batch return at once
  launch_var_finish_rr(ws.part0, np_st, ws.scal, 0, tol * tol, stream);
  if ((rc = var_launched("the partial-sum reduction")) != MONC_OK) return rc;
  int it = 0;
  double rel = 0.0;
  if ((rc = direction(0)) != MONC_OK) return rc;
  // Iterations are queued in batches and the status read once per batch;
  // the next batch's length is the iteration count that the convergence rate
  // seen so far predicts (at least 1, at most 32).
  int queued = 0, batch = 3;
  double rel_prev = 1.0;
  for (;;) {
    const int nb = std::min(batch, maxit - queued);
    for (int b = 0; b < nb; ++b, ++queued) {
      if ((rc = step(queued)) != MONC_OK) return rc;
      if (queued + 1 < maxit && (rc = direction(queued + 1)) != MONC_OK) return rc;
    }
    // the status row and iteration 0's row (<r_0, r_0>) in one read
    double st[2 * kVarSlots];
    if ((rc = read_scalars(ws.scal, st, 2 * kVarSlots, stream)) != MONC_OK) return rc;
    const double rr0 = st[var_slot(0, kVarRR)];
    it = (int)st[kVarLast];
    if (st[kVarDone] == 2.0) {
      if (it == 0) return fail(MONC_EINVAL, "monc_project_var: the divergence of the input is not finite");
      return fail(MONC_EINVAL, "monc_project_var: breakdown at iteration %d (is rho positive everywhere?)", it);
    }
    rel = rr0 > 0.0 ? std::sqrt(st[kVarLastRR] / rr0) : 0.0;
    if (st[kVarDone] != 0.0 || queued >= maxit) break;
    batch = krylov_batch(rel, rel_prev, nb, tol, 32);
    rel_prev = rel;
  }
  // the gauge in FP64: subtract the dz-weighted mean of p (the constants are
  // the operator's null space, so the residual does not change; an FP32
  // preconditioner's rounding would otherwise leave a small mean in p)
  if (it > 0) {
    double wsum = 0.0;
    for (int k = 0; k < pl->nz; ++k) wsum += pl->dz[k];
    launch_var_wsum(g, p, ws.part0, stream);
    if ((rc = var_launched("the gauge sum")) != MONC_OK) return rc;
    launch_var_finish(ws.part0, nullptr, np_pt, ws.scal, kVarGauge, 0, false, stream);
    if ((rc = var_launched("the partial-sum reduction")) != MONC_OK) return rc;
    launch_var_shift(g, ws.scal, kVarGauge, 1.0 / ((double)pl->nx * pl->ny * wsum), p, stream);
    if ((rc = var_launched("the gauge shift")) != MONC_OK) return rc;
  }
  if (iters) *iters = it;
  if (relres) *relres = rel;
  // u = u* - G p, w = 0 on the lid: the FP64 gradient kernel
  Group gr;
  gr.fp64 = true;
  gr.mem.push_back({&pl->h, pl->d_desc, plan_io(pl, u, v, w, p)});
  const std::vector<Group> grad_groups{gr};
  static const std::vector<Phase> grad_seq = {PH_GRAD};
  return run_phases(grad_groups, grad_seq, stream, prof);
}

// ---------------------------------------------------------------------------
// stage-wise access
// ---------------------------------------------------------------------------
extern "C" int monc_debug_stage(monc_plan* pl, int stage, void* const* bufs, int nbufs, void* stream) {
  if (!pl) return fail(MONC_EINVAL, "plan is null");
  if (!bufs) return fail(MONC_EINVAL, "bufs is null");
  int rc = check_device(pl);
  if (rc != MONC_OK) return rc;
  const bool fp64 = pl->dtype == MONC_FP64;
  auto need = [&](int n) { return nbufs == n ? MONC_OK : fail(MONC_EINVAL, "stage %d takes %d buffers (got %d)", stage, n, nbufs); };
  for (int i = 0; i < nbufs; ++i)
    if (!bufs[i] || reinterpret_cast<uintptr_t>(bufs[i]) % 16) return fail(MONC_EINVAL, "buffer %d is null or misaligned", i);
  IoPtrs io;
  std::vector<Phase> seq;
  switch (stage) {
    case MONC_STAGE_FORWARD:
      if ((rc = need(4))) return rc;
      io.u = bufs[0];
      io.v = bufs[1];
      io.w = bufs[2];
      io.spec = bufs[3];
      seq = {PH_XFWD, PH_YFWD};
      break;
    case MONC_STAGE_SOLVE:
      if ((rc = need(1))) return rc;
      io.spec = bufs[0];
      seq = {PH_TRI};
      break;
    case MONC_STAGE_INVERSE:
      if ((rc = need(2))) return rc;
      io.spec = bufs[0];
      io.p = bufs[1];
      seq = {PH_YINV, PH_XINV};
      break;
    case MONC_STAGE_GRADIENT:
      if ((rc = need(4))) return rc;
      if (!fp64) return fail(MONC_EINVAL, "the gradient stage takes an FP64 pressure (FP64 plans only)");
      io.u = bufs[1];
      io.v = bufs[2];
      io.w = bufs[3];
      io.p = bufs[0];
      seq = {PH_GRAD};
      break;
    case MONC_STAGE_RESIDUAL:
      if ((rc = need(5))) return rc;
      if (fp64) return fail(MONC_EINVAL, "the residual stage exists on MIXED plans only");
      io.u = bufs[0];
      io.v = bufs[1];
      io.w = bufs[2];
      io.s2 = static_cast<float*>(bufs[3]);
      io.spec = bufs[4];
      seq = {PH_RESID, PH_YFWD};
      break;
    default:
      return fail(MONC_EINVAL, "unknown stage %d", stage);
  }
  Group g;
  g.fp64 = fp64;
  g.mem.push_back({&pl->h, pl->d_desc, io});
  return run_phases({g}, seq, stream, nullptr);
}

// ---------------------------------------------------------------------------
// batched projection: grouped launches captured in a HIP graph
// ---------------------------------------------------------------------------
struct BatchEntry {
  std::vector<unsigned long long> key;
  std::vector<unsigned long long> plan_ids;
  MemberDesc* d_array = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  unsigned long long last_use = 0;
  ~BatchEntry() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (d_array) (void)hipFree(d_array);
  }
};

static std::mutex g_batch_mu;
static std::vector<std::unique_ptr<BatchEntry>> g_batches;
static unsigned long long g_batch_clock = 0;
static const size_t kBatchCacheSize = 8;

static void drop_batch_cache_for(unsigned long long plan_id) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  g_batches.erase(std::remove_if(g_batches.begin(), g_batches.end(),
                                 [&](const std::unique_ptr<BatchEntry>& e) {
                                   return std::find(e->plan_ids.begin(), e->plan_ids.end(), plan_id) !=
                                          e->plan_ids.end();
                                 }),
                  g_batches.end());
}

// ---------------------------------------------------------------------------
// batch schedule: member order and grouping (tuned by monc_autotune)
// ---------------------------------------------------------------------------
// order 0 puts the largest members first (their workgroups start first, the
// small ones fill the tail), order 1 the smallest first. budget_mb 0 runs
// every phase over all members (one launch per kernel instance and phase);
// otherwise members, in order, are packed into groups whose working set
// (fields, spectral workspace, scratch) stays under budget_mb MB, and the
// groups run one after the other, all phases of a group before the next, so
// that a group's intermediates can stay in the 256 MB Infinity Cache.
struct BatchSchedule {
  int order = 0;
  int budget_mb = 0;
  int branches = 1;  // independent graph branches the groups are dealt to
};

static std::mutex g_sched_mu;
static std::map<std::string, BatchSchedule> g_sched;

// Key of a batch for the tuned schedule: the multiset of member grids and
// the dtype (FNV-1a hash of the sorted grid list).
static std::string batch_key(monc_plan* const* plans, int count) {
  std::vector<std::string> grids;
  for (int i = 0; i < count; ++i) {
    char b[64];
    std::snprintf(b, sizeof b, "%d,%d,%d;", plans[i]->nx, plans[i]->ny, plans[i]->nz);
    grids.push_back(b);
  }
  std::sort(grids.begin(), grids.end());
  unsigned long long h = 1469598103934665603ull;
  for (const auto& g : grids)
    for (char c : g) {
      h ^= (unsigned char)c;
      h *= 1099511628211ull;
    }
  char key[128];
  std::snprintf(key, sizeof key, "gfx950:batch:%d:%016llx:%s", count, h,
                plans[0]->dtype == MONC_FP64 ? "fp64" : "mixed");
  return key;
}

static BatchSchedule lookup_schedule(monc_plan* const* plans, int count) {
  const std::string key = batch_key(plans, count);
  {
    std::lock_guard<std::mutex> lk(g_sched_mu);
    auto it = g_sched.find(key);
    if (it != g_sched.end()) return it->second;
  }
  BatchSchedule sc;
  if (const char* path = std::getenv("MONC_TUNE_CACHE")) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto m = read_cache(path);
    auto it = m.find(key);
    // [order, budget_mb] or [order, budget_mb, branches]
    if (it != m.end() && (it->second.size() == 2 || it->second.size() == 3) &&
        (it->second[0] == 0 || it->second[0] == 1) && it->second[1] >= 0 &&
        (it->second.size() == 2 || (it->second[2] >= 1 && it->second[2] <= MONC_MAX_BRANCHES))) {
      sc.order = it->second[0];
      sc.budget_mb = it->second[1];
      sc.branches = it->second.size() == 3 ? it->second[2] : 1;
    }
  }
  std::lock_guard<std::mutex> lk(g_sched_mu);
  g_sched[key] = sc;
  return sc;
}

static size_t member_bytes(const monc_plan* pl) {
  const size_t n = (size_t)pl->nx * pl->ny * pl->nz;
  return 4 * n * elem_bytes(pl->dtype) + pl->spec_elems * cplx_bytes(pl->dtype) +
         (pl->dtype == MONC_FP64 ? 0 : 2 * n * sizeof(float));
}

static std::vector<int> batch_order(monc_plan* const* plans, int count, int order) {
  std::vector<int> ord(count);
  for (int i = 0; i < count; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    const long long pa = (long long)plans[a]->nx * plans[a]->ny * plans[a]->nz;
    const long long pb = (long long)plans[b]->nx * plans[b]->ny * plans[b]->nz;
    return order == 0 ? pa > pb : pa < pb;
  });
  return ord;
}

static void build_groups(monc_plan* const* plans, int count, void* const* u, void* const* v, void* const* w,
                         void* const* p, const MemberDesc* d_array, const std::vector<int>& ord,
                         const BatchSchedule& sc, std::vector<Group>& groups) {
  groups.clear();
  const size_t budget = (size_t)sc.budget_mb << 20;
  Group g;
  g.fp64 = plans[0]->dtype == MONC_FP64;
  size_t used = 0;
  for (int t = 0; t < count; ++t) {
    const int i = ord[t];
    const size_t mb = member_bytes(plans[i]);
    if (budget && !g.mem.empty() && used + mb > budget) {
      groups.push_back(std::move(g));
      g = Group();
      g.fp64 = plans[0]->dtype == MONC_FP64;
      used = 0;
    }
    g.mem.push_back({&plans[i]->h, d_array + t, plan_io(plans[i], u[i], v[i], w[i], p[i])});
    used += mb;
  }
  groups.push_back(std::move(g));
}

// Every phase over all groups (phase-major), or all phases of each group in
// turn (group-major, the grouped schedules). With side streams (a capture in
// progress on `stream`), group-major group g goes to branch
// g mod (1 + side.size()): the captured graph then holds that many
// independent chains, which the device runs concurrently, so that one
// chain's small launches fill the tails and gaps another leaves.
static int run_batch(const std::vector<Group>& groups, const std::vector<Phase>& seq, bool group_major,
                     void* stream, Profiler* prof, const std::vector<hipStream_t>& side = {}) {
  if (!group_major) return run_phases(groups, seq, stream, prof);
  const size_t nb = 1 + std::min(side.size(), groups.size() ? groups.size() - 1 : 0);
  std::vector<hipEvent_t> ev;
  auto cleanup = [&]() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  };
  if (nb > 1) {  // fork: the side streams start after what the main one holds
    hipEvent_t fork = nullptr;
    if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess)
      return fail(MONC_EHIP, "batch: event creation failed");
    ev.push_back(fork);
    bool ok = hipEventRecord(fork, (hipStream_t)stream) == hipSuccess;
    for (size_t b = 1; b < nb && ok; ++b) ok = hipStreamWaitEvent(side[b - 1], fork, 0) == hipSuccess;
    if (!ok) {
      cleanup();
      return fail(MONC_EHIP, "batch: fork of the graph branches failed");
    }
  }
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    void* st = (gi % nb) ? (void*)side[gi % nb - 1] : stream;
    for (Phase ph : seq) {
      const int rc = launch_phase(groups[gi], ph, st, prof);
      if (rc != MONC_OK) {
        cleanup();
        return rc;
      }
    }
  }
  for (size_t b = 1; b < nb; ++b) {  // join
    hipEvent_t join = nullptr;
    if (hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess) {
      cleanup();
      return fail(MONC_EHIP, "batch: event creation failed");
    }
    ev.push_back(join);
    if (hipEventRecord(join, side[b - 1]) != hipSuccess || hipStreamWaitEvent((hipStream_t)stream, join, 0) != hipSuccess) {
      cleanup();
      return fail(MONC_EHIP, "batch: join of the graph branches failed");
    }
  }
  cleanup();
  return MONC_OK;
}

static int check_batch(monc_plan* const* plans, int count, const char* what) {
  if (!plans) return fail(MONC_EINVAL, "%s: plans is null", what);
  if (count < 1 || count > MONC_MAX_BATCH)
    return fail(MONC_EINVAL, "%s: count must be in [1, %d] (got %d)", what, MONC_MAX_BATCH, count);
  for (int i = 0; i < count; ++i) {
    if (!plans[i]) return fail(MONC_EINVAL, "%s: plans[%d] is null", what, i);
    if (plans[i]->dtype != plans[0]->dtype) return fail(MONC_EINVAL, "batch mixes dtypes (member %d)", i);
    if (plans[i]->device != plans[0]->device) return fail(MONC_EINVAL, "batch spans devices (member %d)", i);
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return fail(MONC_EINVAL, "plan of member %d repeats member %d (one workspace per plan)", i, j);
  }
  return MONC_OK;
}

extern "C" int monc_project_batched(monc_plan* const* plans, int count, void* const* u, void* const* v,
                                    void* const* w, void* const* p, void* stream) {
  if (!plans || !u || !v || !w || !p) return fail(MONC_EINVAL, "null argument array");
  int rc = check_batch(plans, count, "monc_project_batched");
  if (rc != MONC_OK) return rc;
  for (int i = 0; i < count; ++i) {
    void* ptrs[4] = {u[i], v[i], w[i], p[i]};
    char what[64];
    std::snprintf(what, sizeof what, "batch member %d", i);
    rc = check_fields(plans[i], ptrs, 4, what);
    if (rc != MONC_OK) return rc;
  }
  rc = check_device(plans[0]);
  if (rc != MONC_OK) return rc;
  const bool fp64 = plans[0]->dtype == MONC_FP64;
  Profiler* prof = plans[0]->prof.mask ? &plans[0]->prof : nullptr;
  const BatchSchedule sc = lookup_schedule(plans, count);
  const std::vector<int> ord = batch_order(plans, count, sc.order);

  // key: schedule, plan ids, versions and field pointers
  std::vector<unsigned long long> key;
  key.reserve(6 * count + 2);
  key.push_back((unsigned long long)sc.order);
  key.push_back((unsigned long long)sc.budget_mb);
  key.push_back((unsigned long long)sc.branches);
  for (int i = 0; i < count; ++i) {
    key.push_back(plans[i]->id);
    key.push_back(plans[i]->version);
    key.push_back((unsigned long long)(uintptr_t)u[i]);
    key.push_back((unsigned long long)(uintptr_t)v[i]);
    key.push_back((unsigned long long)(uintptr_t)w[i]);
    key.push_back((unsigned long long)(uintptr_t)p[i]);
  }
  std::lock_guard<std::mutex> lk(g_batch_mu);
  BatchEntry* ent = nullptr;
  for (auto& e : g_batches)
    if (e->key == key) ent = e.get();
  if (!ent) {
    auto e = std::make_unique<BatchEntry>();
    e->key = key;
    for (int i = 0; i < count; ++i) e->plan_ids.push_back(plans[i]->id);
    if (hipMalloc((void**)&e->d_array, sizeof(MemberDesc) * count) != hipSuccess)
      return fail(MONC_ENOMEM, "batch descriptor allocation failed");
    std::vector<MemberDesc> hd(count);
    for (int t = 0; t < count; ++t) hd[t] = plans[ord[t]]->h;
    HIP_TRY(hipMemcpy(e->d_array, hd.data(), sizeof(MemberDesc) * count, hipMemcpyHostToDevice));
    if (g_batches.size() >= kBatchCacheSize) {
      auto oldest = std::min_element(g_batches.begin(), g_batches.end(),
                                     [](const std::unique_ptr<BatchEntry>& a, const std::unique_ptr<BatchEntry>& b) {
                                       return a->last_use < b->last_use;
                                     });
      g_batches.erase(oldest);
    }
    ent = e.get();
    g_batches.push_back(std::move(e));
  }
  ent->last_use = ++g_batch_clock;
  std::vector<Group> groups;
  build_groups(plans, count, u, v, w, p, ent->d_array, ord, sc, groups);
  const bool group_major = sc.budget_mb > 0;
  const auto& seq = full_sequence(fp64);
  if (prof) return run_batch(groups, seq, group_major, stream, prof);  // eager launches when timing kernels
  if (!ent->exec) {
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      (void)hipStreamDestroy(cs);
      return fail(MONC_EHIP, "hipStreamBeginCapture failed: %s", hipGetErrorString(e));
    }
    // side streams of the capture: forked from cs and joined back into it,
    // so they record into the same graph
    std::vector<hipStream_t> side;
    for (int b = 1; b < sc.branches && rc == MONC_OK; ++b) {
      hipStream_t s2 = nullptr;
      if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess) rc = fail(MONC_EHIP, "batch: stream creation failed");
      else side.push_back(s2);
    }
    if (rc == MONC_OK) rc = run_batch(groups, seq, group_major, cs, nullptr, side);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    for (hipStream_t s2 : side) (void)hipStreamDestroy(s2);
    if (rc != MONC_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(MONC_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    ent->graph = graph;
    HIP_TRY(hipGraphInstantiate(&ent->exec, graph, nullptr, nullptr, 0));
  }
  HIP_TRY(hipGraphLaunch(ent->exec, (hipStream_t)stream));
  return MONC_OK;
}

extern "C" int monc_batch_schedule(monc_plan* const* plans, int count, int* out) {
  int rc = check_batch(plans, count, "monc_batch_schedule");
  if (rc != MONC_OK) return rc;
  if (!out) return fail(MONC_EINVAL, "monc_batch_schedule: out is null");
  const BatchSchedule sc = lookup_schedule(plans, count);
  const std::vector<int> ord = batch_order(plans, count, sc.order);
  size_t used = 0;
  int ngroups = 1;
  const size_t budget = (size_t)sc.budget_mb << 20;
  for (int t = 0, n = 0; t < count; ++t, ++n) {
    const size_t mb = member_bytes(plans[ord[t]]);
    if (budget && n > 0 && used + mb > budget) {
      ++ngroups;
      used = 0;
    }
    used += mb;
  }
  out[0] = sc.order;
  out[1] = sc.budget_mb;
  out[2] = ngroups;
  out[3] = sc.branches;
  return MONC_OK;
}

extern "C" int monc_batch_set_schedule(monc_plan* const* plans, int count, int order, int budget_mb,
                                       int branches) {
  int rc = check_batch(plans, count, "monc_batch_set_schedule");
  if (rc != MONC_OK) return rc;
  if (order != 0 && order != 1) return fail(MONC_EINVAL, "monc_batch_set_schedule: order must be 0 or 1 (got %d)", order);
  if (budget_mb < 0) return fail(MONC_EINVAL, "monc_batch_set_schedule: budget_mb must be >= 0 (got %d)", budget_mb);
  if (branches < 1 || branches > MONC_MAX_BRANCHES)
    return fail(MONC_EINVAL, "monc_batch_set_schedule: branches must be in [1, %d] (got %d)", MONC_MAX_BRANCHES,
                branches);
  BatchSchedule sc;
  sc.order = order;
  sc.budget_mb = budget_mb;
  sc.branches = branches;
  std::lock_guard<std::mutex> lk(g_sched_mu);
  g_sched[batch_key(plans, count)] = sc;
  return MONC_OK;
}

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------
extern "C" int monc_profile_enable(monc_plan* pl, unsigned mask) {
  if (!pl) return fail(MONC_EINVAL, "plan is null");
  std::lock_guard<std::mutex> lk(pl->prof.mu);
  pl->prof.mask = mask;
  return MONC_OK;
}

extern "C" int monc_profile_read(monc_plan* pl, double* ms, int* launches) {
  if (!pl) return fail(MONC_EINVAL, "plan is null");
  std::lock_guard<std::mutex> lk(pl->prof.mu);
  int rc = MONC_OK;
  for (auto& r : pl->prof.recs) {
    float t = 0.0f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
      rc = fail(MONC_EHIP, "profiling event query failed");
    } else {
      if (ms) ms[r.id] += t;
      if (launches) launches[r.id] += 1;
    }
    pl->prof.pool.push_back(r.a);
    pl->prof.pool.push_back(r.b);
  }
  pl->prof.recs.clear();
  return rc;
}

// ---------------------------------------------------------------------------
// tile parameters and autotuning
// ---------------------------------------------------------------------------
extern "C" int monc_plan_params(const monc_plan* pl, int* out) {
  if (!pl || !out) return fail(MONC_EINVAL, "null argument");
  out[0] = pl->ex;
  out[1] = pl->ey;
  out[2] = pl->ymt;
  out[3] = pl->triP;
  out[4] = pl->h.tricw;
  out[5] = pl->h.xpw;
  out[6] = pl->h.yept;
  return MONC_OK;
}

extern "C" int monc_plan_set_params(monc_plan* pl, const int* in) {
  if (!pl || !in) return fail(MONC_EINVAL, "null argument");
  for (int i = 0; i < MONC_NPARAMS; ++i)
    if (in[i] < 0) return fail(MONC_EINVAL, "parameter %d is negative", i);
  const MemberDesc saved = pl->h;
  const int sv[MONC_NPARAMS] = {pl->ex, pl->ey, pl->ymt, pl->triP, pl->tricw, pl->xpw, pl->yept};
  int rc = configure_tiles(pl, in[0], in[1], in[2], in[3], in[4], in[5], in[6]);
  if (rc != MONC_OK) {
    pl->h = saved;
    pl->ex = sv[0]; pl->ey = sv[1]; pl->ymt = sv[2]; pl->triP = sv[3]; pl->tricw = sv[4]; pl->xpw = sv[5];
    pl->yept = sv[6];
    return rc;
  }
  HIP_TRY(hipDeviceSynchronize());  // in-flight work may still read the old descriptor
  rc = upload_desc(pl);
  if (rc == MONC_OK) ++pl->version;
  return rc;
}

// Tile parameters of one plan: time every candidate value of one parameter,
// all else fixed, one parameter after the other.
static int tune_plan(monc_plan* pl, void* stream) {
  int rc = check_device(pl);
  if (rc != MONC_OK) return rc;
  const size_t bytes = (size_t)pl->nx * pl->ny * pl->nz * elem_bytes(pl->dtype);
  void* buf[4] = {nullptr, nullptr, nullptr, nullptr};
  for (auto& b : buf) {
    if (hipMalloc(&b, bytes) != hipSuccess) {
      for (auto& c : buf) if (c) (void)hipFree(c);
      return fail(MONC_ENOMEM, "autotune scratch allocation failed");
    }
    (void)hipMemset(b, 0, bytes);
  }
  hipStream_t st = (hipStream_t)stream;
  const unsigned saved_mask = pl->prof.mask;
  // time every candidate value of one parameter, all else fixed; the cost of
  // a candidate is the summed time of the kernels that parameter shapes over
  // `reps` projections (enough for a few milliseconds of kernel time, so that
  // small grids are not ranked on noise)
  int reps = 4;
  auto measure = [&](const int* prm, unsigned kmask, double& cost) -> int {
    int r = monc_plan_set_params(pl, prm);
    if (r != MONC_OK) return r;
    pl->prof.mask = kmask;
    for (int it = 0; it < 2; ++it)
      if ((r = monc_project(pl, buf[0], buf[1], buf[2], buf[3], st)) != MONC_OK) return r;
    double ms[MONC_K_COUNT] = {0};
    int cnt[MONC_K_COUNT] = {0};
    monc_profile_read(pl, nullptr, nullptr);  // drop warm-up records
    for (int it = 0; it < reps; ++it)
      if ((r = monc_project(pl, buf[0], buf[1], buf[2], buf[3], st)) != MONC_OK) return r;
    if ((r = monc_profile_read(pl, ms, cnt)) != MONC_OK) return r;
    cost = 0.0;
    for (int k = 0; k < MONC_K_COUNT; ++k) cost += ms[k];
    return MONC_OK;
  };
  int best[MONC_NPARAMS] = {pl->ex, pl->ey, pl->ymt, pl->triP, pl->tricw, pl->h.xpw, pl->h.yept};
  {
    double whole = 0.0;
    const int r = measure(best, (1u << MONC_K_COUNT) - 1, whole);
    if (r != MONC_OK) {
      pl->prof.mask = saved_mask;
      for (auto& b : buf) (void)hipFree(b);
      return r;
    }
    const double per = whole / reps;  // ms per projection
    reps = per > 0.0 ? (int)std::min(64.0, std::max(4.0, std::ceil(3.0 / per))) : 4;
  }
  const unsigned xmask = (1u << MONC_K_DIV_FFTX) | (1u << MONC_K_IFFTX) | (1u << MONC_K_RESID_FFTX);
  const unsigned ymask = (1u << MONC_K_FFTY_FWD) | (1u << MONC_K_FFTY_INV);
  const unsigned tmask = 1u << MONC_K_TRIDIAG;
  struct Axis {
    int idx;
    std::vector<int> vals;
    unsigned mask;
  };
  std::vector<int> pvals;
  for (int P = 1; P <= kTriPmax; P *= 2)
    if (tri_rows(pl->nz, P) != 0 && (P == 1 || (pl->nz + P - 1) / P >= 2)) pvals.push_back(P);
  // elements per thread only shape the runtime-length FFT kernels
  std::vector<Axis> axes;
  if (!ct_supported(pl->nx)) axes.push_back({0, {2, 4, 8}, xmask});
  if (!ct_supported(pl->ny)) axes.push_back({1, {2, 4, 8}, ymask});
  // the radix plan of the compile-time y-FFT (8 or 16 elements per thread;
  // on mixed plans of the lengths it covers also 32, the persistent kernel),
  // timed together with the y tile width, which it bounds (threads per
  // workgroup) and which sets the spectral column blocks that shape the x
  // kernels' spectral traffic
  if (ct_supported(pl->ny) && pl->ny >= 16) {
    if (pl->dtype != MONC_FP64 && pp_supported(pl->ny)) axes.push_back({6, {8, 16, 32}, ymask | xmask});
    else axes.push_back({6, {8, 16}, ymask | xmask});
  }
  axes.push_back({2, {1, 2, 4, 8, 16, 32}, ymask | xmask});
  axes.push_back({3, pvals, tmask});
  axes.push_back({4, {4, 8, 16, 32}, tmask});
  if (ct_supported(pl->nx)) axes.push_back({5, {1, 2, 4}, xmask});
  for (const auto& ax : axes) {
    double best_cost = 1e300;
    int best_val = best[ax.idx];
    for (int val : ax.vals) {
      int prm[MONC_NPARAMS];
      std::copy(best, best + MONC_NPARAMS, prm);
      prm[ax.idx] = val;
      double cost = 0.0;
      if (measure(prm, ax.mask, cost) != MONC_OK) continue;
      int eff[MONC_NPARAMS];
      monc_plan_params(pl, eff);
      if (eff[ax.idx] != val) continue;  // clamped to another candidate
      if (cost < best_cost) {
        best_cost = cost;
        best_val = val;
      }
    }
    best[ax.idx] = best_val;
  }
  pl->prof.mask = saved_mask;
  for (auto& b : buf) (void)hipFree(b);
  rc = monc_plan_set_params(pl, best);
  if (rc != MONC_OK) return rc;
  if (const char* path = std::getenv("MONC_TUNE_CACHE")) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto m = read_cache(path);
    m[cache_key(pl)] = {pl->ex, pl->ey, pl->ymt, pl->triP, pl->tricw, pl->h.xpw, pl->h.yept};
    write_cache(path, m);
  }
  return MONC_OK;
}

// The batch schedule: every candidate (member order x grouping budget) is
// captured and replayed on scratch fields; the fastest replay wins.
static int tune_schedule(monc_plan* const* plans, int count, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const size_t eb = elem_bytes(plans[0]->dtype);
  std::vector<void*> bufs;
  auto release = [&]() {
    for (void* b : bufs) (void)hipFree(b);
    bufs.clear();
  };
  std::vector<void*> f[4];
  for (int i = 0; i < count; ++i) {
    const size_t bytes = (size_t)plans[i]->nx * plans[i]->ny * plans[i]->nz * eb;
    for (int t = 0; t < 4; ++t) {
      void* b = nullptr;
      if (hipMalloc(&b, bytes) != hipSuccess) {
        (void)hipGetLastError();
        release();
        return fail(MONC_ENOMEM, "autotune: scratch fields for the batch do not fit");
      }
      (void)hipMemset(b, 0, bytes);
      bufs.push_back(b);
      f[t].push_back(b);
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    release();
    return fail(MONC_EHIP, "autotune: event creation failed");
  }
  size_t total = 0;
  for (int i = 0; i < count; ++i) total += member_bytes(plans[i]);
  const int budgets[] = {0, 1024, 512, 256, 128, 64};
  const int branch_counts[] = {1, 2, 4};
  BatchSchedule best;
  double best_ms = 1e300;
  int rc = MONC_OK;
  for (int order = 0; order < 2 && rc == MONC_OK; ++order)
    for (int budget : budgets)
      for (int branches : branch_counts) {
        if (rc != MONC_OK) break;
        if (budget && ((size_t)budget << 20) >= total) continue;  // one group anyway
        if (branches > 1 && !budget) continue;                     // one group: one chain
        if (branches > 1 && ((size_t)budget << 20) * (size_t)(branches - 1) >= total)
          continue;  // fewer groups than branches
        rc = monc_batch_set_schedule(plans, count, order, budget, branches);
        for (int r = 0; r < 2 && rc == MONC_OK; ++r)  // capture, then one warm replay
          rc = monc_project_batched(plans, count, f[0].data(), f[1].data(), f[2].data(), f[3].data(), stream);
        if (rc != MONC_OK) break;
        const int reps = 5;
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps && rc == MONC_OK; ++r)
          rc = monc_project_batched(plans, count, f[0].data(), f[1].data(), f[2].data(), f[3].data(), stream);
        (void)hipEventRecord(e1, st);
        float ms = 0.0f;
        if (rc == MONC_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          rc = fail(MONC_EHIP, "autotune: event timing failed");
        if (rc == MONC_OK && ms < best_ms) {
          best_ms = ms;
          best.order = order;
          best.budget_mb = budget;
          best.branches = branches;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // the candidates' graphs hold the scratch pointers: drop them with the fields
  if (hipStreamSynchronize(st) != hipSuccess && rc == MONC_OK) rc = fail(MONC_EHIP, "autotune: stream failed");
  for (int i = 0; i < count; ++i) drop_batch_cache_for(plans[i]->id);
  release();
  if (rc != MONC_OK) return rc;
  rc = monc_batch_set_schedule(plans, count, best.order, best.budget_mb, best.branches);
  if (rc != MONC_OK) return rc;
  if (const char* path = std::getenv("MONC_TUNE_CACHE")) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto m = read_cache(path);
    m[batch_key(plans, count)] = {best.order, best.budget_mb, best.branches};
    write_cache(path, m);
  }
  return MONC_OK;
}

extern "C" int monc_autotune(monc_plan* const* plans, int count, void* stream) {
  int rc = check_batch(plans, count, "monc_autotune");
  if (rc != MONC_OK) return rc;
  // tile parameters: the first plan of every distinct grid is tuned, the
  // others of that grid take its parameters
  for (int i = 0; i < count; ++i) {
    int j = 0;
    while (j < i && !(plans[j]->nx == plans[i]->nx && plans[j]->ny == plans[i]->ny && plans[j]->nz == plans[i]->nz))
      ++j;
    if (j == i) {
      rc = tune_plan(plans[i], stream);
    } else {
      int prm[MONC_NPARAMS];
      monc_plan_params(plans[j], prm);
      rc = monc_plan_set_params(plans[i], prm);
    }
    if (rc != MONC_OK) return rc;
  }
  if (count == 1) return MONC_OK;
  return tune_schedule(plans, count, stream);
}
