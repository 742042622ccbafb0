// Streaming-bandwidth probes: the plainest kernels that move a known number
// of bytes through HBM (read only, write only, copy, and a pointwise update of
// three fields from a fourth, the access mix of the gradient correction).
// They measure the bandwidth a streaming kernel reaches on this device, the
// practical ceiling beside the vendor peak, and their known byte counts
// calibrate the hardware traffic counters. Each thread moves 16-byte
// vectors; every access is bounded by the element count.
#include <hip/hip_runtime.h>

#include "../../include/monc.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

// two vectors per thread, nontemporal loads (the fastest read variant
// measured); a data-dependent store that never fires keeps the loads alive
__global__ void __launch_bounds__(kThreads) k_probe_read(const f4* __restrict__ a, long long n, float* flag) {
  const long long i0 = (long long)blockIdx.x * kThreads * 2 + threadIdx.x;
  f4 s = 0;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const long long i = i0 + (long long)t * kThreads;
    if (i < n) s += __builtin_nontemporal_load(a + i);
  }
  if (s.x + s.y + s.z + s.w == -1.0f) flag[0] = s.x;
}

__global__ void __launch_bounds__(kThreads) k_probe_write(f4* __restrict__ a, long long n) {
  const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) a[i] = (f4)0.0f;
}

__global__ void __launch_bounds__(kThreads) k_probe_copy(const f4* __restrict__ a, f4* __restrict__ b, long long n) {
  const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

// u, v, w -= p in place: 4 reads and 3 writes per element
__global__ void __launch_bounds__(kThreads) k_probe_update(const f4* __restrict__ p, f4* __restrict__ u,
                                                           f4* __restrict__ v, f4* __restrict__ w, long long n) {
  const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) {
    const f4 q = __builtin_nontemporal_load(p + i);
    const f4 a = __builtin_nontemporal_load(u + i) - q;
    const f4 b = __builtin_nontemporal_load(v + i) - q;
    const f4 c = __builtin_nontemporal_load(w + i) - q;
    __builtin_nontemporal_store(a, u + i);
    __builtin_nontemporal_store(b, v + i);
    __builtin_nontemporal_store(c, w + i);
  }
}

}  // namespace

extern "C" int monc_stream_probe(int kind, void* a, void* b, void* c, void* d, size_t bytes, void* stream) {
  if (bytes == 0 || bytes % 16 != 0) return MONC_EINVAL;
  const int need = kind == MONC_PROBE_WRITE ? 1 : kind == MONC_PROBE_READ || kind == MONC_PROBE_COPY ? 2
                 : kind == MONC_PROBE_UPDATE ? 4 : 0;
  if (need == 0) return MONC_EINVAL;
  void* ptrs[4] = {a, b, c, d};
  for (int i = 0; i < need; ++i)
    if (!ptrs[i] || reinterpret_cast<uintptr_t>(ptrs[i]) % 16) return MONC_EINVAL;
  const long long n = (long long)(bytes / 16);
  const long long per = kind == MONC_PROBE_READ ? 2LL * kThreads : kThreads;
  const long long grid = (n + per - 1) / per;
  if (grid > 0x7fffffffLL) return MONC_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  const dim3 g((unsigned)grid), blk(kThreads);
  f4* A = static_cast<f4*>(a);
  switch (kind) {
    case MONC_PROBE_READ:
      hipLaunchKernelGGL(k_probe_read, g, blk, 0, st, A, n, static_cast<float*>(b));
      break;
    case MONC_PROBE_WRITE: hipLaunchKernelGGL(k_probe_write, g, blk, 0, st, A, n); break;
    case MONC_PROBE_COPY: hipLaunchKernelGGL(k_probe_copy, g, blk, 0, st, A, static_cast<f4*>(b), n); break;
    default:
      hipLaunchKernelGGL(k_probe_update, g, blk, 0, st, A, static_cast<f4*>(b), static_cast<f4*>(c),
                         static_cast<f4*>(d), n);
  }
  return hipGetLastError() == hipSuccess ? MONC_OK : MONC_EHIP;
}
