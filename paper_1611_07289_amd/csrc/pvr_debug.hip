// Debug mode: the core entry points check their input arrays on the device
// before they launch (every value finite; patch weights also non-negative),
// synchronise the stream and reject the first offending element by name and
// index.  Off by default; pvr_set_debug switches it, and PVR_DEBUG set in the
// environment (to anything but "" or "0") switches it on at load.  Skipped
// while the stream is being captured into a graph.
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "pvr_internal.h"
#include "pvr_util.h"

using namespace pvr;

namespace {

std::atomic<int> g_debug{-1};  // -1: not yet read from the environment

constexpr unsigned long long NONE = ~0ull;

__global__ void k_set_u64(unsigned long long *dst, unsigned long long v) { *dst = v; }

template <typename T, bool NONNEG>
__global__ void k_first_bad(const T *__restrict__ a, long long n,
                            unsigned long long *__restrict__ first) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const T v = a[i];
    const bool bad = !isfinite(v) || (NONNEG && v < (T)0);
    if (bad) atomicMin(first, (unsigned long long)i);
  }
}

template <typename T>
pvr_status check(const pvr_plan *p, const char *fn, const char *what, const T *a, long long n,
                 bool nonneg, hipStream_t stream) {
  if (!debug_on() || !a || n <= 0) return PVR_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(stream, &cs));
  if (cs != hipStreamCaptureStatusNone) return PVR_OK;
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, stream, p->d_dbg, NONE);
  HIP_TRY(hipGetLastError());
  const int T_ = 256;
  const long long want = (n + T_ - 1) / T_;
  const dim3 grid((unsigned)(want < 4096 ? want : 4096));
  if (nonneg)
    hipLaunchKernelGGL((k_first_bad<T, true>), grid, dim3(T_), 0, stream, a, n, p->d_dbg);
  else
    hipLaunchKernelGGL((k_first_bad<T, false>), grid, dim3(T_), 0, stream, a, n, p->d_dbg);
  HIP_TRY(hipGetLastError());
  unsigned long long first = NONE;
  HIP_TRY(hipMemcpyAsync(&first, p->d_dbg, sizeof first, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (first != NONE)
    return fail(PVR_EINVAL, "%s: %s[%llu] is %s (debug mode)", fn, what, first,
                nonneg ? "negative or not finite" : "not finite");
  return PVR_OK;
}

}  // namespace

bool pvr::debug_on() {
  int v = g_debug.load(std::memory_order_relaxed);
  if (v < 0) {
    const char *e = std::getenv("PVR_DEBUG");
    v = (e && *e && std::strcmp(e, "0") != 0) ? 1 : 0;
    int expect = -1;
    g_debug.compare_exchange_strong(expect, v);
    v = g_debug.load(std::memory_order_relaxed);
  }
  return v == 1;
}

pvr_status pvr::debug_finite(const pvr_plan *p, const char *fn, const char *what, const float *a,
                             long long n, hipStream_t stream) {
  return check<float>(p, fn, what, a, n, false, stream);
}
pvr_status pvr::debug_finite(const pvr_plan *p, const char *fn, const char *what, const double *a,
                             long long n, hipStream_t stream) {
  return check<double>(p, fn, what, a, n, false, stream);
}
pvr_status pvr::debug_weights(const pvr_plan *p, const char *fn, const char *what, const float *a,
                              long long n, hipStream_t stream) {
  return check<float>(p, fn, what, a, n, true, stream);
}
pvr_status pvr::debug_weights(const pvr_plan *p, const char *fn, const char *what, const double *a,
                              long long n, hipStream_t stream) {
  return check<double>(p, fn, what, a, n, true, stream);
}

extern "C" pvr_status pvr_set_debug(int32_t on) {
  g_debug.store(on ? 1 : 0, std::memory_order_relaxed);
  return PVR_OK;
}

extern "C" int32_t pvr_get_debug(void) { return pvr::debug_on() ? 1 : 0; }
