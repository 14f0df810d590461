// Host-side error handling and allocation helpers of the PVR library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>

#include <exception>

#include "pvr_internal.h"

namespace pvr {

pvr_status fail(pvr_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
void plan_free(pvr_plan *p);
pvr_status plan_build_index(pvr_plan *p, hipStream_t stream);
pvr_status launch_bp_prep(const pvr_plan *p, const float *e, const float *pp, hipStream_t stream);
void launch_fill_u8(uint8_t *dst, uint8_t v, long long n, hipStream_t stream);
void launch_fill_i32(int *dst, int v, long long n, hipStream_t stream);
void launch_fill_f32(float *dst, float v, long long n, hipStream_t stream);
void launch_fill_f64(double *dst, double v, long long n, hipStream_t stream);
// The event pair to record around the next launch of kernel k, or nullptr
// when the plan is not timing (or the kernel's slots are full).
hipEvent_t *timing_slot(const pvr_plan *p, int k);

struct PlanGuard {
  pvr_plan *p;
  explicit PlanGuard(pvr_plan *q) : p(q) {}
  ~PlanGuard() { if (p) plan_free(p); }
  void release() { p = nullptr; }
};

}  // namespace pvr

#define PVR_API_BEGIN() \
  pvr::clear_error();   \
  try {
#define PVR_API_END()                                                          \
  }                                                                            \
  catch (const std::exception &e) {                                            \
    return pvr::fail(PVR_EINVAL, "internal error: %s", e.what());              \
  }                                                                            \
  catch (...) {                                                                \
    return pvr::fail(PVR_EINVAL, "internal error");                            \
  }

// Return a non-OK status of a library call from the enclosing entry point.
#define PVR_TRY_STATUS(expr)                                                   \
  do {                                                                         \
    const pvr_status st_try_ = (expr);                                         \
    if (st_try_ != PVR_OK) return st_try_;                                     \
  } while (0)

#define HIP_TRY(expr)                                                          \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess)                                                      \
      return pvr::fail(PVR_EHIP, "%s failed: %s (%s:%d)", #expr,               \
                       hipGetErrorString(e_), __FILE__, __LINE__);             \
  } while (0)

// Device arrays must be aligned to the width the kernels read them with; a
// NULL pointer passes (whether it may be NULL is checked separately).
#define PVR_ALIGNED(fn, ptr, a)                                                \
  do {                                                                         \
    if ((reinterpret_cast<uintptr_t>(ptr) & ((uintptr_t)(a) - 1)) != 0)        \
      return pvr::fail(PVR_EINVAL, "%s: %s is not %d-byte aligned", fn, #ptr,  \
                       (int)(a));                                              \
  } while (0)

// Places `count` elements of T at the next 256-byte boundary of a workspace
// and advances the cursor.  With a NULL base it only measures: the same
// sequence of calls sizes a workspace and then carves it.
struct WsCursor {
  char *base;
  size_t off;
};
template <typename T>
inline T *ws_take(WsCursor &c, long long count) {
  c.off = (c.off + 255) & ~(size_t)255;
  T *r = c.base ? reinterpret_cast<T *>(c.base + c.off) : nullptr;
  c.off += (size_t)(count > 0 ? count : 1) * sizeof(T);
  return r;
}
