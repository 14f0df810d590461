// Kernel timing: event pairs recorded around the hot kernels' launches on
// their own stream, summed on request.
#include "pvr_util.h"

using namespace pvr;

namespace pvr {
hipEvent_t *timing_slot(const pvr_plan *p, int k) {
  if (!p->timing || !p->timers || k < 0 || k >= TIMING_KERNELS) return nullptr;
  KernelTimer &t = const_cast<pvr_plan *>(p)->timers[k];
  if (t.n >= TIMING_CAP) return nullptr;
  return t.ev[t.n++];
}
}  // namespace pvr

extern "C" pvr_status pvr_plan_set_timing(pvr_plan *p, int32_t on) {
  PVR_API_BEGIN();
  if (!p) return fail(PVR_EINVAL, "pvr_plan_set_timing: plan is NULL");
  if (on && !p->timers) {
    KernelTimer *t = (KernelTimer *)calloc(TIMING_KERNELS, sizeof(KernelTimer));
    if (!t) return fail(PVR_ENOMEM, "pvr_plan_set_timing: host allocation failed");
    for (int k = 0; k < TIMING_KERNELS; ++k)
      for (int i = 0; i < TIMING_CAP; ++i)
        for (int j = 0; j < 2; ++j) {
          const hipError_t e = hipEventCreate(&t[k].ev[i][j]);
          if (e != hipSuccess) {
            p->timers = t;  // plan_free destroys what was created
            return fail(PVR_EHIP, "hipEventCreate failed: %s", hipGetErrorString(e));
          }
        }
    p->timers = t;
  }
  p->timing = on != 0;
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_plan_kernel_time(pvr_plan *p, int32_t kernel, double *total_ms,
                                           int32_t *launches) {
  PVR_API_BEGIN();
  if (!p || !total_ms || !launches) return fail(PVR_EINVAL, "pvr_plan_kernel_time: NULL argument");
  if (kernel < 0 || kernel >= TIMING_KERNELS) return fail(PVR_EINVAL, "pvr_plan_kernel_time: unknown kernel %d", kernel);
  *total_ms = 0;
  *launches = 0;
  if (!p->timers) return PVR_OK;
  KernelTimer &t = p->timers[kernel];
  double sum = 0;
  for (int i = 0; i < t.n; ++i) {
    HIP_TRY(hipEventSynchronize(t.ev[i][1]));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, t.ev[i][0], t.ev[i][1]));
    sum += ms;
  }
  *total_ms = sum;
  *launches = t.n;
  t.n = 0;
  return PVR_OK;
  PVR_API_END();
}
