// Error state, plan teardown and fill kernels.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pvr_internal.h"
#include "pvr_util.h"

namespace pvr {

static thread_local char g_err[1024];

pvr_status fail(pvr_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return st;
}

void clear_error() { g_err[0] = 0; }

template <typename T>
__global__ void k_fill(T *__restrict__ dst, T v, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = v;
}

template <typename T>
static void fill(T *dst, T v, long long n, hipStream_t stream) {
  if (n <= 0) return;
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, stream, dst, v, n);
}

void launch_fill_u8(uint8_t *dst, uint8_t v, long long n, hipStream_t s) { fill<uint8_t>(dst, v, n, s); }
void launch_fill_i32(int *dst, int v, long long n, hipStream_t s) { fill<int>(dst, v, n, s); }
void launch_fill_f32(float *dst, float v, long long n, hipStream_t s) { fill<float>(dst, v, n, s); }
void launch_fill_f64(double *dst, double v, long long n, hipStream_t s) { fill<double>(dst, v, n, s); }

void plan_free(pvr_plan *p) {
  if (!p) return;
  // the caller frees the workspace once this returns: let the device finish
  if (p->attached) (void)hipDeviceSynchronize();
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  if (p->ev_join) (void)hipEventDestroy(p->ev_join);
  if (p->side) (void)hipStreamDestroy(p->side);
  if (p->timers) {
    for (int k = 0; k < TIMING_KERNELS; ++k)
      for (int i = 0; i < TIMING_CAP; ++i)
        for (int j = 0; j < 2; ++j)
          if (p->timers[k].ev[i][j]) (void)hipEventDestroy(p->timers[k].ev[i][j]);
    free(p->timers);
  }
  free(p->h_prob);
  free(p->h_stack);
  free(p->h_patch);
  free(p->h_sample_off);
  free(p->h_vol_off);
  free(p->h_sim_blocks);
  free(p->h_brick_prob);
  free(p->h_plane_prob);
  free(p->h_tile_off);
  free(p);
}

}  // namespace pvr

extern "C" const char *pvr_last_error(void) { return pvr::g_err; }

extern "C" const char *pvr_version(void) { return "pvr-mi355x 0.1 (gfx950)"; }
