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
  if (p->d_prob) (void)hipDeviceSynchronize();
  void *dev[] = {p->d_prob, p->d_stack, p->d_patch, p->d_sim_blocks, p->d_tiles, p->d_box_max, p->d_brick_prob, p->d_plane_prob,
                 p->d_theta, p->d_geod, p->d_geof, p->d_bb, p->d_sbox, p->d_invz, p->d_invz64,
                 p->d_mask, p->d_active, p->d_bin_count, p->d_bin_off, p->d_bin_patch, p->d_sub_count, p->d_sub_off, p->d_sub_patch,
                 p->d_rq, p->d_rq64, p->d_pstat, p->d_pbar, p->d_pval, p->d_chunk_stats, p->d_xt, p->d_total,
                 p->d_status};
  for (void *q : dev)
    if (q) (void)hipFree(q);
  if (p->h_total) (void)hipHostFree(p->h_total);
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
  free(p);
}

}  // namespace pvr

extern "C" const char *pvr_last_error(void) { return pvr::g_err; }

extern "C" const char *pvr_version(void) { return "pvr-mi355x 0.1 (gfx950)"; }
