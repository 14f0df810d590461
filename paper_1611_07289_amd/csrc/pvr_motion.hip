// Per-patch motion bookkeeping of the optimisers built on top of the forward
// model: the joint gradient-based registration (steps, acceptance, step
// lengths) and the learned initialiser (motion in the patch's own frame,
// selection, fallback).  One lane per patch; the flat-patch test one
// workgroup per patch.
#include <math.h>

#include "pvr_internal.h"
#include "pvr_util.h"

using namespace pvr;

namespace {

constexpr int MOT_T = 256;

// Half-diagonal of a patch in mm (at least 1): the scale of the rotation
// variables, so that a unit change moves the farthest pixel by about 1 mm.
__device__ __forceinline__ double patch_rho(const PatchDev &pt, const StackDev &st) {
  const double su = st.spacing[0], sv = st.spacing[1];
  const double rho =
      0.5 * sqrt((pt.w - 1) * (pt.w - 1) * su * su + (pt.h - 1) * (pt.h - 1) * sv * sv);
  return rho < 1.0 ? 1.0 : rho;
}

// out = base + A v (inverse = 0) or base + A^-1 v, A = diag(rho F^T, F^T),
// F the stack's unit axes as columns (E is row-major 3x3, E[3r + a] = row r
// of axis a); F is orthogonal, so A^-1 = diag(F / rho, F).
__global__ void __launch_bounds__(MOT_T)
k_motion_frame(const PatchDev *__restrict__ patches, const StackDev *__restrict__ stacks, int M,
               const float *__restrict__ in, int inverse, const float *__restrict__ base,
               float *__restrict__ out) {
  const int s = blockIdx.x * MOT_T + threadIdx.x;
  if (s >= M) return;
  const PatchDev pt = patches[s];
  const StackDev &st = stacks[pt.stack];
  const double rho = patch_rho(pt, st);
  double v[6], r[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) v[a] = in[6 * s + a];
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    const double sc = blk == 0 ? (inverse ? 1.0 / rho : rho) : 1.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double acc = 0;
#pragma unroll
      for (int j = 0; j < 3; ++j)
        acc += (inverse ? st.E[3 * i + j] : st.E[3 * j + i]) * v[3 * blk + j];
      r[3 * blk + i] = sc * acc;
    }
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) out[6 * s + a] = (float)((base ? (double)base[6 * s + a] : 0.0) + r[a]);
}

// trial = theta + delta g_q / |g_q| / sc in the scaled variables q = sc theta
// (sc = rho for the angles, 1 for the translations; g_q = g / sc).
__global__ void __launch_bounds__(MOT_T)
k_motion_step(const PatchDev *__restrict__ patches, const StackDev *__restrict__ stacks, int M,
              const float *__restrict__ theta, const float *__restrict__ grad,
              const float *__restrict__ delta, float step_min, float *__restrict__ trial) {
  const int s = blockIdx.x * MOT_T + threadIdx.x;
  if (s >= M) return;
  const PatchDev pt = patches[s];
  const double rho = patch_rho(pt, stacks[pt.stack]);
  const double d = delta[s];
  double gq[6], n2 = 0;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    gq[a] = (double)grad[6 * s + a] / (a < 3 ? rho : 1.0);
    n2 += gq[a] * gq[a];
  }
  const double n = sqrt(n2) > 1e-30 ? sqrt(n2) : 1e-30;
  const bool live = d >= (double)step_min;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    const double step = live ? d * gq[a] / n / (a < 3 ? rho : 1.0) : 0.0;
    trial[6 * s + a] = (float)((double)theta[6 * s + a] + step);
  }
}

__global__ void __launch_bounds__(MOT_T)
k_motion_accept(int M, const float *__restrict__ cand, const float *__restrict__ score_cand,
                float *__restrict__ theta, float *__restrict__ score, float *__restrict__ delta,
                float step0, float step_min, int *__restrict__ n_live) {
  const int s = blockIdx.x * MOT_T + threadIdx.x;
  const bool in = s < M;
  const bool live = in && (delta ? delta[s] >= step_min : true);
  const bool acc = live && score_cand[s] > score[s];
  if (acc) {
#pragma unroll
    for (int a = 0; a < 6; ++a) theta[6 * s + a] = cand[6 * s + a];
    score[s] = score_cand[s];
  }
  bool still = false;
  if (delta && live) {
    const float d = acc ? fminf(2.f * delta[s], step0) : 0.5f * delta[s];
    delta[s] = d;
    still = d >= step_min;
  }
  if (n_live) {  // patches whose step is still at least step_min: one add per wave
    const unsigned long long b = __ballot(still);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(n_live, (int)__popcll(b));
  }
}

// Population standard deviation of a patch's observed samples (those the
// last build's mask keeps), FP64 sums; delta = step0 if it reaches min_std.
__global__ void __launch_bounds__(MOT_T)
k_motion_init_step(const PatchDev *__restrict__ patches, const uint8_t *__restrict__ mask,
                   const float *__restrict__ y, float step0, double min_std,
                   float *__restrict__ delta) {
  __shared__ double red[3][MOT_T / 64];
  const int s = blockIdx.x;
  const PatchDev pt = patches[s];
  const int n = pt.w * pt.h;
  double a[3] = {0, 0, 0};
  for (int l = threadIdx.x; l < n; l += MOT_T) {
    const long long j = pt.off + l;
    if (!mask[j]) continue;
    const double v = y[j];
    a[0] += 1.0; a[1] += v; a[2] += v * v;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double x = a[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) red[k][wave] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      a[k] = 0;
      for (int w = 0; w < MOT_T / 64; ++w) a[k] += red[k][w];
    }
    double sd = 0;
    if (a[0] > 0) {
      const double m = a[1] / a[0];
      sd = sqrt(fmax(a[2] / a[0] - m * m, 0.0));
    }
    delta[s] = sd >= min_std ? step0 : 0.f;
  }
}

__global__ void __launch_bounds__(MOT_T)
k_motion_fallback(int M, const float *__restrict__ score, float tau,
                  const float *__restrict__ score_ref, const float *__restrict__ theta_ref,
                  float *__restrict__ theta, const uint8_t *__restrict__ active,
                  uint8_t *__restrict__ flag, uint8_t *__restrict__ keep) {
  const int s = blockIdx.x * MOT_T + threadIdx.x;
  if (s >= M) return;
  const bool act = active ? active[s] != 0 : true;
  const float thr = score_ref ? score_ref[s] + tau : tau;
  const bool back = act && score[s] < thr;
  if (back) {
#pragma unroll
    for (int a = 0; a < 6; ++a) theta[6 * s + a] = theta_ref[6 * s + a];
  }
  flag[s] = back ? 1 : 0;
  if (keep) keep[s] = act && !back ? 1 : 0;
}

__global__ void __launch_bounds__(MOT_T)
k_motion_live(int M, const float *__restrict__ delta, float step_min,
              const uint8_t *__restrict__ active, uint8_t *__restrict__ live) {
  const int s = blockIdx.x * MOT_T + threadIdx.x;
  if (s >= M) return;
  const bool act = active ? active[s] != 0 : true;
  live[s] = act && delta[s] >= step_min ? 1 : 0;
}

inline unsigned lanes(int M) { return (unsigned)((M + MOT_T - 1) / MOT_T); }

}  // namespace

extern "C" pvr_status pvr_motion_frame(const pvr_plan *p, const float *in, int32_t inverse,
                                       const float *base, float *out, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_motion_frame", in, 4);
  PVR_ALIGNED("pvr_motion_frame", base, 4);
  PVR_ALIGNED("pvr_motion_frame", out, 4);
  if (!p || !in || !out) return fail(PVR_EINVAL, "pvr_motion_frame: NULL argument");
  if (!p->attached) return fail(PVR_EINVAL, "pvr_motion_frame: no workspace attached");
  hipLaunchKernelGGL(k_motion_frame, dim3(lanes(p->M)), dim3(MOT_T), 0, stream, p->d_patch,
                     p->d_stack, p->M, in, inverse ? 1 : 0, base, out);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_motion_step(const pvr_plan *p, const float *theta,
                                      const float *grad_theta, const float *delta,
                                      float step_min, float *trial, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_motion_step", theta, 4);
  PVR_ALIGNED("pvr_motion_step", grad_theta, 4);
  PVR_ALIGNED("pvr_motion_step", delta, 4);
  PVR_ALIGNED("pvr_motion_step", trial, 4);
  if (!p || !theta || !grad_theta || !delta || !trial)
    return fail(PVR_EINVAL, "pvr_motion_step: NULL argument");
  if (!p->attached) return fail(PVR_EINVAL, "pvr_motion_step: no workspace attached");
  hipLaunchKernelGGL(k_motion_step, dim3(lanes(p->M)), dim3(MOT_T), 0, stream, p->d_patch,
                     p->d_stack, p->M, theta, grad_theta, delta, step_min, trial);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_motion_accept(const pvr_plan *p, const float *cand,
                                        const float *score_cand, float *theta, float *score,
                                        float *delta, float step0, float step_min,
                                        int32_t *n_live, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_motion_accept", cand, 4);
  PVR_ALIGNED("pvr_motion_accept", score_cand, 4);
  PVR_ALIGNED("pvr_motion_accept", theta, 4);
  PVR_ALIGNED("pvr_motion_accept", score, 4);
  PVR_ALIGNED("pvr_motion_accept", delta, 4);
  PVR_ALIGNED("pvr_motion_accept", n_live, 4);
  if (!p || !cand || !score_cand || !theta || !score)
    return fail(PVR_EINVAL, "pvr_motion_accept: NULL argument");
  hipLaunchKernelGGL(k_motion_accept, dim3(lanes(p->M)), dim3(MOT_T), 0, stream, p->M, cand,
                     score_cand, theta, score, delta, step0, step_min, n_live);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_motion_init_step(const pvr_plan *p, const float *y_obs, float step0,
                                           double min_std, float *delta, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_motion_init_step", y_obs, 4);
  PVR_ALIGNED("pvr_motion_init_step", delta, 4);
  if (!p || !y_obs || !delta) return fail(PVR_EINVAL, "pvr_motion_init_step: NULL argument");
  if (!p->built) return fail(PVR_EINVAL, "pvr_motion_init_step: plan has not been built");
  hipLaunchKernelGGL(k_motion_init_step, dim3(p->M), dim3(MOT_T), 0, stream, p->d_patch,
                     p->d_mask, y_obs, step0, min_std, delta);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_motion_fallback(const pvr_plan *p, const float *score, float tau,
                                          const float *score_ref, const float *theta_ref,
                                          float *theta, const uint8_t *active, uint8_t *flag,
                                          uint8_t *keep, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_motion_fallback", score, 4);
  PVR_ALIGNED("pvr_motion_fallback", score_ref, 4);
  PVR_ALIGNED("pvr_motion_fallback", theta_ref, 4);
  PVR_ALIGNED("pvr_motion_fallback", theta, 4);
  if (!p || !score || !theta_ref || !theta || !flag)
    return fail(PVR_EINVAL, "pvr_motion_fallback: NULL argument");
  hipLaunchKernelGGL(k_motion_fallback, dim3(lanes(p->M)), dim3(MOT_T), 0, stream, p->M, score,
                     tau, score_ref, theta_ref, theta, active, flag, keep);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_motion_live(const pvr_plan *p, const float *delta, float step_min,
                                      const uint8_t *active, uint8_t *live, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_motion_live", delta, 4);
  if (!p || !delta || !live) return fail(PVR_EINVAL, "pvr_motion_live: NULL argument");
  hipLaunchKernelGGL(k_motion_live, dim3(lanes(p->M)), dim3(MOT_T), 0, stream, p->M, delta,
                     step_min, active, live);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}
