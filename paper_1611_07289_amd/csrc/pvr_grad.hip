// Derivative of the forward model with respect to the per-patch motion:
//   grad_theta_s = sum_{j in s} g_j d y_hat_j / d theta_s.
//
// y_hat_j = sum_i g_hat_ji X_i / Z_j with Z_j = sum_i g_hat_ji, so
//   d y_hat_j / d theta = sum_i (X_i - y_hat_j) d g_hat_ji / d theta / Z_j,
// with d g_hat / d theta as derived in pvr_grad.h.
//
// One workgroup per patch; FP64 accumulation of the six per-patch sums.  In
// FP32 one walk per sample gathers the nine offset moments of pvr_grad.h
// (the exact registration's walk, grouped loads through a buffer resource)
// and forms the six derivatives once per sample; in FP64 two walks (y_hat,
// then the derivative evaluated at every voxel) keep the direct form.
#include <math.h>

#include "pvr_geometry.h"
#include "pvr_grad.h"
#include "pvr_internal.h"
#include "pvr_util.h"

using namespace pvr;

constexpr int GR_THREADS = 256;

template <typename T>
__global__ void __launch_bounds__(GR_THREADS)
k_grad_theta(const ProbDev *__restrict__ probs, const StackDev *__restrict__ stacks,
             const PatchDev *__restrict__ patches, const typename GeoOf<T>::type *__restrict__ geo,
             const double *__restrict__ theta, const T *__restrict__ invz,
             const T *__restrict__ X, const T *__restrict__ gy, T *__restrict__ grad) {
  __shared__ double red[6][GR_THREADS / 64];
  const int s = blockIdx.x;
  const PatchDev pt = patches[s];
  const ProbDev pr = probs[pt.problem];
  const StackDev st = stacks[pt.stack];
  const typename GeoOf<T>::type &g = geo[s];
  GradConst gc;
  make_grad_const(pr, st, pt, theta + 6 * s, gc);
  const T *Xp = X + pr.vol_off;
  GradMom gm;
  if constexpr (sizeof(T) == 4) make_grad_mom(gc, g.perm, gm);
  const unsigned nbytes = (unsigned)(pr.nx * pr.ny * pr.nz) * (unsigned)sizeof(T);
  const __amdgpu_buffer_rsrc_t xr = raw_buffer(Xp, nbytes);
  double sum6[6] = {0, 0, 0, 0, 0, 0};
  const int n = pt.w * pt.h;
  for (int l = threadIdx.x; l < n; l += GR_THREADS) {
    const long long j = pt.off + l;
    const T iz = invz[j];
    if (!(iz > (T)0)) continue;
    const T gj = gy[j];
    if (gj == (T)0) continue;
    const int u = pt.x0 + l % pt.w, v = pt.y0 + l / pt.w;
    int b[3];
    T f[3];
    sample_centre(g, pr, u, v, pt.slice, b, f);
    // q = x_world - (c + t), x_world = Vl x_vox + o
    double xv[3], q[3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
      xv[r] = fma(g.H[4 * r], (double)u, fma(g.H[4 * r + 1], (double)v,
                                             fma(g.H[4 * r + 2], (double)pt.slice, g.H[4 * r + 3])));
#pragma unroll
    for (int r = 0; r < 3; ++r)
      q[r] = gc.Vl[3 * r] * xv[0] + gc.Vl[3 * r + 1] * xv[1] + gc.Vl[3 * r + 2] * xv[2] +
             gc.v2w_o[r] - gc.ct[r];
    const T qt[3] = {(T)q[0], (T)q[1], (T)q[2]};
    T a6[6] = {0, 0, 0, 0, 0, 0};
    if constexpr (sizeof(T) == 4) {
      // moments of w_i = e^{-Q_i/2} (X_i - y_hat) from those relative to the
      // centre voxel's value X_b: y_hat - X_b = sum g_hat (X - X_b) / Z
      float xb, a, z, mx[9], me[9];
      if (g.perm[2] == 0)
        psf_walk_grad<1, false>(g, pr, b, f, xr, nbytes, xb, a, z, mx, me);
      else
        psf_walk_grad<2, false>(g, pr, b, f, xr, nbytes, xb, a, z, mx, me);
      const float dl = a * iz;
      float m[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) m[c] = fma(-dl, me[c], mx[c]);
      grad_from_moments(gm, m, qt, a6);
    } else {
      T z = 0, acc = 0;
      psf_walk<T, typename GeoOf<T>::type, true>(g, pr, b, f, Xp, z, acc);
      const T yh = acc * iz;
      grad_walk<T>(g, pr, gc, b, f, qt, Xp, yh, a6);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) sum6[k] += (double)gj * (double)(a6[k] * iz);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double x = sum6[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) red[k][wave] = x;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double x = 0;
    for (int w = 0; w < GR_THREADS / 64; ++w) x += red[threadIdx.x][w];
    grad[6 * s + threadIdx.x] = (T)x;
  }
}

template <typename T>
static pvr_status grad_impl(const pvr_plan *p, const T *X, const T *gy, T *grad, const T *invz,
                            hipStream_t stream) {
  if (!X || !gy || !grad) return fail(PVR_EINVAL, "pvr_simulate_grad_theta: NULL argument");
  if (p->psf != PVR_PSF_GAUSSIAN)
    return fail(PVR_EUNSUPPORTED, "pvr_simulate_grad_theta: the theta-derivative is implemented for the Gaussian PSF");
  const void *geo = sizeof(T) == 4 ? (const void *)p->d_geof : (const void *)p->d_geod;
  hipLaunchKernelGGL(k_grad_theta<T>, dim3(p->M), dim3(GR_THREADS), 0, stream, p->d_prob,
                     p->d_stack, p->d_patch, (const typename GeoOf<T>::type *)geo, p->d_theta,
                     invz, X, gy, grad);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
}

extern "C" pvr_status pvr_simulate_grad_theta(const pvr_plan *p, const float *X, const float *gy,
                                              float *grad_theta, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_simulate_grad_theta", X, 4);
  PVR_ALIGNED("pvr_simulate_grad_theta", gy, 4);
  PVR_ALIGNED("pvr_simulate_grad_theta", grad_theta, 4);
  if (!p) return fail(PVR_EINVAL, "pvr_simulate_grad_theta: plan is NULL");
  if (!p->built) return fail(PVR_EINVAL, "pvr_simulate_grad_theta: plan has not been built");
  PVR_TRY_STATUS(debug_finite(p, "pvr_simulate_grad_theta", "X", X, p->V, stream));
  PVR_TRY_STATUS(debug_finite(p, "pvr_simulate_grad_theta", "grad_y", gy, p->N, stream));
  return grad_impl<float>(p, X, gy, grad_theta, p->d_invz, stream);
  PVR_API_END();
}

extern "C" pvr_status pvr_simulate_grad_theta_f64(const pvr_plan *p, const double *X,
                                                  const double *gy, double *grad_theta,
                                                  hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_simulate_grad_theta_f64", X, 8);
  PVR_ALIGNED("pvr_simulate_grad_theta_f64", gy, 8);
  PVR_ALIGNED("pvr_simulate_grad_theta_f64", grad_theta, 8);
  if (!p) return fail(PVR_EINVAL, "pvr_simulate_grad_theta_f64: plan is NULL");
  if (!p->built || !p->built64)
    return fail(PVR_EINVAL, "pvr_simulate_grad_theta_f64: plan needs pvr_plan_build_f64 on a "
                            "workspace attached with PVR_WS_F64");
  PVR_TRY_STATUS(debug_finite(p, "pvr_simulate_grad_theta_f64", "X", X, p->V, stream));
  PVR_TRY_STATUS(debug_finite(p, "pvr_simulate_grad_theta_f64", "grad_y", gy, p->N, stream));
  return grad_impl<double>(p, X, gy, grad_theta, p->d_invz64, stream);
  PVR_API_END();
}

// ---------------------------------------------------------------------------
// Cross-correlation of every patch with its simulation and its derivative
// with respect to the simulated samples (Sec. IV-A eq. CC over the samples
// valid at the last build, population statistics):
//   NCC_s = cov(y, yh) / (sd_y sd_yh),
//   d NCC_s / d yh_j = ((y_j - mu_y) / (sd_y sd_yh)
//                       - NCC_s (yh_j - mu_yh) / sd_yh^2) / n_s.
// Flat patches (a variance at or below 1e-12 of the squared mean) get NCC 0
// and a zero derivative.  One workgroup per patch.
__global__ void __launch_bounds__(GR_THREADS)
k_ncc_grad(const PatchDev *__restrict__ patches, const float *__restrict__ invz,
           const float *__restrict__ y, const float *__restrict__ yh,
           float *__restrict__ gout, float *__restrict__ ncc) {
  __shared__ double red[6][GR_THREADS / 64];
  const int s = blockIdx.x;
  const PatchDev pt = patches[s];
  const int n = pt.w * pt.h;
  double a6[6] = {0, 0, 0, 0, 0, 0};
  for (int l = threadIdx.x; l < n; l += GR_THREADS) {
    const long long j = pt.off + l;
    if (!(invz[j] > 0.f)) continue;
    const double yo = y[j], ys = yh[j];
    a6[0] += 1.0; a6[1] += yo; a6[2] += yo * yo; a6[3] += ys; a6[4] += ys * ys; a6[5] += yo * ys;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double x = a6[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) red[k][wave] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double x = 0;
    for (int w = 0; w < GR_THREADS / 64; ++w) x += red[k][w];
    a6[k] = x;
  }
  const double cnt = a6[0];
  double my = 0, mh = 0, vy = 0, vh = 0, cv = 0, r = 0;
  bool ok = cnt > 0;
  if (ok) {
    my = a6[1] / cnt; mh = a6[3] / cnt;
    vy = a6[2] / cnt - my * my; vh = a6[4] / cnt - mh * mh; cv = a6[5] / cnt - my * mh;
    ok = vy > 1e-12 * my * my && vh > 1e-12 * mh * mh && vy > 0 && vh > 0;
  }
  double sy = 0, sh = 0;
  if (ok) {
    sy = sqrt(vy); sh = sqrt(vh);
    r = cv / (sy * sh);
  }
  if (ncc && threadIdx.x == 0) ncc[s] = (float)r;
  if (!gout) return;
  for (int l = threadIdx.x; l < n; l += GR_THREADS) {
    const long long j = pt.off + l;
    float gj = 0.f;
    if (ok && invz[j] > 0.f) {
      const double yo = y[j], ys = yh[j];
      gj = (float)(((yo - my) / (sy * sh) - r * (ys - mh) / vh) / cnt);
    }
    gout[j] = gj;
  }
}

extern "C" pvr_status pvr_ncc_grad(const pvr_plan *p, const float *y_obs, const float *y_sim,
                                   float *grad_y, float *ncc, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_ncc_grad", y_obs, 4);
  PVR_ALIGNED("pvr_ncc_grad", y_sim, 4);
  PVR_ALIGNED("pvr_ncc_grad", grad_y, 4);
  PVR_ALIGNED("pvr_ncc_grad", ncc, 4);
  if (!p || !y_obs || !y_sim) return fail(PVR_EINVAL, "pvr_ncc_grad: NULL argument");
  if (!p->built) return fail(PVR_EINVAL, "pvr_ncc_grad: plan has not been built");
  hipLaunchKernelGGL(k_ncc_grad, dim3(p->M), dim3(GR_THREADS), 0, stream, p->d_patch, p->d_invz,
                     y_obs, y_sim, grad_y, ncc);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}
