// EM robust weights of one SR iteration (inlier Gaussian, uniform outlier
// density, inlier posterior p, patch potential p_bar, patch classification,
// M-step).  All sums are FP64 and reduced in a fixed order.
//
// Kernels, in call order:
//   k_em_patch_stats  one workgroup per patch: min / max residual, max |y|,
//                     sum e^2 and count over the patch's valid samples
//   k_em_problem      one workgroup per problem: m = 1/(max e - min e), and at
//                     the start of a cycle sigma^2 = mean(e^2), c = 0.9
//   k_em_estep        one workgroup per patch: p_j, N_s, sum p^2, sum p,
//                     sum p e^2, p_bar_s
//   k_em_patches      one workgroup per problem: two-component mixture on
//                     {p_bar_s} (median split start, 20 EM iterations), W_s,
//                     and the M-step for the next iteration
#include <math.h>

#include "pvr_internal.h"
#include "pvr_util.h"

using namespace pvr;

constexpr int EM_T = 256;     // per-patch workgroups
constexpr int EMP_T = 1024;   // per-problem workgroups
constexpr int PSTAT = 10;     // doubles per patch in the scratch table

template <int NT>
__device__ __forceinline__ double bsum(double v, double *lds) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) lds[t] += lds[t + s];
    __syncthreads();
  }
  const double r = lds[0];
  __syncthreads();
  return r;
}

template <int NT>
__device__ __forceinline__ double bmin(double v, double *lds) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) lds[t] = fmin(lds[t], lds[t + s]);
    __syncthreads();
  }
  const double r = lds[0];
  __syncthreads();
  return r;
}

template <int NT>
__device__ __forceinline__ double bmax(double v, double *lds) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) lds[t] = fmax(lds[t], lds[t + s]);
    __syncthreads();
  }
  const double r = lds[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(EM_T)
k_em_patch_stats(const PatchDev *__restrict__ patches, const float *__restrict__ invz,
                 const float *__restrict__ e, const float *__restrict__ y,
                 double *__restrict__ pstat) {
  __shared__ double lds[EM_T];
  const int s = blockIdx.x;
  const PatchDev pt = patches[s];
  const int n = pt.w * pt.h;
  double mn = INFINITY, mx = -INFINITY, ym = 0, se2 = 0, cnt = 0;
  for (int l = threadIdx.x; l < n; l += EM_T) {
    const long long j = pt.off + l;
    if (!(invz[j] > 0.f)) continue;
    const double ev = e[j];
    mn = fmin(mn, ev);
    mx = fmax(mx, ev);
    ym = fmax(ym, fabs((double)y[j]));
    se2 += ev * ev;
    cnt += 1.0;
  }
  mn = bmin<EM_T>(mn, lds);
  mx = bmax<EM_T>(mx, lds);
  ym = bmax<EM_T>(ym, lds);
  se2 = bsum<EM_T>(se2, lds);
  cnt = bsum<EM_T>(cnt, lds);
  if (threadIdx.x == 0) {
    double *o = pstat + PSTAT * s;
    o[0] = mn; o[1] = mx; o[2] = ym; o[3] = se2; o[4] = cnt;
  }
}

__global__ void __launch_bounds__(EMP_T)
k_em_problem(const ProbDev *__restrict__ probs, const double *__restrict__ pstat,
             pvr_em_state *__restrict__ em, int init) {
  __shared__ double lds[EMP_T];
  const ProbDev pr = probs[blockIdx.x];
  double mn = INFINITY, mx = -INFINITY, ym = 0, se2 = 0, cnt = 0;
  for (int s = pr.patch_begin + threadIdx.x; s < pr.patch_end; s += EMP_T) {
    const double *o = pstat + PSTAT * s;
    mn = fmin(mn, o[0]);
    mx = fmax(mx, o[1]);
    ym = fmax(ym, o[2]);
    se2 += o[3];
    cnt += o[4];
  }
  mn = bmin<EMP_T>(mn, lds);
  mx = bmax<EMP_T>(mx, lds);
  ym = bmax<EMP_T>(ym, lds);
  se2 = bsum<EMP_T>(se2, lds);
  cnt = bsum<EMP_T>(cnt, lds);
  if (threadIdx.x == 0) {
    pvr_em_state &st = em[blockIdx.x];
    const double eps = 1e-6 * ym;
    const double range = cnt > 0 ? fmax(mx - mn, eps) : 0.0;
    st.m = range > 0 ? 1.0 / range : 1.0;
    st.y_abs_max = ym;
    if (init || !st.started) {
      const double floor2 = (1e-4 * ym) * (1e-4 * ym);
      double s2 = cnt > 0 ? se2 / cnt : 0.0;
      s2 = s2 > 0 ? fmax(s2, floor2) : fmax(floor2, 1.0);
      st.sigma2 = s2;
      st.c = 0.9;
      st.started = 1;
    }
  }
}

__global__ void __launch_bounds__(EM_T)
k_em_estep(const PatchDev *__restrict__ patches, const float *__restrict__ invz,
           const float *__restrict__ e, const pvr_em_state *__restrict__ em,
           float *__restrict__ p_out, float *__restrict__ pbar, double *__restrict__ pstat) {
  __shared__ double lds[EM_T];
  const int s = blockIdx.x;
  const PatchDev pt = patches[s];
  const pvr_em_state st = em[pt.problem];
  const float sigma2 = (float)st.sigma2;
  const float inv2s2 = (float)(0.5 / st.sigma2);
  const float cG0 = (float)(st.c / sqrt(2.0 * M_PI * st.sigma2));
  const float mo = (float)(st.m * (1.0 - st.c));
  (void)sigma2;
  const int n = pt.w * pt.h;
  double ns = 0, sp2 = 0, sp = 0, spe2 = 0;
  for (int l = threadIdx.x; l < n; l += EM_T) {
    const long long j = pt.off + l;
    float pj = 0.f;
    if (invz[j] > 0.f) {
      const float ev = e[j];
      const float Gc = cG0 * expf(-ev * ev * inv2s2);
      const float dd = Gc + mo;
      pj = dd > 0.f ? Gc / dd : 0.f;
      ns += 1.0;
      sp2 += (double)pj * pj;
      sp += pj;
      spe2 += (double)pj * ev * ev;
    }
    if (p_out) p_out[j] = pj;
  }
  ns = bsum<EM_T>(ns, lds);
  sp2 = bsum<EM_T>(sp2, lds);
  sp = bsum<EM_T>(sp, lds);
  spe2 = bsum<EM_T>(spe2, lds);
  if (threadIdx.x == 0) {
    double *o = pstat + PSTAT * s;
    o[5] = ns; o[6] = sp2; o[7] = sp; o[8] = spe2;
    if (pbar) pbar[s] = ns > 0 ? (float)sqrt(sp2 / ns) : 0.f;
  }
}

__device__ __forceinline__ double log_normal(double v, double mu, double sd) {
  const double z = (v - mu) / sd;
  return -0.5 * z * z - log(sd) - 0.91893853320467274178;  // 0.5 log(2 pi)
}

__device__ __forceinline__ double inlier_resp(double v, double mu0, double sd0, double mu1,
                                              double sd1, double w1) {
  const double l1 = w1 > 0 ? log(w1) + log_normal(v, mu1, sd1) : -INFINITY;
  const double l0 = w1 < 1 ? log(1.0 - w1) + log_normal(v, mu0, sd0) : -INFINITY;
  return 1.0 / (1.0 + exp(l0 - l1));
}

// Two-component mixture on the potentials of one problem, patch weights and
// the M-step.  The start splits the potentials at the median: the n/2 smallest
// form the low component.  The split value is found exactly by a radix select
// on the float bit patterns (potentials are >= 0, so the patterns are ordered
// like the values).
__global__ void __launch_bounds__(EMP_T)
k_em_patches(const ProbDev *__restrict__ probs, const float *__restrict__ pbar,
             const uint8_t *__restrict__ active, double *__restrict__ pstat,
             double *__restrict__ resp, float *__restrict__ patch_w, pvr_em_state *__restrict__ em,
             int fix_w) {
  __shared__ double lds[EMP_T];
  __shared__ unsigned int hist[256];
  __shared__ unsigned int sel_prefix, sel_rank;
  const ProbDev pr = probs[blockIdx.x];
  const int t = threadIdx.x;
  const int pb = pr.patch_begin, pe = pr.patch_end;
  auto used = [&](int s) -> bool { return pstat[PSTAT * s + 5] > 0 && active[s] != 0; };
  double n = 0;
  for (int s = pb + t; s < pe; s += EMP_T) n += used(s) ? 1.0 : 0.0;
  n = bsum<EMP_T>(n, lds);
  const int nu = (int)n;
  double mu0 = 0, sd0 = 1, mu1 = 0, sd1 = 1, w1 = 0.9;
  bool fit = nu >= 2;
  if (fit) {
    const int n_lo = nu / 2;
    // radix select of the value of rank n_lo - 1
    if (t == 0) { sel_prefix = 0; sel_rank = (unsigned)(n_lo - 1); }
    __syncthreads();
    for (int pass = 0; pass < 4; ++pass) {
      const int shift = 24 - 8 * pass;
      for (int b = t; b < 256; b += EMP_T) hist[b] = 0;
      __syncthreads();
      const unsigned pref = sel_prefix;
      const unsigned mask_hi = pass == 0 ? 0u : (0xffffffffu << (32 - 8 * pass));
      for (int s = pb + t; s < pe; s += EMP_T) {
        if (!used(s)) continue;
        const unsigned bits = __float_as_uint(pbar[s]);
        if ((bits & mask_hi) == pref) atomicAdd(&hist[(bits >> shift) & 255u], 1u);
      }
      __syncthreads();
      if (t == 0) {
        unsigned r = sel_rank, acc = 0;
        int b = 0;
        for (; b < 256; ++b) {
          if (acc + hist[b] > r) break;
          acc += hist[b];
        }
        sel_prefix = pref | ((unsigned)b << shift);
        sel_rank = r - acc;
      }
      __syncthreads();
    }
    const double tv = (double)__uint_as_float(sel_prefix);
    double c_lt = 0, s_lt = 0, q_lt = 0, s_all = 0, q_all = 0;
    for (int s = pb + t; s < pe; s += EMP_T) {
      if (!used(s)) continue;
      const double v = pbar[s];
      s_all += v;
      q_all += v * v;
      if (v < tv) { c_lt += 1; s_lt += v; q_lt += v * v; }
    }
    c_lt = bsum<EMP_T>(c_lt, lds);
    s_lt = bsum<EMP_T>(s_lt, lds);
    q_lt = bsum<EMP_T>(q_lt, lds);
    s_all = bsum<EMP_T>(s_all, lds);
    q_all = bsum<EMP_T>(q_all, lds);
    const double fill = n_lo - c_lt;
    const double s0 = s_lt + fill * tv, q0 = q_lt + fill * tv * tv;
    const double n_hi = nu - n_lo;
    mu0 = s0 / n_lo;
    sd0 = fmax(sqrt(fmax(q0 / n_lo - mu0 * mu0, 0.0)), 1e-3);
    mu1 = (s_all - s0) / n_hi;
    sd1 = fmax(sqrt(fmax((q_all - q0) / n_hi - mu1 * mu1, 0.0)), 1e-3);
    w1 = 0.9;
    for (int it = 0; it < 20; ++it) {
      double r1s = 0, r0s = 0, r1v = 0, r0v = 0;
      for (int s = pb + t; s < pe; s += EMP_T) {
        if (!used(s)) continue;
        const double v = pbar[s];
        const double r1 = inlier_resp(v, mu0, sd0, mu1, sd1, w1);
        resp[s] = r1;
        r1s += r1;
        r0s += 1.0 - r1;
        r1v += r1 * v;
        r0v += (1.0 - r1) * v;
      }
      r1s = bsum<EMP_T>(r1s, lds);
      r0s = bsum<EMP_T>(r0s, lds);
      r1v = bsum<EMP_T>(r1v, lds);
      r0v = bsum<EMP_T>(r0v, lds);
      if (!(r1s > 0) || !(r0s > 0)) break;
      const double nmu1 = r1v / r1s, nmu0 = r0v / r0s;
      double d1 = 0, d0 = 0;
      for (int s = pb + t; s < pe; s += EMP_T) {
        if (!used(s)) continue;
        const double v = pbar[s];
        const double r1 = resp[s];
        d1 += r1 * (v - nmu1) * (v - nmu1);
        d0 += (1.0 - r1) * (v - nmu0) * (v - nmu0);
      }
      d1 = bsum<EMP_T>(d1, lds);
      d0 = bsum<EMP_T>(d0, lds);
      w1 = r1s / nu;
      mu1 = nmu1;
      mu0 = nmu0;
      sd1 = fmax(sqrt(d1 / r1s), 1e-3);
      sd0 = fmax(sqrt(d0 / r0s), 1e-3);
    }
  }
  const bool swap = fit && mu0 > mu1;
  // patch weights, then the M-step sums over the problem's patches
  double swpe2 = 0, swp = 0, sw = 0, nex = 0;
  for (int s = pb + t; s < pe; s += EMP_T) {
    double W;
    const bool u = used(s);
    if (fix_w) {
      W = patch_w[s];
    } else {
      double pi = 0;
      if (u) {
        pi = fit ? inlier_resp((double)pbar[s], mu0, sd0, mu1, sd1, w1) : 1.0;
        if (swap) pi = 1.0 - pi;
      }
      W = (u && pi >= 0.5) ? pi : 0.0;
      patch_w[s] = (float)W;
      W = (double)(float)W;
    }
    const double *o = pstat + PSTAT * s;
    swpe2 += W * o[8];
    swp += W * o[7];
    sw += W * o[5];
    nex += (u && W == 0) ? 1.0 : 0.0;
  }
  swpe2 = bsum<EMP_T>(swpe2, lds);
  swp = bsum<EMP_T>(swp, lds);
  sw = bsum<EMP_T>(sw, lds);
  nex = bsum<EMP_T>(nex, lds);
  if (t == 0) {
    pvr_em_state &st = em[blockIdx.x];
    const double floor2 = (1e-4 * st.y_abs_max) * (1e-4 * st.y_abs_max);
    st.sum_wp = swp;
    st.sum_wpe2 = swpe2;
    st.sum_w = sw;
    if (swp > 0) st.sigma2 = fmax(swpe2 / swp, floor2);
    if (sw > 0) st.c = swp / sw;
    st.n_used = nu;
    st.n_excluded = (int)nex;
  }
}

extern "C" pvr_status pvr_robust_weights(pvr_plan *p, const float *resid, const float *y_obs,
                                         pvr_em_state *em, float *pp, float *pbar,
                                         float *patch_w, int32_t flags, hipStream_t stream) {
  PVR_API_BEGIN();
  if (!p || !resid || !y_obs || !em || !patch_w) return fail(PVR_EINVAL, "pvr_robust_weights: NULL argument");
  if (!p->built) return fail(PVR_EINVAL, "pvr_robust_weights: plan has not been built");
  const int init = (flags & PVR_EM_INIT) != 0;
  const int fix = (flags & PVR_EM_FIX_W) != 0;
  // p_bar is needed by the classification even when the caller does not want it
  float *pb = pbar ? pbar : p->d_pbar;
  hipLaunchKernelGGL(k_em_patch_stats, dim3(p->M), dim3(EM_T), 0, stream, p->d_patch, p->d_invz,
                     resid, y_obs, p->d_pstat);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_em_problem, dim3(p->P), dim3(EMP_T), 0, stream, p->d_prob, p->d_pstat, em,
                     init);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_em_estep, dim3(p->M), dim3(EM_T), 0, stream, p->d_patch, p->d_invz, resid,
                     em, pp, pb, p->d_pstat);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_em_patches, dim3(p->P), dim3(EMP_T), 0, stream, p->d_prob, pb, p->d_active,
                     p->d_pstat, p->d_resp, patch_w, em, fix);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}
