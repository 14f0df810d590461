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
constexpr int EMP_LDS = 12288; // patches per problem whose potentials fit the LDS copy

// Workgroup reductions in a fixed order: a butterfly inside every wave, then
// the wave results combined in wave order by every lane.  lds must hold
// NT / 64 doubles per reduced value.
enum class Op { Sum, Min, Max };

template <Op OP>
__device__ __forceinline__ double combine(double a, double b) {
  if (OP == Op::Sum) return a + b;
  if (OP == Op::Min) return fmin(a, b);
  return fmax(a, b);
}

template <int NT, Op OP>
__device__ __forceinline__ double breduce(double v, double *lds) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = combine<OP>(v, __shfl_xor(v, o, 64));
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double r = lds[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) r = combine<OP>(r, lds[w]);
  __syncthreads();
  return r;
}

// K sums at once (one pair of barriers)
template <int NT, int K>
__device__ __forceinline__ void bsumk(double (&v)[K], double *lds) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    double x = v[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) lds[q * NW + wave] = x;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < K; ++q) {
    double r = lds[q * NW];
#pragma unroll
    for (int w = 1; w < NW; ++w) r += lds[q * NW + w];
    v[q] = r;
  }
  __syncthreads();
}

template <int NT> __device__ __forceinline__ double bsum(double v, double *lds) { return breduce<NT, Op::Sum>(v, lds); }
template <int NT> __device__ __forceinline__ double bmin(double v, double *lds) { return breduce<NT, Op::Min>(v, lds); }
template <int NT> __device__ __forceinline__ double bmax(double v, double *lds) { return breduce<NT, Op::Max>(v, lds); }

__global__ void __launch_bounds__(EM_T)
k_em_patch_stats(const PatchDev *__restrict__ patches, const float *__restrict__ invz,
                 const float *__restrict__ e, const float *__restrict__ y,
                 double *__restrict__ pstat) {
  __shared__ double lds[8 * (EM_T / 64)];
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
  double red[2] = {se2, cnt};
  bsumk<EM_T, 2>(red, lds);
  se2 = red[0]; cnt = red[1];
  if (threadIdx.x == 0) {
    double *o = pstat + PSTAT * s;
    o[0] = mn; o[1] = mx; o[2] = ym; o[3] = se2; o[4] = cnt;
  }
}

// Per-problem reduction of the residual statistics: from the per-patch table
// (pstat, stride PSTAT), or with chunk_stats from the forward kernel's
// per-chunk records (stride 5) over the problem's chunk range.
__global__ void __launch_bounds__(EMP_T)
k_em_problem(const ProbDev *__restrict__ probs, const double *__restrict__ pstat,
             const double *__restrict__ chunk_stats, pvr_em_state *__restrict__ em, int init,
             unsigned *__restrict__ status) {
  __shared__ double lds[8 * (EMP_T / 64)];
  const ProbDev pr = probs[blockIdx.x];
  double mn = INFINITY, mx = -INFINITY, ym = 0, se2 = 0, cnt = 0;
  const int r0 = chunk_stats ? pr.chunk_begin : pr.patch_begin;
  const int r1 = chunk_stats ? pr.chunk_end : pr.patch_end;
  for (int s = r0 + threadIdx.x; s < r1; s += EMP_T) {
    const double *o = chunk_stats ? chunk_stats + 5 * (long long)s : pstat + PSTAT * s;
    mn = fmin(mn, o[0]);
    mx = fmax(mx, o[1]);
    ym = fmax(ym, o[2]);
    se2 += o[3];
    cnt += o[4];
  }
  // the five reductions at once: a butterfly inside every wave, then thread 0
  // combines the wave results in wave order (the order of breduce / bsumk)
  {
    constexpr int NW = EMP_T / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      mn = fmin(mn, __shfl_xor(mn, o, 64));
      mx = fmax(mx, __shfl_xor(mx, o, 64));
      ym = fmax(ym, __shfl_xor(ym, o, 64));
      se2 += __shfl_xor(se2, o, 64);
      cnt += __shfl_xor(cnt, o, 64);
    }
    if (lane == 0) {
      lds[0 * NW + wave] = mn;
      lds[1 * NW + wave] = mx;
      lds[2 * NW + wave] = ym;
      lds[3 * NW + wave] = se2;
      lds[4 * NW + wave] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      mn = lds[0]; mx = lds[NW]; ym = lds[2 * NW]; se2 = lds[3 * NW]; cnt = lds[4 * NW];
      for (int w = 1; w < NW; ++w) {
        mn = fmin(mn, lds[w]);
        mx = fmax(mx, lds[NW + w]);
        ym = fmax(ym, lds[2 * NW + w]);
        se2 += lds[3 * NW + w];
        cnt += lds[4 * NW + w];
      }
    }
  }
  if (threadIdx.x == 0) {
    // min / max skip NaN residuals, their squares' sum does not
    if (!isfinite(se2) || !isfinite(mx - mn) || !isfinite(ym)) atomicOr(status, PVR_FAULT_RESIDUAL);
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
  __shared__ double lds[8 * (EM_T / 64)];
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
  // one sample: the posterior and the sums (invalid samples, 1/Z = 0, get 0)
  auto one = [&](long long j, float iz, float ev) {
    float pj = 0.f;
    if (iz > 0.f) {
      const float Gc = cG0 * expf(-ev * ev * inv2s2);
      const float dd = Gc + mo;
      pj = dd > 0.f ? Gc / dd : 0.f;
      ns += 1.0;
      sp2 += (double)pj * pj;
      sp += pj;
      spe2 += (double)pj * ev * ev;
    }
    if (p_out) p_out[j] = pj;
  };
  // four samples per thread in flight (the loop is latency-bound), taken in
  // the same order as one at a time; e is read for invalid samples too (it
  // is defined for every sample)
  int l = threadIdx.x;
  for (; l + 3 * EM_T < n; l += 4 * EM_T) {
    float iz[4], ev[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long j = pt.off + l + u * EM_T;
      iz[u] = invz[j];
      ev[u] = e[j];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) one(pt.off + l + u * EM_T, iz[u], ev[u]);
  }
  for (; l < n; l += EM_T) {
    const long long j = pt.off + l;
    one(j, invz[j], e[j]);
  }
  double red[4] = {ns, sp2, sp, spe2};
  bsumk<EM_T, 4>(red, lds);
  ns = red[0]; sp2 = red[1]; sp = red[2]; spe2 = red[3];
  if (threadIdx.x == 0) {
    double *o = pstat + PSTAT * s;
    o[5] = ns; o[6] = sp2; o[7] = sp; o[8] = spe2;
    if (pbar) pbar[s] = ns > 0 ? (float)sqrt(sp2 / ns) : 0.f;
  }
}

// Inlier responsibility 1 / (1 + exp(l0 - l1)) with
// l_c = log(weight_c) - log(sd_c) - (v - mu_c)^2 / (2 sd_c^2); the constant
// 0.5 log(2 pi) cancels.  The per-component constants are computed once per
// mixture iteration.
struct Mix {
  double mu0, mu1, h0, h1, c0, c1;  // h = 1 / (2 sd^2), c = log(weight) - log(sd)
};

__device__ __forceinline__ Mix make_mix(double mu0, double sd0, double mu1, double sd1, double w1) {
  Mix m;
  m.mu0 = mu0; m.mu1 = mu1;
  m.h0 = 0.5 / (sd0 * sd0); m.h1 = 0.5 / (sd1 * sd1);
  m.c1 = w1 > 0 ? log(w1) - log(sd1) : -INFINITY;
  m.c0 = w1 < 1 ? log(1.0 - w1) - log(sd0) : -INFINITY;
  return m;
}

__device__ __forceinline__ double inlier_resp(double v, const Mix &m) {
  const double d0 = v - m.mu0, d1 = v - m.mu1;
  const double l1 = m.c1 - d1 * d1 * m.h1;
  const double l0 = m.c0 - d0 * d0 * m.h0;
  return 1.0 / (1.0 + exp(l0 - l1));
}

// The same in single precision for the mixture iterations (the sums over
// patches stay FP64; the responsibilities differ from the FP64 ones by ~1e-7
// relative, which moves the fitted parameters by as little).  The final
// patch posteriors use inlier_resp.
struct MixF {
  float mu0, mu1, h0, h1, c0, c1;
};
// The constants of make_mix in single precision from the FP64 parameters
// (single-precision logarithms: the constants only enter inlier_resp_f).
__device__ __forceinline__ MixF make_mix_f(double mu0, double sd0, double mu1, double sd1,
                                          double w1) {
  const float s0 = (float)sd0, s1 = (float)sd1, wf = (float)w1;
  MixF m;
  m.mu0 = (float)mu0;
  m.mu1 = (float)mu1;
  m.h0 = 0.5f / (s0 * s0);
  m.h1 = 0.5f / (s1 * s1);
  m.c1 = w1 > 0 ? __logf(wf) - __logf(s1) : -INFINITY;
  m.c0 = w1 < 1 ? __logf(1.f - wf) - __logf(s0) : -INFINITY;
  return m;
}
__device__ __forceinline__ float inlier_resp_f(float v, const MixF &m) {
  const float d0 = v - m.mu0, d1 = v - m.mu1;
  const float l = (m.c0 - d0 * d0 * m.h0) - (m.c1 - d1 * d1 * m.h1);
  // l = +-inf when a component has zero weight: exp gives inf or 0, 1/(1+inf) = 0
  return __builtin_amdgcn_rcpf(1.f + __expf(l));
}

// Two-component mixture on the potentials of one problem, patch weights and
// the M-step.  The start splits the potentials at the median: the n/2 smallest
// form the low component.  The split value is found exactly by a radix select
// on the float bit patterns (potentials are >= 0, so the patterns are ordered
// like the values).
//
// The potentials of the problem's patches are first copied to a compact
// array (-1 marks a patch that takes no part): in LDS when the problem has
// at most EMP_LDS patches, else in the plan's scratch array, so the 20
// mixture iterations touch only that array.  One pass per iteration gathers
// the high component's sums of r, r v and r v^2; the low component's follow
// from the totals (sum 1, sum v, sum v^2), and each variance is
// E[v^2] - mean^2 (values in [0, 1], FP64: the cancellation costs ~1e-16 /
// var relative, against a floor of 1e-6 on the variance).  Inside the
// iterations the responsibilities are single precision (inlier_resp_f).
__global__ void __launch_bounds__(EMP_T)
k_em_patches(const ProbDev *__restrict__ probs, const float *__restrict__ pbar,
             const uint8_t *__restrict__ active, const double *__restrict__ pstat,
             float *__restrict__ gval, float *__restrict__ patch_w, pvr_em_state *__restrict__ em,
             int fix_w, int use_lds) {
  __shared__ double lds[8 * (EMP_T / 64)];
  __shared__ unsigned int hist[256];
  __shared__ unsigned int sel_prefix, sel_rank;
  __shared__ double mixp[5];  // mu0, sd0, mu1, sd1, w1
  __shared__ MixF mixf;
  __shared__ int mix_stop;
  extern __shared__ float sval[];
  const ProbDev pr = probs[blockIdx.x];
  const int t = threadIdx.x;
  const int pb = pr.patch_begin, np = pr.patch_end - pr.patch_begin;
  float *V = use_lds ? sval : gval + pb;
  double n = 0, s_all = 0, q_all = 0;
  // the patches taking part (valid samples, active) and their potentials;
  // the three reads of a patch are independent and four patches per thread
  // are in flight, taken in the same order as one at a time
  auto take = [&](int q, double ns, uint8_t act, float pv) {
    const float v = (ns > 0 && act != 0) ? pv : -1.f;
    V[q] = v;
    if (v >= 0.f) {
      n += 1.0;
      s_all += (double)v;
      q_all += (double)v * (double)v;
    }
  };
  {
    int q = t;
    for (; q + 3 * EMP_T < np; q += 4 * EMP_T) {
      double ns[4];
      uint8_t act[4];
      float pv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int s = pb + q + u * EMP_T;
        ns[u] = pstat[PSTAT * s + 5];
        act[u] = active[s];
        pv[u] = pbar[s];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) take(q + u * EMP_T, ns[u], act[u], pv[u]);
    }
    for (; q < np; q += EMP_T) {
      const int s = pb + q;
      take(q, pstat[PSTAT * s + 5], active[s], pbar[s]);
    }
  }
  {
    double r3[3] = {n, s_all, q_all};
    bsumk<EMP_T, 3>(r3, lds);  // its barriers also publish V
    n = r3[0]; s_all = r3[1]; q_all = r3[2];
  }
  const int nu = (int)n;
  double mu0 = 0, sd0 = 1, mu1 = 0, sd1 = 1, w1 = 0.9;
  const bool fit = nu >= 2;
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
      for (int q = t; q < np; q += EMP_T) {
        const float v = V[q];
        if (!(v >= 0.f)) continue;
        const unsigned bits = __float_as_uint(v);
        if ((bits & mask_hi) == pref) atomicAdd(&hist[(bits >> shift) & 255u], 1u);
      }
      __syncthreads();
      // the bin holding rank r: wave 0 scans the 256 counts (4 per lane)
      if (t < 64) {
        const unsigned r = sel_rank;
        const unsigned h0 = hist[4 * t], h1 = hist[4 * t + 1], h2 = hist[4 * t + 2],
                       h3 = hist[4 * t + 3];
        const unsigned tot = h0 + h1 + h2 + h3;
        unsigned incl = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const unsigned v = __shfl_up(incl, o, 64);
          if (t >= o) incl += v;
        }
        const unsigned long long hit = __ballot(incl > r);
        if (hit != 0ull && t == __ffsll((long long)hit) - 1) {
          unsigned acc = incl - tot;
          int b = 4 * t;
          if (acc + h0 <= r) {
            acc += h0; ++b;
            if (acc + h1 <= r) {
              acc += h1; ++b;
              if (acc + h2 <= r) { acc += h2; ++b; }
            }
          }
          sel_prefix = pref | ((unsigned)b << shift);
          sel_rank = r - acc;
        }
      }
      __syncthreads();
    }
    const double tv = (double)__uint_as_float(sel_prefix);
    double c_lt = 0, s_lt = 0, q_lt = 0;
    for (int q = t; q < np; q += EMP_T) {
      const double v = V[q];
      if (v >= 0 && v < tv) { c_lt += 1; s_lt += v; q_lt += v * v; }
    }
    double red3[3] = {c_lt, s_lt, q_lt};
    bsumk<EMP_T, 3>(red3, lds);
    c_lt = red3[0]; s_lt = red3[1]; q_lt = red3[2];
    // the mixture state lives in LDS and is updated by one lane: its FP64
    // divisions, square roots and logarithms would otherwise run in all 16
    // waves of the workgroup
    if (t == 0) {
      const double fill = n_lo - c_lt;
      const double s0 = s_lt + fill * tv, q0 = q_lt + fill * tv * tv;
      const double n_hi = nu - n_lo;
      const double m0 = s0 / n_lo, m1 = (s_all - s0) / n_hi;
      mixp[0] = m0;
      mixp[1] = fmax(sqrt(fmax(q0 / n_lo - m0 * m0, 0.0)), 1e-3);
      mixp[2] = m1;
      mixp[3] = fmax(sqrt(fmax((q_all - q0) / n_hi - m1 * m1, 0.0)), 1e-3);
      mixp[4] = 0.9;
      mixf = make_mix_f(mixp[0], mixp[1], mixp[2], mixp[3], mixp[4]);
      mix_stop = 0;
    }
    __syncthreads();
    for (int it = 0; it < 20; ++it) {
      double r1s = 0, r1v = 0, r1q = 0;
      const MixF mx = mixf;
      for (int q = t; q < np; q += EMP_T) {
        const float vf = V[q];
        if (!(vf >= 0.f)) continue;
        const double v = vf;
        const double r1 = inlier_resp_f(vf, mx);
        r1s += r1;
        r1v += r1 * v;
        r1q += r1 * v * v;
      }
      double red[3] = {r1s, r1v, r1q};
      bsumk<EMP_T, 3>(red, lds);
      if (t == 0) {
        r1s = red[0]; r1v = red[1]; r1q = red[2];
        const double r0s = nu - r1s;
        if (!(r1s > 0) || !(r0s > 0)) {
          mix_stop = 1;
        } else {
          const double m1 = r1v / r1s, m0 = (s_all - r1v) / r0s;
          mixp[2] = m1;
          mixp[0] = m0;
          mixp[3] = fmax(sqrt(fmax(r1q / r1s - m1 * m1, 0.0)), 1e-3);
          mixp[1] = fmax(sqrt(fmax((q_all - r1q) / r0s - m0 * m0, 0.0)), 1e-3);
          mixp[4] = r1s / nu;
          mixf = make_mix_f(mixp[0], mixp[1], mixp[2], mixp[3], mixp[4]);
        }
      }
      __syncthreads();
      if (mix_stop) break;
    }
    mu0 = mixp[0]; sd0 = mixp[1]; mu1 = mixp[2]; sd1 = mixp[3]; w1 = mixp[4];
  }
  const bool swap = fit && mu0 > mu1;
  const Mix mfin = make_mix(mu0, sd0, mu1, sd1, w1);
  // patch weights, then the M-step sums over the problem's patches
  double swpe2 = 0, swp = 0, sw = 0, nex = 0;
  // one patch: its weight (given, or from the fitted mixture) and its terms
  // of the M-step sums, from its partials o = (N_s, sum p, sum p e^2)
  auto weigh = [&](int q, double o5, double o7, double o8, float wgiven) {
    const int s = pb + q;
    double W;
    const bool u = V[q] >= 0.f;
    if (fix_w) {
      W = wgiven;
    } else {
      double pi = 0;
      if (u) {
        pi = fit ? inlier_resp((double)V[q], mfin) : 1.0;
        if (swap) pi = 1.0 - pi;
      }
      W = (u && pi >= 0.5) ? pi : 0.0;
      patch_w[s] = (float)W;
      W = (double)(float)W;
    }
    swpe2 += W * o8;
    swp += W * o7;
    sw += W * o5;
    nex += (u && W == 0) ? 1.0 : 0.0;
  };
  // four patches' partials per thread in flight, in the order of one at a time
  {
    int q = t;
    for (; q + 3 * EMP_T < np; q += 4 * EMP_T) {
      double o5[4], o7[4], o8[4];
      float wg[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int s = pb + q + u * EMP_T;
        const double *o = pstat + PSTAT * s;
        o5[u] = o[5];
        o7[u] = o[7];
        o8[u] = o[8];
        wg[u] = fix_w ? patch_w[s] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) weigh(q + u * EMP_T, o5[u], o7[u], o8[u], wg[u]);
    }
    for (; q < np; q += EMP_T) {
      const int s = pb + q;
      const double *o = pstat + PSTAT * s;
      weigh(q, o[5], o[7], o[8], fix_w ? patch_w[s] : 0.f);
    }
  }
  double red4b[4] = {swpe2, swp, sw, nex};
  bsumk<EMP_T, 4>(red4b, lds);
  swpe2 = red4b[0]; swp = red4b[1]; sw = red4b[2]; nex = red4b[3];
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
  PVR_ALIGNED("pvr_robust_weights", resid, 4);
  PVR_ALIGNED("pvr_robust_weights", y_obs, 4);
  PVR_ALIGNED("pvr_robust_weights", em, 8);
  PVR_ALIGNED("pvr_robust_weights", pp, 4);
  PVR_ALIGNED("pvr_robust_weights", pbar, 4);
  PVR_ALIGNED("pvr_robust_weights", patch_w, 4);
  if (!p || !resid || !y_obs || !em || !patch_w) return fail(PVR_EINVAL, "pvr_robust_weights: NULL argument");
  if (!p->built) return fail(PVR_EINVAL, "pvr_robust_weights: plan has not been built");
  PVR_TRY_STATUS(debug_finite(p, "pvr_robust_weights", "resid", resid, p->N, stream));
  PVR_TRY_STATUS(debug_finite(p, "pvr_robust_weights", "y_obs", y_obs, p->N, stream));
  const int init = (flags & PVR_EM_INIT) != 0;
  const int fix = (flags & PVR_EM_FIX_W) != 0;
  // p_bar is needed by the classification even when the caller does not want it
  float *pb = pbar ? pbar : p->d_pbar;
  // residual statistics: reused from the forward kernel when the caller vouches
  // that resid is unchanged since the plan's last pvr_simulate wrote it
  const bool fresh = (flags & PVR_EM_RESID_FRESH) && p->stats_valid && p->stats_resid == resid &&
                     p->stats_y == y_obs;
  if (!fresh) {
    hipLaunchKernelGGL(k_em_patch_stats, dim3(p->M), dim3(EM_T), 0, stream, p->d_patch, p->d_invz,
                       resid, y_obs, p->d_pstat);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_em_problem, dim3(p->P), dim3(EMP_T), 0, stream, p->d_prob, p->d_pstat,
                     fresh ? (const double *)p->d_chunk_stats : nullptr, em, init, p->d_status);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_em_estep, dim3(p->M), dim3(EM_T), 0, stream, p->d_patch, p->d_invz, resid,
                     em, pp, pb, p->d_pstat);
  HIP_TRY(hipGetLastError());
  // the adjoint's inputs need the posteriors only, not the patch weights: on
  // request they are prepared on the plan's second stream while the patch
  // classification (one workgroup per problem) runs on this one
  const bool prep = (flags & PVR_EM_PREP_ADJOINT) && pp != nullptr;
  p->rq_fresh = false;
  if (prep) {
    HIP_TRY(hipEventRecord(p->ev_fork, stream));
    HIP_TRY(hipStreamWaitEvent(p->side, p->ev_fork, 0));
    const pvr_status st = launch_bp_prep(p, resid, pp, p->side);
    if (st != PVR_OK) return st;
    HIP_TRY(hipEventRecord(p->ev_join, p->side));
  }
  const int use_lds = p->max_problem_patches <= EMP_LDS;
  hipLaunchKernelGGL(k_em_patches, dim3(p->P), dim3(EMP_T),
                     use_lds ? (size_t)p->max_problem_patches * sizeof(float) : 0, stream,
                     p->d_prob, pb, p->d_active, p->d_pstat, p->d_pval, patch_w, em, fix, use_lds);
  HIP_TRY(hipGetLastError());
  if (prep) {
    HIP_TRY(hipStreamWaitEvent(stream, p->ev_join, 0));
    p->rq_fresh = true;
    p->rq_e = resid;
    p->rq_p = pp;
  }
  return PVR_OK;
  PVR_API_END();
}
