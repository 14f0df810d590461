// Adjoint direction ("pixel-volume") as a gather: every voxel sums, in a fixed
// order, the contributions of the samples whose PSF support covers it, so no
// two lanes ever write the same address and the result is bitwise repeatable.
//
// Patches are indexed per 4^3 sub-brick (one wavefront), in patch order.  For
// a voxel and a patch, the voxel is mapped (FP64 affine G) into the patch's
// unmoved pixel frame; the PSF is axis-aligned there, so the candidate pixels
// are the integer (u, v) inside an ellipse around the mapped point, on the
// patch's single slice.
#include <math.h>

#include "pvr_internal.h"
#include "pvr_util.h"

using namespace pvr;

constexpr int BP_THREADS = BRICK * BRICK * BRICK;

template <typename T> struct Vec2Of;
template <> struct Vec2Of<float> { using type = float2; };
template <> struct Vec2Of<double> { using type = double2; };

// rq_j = (p_j e_j / Z_j, p_j / Z_j) for valid samples, 0 otherwise (the
// patch weight W_s is applied by the gather, per patch).
template <typename T>
__global__ void __launch_bounds__(SIM_THREADS)
k_bp_prep(const PatchDev *__restrict__ patches, const BlockWork *__restrict__ work,
          const T *__restrict__ invz, const T *__restrict__ e, const T *__restrict__ p,
          typename Vec2Of<T>::type *__restrict__ rq) {
  const BlockWork wk = work[blockIdx.x];
  const PatchDev pt = patches[wk.patch];
  const int n = pt.w * pt.h;
  const int l1 = min(n, wk.l0 + SIM_CHUNK);
  // one sample (invalid samples, 1/Z = 0, get 0)
  auto one = [&](long long j, T iz, T pj, T ej) {
    typename Vec2Of<T>::type o;
    if (iz > (T)0) {
      const T q = pj * iz;
      o.x = q * ej;
      o.y = q;
    } else {
      o.x = 0;
      o.y = 0;
    }
    rq[j] = o;
  };
  // four samples per thread in flight: their reads are independent (e and p
  // are defined for every sample)
  int l = wk.l0 + threadIdx.x;
  for (; l + 3 * SIM_THREADS < l1; l += 4 * SIM_THREADS) {
    T iz[4], pj[4], ej[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long j = pt.off + l + u * SIM_THREADS;
      iz[u] = invz[j];
      pj[u] = p ? p[j] : (T)1;
      ej[u] = e[j];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) one(pt.off + l + u * SIM_THREADS, iz[u], pj[u], ej[u]);
  }
  for (; l < l1; l += SIM_THREADS) {
    const long long j = pt.off + l;
    one(j, invz[j], p ? p[j] : (T)1, e[j]);
  }
}

// Raw buffer view of one patch's n rq entries plus one entry on either side
// (the neighbouring patches' entries, or the zero guards around the whole
// array), so byte offset (i + 1) sizeof(V2) addresses entry i, i in [-1, n].
// A buffer load never faults: outside the view it returns 0, so candidate
// pixels off the patch need no address clamp.  Their weights are zeroed
// explicitly, so whatever such a load returns never contributes.  The one
// entry of margin matters because the compiler merges the loads of two
// adjacent candidates into one 16-byte load, and a partly out-of-range load
// may return 0 for all of it: with the margin, a pair holding an in-patch
// entry is always wholly in range.
template <typename V2>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t patch_rsrc(const V2 *patch_base, int n) {
  return raw_buffer(patch_base - 1, (unsigned)(n + 2) * (unsigned)sizeof(V2));
}

template <typename V2> __device__ __forceinline__ V2 load_rq(__amdgpu_buffer_rsrc_t r, int off);
template <> __device__ __forceinline__ float2 load_rq<float2>(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <> __device__ __forceinline__ double2 load_rq<double2>(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

// max(a b - c, 0) for a b - c in [-1, 1]: one FMA with the output clamp.
template <typename T> __device__ __forceinline__ T fma_clamp0(T a, T b, T c);
template <> __device__ __forceinline__ float fma_clamp0<float>(float a, float b, float c) {
  return __builtin_amdgcn_fmed3f(fmaf(a, b, -c), 0.f, 1.f);
}
template <> __device__ __forceinline__ double fma_clamp0<double>(double a, double b, double c) {
  return fmax(fma(a, b, -c), 0.0);
}

// Contribution of one patch to one voxel mapped to pixel coordinates
// (pu, pv) with normalised through-plane term qk.  The candidate pixels are
// rint(p) + [-HU, HU] x [-HV, HV] (a superset of the integers inside the
// in-plane support ellipse).  The weight factorises over the axes of the
// patch frame, 2^-Q = 2^-(qk + wv^2) 2^-(wu^2), so a candidate costs one
// product; rows and columns outside the patch get the factor 0, and
// 2^-Q - 2^-K2 is clamped at 0 outside the support (every value lies in
// [-1, 1], so the clamp to [0, 1] is exact).
template <typename T, typename GEO, typename V2, int HU, int HV, bool DEN>
__device__ __forceinline__ void adj_patch(const GEO &g, const PatchDev &pt, double pu, double pv,
                                          T qk, const V2 *__restrict__ rq, T &sn, T &sd) {
  const double rud = rint(pu), rvd = rint(pv);
  const int ru = (int)rud - pt.x0, rv = (int)rvd - pt.y0;  // patch-local nearest pixel
  const T fu = (T)(pu - rud), fv = (T)(pv - rvd);
  const T cu = (T)g.cu, cv = (T)g.cv, cut = (T)g.cut;
  T U[2 * HU + 1], E[2 * HV + 1];
#pragma unroll
  for (int a = -HU; a <= HU; ++a) {
    const T wu = ((T)a - fu) * cu;
    const bool in = (unsigned)(ru + a) < (unsigned)pt.w;
    U[a + HU] = in ? fast_exp2<T>(-wu * wu) : (T)0;
  }
#pragma unroll
  for (int b = -HV; b <= HV; ++b) {
    const T wv = ((T)b - fv) * cv;
    const bool in = (unsigned)(rv + b) < (unsigned)pt.h;
    E[b + HV] = in ? fast_exp2<T>(-fma(wv, wv, qk)) : (T)0;
  }
  const __amdgpu_buffer_rsrc_t r = patch_rsrc(rq + pt.off, pt.w * pt.h);
  const int row_bytes = pt.w * (int)sizeof(V2);
  int off = ((rv - HV) * pt.w + (ru - HU) + 1) * (int)sizeof(V2);
#pragma unroll
  for (int b = 0; b < 2 * HV + 1; ++b) {
#pragma unroll
    for (int a = 0; a < 2 * HU + 1; ++a) {
      const T gh = fma_clamp0<T>(E[b], U[a], cut);
      const V2 q = load_rq<V2>(r, off + a * (int)sizeof(V2));
      sn = fma(gh, q.x, sn);
      if (DEN) sd = fma(gh, q.y, sd);
    }
    off += row_bytes;
  }
}

// Candidate grids wider than the unrolled shapes (PSF much wider than a
// pixel): the same arithmetic with run-time half-widths, one exponential
// per candidate.
template <typename T, typename GEO, typename V2, bool DEN>
__device__ __forceinline__ void adj_patch_rt(const GEO &g, const PatchDev &pt, double pu, double pv,
                                             T qk, const V2 *__restrict__ rq, T &sn, T &sd) {
  const int hu = g.hu, hv = g.hv;
  const double rud = rint(pu), rvd = rint(pv);
  const int ru = (int)rud - pt.x0, rv = (int)rvd - pt.y0;
  const T fu = (T)(pu - rud), fv = (T)(pv - rvd);
  const T cu = (T)g.cu, cv = (T)g.cv, cut = (T)g.cut;
  const __amdgpu_buffer_rsrc_t r = patch_rsrc(rq + pt.off, pt.w * pt.h);
  for (int b = -hv; b <= hv; ++b) {
    const T wv = ((T)b - fv) * cv;
    const T qkv = fma(wv, wv, qk);
    const int row = (rv + b) * pt.w;
    for (int a = -hu; a <= hu; ++a) {
      const T wu = ((T)a - fu) * cu;
      const bool in = ((unsigned)(ru + a) < (unsigned)pt.w) & ((unsigned)(rv + b) < (unsigned)pt.h);
      const T gh = in ? fma_clamp0<T>(fast_exp2<T>(-fma(wu, wu, qkv)), (T)1, cut) : (T)0;
      const V2 q = load_rq<V2>(r, (row + ru + a + 1) * (int)sizeof(V2));
      sn = fma(gh, q.x, sn);
      if (DEN) sd = fma(gh, q.y, sd);
    }
  }
}

// The sinc PSF (PVR_PSF_SINC): the weight factorises over the patch frame as
// s(t_u) s(t_v) g(t_n) with t = pixel offset * (spacing / first zero) in-plane
// and g = 2^-qk - 2^-K2 (clamped at 0) through-plane; candidates outside the
// main lobe (|t| >= 1) or the patch get the factor 0.  HU, HV > 0: the
// candidate half-widths every patch fits; 0 reads them per patch.
template <typename T, typename GEO, typename V2, int HU, int HV, bool DEN>
__device__ __forceinline__ void adj_patch_sinc(const GEO &g, const PatchDev &pt, double pu,
                                               double pv, T qk, const V2 *__restrict__ rq, T &sn,
                                               T &sd) {
  const int hu = HU > 0 ? HU : g.hu, hv = HV > 0 ? HV : g.hv;
  const double rud = rint(pu), rvd = rint(pv);
  const int ru = (int)rud - pt.x0, rv = (int)rvd - pt.y0;
  const T fu = (T)(pu - rud), fv = (T)(pv - rvd);
  const T cu = (T)g.cu, cv = (T)g.cv, cut = (T)g.cut;
  T gz = fast_exp2<T>(-qk) - cut;
  gz = gz > (T)0 ? gz : (T)0;
  const __amdgpu_buffer_rsrc_t r = patch_rsrc(rq + pt.off, pt.w * pt.h);
  for (int b = -hv; b <= hv; ++b) {
    const T tv = ((T)b - fv) * cv;
    const bool inb = ((unsigned)(rv + b) < (unsigned)pt.h) & (fabs(tv) < (T)1);
    const T e = inb ? sinc_poly<T>(tv) * gz : (T)0;
    const int row = (rv + b) * pt.w;
    for (int a = -hu; a <= hu; ++a) {
      const T tu = ((T)a - fu) * cu;
      const bool ina = ((unsigned)(ru + a) < (unsigned)pt.w) & (fabs(tu) < (T)1);
      const T gh = ina ? sinc_poly<T>(tu) * e : (T)0;
      const V2 q = load_rq<V2>(r, (row + ru + a + 1) * (int)sizeof(V2));
      sn = fma(gh, q.x, sn);
      if (DEN) sd = fma(gh, q.y, sd);
    }
  }
}

// One workgroup = one 8^3 brick; each wavefront owns one 4^3 sub-brick and
// walks that sub-brick's patch list (wave-uniform), one voxel per lane.
// HW: the candidate half-width every patch of the plan fits (1 or 2, fixed
// at compile time), or 0 to read it per patch.
template <typename T, bool DEN, int HW, bool SINC>
__global__ void __launch_bounds__(BP_THREADS)
k_backproject(const ProbDev *__restrict__ probs, const PatchDev *__restrict__ patches,
              const typename GeoOf<T>::type *__restrict__ geo, const int *__restrict__ brick_prob,
              const int *__restrict__ sub_off, const int *__restrict__ sub_patch,
              const typename Vec2Of<T>::type *__restrict__ rq, const T *__restrict__ patch_w,
              T *__restrict__ num, T *__restrict__ den, int n_bricks, int granule) {
  using GEO = typename GeoOf<T>::type;
  using V2 = typename Vec2Of<T>::type;
  const int bi = xcd_work(blockIdx.x, granule);
  if (bi >= n_bricks) return;
  const ProbDev pr = probs[brick_prob[bi]];
  const int local = bi - pr.brick_base;
  const int bx = local % pr.nbx, by = (local / pr.nbx) % pr.nby, bz = local / (pr.nbx * pr.nby);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  const int i = bx * BRICK + (w & 1) * SUB + (l & 3);
  const int jj = by * BRICK + ((w >> 1) & 1) * SUB + ((l >> 2) & 3);
  const int kk = bz * BRICK + (w >> 2) * SUB + (l >> 4);
  const bool inside = i < pr.nx && jj < pr.ny && kk < pr.nz;
  T sn = 0, sd = 0;
  const int sbi = bi * 8 + w;
  const int q0 = sub_off[sbi], q1 = sub_off[sbi + 1];
  const double fi = i, fj = jj, fk = kk;
  for (int q = q0; q < q1; ++q) {
    const int s = sub_patch[q];
    // the patch weight scales the patch's whole contribution; an excluded
    // patch (weight 0) is skipped
    const T ws = patch_w ? patch_w[s] : (T)1;
    if (ws == (T)0) continue;
    const GEO &g = geo[s];
    const PatchDev pt = patches[s];
    const double pk = fma(g.G[8], fi, fma(g.G[9], fj, fma(g.G[10], fk, g.G[11])));
    const T wk = (T)(pk - (double)pt.slice) * (T)g.ck;
    const T qk = wk * wk;
    if (!(qk <= (T)g.K2)) continue;
    const double pu = fma(g.G[0], fi, fma(g.G[1], fj, fma(g.G[2], fk, g.G[3])));
    const double pv = fma(g.G[4], fi, fma(g.G[5], fj, fma(g.G[6], fk, g.G[7])));
    T pn = 0, pd = 0;
    if (SINC)
      adj_patch_sinc<T, GEO, V2, HW, HW, DEN>(g, pt, pu, pv, qk, rq, pn, pd);
    else if (HW == 1)
      adj_patch<T, GEO, V2, 1, 1, DEN>(g, pt, pu, pv, qk, rq, pn, pd);
    else if (HW == 2)
      adj_patch<T, GEO, V2, 2, 2, DEN>(g, pt, pu, pv, qk, rq, pn, pd);
    else
      adj_patch_rt<T, GEO, V2, DEN>(g, pt, pu, pv, qk, rq, pn, pd);
    sn = fma(ws, pn, sn);
    if (DEN) sd = fma(ws, pd, sd);
  }
  if (inside) {
    const long long idx = pr.vol_off + ((long long)kk * pr.ny + jj) * pr.nx + i;
    num[idx] = sn;
    if (DEN) den[idx] = sd;
  }
}

// The preparation pass on its own (FP32), for pvr_robust_weights.
pvr_status pvr::launch_bp_prep(const pvr_plan *p, const float *e, const float *pp,
                               hipStream_t stream) {
  hipLaunchKernelGGL(k_bp_prep<float>, dim3(p->n_sim_blocks), dim3(SIM_THREADS), 0, stream,
                     p->d_patch, p->d_sim_blocks, p->d_invz, e, pp, p->d_rq + 1);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
}

template <typename T>
static pvr_status backproject_impl(const pvr_plan *p, const T *e, const T *pp, const T *patch_w,
                                   T *num, T *den, const T *invz, typename Vec2Of<T>::type *rq,
                                   hipStream_t stream) {
  if (!e || !num) return fail(PVR_EINVAL, "pvr_backproject: e and num are required");
  if (!p->index_valid) {
    const pvr_status st = plan_build_index(const_cast<pvr_plan *>(p), stream);
    if (st != PVR_OK) return st;
  }
  // the preparation pass, unless pvr_robust_weights (PVR_EM_PREP_ADJOINT)
  // already ran it for these residuals and posteriors
  const bool prepared = sizeof(T) == 4 && p->rq_fresh && p->rq_e == (const void *)e &&
                        p->rq_p == (const void *)pp;
  if (!prepared) {
    hipLaunchKernelGGL(k_bp_prep<T>, dim3(p->n_sim_blocks), dim3(SIM_THREADS), 0, stream,
                       p->d_patch, p->d_sim_blocks, invz, e, pp, rq);
    HIP_TRY(hipGetLastError());
  }
  const void *geo = sizeof(T) == 4 ? (const void *)p->d_geof : (const void *)p->d_geod;
  const dim3 grid(xcd_blocks(p->n_bricks, p->bp_granule));
  hipEvent_t *ev = timing_slot(p, PVR_KERNEL_BACKPROJECT);
  if (ev) HIP_TRY(hipEventRecord(ev[0], stream));
  const int hw = (p->max_hu <= 1 && p->max_hv <= 1) ? 1 : (p->max_hu <= 2 && p->max_hv <= 2) ? 2 : 0;
  const auto *geot = (const typename GeoOf<T>::type *)geo;
#define BP_LAUNCH(D, H, SC)                                                                     \
  hipLaunchKernelGGL((k_backproject<T, D, H, SC>), grid, dim3(BP_THREADS), 0, stream, p->d_prob, \
                     p->d_patch, geot, p->d_brick_prob, p->d_sub_off, p->d_sub_patch, rq,         \
                     patch_w, num, den, p->n_bricks, p->bp_granule)
#define BP_LAUNCH_HW(D, SC)            \
  if (hw == 1) BP_LAUNCH(D, 1, SC);    \
  else if (hw == 2) BP_LAUNCH(D, 2, SC); \
  else BP_LAUNCH(D, 0, SC)
  const bool sinc = p->psf == PVR_PSF_SINC;
  if (den) {
    if (sinc) { BP_LAUNCH_HW(true, true); }
    else { BP_LAUNCH_HW(true, false); }
  } else {
    if (sinc) { BP_LAUNCH_HW(false, true); }
    else { BP_LAUNCH_HW(false, false); }
  }
#undef BP_LAUNCH_HW
#undef BP_LAUNCH
  HIP_TRY(hipGetLastError());
  if (ev) HIP_TRY(hipEventRecord(ev[1], stream));
  return PVR_OK;
}

extern "C" pvr_status pvr_backproject(const pvr_plan *p, const float *e, const float *pp,
                                      const float *patch_w, float *num, float *den,
                                      hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_backproject", e, 4);
  PVR_ALIGNED("pvr_backproject", pp, 4);
  PVR_ALIGNED("pvr_backproject", patch_w, 4);
  PVR_ALIGNED("pvr_backproject", num, 4);
  PVR_ALIGNED("pvr_backproject", den, 4);
  if (!p) return fail(PVR_EINVAL, "pvr_backproject: plan is NULL");
  if (!p->built) return fail(PVR_EINVAL, "pvr_backproject: plan has not been built");
  PVR_TRY_STATUS(debug_finite(p, "pvr_backproject", "e", e, p->N, stream));
  PVR_TRY_STATUS(debug_finite(p, "pvr_backproject", "p", pp, p->N, stream));
  PVR_TRY_STATUS(debug_weights(p, "pvr_backproject", "patch_w", patch_w, p->M, stream));
  return backproject_impl<float>(p, e, pp, patch_w, num, den, p->d_invz, p->d_rq + 1, stream);
  PVR_API_END();
}

extern "C" pvr_status pvr_backproject_f64(const pvr_plan *p, const double *e, const double *pp,
                                          const double *patch_w, double *num, double *den,
                                          hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_backproject_f64", e, 8);
  PVR_ALIGNED("pvr_backproject_f64", pp, 8);
  PVR_ALIGNED("pvr_backproject_f64", patch_w, 8);
  PVR_ALIGNED("pvr_backproject_f64", num, 8);
  PVR_ALIGNED("pvr_backproject_f64", den, 8);
  if (!p) return fail(PVR_EINVAL, "pvr_backproject_f64: plan is NULL");
  if (!p->built || !p->built64)
    return fail(PVR_EINVAL, "pvr_backproject_f64: plan needs pvr_plan_build_f64 on a workspace "
                            "attached with PVR_WS_F64");
  PVR_TRY_STATUS(debug_finite(p, "pvr_backproject_f64", "e", e, p->N, stream));
  PVR_TRY_STATUS(debug_finite(p, "pvr_backproject_f64", "p", pp, p->N, stream));
  PVR_TRY_STATUS(debug_weights(p, "pvr_backproject_f64", "patch_w", patch_w, p->M, stream));
  return backproject_impl<double>(p, e, pp, patch_w, num, den, p->d_invz64, p->d_rq64 + 1, stream);
  PVR_API_END();
}
