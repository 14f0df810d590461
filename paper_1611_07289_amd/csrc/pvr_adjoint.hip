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

// rq_j = (W_s p_j e_j / Z_j, W_s p_j / Z_j) for valid samples, 0 otherwise.
template <typename T>
__global__ void __launch_bounds__(SIM_THREADS)
k_bp_prep(const PatchDev *__restrict__ patches, const BlockWork *__restrict__ work,
          const T *__restrict__ invz, const T *__restrict__ e, const T *__restrict__ p,
          const T *__restrict__ patch_w, typename Vec2Of<T>::type *__restrict__ rq) {
  const BlockWork wk = work[blockIdx.x];
  const PatchDev pt = patches[wk.patch];
  const T w = patch_w ? patch_w[wk.patch] : (T)1;
  const int n = pt.w * pt.h;
  const int l1 = min(n, wk.l0 + SIM_CHUNK);
  for (int l = wk.l0 + threadIdx.x; l < l1; l += SIM_THREADS) {
    const long long j = pt.off + l;
    const T iz = invz[j];
    typename Vec2Of<T>::type o;
    if (iz > (T)0 && w != (T)0) {
      const T q = w * (p ? p[j] : (T)1) * iz;
      o.x = q * e[j];
      o.y = q;
    } else {
      o.x = 0;
      o.y = 0;
    }
    rq[j] = o;
  }
}

// Contribution of one patch to one voxel mapped to pixel coordinates
// (pu, pv) with normalised through-plane term qk.  The candidate pixels are
// rint(p) + [-h, h] on both axes (a superset of the integers inside the
// in-plane support ellipse); candidates outside the support or the patch get
// weight 0 and read a clamped, in-patch address.
template <typename T, typename GEO, typename V2, int HU, int HV>
__device__ __forceinline__ void adj_patch(const GEO &g, const PatchDev &pt, double pu, double pv,
                                          T qk, int hu_rt, int hv_rt,
                                          const V2 *__restrict__ rq, T &sn, T &sd) {
  const int hu = HU > 0 ? HU : hu_rt, hv = HV > 0 ? HV : hv_rt;
  const double rud = rint(pu), rvd = rint(pv);
  const int ru = (int)rud, rv = (int)rvd;
  const T fu = (T)(pu - rud), fv = (T)(pv - rvd);
  const T cu = (T)g.cu, cv = (T)g.cv, K2 = (T)g.K2, cut = (T)g.cut;
  const int x1 = pt.x0 + pt.w - 1, y1 = pt.y0 + pt.h - 1;
  const V2 *base = rq + pt.off;
#pragma unroll
  for (int b = -hv; b <= hv; ++b) {
    const int v = rv + b;
    const T wv = ((T)b - fv) * cv;
    const T qkv = fma(wv, wv, qk);
    const bool vok = (v >= pt.y0) & (v <= y1);
    const int vrow = (min(max(v, pt.y0), y1) - pt.y0) * pt.w;
#pragma unroll
    for (int a = -hu; a <= hu; ++a) {
      const int u = ru + a;
      const T wu = ((T)a - fu) * cu;
      const T Q = fma(wu, wu, qkv);
      const bool ok = vok & (u >= pt.x0) & (u <= x1) & (Q <= K2);
      T gh = fast_exp2<T>(-Q) - cut;
      gh = ok ? (gh > (T)0 ? gh : (T)0) : (T)0;
      const V2 r = base[vrow + (min(max(u, pt.x0), x1) - pt.x0)];
      sn = fma(gh, r.x, sn);
      sd = fma(gh, r.y, sd);
    }
  }
}

// One workgroup = one 8^3 brick; each wavefront owns one 4^3 sub-brick and
// walks that sub-brick's patch list (wave-uniform), one voxel per lane.
template <typename T, bool DEN>
__global__ void __launch_bounds__(BP_THREADS)
k_backproject(const ProbDev *__restrict__ probs, const PatchDev *__restrict__ patches,
              const typename GeoOf<T>::type *__restrict__ geo, const int *__restrict__ brick_prob,
              const int *__restrict__ sub_off, const int *__restrict__ sub_patch,
              const typename Vec2Of<T>::type *__restrict__ rq, T *__restrict__ num,
              T *__restrict__ den) {
  using GEO = typename GeoOf<T>::type;
  using V2 = typename Vec2Of<T>::type;
  const int bi = blockIdx.x;
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
    const GEO &g = geo[s];
    const PatchDev pt = patches[s];
    const double pk = fma(g.G[8], fi, fma(g.G[9], fj, fma(g.G[10], fk, g.G[11])));
    const T wk = (T)(pk - (double)pt.slice) * (T)g.ck;
    const T qk = wk * wk;
    if (!(qk <= (T)g.K2)) continue;
    const double pu = fma(g.G[0], fi, fma(g.G[1], fj, fma(g.G[2], fk, g.G[3])));
    const double pv = fma(g.G[4], fi, fma(g.G[5], fj, fma(g.G[6], fk, g.G[7])));
    if (g.hu == 1 && g.hv == 1)
      adj_patch<T, GEO, V2, 1, 1>(g, pt, pu, pv, qk, 1, 1, rq, sn, sd);
    else
      adj_patch<T, GEO, V2, 0, 0>(g, pt, pu, pv, qk, g.hu, g.hv, rq, sn, sd);
  }
  if (inside) {
    const long long idx = pr.vol_off + ((long long)kk * pr.ny + jj) * pr.nx + i;
    num[idx] = sn;
    if (DEN) den[idx] = sd;
  }
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
  hipLaunchKernelGGL(k_bp_prep<T>, dim3(p->n_sim_blocks), dim3(SIM_THREADS), 0, stream, p->d_patch,
                     p->d_sim_blocks, invz, e, pp, patch_w, rq);
  HIP_TRY(hipGetLastError());
  const void *geo = sizeof(T) == 4 ? (const void *)p->d_geof : (const void *)p->d_geod;
  if (den)
    hipLaunchKernelGGL((k_backproject<T, true>), dim3(p->n_bricks), dim3(BP_THREADS), 0, stream,
                       p->d_prob, p->d_patch, (const typename GeoOf<T>::type *)geo, p->d_brick_prob,
                       p->d_sub_off, p->d_sub_patch, rq, num, den);
  else
    hipLaunchKernelGGL((k_backproject<T, false>), dim3(p->n_bricks), dim3(BP_THREADS), 0, stream,
                       p->d_prob, p->d_patch, (const typename GeoOf<T>::type *)geo, p->d_brick_prob,
                       p->d_sub_off, p->d_sub_patch, rq, num, den);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
}

extern "C" pvr_status pvr_backproject(const pvr_plan *p, const float *e, const float *pp,
                                      const float *patch_w, float *num, float *den,
                                      hipStream_t stream) {
  PVR_API_BEGIN();
  if (!p) return fail(PVR_EINVAL, "pvr_backproject: plan is NULL");
  if (!p->built) return fail(PVR_EINVAL, "pvr_backproject: plan has not been built");
  return backproject_impl<float>(p, e, pp, patch_w, num, den, p->d_invz, p->d_rq, stream);
  PVR_API_END();
}

extern "C" pvr_status pvr_backproject_f64(const pvr_plan *p, const double *e, const double *pp,
                                          const double *patch_w, double *num, double *den,
                                          hipStream_t stream) {
  PVR_API_BEGIN();
  if (!p) return fail(PVR_EINVAL, "pvr_backproject_f64: plan is NULL");
  if (!p->built || !p->built64) return fail(PVR_EINVAL, "pvr_backproject_f64: plan needs pvr_plan_build_f64");
  pvr_plan *mp = const_cast<pvr_plan *>(p);
  if (!mp->d_rq64) DEV_ALLOC(mp, mp->d_rq64, mp->N);
  return backproject_impl<double>(p, e, pp, patch_w, num, den, p->d_invz64, mp->d_rq64, stream);
  PVR_API_END();
}
