// Per-patch motion geometry shared by the plan build and the registration
// kernel (which rebuilds it for every trial transform).
#pragma once

#include "pvr_internal.h"

namespace pvr {

// ---------------------------------------------------------------------------
// small 3x3 / 3x4 helpers (row-major), host and device
// ---------------------------------------------------------------------------
__host__ __device__ static inline void mat3_mul(const double *a, const double *b,
                                                double *c) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      c[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}

__host__ __device__ static inline double mat3_inv(const double *m, double *o) {
  double det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
               m[2] * (m[3] * m[7] - m[4] * m[6]);
  double id = 1.0 / det;
  o[0] = (m[4] * m[8] - m[5] * m[7]) * id;
  o[1] = (m[2] * m[7] - m[1] * m[8]) * id;
  o[2] = (m[1] * m[5] - m[2] * m[4]) * id;
  o[3] = (m[5] * m[6] - m[3] * m[8]) * id;
  o[4] = (m[0] * m[8] - m[2] * m[6]) * id;
  o[5] = (m[2] * m[3] - m[0] * m[5]) * id;
  o[6] = (m[3] * m[7] - m[4] * m[6]) * id;
  o[7] = (m[1] * m[6] - m[0] * m[7]) * id;
  o[8] = (m[0] * m[4] - m[1] * m[3]) * id;
  return det;
}

// affine a (3x4) -> linear L (3x3) and offset t
__host__ __device__ static inline void aff_split(const double *a, double *L, double *t) {
  for (int r = 0; r < 3; ++r) {
    L[3 * r] = a[4 * r]; L[3 * r + 1] = a[4 * r + 1]; L[3 * r + 2] = a[4 * r + 2];
    t[r] = a[4 * r + 3];
  }
}

__host__ __device__ static inline void aff_join(const double *L, const double *t, double *a) {
  for (int r = 0; r < 3; ++r) {
    a[4 * r] = L[3 * r]; a[4 * r + 1] = L[3 * r + 1]; a[4 * r + 2] = L[3 * r + 2];
    a[4 * r + 3] = t[r];
  }
}

__host__ __device__ static inline void aff_inv(const double *a, double *o) {
  double L[9], t[3], Li[9], ti[3];
  aff_split(a, L, t);
  mat3_inv(L, Li);
  for (int r = 0; r < 3; ++r) ti[r] = -(Li[3 * r] * t[0] + Li[3 * r + 1] * t[1] + Li[3 * r + 2] * t[2]);
  aff_join(Li, ti, o);
}

// Integer pixels within the in-plane support radius sqrt(K2) / c of a point
// lie among rint(p) + [-h, h] with h = floor(R + 1/2); c = sqrt(kappa) *
// spacing / sigma along the axis.  Depends on the stack only (not on the
// motion), so the plan sizes the adjoint's candidate grid from it.
__host__ __device__ static inline int cand_halfwidth(double K2, double c) {
  return (int)floor(sqrt(K2) / c + 0.5);
}

// The same for the sinc PSF's main lobe |t| < 1 with t = pixel offset * c.
__host__ __device__ static inline int sinc_halfwidth(double c) {
  return (int)floor(1.0 / c + 0.5);
}

// R = Rz(rz) Ry(ry) Rx(rx)
__host__ __device__ static inline void rot_zyx(const double *th, double *R) {
  double cx = cos(th[0]), sx = sin(th[0]), cy = cos(th[1]), sy = sin(th[1]);
  double cz = cos(th[2]), sz = sin(th[2]);
  R[0] = cz * cy; R[1] = cz * sy * sx - sz * cx; R[2] = cz * sy * cx + sz * sx;
  R[3] = sz * cy; R[4] = sz * sy * sx + cz * cx; R[5] = sz * sy * cx - cz * sx;
  R[6] = -sy;     R[7] = cy * sx;                R[8] = cy * cx;
}

// Per-patch motion geometry (see pvr_internal.h).  One thread per patch.
// PSF: PVR_PSF_GAUSSIAN or PVR_PSF_SINC, a template parameter so that code
// which only ever uses one PSF (registration) carries no code for the other.
template <int PSF = PVR_PSF_GAUSSIAN>
__device__ inline void make_geometry(const ProbDev &pr, const StackDev &st, const PatchDev &pt,
                              const double *th, double k, GeoD &g, GeoF &gf, int *bb) {
  constexpr int psf = PSF;
  double R[9];
  rot_zyx(th, R);
  double A[9], o[3];
  aff_split(st.p2w, A, o);
  double pc[3] = {pt.x0 + 0.5 * (pt.w - 1), pt.y0 + 0.5 * (pt.h - 1), (double)pt.slice};
  double c[3];
  for (int r = 0; r < 3; ++r) c[r] = A[3 * r] * pc[0] + A[3 * r + 1] * pc[1] + A[3 * r + 2] * pc[2] + o[r];
  // motion x -> R x + m0 with m0 = c - R c + t
  double m0[3];
  for (int r = 0; r < 3; ++r)
    m0[r] = c[r] - (R[3 * r] * c[0] + R[3 * r + 1] * c[1] + R[3 * r + 2] * c[2]) + th[3 + r];
  double Wl[9], wo[3];
  aff_split(pr.w2v, Wl, wo);
  double RA[9], HL[9];
  mat3_mul(R, A, RA);
  mat3_mul(Wl, RA, HL);
  double Ro[3], Ho[3];
  for (int r = 0; r < 3; ++r) Ro[r] = R[3 * r] * o[0] + R[3 * r + 1] * o[1] + R[3 * r + 2] * o[2] + m0[r];
  for (int r = 0; r < 3; ++r) Ho[r] = Wl[3 * r] * Ro[0] + Wl[3 * r + 1] * Ro[1] + Wl[3 * r + 2] * Ro[2] + wo[r];
  aff_join(HL, Ho, g.H);
  aff_inv(g.H, g.G);
  // quadratic form in voxel offsets: L = diag(1/sigma) F^T Vl, A' = kappa L^T L
  double F[9], Vl[9], vo[3];
  mat3_mul(R, st.E, F);
  aff_split(pr.v2w, Vl, vo);
  double L[9];
  for (int a = 0; a < 3; ++a)
    for (int j = 0; j < 3; ++j)
      L[3 * a + j] = (F[a] * Vl[j] + F[3 + a] * Vl[3 + j] + F[6 + a] * Vl[6 + j]) / st.sigma[a];
  double Aq[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      Aq[3 * i + j] = KAPPA * (L[i] * L[j] + L[3 + i] * L[3 + j] + L[6 + i] * L[6 + j]);
  double Ai[9];
  mat3_inv(Aq, Ai);
  const double K2 = KAPPA * k * k;
  double ext[3];
  for (int b = 0; b < 3; ++b) ext[b] = sqrt(K2 * Ai[4 * b]);
  if constexpr (psf == PVR_PSF_SINC) {
    // support box |t_u| < 1, |t_v| < 1, |t_n| <= k with t = diag(1/w_u, 1/w_v,
    // 1/sigma_n) F^T Vl (voxel offset): its half extent along voxel axis b is
    // sum_a |(Wl F)_{b a}| h_a, h = (w_u, w_v, k sigma_n)
    const double hw[3] = {st.wz[0], st.wz[1], k * st.sigma[2]};
    const double sc[3] = {1.0 / st.wz[0], 1.0 / st.wz[1], 1.0 / st.sigma[2]};
    for (int a = 0; a < 3; ++a)
      for (int j = 0; j < 3; ++j)
        g.L[3 * a + j] = (F[a] * Vl[j] + F[3 + a] * Vl[3 + j] + F[6 + a] * Vl[6 + j]) * sc[a];
    double WF[9];
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a)
        WF[3 * b + a] = Wl[3 * b] * F[a] + Wl[3 * b + 1] * F[3 + a] + Wl[3 * b + 2] * F[6 + a];
    for (int b = 0; b < 3; ++b)
      ext[b] = fabs(WF[3 * b]) * hw[0] + fabs(WF[3 * b + 1]) * hw[1] + fabs(WF[3 * b + 2]) * hw[2];
  }
  g.psf = psf;
  g.kcut = k;  // (L is set for the sinc PSF only)
  for (int b = 0; b < 3; ++b) { g.ext[b] = ext[b]; gf.ext[b] = (float)ext[b]; }
  int ic = 0;
  if (ext[1] > ext[ic]) ic = 1;
  if (ext[2] > ext[ic]) ic = 2;
  int ia = ic == 0 ? 1 : 0;
  int ib = 3 - ic - ia;
  g.perm[0] = ia; g.perm[1] = ib; g.perm[2] = ic;
  const double Acc = Aq[4 * ic];
  const double Aca = Aq[3 * ic + ia], Acb = Aq[3 * ic + ib];
  g.Acc = Acc; g.Aca = Aca; g.Acb = Acb;
  g.Saa = Aq[4 * ia] - Aca * Aca / Acc;
  g.Sab = Aq[3 * ia + ib] - Aca * Acb / Acc;
  g.Sbb = Aq[4 * ib] - Acb * Acb / Acc;
  g.iAinv_aa = 1.0 / Ai[4 * ia];
  g.ha = ext[ia];
  g.inv_Acc = 1.0 / Acc;
  g.inv_Sbb = 1.0 / g.Sbb;
  g.nSab_Sbb = -g.Sab / g.Sbb;
  g.K2 = K2;
  g.cut = exp2(-K2);
  const double sk = sqrt(KAPPA);
  g.cu = sk * st.spacing[0] / st.sigma[0];
  g.cv = sk * st.spacing[1] / st.sigma[1];
  g.ck = sk * st.spacing[2] / st.sigma[2];
  if constexpr (psf == PVR_PSF_SINC) {
    // in-plane: pixel offset -> t (the sinc's argument over pi)
    g.cu = st.spacing[0] / st.wz[0];
    g.cv = st.spacing[1] / st.wz[1];
  }
  // brick range of the union of the patch's supports: the pixel box grown by
  // the support's half widths along every stack axis, mapped by H
  double r3[3];
  for (int a = 0; a < 3; ++a) r3[a] = k * st.sigma[a] / st.spacing[a];
  if constexpr (psf == PVR_PSF_SINC)
    for (int a = 0; a < 2; ++a) r3[a] = st.wz[a] / st.spacing[a];
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int q = 0; q < 8; ++q) {
    double cu = (q & 1) ? pt.x0 + pt.w - 1 + r3[0] : pt.x0 - r3[0];
    double cv = (q & 2) ? pt.y0 + pt.h - 1 + r3[1] : pt.y0 - r3[1];
    double cs = (q & 4) ? pt.slice + r3[2] : pt.slice - r3[2];
    for (int r = 0; r < 3; ++r) {
      double x = g.H[4 * r] * cu + g.H[4 * r + 1] * cv + g.H[4 * r + 2] * cs + g.H[4 * r + 3];
      lo[r] = fmin(lo[r], x);
      hi[r] = fmax(hi[r], x);
    }
  }
  const int nb[3] = {pr.nbx, pr.nby, pr.nbz};
  for (int r = 0; r < 3; ++r) {
    // clamped before the conversion, so that a non-finite motion gives an
    // empty range instead of an out-of-range integer
    const double span = (double)BRICK * (nb[r] + 2);
    double l = fmin(fmax(floor(lo[r]) - 1.0, -span), span);
    double h = fmin(fmax(ceil(hi[r]) + 1.0, -span), span);
    int bl = (int)floor(l / BRICK), bh = (int)floor(h / BRICK);
    bl = bl < 0 ? 0 : bl;
    bh = bh > nb[r] - 1 ? nb[r] - 1 : bh;
    g.bb_lo[r] = bl; g.bb_hi[r] = bh;
    bb[r] = bl; bb[3 + r] = bh;
  }
  // single-precision copy
  for (int q = 0; q < 12; ++q) { gf.H[q] = g.H[q]; gf.G[q] = g.G[q]; }
  gf.Acc = (float)g.Acc; gf.Aca = (float)g.Aca; gf.Acb = (float)g.Acb;
  gf.Saa = (float)g.Saa; gf.Sab = (float)g.Sab; gf.Sbb = (float)g.Sbb;
  gf.iAinv_aa = (float)g.iAinv_aa; gf.ha = (float)g.ha;
  gf.inv_Acc = (float)g.inv_Acc; gf.inv_Sbb = (float)g.inv_Sbb; gf.nSab_Sbb = (float)g.nSab_Sbb;
  gf.K2 = (float)g.K2; gf.cut = (float)g.cut;
  gf.cu = (float)g.cu; gf.cv = (float)g.cv; gf.ck = (float)g.ck;
  g.inv_cu = 1.0 / g.cu; g.inv_cv = 1.0 / g.cv;
  // integer pixels within the in-plane support radius R of a point p are
  // among rint(p) + [-h, h] with h = floor(R + 1/2)
  g.hu = psf == PVR_PSF_SINC ? sinc_halfwidth(g.cu) : cand_halfwidth(K2, g.cu);
  g.hv = psf == PVR_PSF_SINC ? sinc_halfwidth(g.cv) : cand_halfwidth(K2, g.cv);
  gf.hu = g.hu; gf.hv = g.hv;
  gf.psf = g.psf;
  if constexpr (psf == PVR_PSF_SINC) {
    gf.kcut = (float)g.kcut;
    for (int q = 0; q < 9; ++q) gf.L[q] = (float)g.L[q];
  }
  gf.inv_cu = (float)g.inv_cu; gf.inv_cv = (float)g.inv_cv;
  for (int q = 0; q < 3; ++q) gf.perm[q] = g.perm[q];
}


}  // namespace pvr
