// Derivative of the forward model's PSF weights with respect to the
// per-patch motion, shared by the theta-gradient kernel and the exact-gradient
// registration.
//
// Inside the support g_hat = exp(-Q/2) - exp(-k^2/2) and
//   Q = D^T M D,  D = v_i - x_j (world),  M = F diag(1/sigma^2) F^T,
// with x_j = R (P_j - c) + c + t and F = R E.  Writing z = M D and
// y = v_i - c - t = D + R (P_j - c):
//   dQ/dt   = -2 z,
//   dQ/dr_k = 2 omega_k . (z x y),
// where omega_k is the world axis of the k-th elementary rotation of
// R = Rz Ry Rx (omega_x = Rz Ry e_x, omega_y = Rz e_y, omega_z = e_z), since
// dR/dr_k = [omega_k]_x R.  Hence d g_hat / d theta = exp(-Q/2) *
// (-omega_k . (z x y), z).  The support boundary itself does not move the sum
// because g_hat vanishes there.
#pragma once

#include "pvr_geometry.h"
#include "pvr_internal.h"

namespace pvr {

struct GradConst {
  double M[9];      // F diag(1/sigma^2) F^T (world, mm^-2)
  double om[9];     // omega_x, omega_y, omega_z as rows
  double Vl[9];     // vox2world linear part
  double ct[3];     // c + t (world)
  double v2w_o[3];  // vox2world offset
};

__device__ inline void make_grad_const(const ProbDev &pr, const StackDev &st, const PatchDev &pt,
                                const double *th, GradConst &gc) {
  double R[9];
  rot_zyx(th, R);
  double F[9];
  mat3_mul(R, st.E, F);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int a = 0; a < 3; ++a) s += F[3 * i + a] * F[3 * j + a] / (st.sigma[a] * st.sigma[a]);
      gc.M[3 * i + j] = s;
    }
  const double cz = cos(th[2]), sz = sin(th[2]), cy = cos(th[1]), sy = sin(th[1]);
  // omega_x = Rz Ry e_x, omega_y = Rz e_y, omega_z = e_z
  gc.om[0] = cz * cy; gc.om[1] = sz * cy; gc.om[2] = -sy;
  gc.om[3] = -sz;     gc.om[4] = cz;      gc.om[5] = 0.0;
  gc.om[6] = 0.0;     gc.om[7] = 0.0;     gc.om[8] = 1.0;
  double A[9], o[3];
  aff_split(st.p2w, A, o);
  const double pc[3] = {pt.x0 + 0.5 * (pt.w - 1), pt.y0 + 0.5 * (pt.h - 1), (double)pt.slice};
  for (int r = 0; r < 3; ++r)
    gc.ct[r] = A[3 * r] * pc[0] + A[3 * r + 1] * pc[1] + A[3 * r + 2] * pc[2] + o[r] + th[3 + r];
  aff_split(pr.v2w, gc.Vl, gc.v2w_o);
}

// Derivative walk over the support of one sample: accumulates
// sum_i (X_i - yh) d g_hat / d theta (six values, in T) over in-grid voxels.
template <typename T, typename GEO>
__device__ __forceinline__ void grad_walk(const GEO &g, const ProbDev &p, const GradConst &gc,
                                          const int b[3], const T f[3], const T q[3],
                                          const T *__restrict__ Xp, T yh, T acc6[6]) {
  const int ia = g.perm[0], ib = g.perm[1], ic = g.perm[2];
  const int n_a = sel3(ia, p.nx, p.ny, p.nz), n_b = sel3(ib, p.nx, p.ny, p.nz),
            n_c = sel3(ic, p.nx, p.ny, p.nz);
  const int sy = p.nx, sz = p.nx * p.ny;
  const int st_a = sel3(ia, 1, sy, sz), st_b = sel3(ib, 1, sy, sz), st_c = sel3(ic, 1, sy, sz);
  const int b_a = sel3(ia, b[0], b[1], b[2]), b_b = sel3(ib, b[0], b[1], b[2]),
            b_c = sel3(ic, b[0], b[1], b[2]);
  const T f_a = sel3f<T>(ia, f[0], f[1], f[2]), f_b = sel3f<T>(ib, f[0], f[1], f[2]),
          f_c = sel3f<T>(ic, f[0], f[1], f[2]);
  const T K2 = (T)g.K2, cut = (T)g.cut, Acc = (T)g.Acc, Aca = (T)g.Aca, Acb = (T)g.Acb,
          Saa = (T)g.Saa, Sab = (T)g.Sab, Sbb = (T)g.Sbb, iAaa = (T)g.iAinv_aa, ha = (T)g.ha,
          iAcc = (T)g.inv_Acc, iSbb = (T)g.inv_Sbb, nSab = (T)g.nSab_Sbb;
  // world step per unit of each permuted voxel axis (columns of Vl)
  T Va[3], Vb[3], Vc[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    Va[r] = (T)gc.Vl[3 * r + ia];
    Vb[r] = (T)gc.Vl[3 * r + ib];
    Vc[r] = (T)gc.Vl[3 * r + ic];
  }
  T M[9], om[9];
#pragma unroll
  for (int r = 0; r < 9; ++r) { M[r] = (T)gc.M[r]; om[r] = (T)gc.om[r]; }
  const T *Xb = Xp + ((long long)b[2] * p.ny + b[1]) * p.nx + b[0];
  const int lo_a = max((int)ceil(f_a - ha), -b_a);
  const int hi_a = min((int)floor(f_a + ha), n_a - 1 - b_a);
  for (int oa = lo_a; oa <= hi_a; ++oa) {
    const T wa = (T)oa - f_a;
    const T rem = K2 - wa * wa * iAaa;
    if (rem < (T)0) continue;
    const T wbc = nSab * wa;
    const T rb = sqrt(rem * iSbb);
    const int lo_b = max((int)ceil(f_b + wbc - rb), -b_b);
    const int hi_b = min((int)floor(f_b + wbc + rb), n_b - 1 - b_b);
    const T qa = Saa * wa * wa;
    const T sa2 = (T)2 * Sab * wa;
    for (int ob = lo_b; ob <= hi_b; ++ob) {
      const T wb = (T)ob - f_b;
      const T q1 = qa + wb * (sa2 + Sbb * wb);
      const T rem2 = K2 - q1;
      if (rem2 < (T)0) continue;
      const T wcc = -(Aca * wa + Acb * wb) * iAcc;
      const T rc = sqrt(rem2 * iAcc);
      const int lo_c = max((int)ceil(f_c + wcc - rc), -b_c);
      const int hi_c = min((int)floor(f_c + wcc + rc), n_c - 1 - b_c);
      T d = ((T)lo_c - f_c) - wcc;
      T wc = (T)lo_c - f_c;
      int off = oa * st_a + ob * st_b + lo_c * st_c;
      for (int oc = lo_c; oc <= hi_c; ++oc) {
        const T Qs = fma(Acc * d, d, q1);
        const T e2 = fast_exp2<T>(-Qs);
        if (e2 - cut > (T)0) {
          T D[3];
#pragma unroll
          for (int r = 0; r < 3; ++r) D[r] = Va[r] * wa + Vb[r] * wb + Vc[r] * wc;
          T zz[3];
#pragma unroll
          for (int r = 0; r < 3; ++r) zz[r] = M[3 * r] * D[0] + M[3 * r + 1] * D[1] + M[3 * r + 2] * D[2];
          const T y0 = D[0] + q[0], y1 = D[1] + q[1], y2 = D[2] + q[2];
          const T cr0 = zz[1] * y2 - zz[2] * y1, cr1 = zz[2] * y0 - zz[0] * y2,
                  cr2 = zz[0] * y1 - zz[1] * y0;
          const T wgt = e2 * (Xb[off] - yh);
#pragma unroll
          for (int k = 0; k < 3; ++k)
            acc6[k] -= wgt * (om[3 * k] * cr0 + om[3 * k + 1] * cr1 + om[3 * k + 2] * cr2);
          acc6[3] += wgt * zz[0];
          acc6[4] += wgt * zz[1];
          acc6[5] += wgt * zz[2];
        }
        off += st_c;
        d += (T)1;
        wc += (T)1;
      }
    }
  }
}


// ---------------------------------------------------------------------------
// Moment form of the derivative sums, for one sample x_j.  With voxel offsets
// u = (w_a, w_b, w_c) from the sample centre along the walk's permuted voxel
// axes and V the world step per unit of each (so D = V u), the derivative
// weights w_i = e^{-Q_i/2} (X_i - y_hat) over the support enter only through
//   n = sum_i w_i u_i  and  S = sum_i w_i u_i u_i^T:
//   sum_i w_i z_i          = M V n = P n                    (translations),
//   sum_i w_i z_i x y_i    = c + (P n) x q,  c_r = eps_rst (P S V^T)_st,
// with q = x_j - (c_s + t), since z x y = (M D) x D + (M D) x q.  The walk
// therefore accumulates nine moments per weight set instead of evaluating
// the derivative at every voxel.
struct GradMom {
  float V[9];   // V[3 r + a]: world component r of the step along walk axis a
  float P[9];   // M V
  float om[9];  // rotation axes omega_k as rows
};

__device__ inline void make_grad_mom(const GradConst &gc, const int perm[3], GradMom &gm) {
  for (int r = 0; r < 3; ++r)
    for (int a = 0; a < 3; ++a) gm.V[3 * r + a] = (float)gc.Vl[3 * r + perm[a]];
  for (int r = 0; r < 3; ++r)
    for (int a = 0; a < 3; ++a) {
      double s = 0;
      for (int m = 0; m < 3; ++m) s += gc.M[3 * r + m] * gc.Vl[3 * m + perm[a]];
      gm.P[3 * r + a] = (float)s;
    }
  for (int q = 0; q < 9; ++q) gm.om[q] = (float)gc.om[q];
}

// One walk over the support of a sample (as psf_walk_fwd, FP32, with its ROW
// and XT): the PSF sums
// relative to the centre voxel's value X_b (A' = sum g_hat (X - X_b),
// Z = sum g_hat, so y_hat = X_b + A'/Z) and the nine offset moments of
// e^{-Q/2} (X - X_b) and of e^{-Q/2} (first moments a, b, c, then the second
// moments aa, ab, ac, bb, bc, cc).  The moments of the weights w_i follow as
// mx - (y_hat - X_b) me; the reference X_b keeps that difference accurate.
template <int ROW, bool XT>
__device__ __forceinline__ void psf_walk_grad(const GeoF &g, const ProbDev &p, const int b[3],
                                              const float f[3], __amdgpu_buffer_rsrc_t xr,
                                              unsigned nbytes, float &xb_out, float &a_out,
                                              float &z_out, float mx[9], float me[9]) {
  const int sx = XT ? p.ny : 1, sy = XT ? 1 : p.nx, sz = p.nx * p.ny;
  const int ia = g.perm[0], ib = g.perm[1], ic = g.perm[2];
  const int st_a = sel3(ia, sx, sy, sz), st_b = sel3(ib, sx, sy, sz), st_c = sel3(ic, sx, sy, sz);
  const int b_a = sel3(ia, b[0], b[1], b[2]), b_b = sel3(ib, b[0], b[1], b[2]),
            b_c = sel3(ic, b[0], b[1], b[2]);
  const int n_a = sel3(ia, p.nx, p.ny, p.nz), n_b = sel3(ib, p.nx, p.ny, p.nz),
            n_c = sel3(ic, p.nx, p.ny, p.nz);
  const float f_a = sel3f<float>(ia, f[0], f[1], f[2]), f_b = sel3f<float>(ib, f[0], f[1], f[2]),
              f_c = sel3f<float>(ic, f[0], f[1], f[2]);
  const float K2 = g.K2, cut = g.cut, Acc = g.Acc, Aca = g.Aca, Acb = g.Acb, Saa = g.Saa,
              Sab = g.Sab, Sbb = g.Sbb, iAaa = g.iAinv_aa, ha = g.ha, iAcc = g.inv_Acc,
              iSbb = g.inv_Sbb, nSab = g.nSab_Sbb;
  const int lo_a = max((int)ceil(f_a - ha), -b_a);
  const int hi_a = min((int)floor(f_a + ha), n_a - 1 - b_a);
  const int cl_b = -b_b, ch_b = n_b - 1 - b_b, cl_c = -b_c, ch_c = n_c - 1 - b_c;
  const int vb = b[0] * sx + b[1] * sy + b[2] * sz;
  const unsigned step = (unsigned)st_c * 4u;
  const float xb = load_vox<float>(xr, (unsigned)vb * 4u);
  float acc = 0.f, z = 0.f;
#pragma unroll
  for (int q = 0; q < 9; ++q) { mx[q] = 0.f; me[q] = 0.f; }
  for (int oa = lo_a; oa <= hi_a; ++oa) {
    const float wa = (float)oa - f_a;
    const float rem = K2 - wa * wa * iAaa;
    if (rem < 0.f) continue;
    const float wbc = nSab * wa;
    const float rb = fast_sqrt<float>(rem * iSbb);
    const int lo_b = max((int)ceil(f_b + wbc - rb), cl_b);
    const int hi_b = min((int)floor(f_b + wbc + rb), ch_b);
    const float qa = Saa * wa * wa;
    const float sa2 = 2.f * Sab * wa;
    for (int ob = lo_b; ob <= hi_b; ++ob) {
      const float wb = (float)ob - f_b;
      const float q1 = qa + wb * (sa2 + Sbb * wb);
      const float rem2 = K2 - q1;
      if (rem2 < 0.f) continue;
      const float wcc = -(Aca * wa + Acb * wb) * iAcc;
      const float rc = fast_sqrt<float>(rem2 * iAcc);
      const int lo_c = max((int)ceil(f_c + wcc - rc), cl_c);
      const int hi_c = min((int)floor(f_c + wcc + rc), ch_c);
      const int n = hi_c - lo_c + 1;
      float d = ((float)lo_c - f_c) - wcc;
      float wc = (float)lo_c - f_c;
      unsigned off = (unsigned)(vb + oa * st_a + ob * st_b + lo_c * st_c) * 4u;
      float r0x = 0.f, r1x = 0.f, r2x = 0.f, r0e = 0.f, r1e = 0.f, r2e = 0.f;
      for (int k0 = 0; k0 < n; k0 += 4) {
        float x[4];
        load_group<float, ROW>(xr, off, step, nbytes, x);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float Q = fma(Acc * d, d, q1);
          const float e2 = fast_exp2<float>(-Q);
          const float gh = k0 + k < n ? clamp01<float>(e2 - cut) : 0.f;
          const float em = gh > 0.f ? e2 : 0.f;
          const float xd = x[k] - xb;
          acc = fma(gh, xd, acc);
          z += gh;
          const float ex = em * xd;
          const float tx = ex * wc, te = em * wc;
          r0x += ex;
          r1x += tx;
          r2x = fma(tx, wc, r2x);
          r0e += em;
          r1e += te;
          r2e = fma(te, wc, r2e);
          d += 1.f;
          wc += 1.f;
        }
        off += 4 * step;
      }
      const float wab = wa * wb, waa = wa * wa, wbb = wb * wb;
      mx[0] = fma(wa, r0x, mx[0]);  me[0] = fma(wa, r0e, me[0]);
      mx[1] = fma(wb, r0x, mx[1]);  me[1] = fma(wb, r0e, me[1]);
      mx[2] += r1x;                 me[2] += r1e;
      mx[3] = fma(waa, r0x, mx[3]); me[3] = fma(waa, r0e, me[3]);
      mx[4] = fma(wab, r0x, mx[4]); me[4] = fma(wab, r0e, me[4]);
      mx[5] = fma(wa, r1x, mx[5]);  me[5] = fma(wa, r1e, me[5]);
      mx[6] = fma(wbb, r0x, mx[6]); me[6] = fma(wbb, r0e, me[6]);
      mx[7] = fma(wb, r1x, mx[7]);  me[7] = fma(wb, r1e, me[7]);
      mx[8] += r2x;                 me[8] += r2e;
    }
  }
  xb_out = xb;
  a_out = acc;
  z_out = z;
}

// The six derivative sums sum_i w_i d g_hat_i / d theta (rotations, then
// translations) from the nine moments m of the weights w_i (see GradMom).
__device__ __forceinline__ void grad_from_moments(const GradMom &gm, const float m[9],
                                                  const float q[3], float a6[6]) {
  // t = P n
  float t[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) t[r] = gm.P[3 * r] * m[0] + gm.P[3 * r + 1] * m[1] + gm.P[3 * r + 2] * m[2];
  const float S[9] = {m[3], m[4], m[5], m[4], m[6], m[7], m[5], m[7], m[8]};
  // T = S V^T: T[u][c] = sum_v S[u][v] V[c][v]
  float T[9];
#pragma unroll
  for (int u = 0; u < 3; ++u)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      T[3 * u + c] = S[3 * u] * gm.V[3 * c] + S[3 * u + 1] * gm.V[3 * c + 1] + S[3 * u + 2] * gm.V[3 * c + 2];
  // C = P T; only its antisymmetric part enters
  auto C = [&](int r, int c) {
    return gm.P[3 * r] * T[c] + gm.P[3 * r + 1] * T[3 + c] + gm.P[3 * r + 2] * T[6 + c];
  };
  const float c0 = C(1, 2) - C(2, 1) + (t[1] * q[2] - t[2] * q[1]);
  const float c1 = C(2, 0) - C(0, 2) + (t[2] * q[0] - t[0] * q[2]);
  const float c2 = C(0, 1) - C(1, 0) + (t[0] * q[1] - t[1] * q[0]);
#pragma unroll
  for (int k = 0; k < 3; ++k) a6[k] = -(gm.om[3 * k] * c0 + gm.om[3 * k + 1] * c1 + gm.om[3 * k + 2] * c2);
  a6[3] = t[0];
  a6[4] = t[1];
  a6[5] = t[2];
}

}  // namespace pvr
