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

}  // namespace pvr
