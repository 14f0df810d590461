// Derivative of the forward model with respect to the per-patch motion:
//   grad_theta_s = sum_{j in s} g_j d y_hat_j / d theta_s.
//
// y_hat_j = sum_i g_hat_ji X_i / Z_j with Z_j = sum_i g_hat_ji, so
//   d y_hat_j / d theta = sum_i (X_i - y_hat_j) d g_hat_ji / d theta / Z_j.
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
//
// One workgroup per patch; two walks per sample (y_hat, then the derivative
// sums); FP64 accumulation of the six per-patch sums.
#include <math.h>

#include "pvr_geometry.h"
#include "pvr_internal.h"
#include "pvr_util.h"

using namespace pvr;

constexpr int GR_THREADS = 256;

struct GradConst {
  double M[9];      // F diag(1/sigma^2) F^T (world, mm^-2)
  double om[9];     // omega_x, omega_y, omega_z as rows
  double Vl[9];     // vox2world linear part
  double ct[3];     // c + t (world)
  double v2w_o[3];  // vox2world offset
};

__device__ void make_grad_const(const ProbDev &pr, const StackDev &st, const PatchDev &pt,
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
    T z = 0, acc = 0;
    psf_walk<T, typename GeoOf<T>::type, true>(g, pr, b, f, Xp, z, acc);
    const T yh = acc * iz;
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
    grad_walk<T>(g, pr, gc, b, f, qt, Xp, yh, a6);
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
  if (!p) return fail(PVR_EINVAL, "pvr_simulate_grad_theta: plan is NULL");
  if (!p->built) return fail(PVR_EINVAL, "pvr_simulate_grad_theta: plan has not been built");
  return grad_impl<float>(p, X, gy, grad_theta, p->d_invz, stream);
  PVR_API_END();
}

extern "C" pvr_status pvr_simulate_grad_theta_f64(const pvr_plan *p, const double *X,
                                                  const double *gy, double *grad_theta,
                                                  hipStream_t stream) {
  PVR_API_BEGIN();
  if (!p) return fail(PVR_EINVAL, "pvr_simulate_grad_theta_f64: plan is NULL");
  if (!p->built || !p->built64)
    return fail(PVR_EINVAL, "pvr_simulate_grad_theta_f64: plan needs pvr_plan_build_f64");
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
  if (!p || !y_obs || !y_sim) return fail(PVR_EINVAL, "pvr_ncc_grad: NULL argument");
  if (!p->built) return fail(PVR_EINVAL, "pvr_ncc_grad: plan has not been built");
  hipLaunchKernelGGL(k_ncc_grad, dim3(p->M), dim3(GR_THREADS), 0, stream, p->d_patch, p->d_invz,
                     y_obs, y_sim, grad_y, ncc);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}
