// Edge-preserving SR volume update ("volume-volume"): one lane per voxel,
// Jacobi form (reads X, writes X_out), 26-neighbour diffusion regulariser.
#include <math.h>

#include "pvr_internal.h"
#include "pvr_util.h"

using namespace pvr;

__global__ void __launch_bounds__(256)
k_sr_update(const ProbDev *__restrict__ probs, int P, long long V, const float *__restrict__ X,
            const float *__restrict__ num, const float *__restrict__ den, pvr_sr_params prm,
            float *__restrict__ Xo) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= V) return;
  int lo = 0, hi = P - 1;  // problem holding gid
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].vol_off <= gid) lo = mid; else hi = mid - 1;
  }
  const ProbDev pr = probs[lo];
  const long long loc = gid - pr.vol_off;
  const int i = (int)(loc % pr.nx);
  const int j = (int)((loc / pr.nx) % pr.ny);
  const int k = (int)(loc / ((long long)pr.nx * pr.ny));
  const float x = X[gid];
  const float dn = den[gid];
  const float step = dn > prm.den_eps ? num[gid] / dn : 0.f;
  float R = 0.f;
  if (prm.lambda != 0.f) {
    const float inv_delta = 1.f / prm.delta;
    const float bw[4] = {0.f, 1.f, 0.70710678118654752f, 0.57735026918962576f};
    const long long sy = pr.nx, sz = (long long)pr.nx * pr.ny;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int nnz = (dx != 0) + (dy != 0) + (dz != 0);
          if (nnz == 0) continue;
          const int ii = i + dx, jj = j + dy, kk = k + dz;
          if (ii < 0 || ii >= pr.nx || jj < 0 || jj >= pr.ny || kk < 0 || kk >= pr.nz) continue;
          const float D = X[gid + dx + dy * sy + dz * sz] - x;
          const float t = D * inv_delta;
          R = fmaf(bw[nnz] * D, 1.f / sqrtf(fmaf(t, t, 1.f)), R);
        }
      }
    }
  }
  float out = fmaf(prm.alpha, step, x);
  out = fmaf(prm.alpha * prm.lambda, R, out);
  if (prm.use_clamp) out = fmaxf(out, prm.clamp_min);
  Xo[gid] = out;
}

extern "C" pvr_status pvr_sr_update(const pvr_plan *p, const float *X, const float *num,
                                    const float *den, const pvr_sr_params *prm, float *X_out,
                                    hipStream_t stream) {
  PVR_API_BEGIN();
  if (!p || !X || !num || !den || !prm || !X_out) return fail(PVR_EINVAL, "pvr_sr_update: NULL argument");
  if (X_out == X) return fail(PVR_EINVAL, "pvr_sr_update: X_out must not alias X");
  if (!(prm->delta > 0)) return fail(PVR_EINVAL, "pvr_sr_update: delta must be > 0");
  const long long V = p->V;
  const long long blocks = (V + 255) / 256;
  hipLaunchKernelGGL(k_sr_update, dim3((unsigned)blocks), dim3(256), 0, stream, p->d_prob, p->P, V,
                     X, num, den, *prm, X_out);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}
