// Edge-preserving SR volume update ("volume-volume"): one lane per voxel,
// Jacobi form (reads X, writes X_out), 26-neighbour diffusion regulariser.
#include <math.h>

#include "pvr_internal.h"
#include "pvr_util.h"

using namespace pvr;

// One workgroup = a 64 x 4 tile of one z-plane of one problem (grid
// x = tiles over x, y = tiles over y, z = planes of all problems stacked).
// A neighbour outside the grid (whose term the Neumann border drops) is not
// branched around: its load reads the centre voxel instead, so its
// difference D is exactly 0 and so is its term, and every load stays inside
// the problem's volume.  1/sqrt uses the hardware reciprocal square root
// (about 1 ulp).
__global__ void __launch_bounds__(256)
k_sr_update(const ProbDev *__restrict__ probs, const int *__restrict__ plane_prob,
            const float *__restrict__ X, const float *__restrict__ num,
            const float *__restrict__ den, pvr_sr_params prm, float *__restrict__ Xo,
            unsigned *__restrict__ status) {
  const int zg = blockIdx.z;
  const ProbDev pr = probs[plane_prob[zg]];
  const int k = zg - plane_prob[gridDim.z + plane_prob[zg]];
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= pr.nx || j >= pr.ny) return;
  const int sy = pr.nx, sz = pr.nx * pr.ny;
  const int c = k * sz + j * sy + i;
  const float *Xp = X + pr.vol_off;
  const float x = Xp[c];
  const float dn = den[pr.vol_off + c];
  const float step = dn > prm.den_eps ? num[pr.vol_off + c] / dn : 0.f;
  float R = 0.f;
  if (prm.lambda != 0.f) {
    const __amdgpu_buffer_rsrc_t xr = raw_buffer(Xp, (unsigned)(sz * pr.nz) * (unsigned)sizeof(float));
    const float inv_delta = 1.f / prm.delta;
    const float bw[4] = {0.f, 1.f, 0.70710678118654752f, 0.57735026918962576f};
    const bool okx[3] = {i > 0, true, i < pr.nx - 1};
    const bool oky[3] = {j > 0, true, j < pr.ny - 1};
    const bool okz[3] = {k > 0, true, k < pr.nz - 1};
    const int vo = c * (int)sizeof(float);
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int nnz = (dx != 0) + (dy != 0) + (dz != 0);
          if (nnz == 0) continue;
          const bool ok = okx[dx + 1] & oky[dy + 1] & okz[dz + 1];
          const int so = (dx + dy * sy + dz * sz) * (int)sizeof(float);
          const float v = __builtin_bit_cast(
              float, __builtin_amdgcn_raw_buffer_load_b32(xr, ok ? vo + so : vo, 0, 0));
          const float D = v - x;
          const float t = D * inv_delta;
          R = fmaf(bw[nnz] * D, __builtin_amdgcn_rsqf(fmaf(t, t, 1.f)), R);
        }
      }
    }
  }
  float out = fmaf(prm.alpha, step, x);
  out = fmaf(prm.alpha * prm.lambda, R, out);
  // a non-finite value before the clamp (which would hide a NaN) raises the
  // volume flag once per wave
  const unsigned long long bad = __ballot(!__builtin_isfinite(out));
  if (bad && (threadIdx.x & 63) == (unsigned)__builtin_ctzll(bad)) atomicOr(status, PVR_FAULT_VOLUME);
  if (prm.use_clamp) out = fmaxf(out, prm.clamp_min);
  Xo[pr.vol_off + c] = out;
}

extern "C" pvr_status pvr_sr_update(const pvr_plan *p, const float *X, const float *num,
                                    const float *den, const pvr_sr_params *prm, float *X_out,
                                    hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_sr_update", X, 4);
  PVR_ALIGNED("pvr_sr_update", num, 4);
  PVR_ALIGNED("pvr_sr_update", den, 4);
  PVR_ALIGNED("pvr_sr_update", X_out, 4);
  if (!p || !X || !num || !den || !prm || !X_out) return fail(PVR_EINVAL, "pvr_sr_update: NULL argument");
  if (X_out == X) return fail(PVR_EINVAL, "pvr_sr_update: X_out must not alias X");
  if (!p->attached) return fail(PVR_EINVAL, "pvr_sr_update: no workspace attached (pvr_plan_attach)");
  if (!(prm->delta > 0)) return fail(PVR_EINVAL, "pvr_sr_update: delta must be > 0");
  PVR_TRY_STATUS(debug_finite(p, "pvr_sr_update", "X", X, p->V, stream));
  PVR_TRY_STATUS(debug_finite(p, "pvr_sr_update", "num", num, p->V, stream));
  PVR_TRY_STATUS(debug_finite(p, "pvr_sr_update", "den", den, p->V, stream));
  hipLaunchKernelGGL(k_sr_update, dim3((p->max_nx + 63) / 64, (p->max_ny + 3) / 4, p->n_planes),
                     dim3(256), 0, stream, p->d_prob, p->d_plane_prob, X, num, den, *prm, X_out,
                     p->d_status);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}
