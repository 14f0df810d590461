// Plan creation and the motion-dependent build: per-patch geometry, per-sample
// PSF normalisers and the brick -> patch index of the gather adjoint.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "pvr_internal.h"
#include "pvr_util.h"
#include "pvr_geometry.h"

using namespace pvr;

__global__ void k_theta_to_f64(const float *__restrict__ th, double *__restrict__ out, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)th[i];
}

__global__ void k_copy_theta(const double *__restrict__ th, double *__restrict__ out, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = th[i];
}

__global__ void k_geometry(const ProbDev *__restrict__ probs, const StackDev *__restrict__ stacks,
                           const PatchDev *__restrict__ patches, const double *__restrict__ theta,
                           int M, double k, GeoD *__restrict__ gd, GeoF *__restrict__ gf,
                           int *__restrict__ bb) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= M) return;
  const PatchDev pt = patches[s];
  GeoD g;
  GeoF f;
  make_geometry(probs[pt.problem], stacks[pt.stack], pt, theta + 6 * s, k, g, f, bb + 6 * s);
  gd[s] = g;
  gf[s] = f;
}

// Per-sample inverse normaliser 1/Z_j (0 marks an invalid sample).
template <typename T>
__global__ void __launch_bounds__(SIM_THREADS)
k_normalisers(const ProbDev *__restrict__ probs, const PatchDev *__restrict__ patches,
              const BlockWork *__restrict__ work, const typename GeoOf<T>::type *__restrict__ geo,
              const uint8_t *__restrict__ mask, const uint8_t *__restrict__ active,
              float *__restrict__ invz, double *__restrict__ invz64) {
  const BlockWork wk = work[blockIdx.x];
  const PatchDev pt = patches[wk.patch];
  const ProbDev pr = probs[pt.problem];
  const typename GeoOf<T>::type &g = geo[wk.patch];
  const int n = pt.w * pt.h;
  const int l1 = min(n, wk.l0 + SIM_CHUNK);
  const bool act = active ? active[wk.patch] != 0 : true;
  for (int l = wk.l0 + threadIdx.x; l < l1; l += SIM_THREADS) {
    const long long j = pt.off + l;
    const int u = pt.x0 + l % pt.w, v = pt.y0 + l / pt.w;
    int b[3];
    T f[3];
    bool ok = sample_centre(g, pr, u, v, pt.slice, b, f) && act && (!mask || mask[j]);
    T z = 0, acc = 0;
    if (ok) psf_walk<T, typename GeoOf<T>::type, false>(g, pr, b, f, nullptr, z, acc);
    ok = ok && z > (T)0;
    const T iz = ok ? (T)1 / z : (T)0;
    invz[j] = (float)iz;
    if (invz64) invz64[j] = (double)iz;
  }
}

// brick -> patch index: count, scan, fill.  Every brick scans the patches of
// its problem in order, so each list is sorted by patch (deterministic).
__global__ void k_bin_count(const ProbDev *__restrict__ probs, const int *__restrict__ brick_prob,
                            const int *__restrict__ bb, int nb, int *__restrict__ count) {
  int bi = blockIdx.x * blockDim.x + threadIdx.x;
  if (bi >= nb) return;
  const ProbDev pr = probs[brick_prob[bi]];
  const int local = bi - pr.brick_base;
  const int bx = local % pr.nbx, by = (local / pr.nbx) % pr.nby, bz = local / (pr.nbx * pr.nby);
  int c = 0;
  for (int s = pr.patch_begin; s < pr.patch_end; ++s) {
    const int *r = bb + 6 * s;
    c += (bx >= r[0]) & (bx <= r[3]) & (by >= r[1]) & (by <= r[4]) & (bz >= r[2]) & (bz <= r[5]);
  }
  count[bi] = c;
}

__global__ void k_bin_fill(const ProbDev *__restrict__ probs, const int *__restrict__ brick_prob,
                           const int *__restrict__ bb, int nb, const int *__restrict__ off,
                           int *__restrict__ list) {
  int bi = blockIdx.x * blockDim.x + threadIdx.x;
  if (bi >= nb) return;
  const ProbDev pr = probs[brick_prob[bi]];
  const int local = bi - pr.brick_base;
  const int bx = local % pr.nbx, by = (local / pr.nbx) % pr.nby, bz = local / (pr.nbx * pr.nby);
  int c = off[bi];
  for (int s = pr.patch_begin; s < pr.patch_end; ++s) {
    const int *r = bb + 6 * s;
    if ((bx >= r[0]) & (bx <= r[3]) & (by >= r[1]) & (by <= r[4]) & (bz >= r[2]) & (bz <= r[5]))
      list[c++] = s;
  }
}

// Exclusive scan of count[0..n) into off[0..n], off[n] = total, by one
// workgroup of 1024 threads (each owns a contiguous run).
__global__ void __launch_bounds__(1024) k_scan(const int *__restrict__ count, int n,
                                               int *__restrict__ off, int *__restrict__ total) {
  __shared__ long long lds[1024];
  const int tid = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int a = min(n, tid * per), b = min(n, a + per);
  long long s = 0;
  for (int i = a; i < b; ++i) s += count[i];
  lds[tid] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    long long v = tid >= d ? lds[tid - d] : 0;
    __syncthreads();
    lds[tid] += v;
    __syncthreads();
  }
  long long run = lds[tid] - s;
  for (int i = a; i < b; ++i) {
    off[i] = (int)run;
    run += count[i];
  }
  if (tid == 1023) {
    off[n] = (int)lds[1023];
    total[0] = (int)min(lds[1023], (long long)0x7fffffff);
  }
}

// ---------------------------------------------------------------------------
// host API
// ---------------------------------------------------------------------------
static void host_mat3_from_aff(const double *a, double *L) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) L[3 * r + c] = a[4 * r + c];
}

extern "C" pvr_status pvr_plan_create(const pvr_grid *grids, int32_t n_problems,
                                      const pvr_stack *stacks, int32_t n_stacks,
                                      const pvr_patch *patches, int32_t n_patches,
                                      double cutoff_k, pvr_plan **out) {
  PVR_API_BEGIN();
  if (!out) return fail(PVR_EINVAL, "pvr_plan_create: out is NULL");
  *out = nullptr;
  if (!grids || !stacks || !patches) return fail(PVR_EINVAL, "pvr_plan_create: NULL descriptor array");
  if (n_problems <= 0 || n_stacks <= 0 || n_patches <= 0)
    return fail(PVR_ESHAPE, "pvr_plan_create: empty problem / stack / patch set");
  if (!(cutoff_k > 0 && cutoff_k < 20)) return fail(PVR_EINVAL, "pvr_plan_create: cutoff_k out of (0, 20)");
  pvr_plan *p = (pvr_plan *)calloc(1, sizeof(pvr_plan));
  PlanGuard guard(p);
  p->P = n_problems; p->S = n_stacks; p->M = n_patches; p->k = cutoff_k;
  p->h_prob = (ProbDev *)calloc(n_problems, sizeof(ProbDev));
  p->h_stack = (StackDev *)calloc(n_stacks, sizeof(StackDev));
  p->h_patch = (PatchDev *)calloc(n_patches, sizeof(PatchDev));
  p->h_sample_off = (long long *)calloc(n_patches + 1, sizeof(long long));
  p->h_vol_off = (long long *)calloc(n_problems + 1, sizeof(long long));
  // problems
  long long vo = 0;
  int nbr = 0;
  for (int b = 0; b < n_problems; ++b) {
    const pvr_grid &g = grids[b];
    if (g.nx <= 0 || g.ny <= 0 || g.nz <= 0) return fail(PVR_ESHAPE, "pvr_plan_create: grid %d has an empty size", b);
    ProbDev &d = p->h_prob[b];
    d.nx = g.nx; d.ny = g.ny; d.nz = g.nz;
    d.nbx = (g.nx + BRICK - 1) / BRICK; d.nby = (g.ny + BRICK - 1) / BRICK; d.nbz = (g.nz + BRICK - 1) / BRICK;
    d.brick_base = nbr;
    d.n_bricks = d.nbx * d.nby * d.nbz;
    nbr += d.n_bricks;
    d.vol_off = vo;
    p->h_vol_off[b] = vo;
    vo += (long long)g.nx * g.ny * g.nz;
    memcpy(d.v2w, g.vox2world, sizeof(d.v2w));
    double L[9], Li[9];
    host_mat3_from_aff(g.vox2world, L);
    double det = mat3_inv(L, Li);
    if (!(fabs(det) > 1e-12)) return fail(PVR_ESHAPE, "pvr_plan_create: grid %d vox2world is singular", b);
    aff_inv(g.vox2world, d.w2v);
  }
  p->h_vol_off[n_problems] = vo;
  p->V = vo;
  p->n_bricks = nbr;
  // stacks
  for (int s = 0; s < n_stacks; ++s) {
    const pvr_stack &st = stacks[s];
    if (st.problem < 0 || st.problem >= n_problems) return fail(PVR_EINVAL, "pvr_plan_create: stack %d names problem %d", s, st.problem);
    if (st.nx <= 0 || st.ny <= 0 || st.nslices <= 0) return fail(PVR_ESHAPE, "pvr_plan_create: stack %d has an empty size", s);
    StackDev &d = p->h_stack[s];
    d.problem = st.problem; d.nx = st.nx; d.ny = st.ny; d.ns = st.nslices;
    memcpy(d.p2w, st.pix2world, sizeof(d.p2w));
    double L[9];
    host_mat3_from_aff(st.pix2world, L);
    for (int a = 0; a < 3; ++a) {
      double n = sqrt(L[a] * L[a] + L[3 + a] * L[3 + a] + L[6 + a] * L[6 + a]);
      if (!(n > 0)) return fail(PVR_ESHAPE, "pvr_plan_create: stack %d axis %d has zero length", s, a);
      d.spacing[a] = n;
      for (int r = 0; r < 3; ++r) d.E[3 * r + a] = L[3 * r + a] / n;
      if (!(st.fwhm_mm[a] > 0)) return fail(PVR_EINVAL, "pvr_plan_create: stack %d fwhm[%d] <= 0", s, a);
      d.sigma[a] = st.fwhm_mm[a] / (2.0 * sqrt(2.0 * log(2.0)));
    }
    for (int a = 0; a < 3; ++a)
      for (int c = a + 1; c < 3; ++c) {
        double dt = d.E[a] * d.E[c] + d.E[3 + a] * d.E[3 + c] + d.E[6 + a] * d.E[6 + c];
        if (fabs(dt) > 1e-9) return fail(PVR_ESHAPE, "pvr_plan_create: stack %d axes %d and %d are not orthogonal", s, a, c);
      }
  }
  // patches: grouped by problem in problem order, each inside its slice
  long long so = 0;
  int prev_prob = 0;
  std::vector<BlockWork> blocks;
  std::vector<int> pcount(n_problems, 0);
  std::vector<long long> scount(n_problems, 0);
  for (int s = 0; s < n_patches; ++s) {
    const pvr_patch &q = patches[s];
    if (q.stack < 0 || q.stack >= n_stacks) return fail(PVR_EINVAL, "pvr_plan_create: patch %d names stack %d", s, q.stack);
    const StackDev &st = p->h_stack[q.stack];
    if (q.w <= 0 || q.h <= 0 || q.x0 < 0 || q.y0 < 0 || q.x0 + q.w > st.nx || q.y0 + q.h > st.ny ||
        q.slice < 0 || q.slice >= st.ns)
      return fail(PVR_ESHAPE, "pvr_plan_create: patch %d does not fit its slice", s);
    const int prob = st.problem;
    if (prob < prev_prob) return fail(PVR_EINVAL, "pvr_plan_create: patches must be ordered by problem (patch %d)", s);
    prev_prob = prob;
    PatchDev &d = p->h_patch[s];
    d.stack = q.stack; d.slice = q.slice; d.x0 = q.x0; d.y0 = q.y0; d.w = q.w; d.h = q.h;
    d.problem = prob; d.off = so;
    p->h_sample_off[s] = so;
    const int n = q.w * q.h;
    for (int l0 = 0; l0 < n; l0 += SIM_CHUNK) blocks.push_back(BlockWork{s, l0});
    so += n;
    pcount[prob] += 1;
    scount[prob] += n;
  }
  {
    int pb = 0;
    long long sb = 0;
    for (int b = 0; b < n_problems; ++b) {
      p->h_prob[b].patch_begin = pb; p->h_prob[b].patch_end = pb + pcount[b];
      p->h_prob[b].sample_begin = sb; p->h_prob[b].sample_end = sb + scount[b];
      pb += pcount[b];
      sb += scount[b];
    }
  }
  p->h_sample_off[n_patches] = so;
  p->N = so;
  if (so > 0x7fffffffLL * 4) return fail(PVR_ESHAPE, "pvr_plan_create: too many samples");
  p->n_sim_blocks = (int)blocks.size();
  std::vector<int> brick_prob(nbr);
  for (int b = 0; b < n_problems; ++b)
    for (int i = 0; i < p->h_prob[b].n_bricks; ++i) brick_prob[p->h_prob[b].brick_base + i] = b;
  // device buffers (all host-side validation is done above)
  HIP_TRY(hipGetDevice(&p->device));
  DEV_ALLOC(p, p->d_prob, n_problems);
  DEV_ALLOC(p, p->d_stack, n_stacks);
  DEV_ALLOC(p, p->d_patch, n_patches);
  DEV_ALLOC(p, p->d_sim_blocks, p->n_sim_blocks);
  DEV_ALLOC(p, p->d_brick_prob, nbr);
  DEV_ALLOC(p, p->d_theta, 6 * (size_t)n_patches);
  DEV_ALLOC(p, p->d_geod, n_patches);
  DEV_ALLOC(p, p->d_geof, n_patches);
  DEV_ALLOC(p, p->d_bb, 6 * (size_t)n_patches);
  DEV_ALLOC(p, p->d_invz, p->N);
  DEV_ALLOC(p, p->d_mask, p->N);
  DEV_ALLOC(p, p->d_active, n_patches);
  DEV_ALLOC(p, p->d_bin_count, nbr);
  DEV_ALLOC(p, p->d_bin_off, nbr + 1);
  DEV_ALLOC(p, p->d_rq, p->N);
  DEV_ALLOC(p, p->d_pstat, 10 * (size_t)n_patches);
  DEV_ALLOC(p, p->d_resp, n_patches);
  DEV_ALLOC(p, p->d_pbar, n_patches);
  DEV_ALLOC(p, p->d_total, 4);
  HIP_TRY(hipHostMalloc((void **)&p->h_total, sizeof(int) * 4, hipHostMallocDefault));
  HIP_TRY(hipMemcpy(p->d_prob, p->h_prob, sizeof(ProbDev) * n_problems, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->d_stack, p->h_stack, sizeof(StackDev) * n_stacks, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->d_patch, p->h_patch, sizeof(PatchDev) * n_patches, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->d_sim_blocks, blocks.data(), sizeof(BlockWork) * blocks.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->d_brick_prob, brick_prob.data(), sizeof(int) * nbr, hipMemcpyHostToDevice));
  HIP_TRY(hipDeviceSynchronize());
  guard.release();
  *out = p;
  return PVR_OK;
  PVR_API_END();
}

extern "C" void pvr_plan_destroy(pvr_plan *p) {
  if (!p) return;
  plan_free(p);
}

extern "C" pvr_status pvr_plan_info(const pvr_plan *p, pvr_plan_sizes *out) {
  PVR_API_BEGIN();
  if (!p || !out) return fail(PVR_EINVAL, "pvr_plan_info: NULL argument");
  out->n_samples = p->N;
  out->n_voxels = p->V;
  out->n_patches = p->M;
  out->n_problems = p->P;
  out->n_stacks = p->S;
  out->n_bricks = p->n_bricks;
  out->n_bin_pairs = p->n_pairs;
  out->device_bytes = p->device_bytes;
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_plan_offsets(const pvr_plan *p, int64_t *sample_off, int64_t *vol_off) {
  PVR_API_BEGIN();
  if (!p) return fail(PVR_EINVAL, "pvr_plan_offsets: plan is NULL");
  if (sample_off) for (int s = 0; s <= p->M; ++s) sample_off[s] = p->h_sample_off[s];
  if (vol_off) for (int b = 0; b <= p->P; ++b) vol_off[b] = p->h_vol_off[b];
  return PVR_OK;
  PVR_API_END();
}

extern "C" const float *pvr_plan_inv_z(const pvr_plan *p) { return p ? p->d_invz : nullptr; }

static pvr_status plan_build_common(pvr_plan *p, const uint8_t *active, const uint8_t *mask,
                                    bool f64, hipStream_t stream) {
  const int M = p->M;
  const int T = 256;
  if (active) {
    HIP_TRY(hipMemcpyAsync(p->d_active, active, M, hipMemcpyDeviceToDevice, stream));
  } else {
    launch_fill_u8(p->d_active, 1, M, stream);
  }
  if (mask) {
    HIP_TRY(hipMemcpyAsync(p->d_mask, mask, p->N, hipMemcpyDeviceToDevice, stream));
  } else {
    launch_fill_u8(p->d_mask, 1, p->N, stream);
  }
  hipLaunchKernelGGL(k_geometry, dim3((M + T - 1) / T), dim3(T), 0, stream, p->d_prob, p->d_stack,
                     p->d_patch, p->d_theta, M, p->k, p->d_geod, p->d_geof, p->d_bb);
  HIP_TRY(hipGetLastError());
  if (f64) {
    if (!p->d_invz64) DEV_ALLOC(p, p->d_invz64, p->N);
    hipLaunchKernelGGL(k_normalisers<double>, dim3(p->n_sim_blocks), dim3(SIM_THREADS), 0, stream,
                       p->d_prob, p->d_patch, p->d_sim_blocks, p->d_geod, p->d_mask, p->d_active,
                       p->d_invz, p->d_invz64);
  } else {
    hipLaunchKernelGGL(k_normalisers<float>, dim3(p->n_sim_blocks), dim3(SIM_THREADS), 0, stream,
                       p->d_prob, p->d_patch, p->d_sim_blocks, p->d_geof, p->d_mask, p->d_active,
                       p->d_invz, (double *)nullptr);
  }
  HIP_TRY(hipGetLastError());
  const int nb = p->n_bricks;
  hipLaunchKernelGGL(k_bin_count, dim3((nb + T - 1) / T), dim3(T), 0, stream, p->d_prob,
                     p->d_brick_prob, p->d_bb, nb, p->d_bin_count);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, stream, p->d_bin_count, nb, p->d_bin_off,
                     p->d_total);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(p->h_total, p->d_total, sizeof(int), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  const long long pairs = p->h_total[0];
  if (pairs >= 0x7fffffffLL) return fail(PVR_ESHAPE, "pvr_plan_build: brick index exceeds 2^31 pairs");
  if (pairs > p->bin_cap) {
    if (p->d_bin_patch) { HIP_TRY(hipFree(p->d_bin_patch)); p->device_bytes -= p->bin_cap * 4; }
    p->d_bin_patch = nullptr;
    long long cap = pairs + pairs / 8 + 1024;
    DEV_ALLOC(p, p->d_bin_patch, cap);
    p->bin_cap = cap;
  }
  p->n_pairs = pairs;
  hipLaunchKernelGGL(k_bin_fill, dim3((nb + T - 1) / T), dim3(T), 0, stream, p->d_prob,
                     p->d_brick_prob, p->d_bb, nb, p->d_bin_off, p->d_bin_patch);
  HIP_TRY(hipGetLastError());
  p->built = true;
  p->built64 = f64;
  return PVR_OK;
}

extern "C" pvr_status pvr_plan_build(pvr_plan *p, const float *theta, const uint8_t *active,
                                     const uint8_t *sample_mask, hipStream_t stream) {
  PVR_API_BEGIN();
  if (!p || !theta) return fail(PVR_EINVAL, "pvr_plan_build: NULL plan or theta");
  const int n = 6 * p->M;
  hipLaunchKernelGGL(k_theta_to_f64, dim3((n + 255) / 256), dim3(256), 0, stream, theta, p->d_theta, n);
  HIP_TRY(hipGetLastError());
  return plan_build_common(p, active, sample_mask, false, stream);
  PVR_API_END();
}

extern "C" pvr_status pvr_plan_build_f64(pvr_plan *p, const double *theta, const uint8_t *active,
                                         const uint8_t *sample_mask, hipStream_t stream) {
  PVR_API_BEGIN();
  if (!p || !theta) return fail(PVR_EINVAL, "pvr_plan_build_f64: NULL plan or theta");
  const int n = 6 * p->M;
  hipLaunchKernelGGL(k_copy_theta, dim3((n + 255) / 256), dim3(256), 0, stream, theta, p->d_theta, n);
  HIP_TRY(hipGetLastError());
  return plan_build_common(p, active, sample_mask, true, stream);
  PVR_API_END();
}
