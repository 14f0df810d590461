// Forward direction ("volume-pixel"): PSF-weighted simulation of moved patch
// samples, and the per-patch NCC registration built on the same PSF walk.
//
// One workgroup (256 lanes = 4 waves) covers a chunk of up to 1024 samples of
// one patch, so the patch's geometry is uniform across the workgroup; lanes
// take consecutive pixels of a patch row, whose supports are near-identical
// shapes shifted by one pixel, so the volume reads of a wave coalesce along
// the row direction.
#include <math.h>

#include "pvr_geometry.h"
#include "pvr_grad.h"
#include "pvr_internal.h"
#include "pvr_util.h"

using namespace pvr;

// With resid and chunk_stats, the workgroup also reduces its chunk's
// residual statistics over valid samples -- min e, max e, max |y|, sum e^2
// and the count (FP64, fixed order) -- into chunk_stats[5 * chunk], which the
// robust weights then read instead of passing over e once more.
template <typename T>
__global__ void __launch_bounds__(SIM_THREADS)
k_simulate(const ProbDev *__restrict__ probs, const PatchDev *__restrict__ patches,
           const BlockWork *__restrict__ work, const typename GeoOf<T>::type *__restrict__ geo,
           const T *__restrict__ invz, const T *__restrict__ X, const T *__restrict__ XT,
           const T *__restrict__ y_obs, T *__restrict__ y_sim, T *__restrict__ resid,
           double *__restrict__ chunk_stats, int n_work, int granule) {
  const int wi = xcd_work(blockIdx.x, granule);
  if (wi >= n_work) return;
  const BlockWork wk = work[wi];
  const PatchDev pt = patches[wk.patch];
  const ProbDev pr = probs[pt.problem];
  const typename GeoOf<T>::type &g = geo[wk.patch];
  const unsigned nbytes = (unsigned)(pr.nx * pr.ny * pr.nz) * (unsigned)sizeof(T);
  // patches whose rows run along y read the y-fastest copy, so that the lanes
  // of a wave (consecutive pixels of a row) read consecutive addresses
  const bool sinc = g.psf == PVR_PSF_SINC;
  const bool xt = XT != nullptr && pt.layout == 1;
  const __amdgpu_buffer_rsrc_t xr = raw_buffer((xt ? XT : X) + pr.vol_off, nbytes);
  const int n = pt.w * pt.h;
  const int l1 = min(n, wk.l0 + SIM_CHUNK);
  double st[5] = {INFINITY, -INFINITY, 0.0, 0.0, 0.0};  // min e, max e, max|y|, sum e^2, count
  for (int l = wk.l0 + threadIdx.x; l < l1; l += SIM_THREADS) {
    const long long j = pt.off + l;
    const T iz = invz[j];
    T yh = (T)0;
    if (iz > (T)0) {
      const int u = pt.x0 + l % pt.w, v = pt.y0 + l / pt.w;
      int b[3];
      T f[3];
      sample_centre(g, pr, u, v, pt.slice, b, f);
      // the layout, and whether the walk's inner axis is the layout's fastest
      // one, are uniform over the chunk: one branch per chunk picks the walk
      using G = typename GeoOf<T>::type;
      if (sinc) {
        T z;
        if (xt)
          yh = (g.perm[2] == 1 ? psf_walk_sinc<T, G, true, 1, true>(g, pr, b, f, xr, nbytes, &z)
                               : psf_walk_sinc<T, G, true, 2, true>(g, pr, b, f, xr, nbytes, &z)) * iz;
        else
          yh = (g.perm[2] == 0 ? psf_walk_sinc<T, G, true, 1>(g, pr, b, f, xr, nbytes, &z)
                               : psf_walk_sinc<T, G, true, 2>(g, pr, b, f, xr, nbytes, &z)) * iz;
      } else if (xt)
        yh = (g.perm[2] == 1 ? psf_walk_fwd<T, G, false, 1, true>(g, pr, b, f, xr, nbytes)
                             : psf_walk_fwd<T, G, false, 2, true>(g, pr, b, f, xr, nbytes)) * iz;
      else
        yh = (g.perm[2] == 0 ? psf_walk_fwd<T, G, false, 1>(g, pr, b, f, xr, nbytes)
                             : psf_walk_fwd<T, G, false, 2>(g, pr, b, f, xr, nbytes)) * iz;
    }
    if (y_sim) y_sim[j] = yh;
    if (resid) {
      const T e = iz > (T)0 ? y_obs[j] - yh : (T)0;
      resid[j] = e;
      if (chunk_stats && iz > (T)0) {
        const double ev = (double)e;
        st[0] = fmin(st[0], ev);
        st[1] = fmax(st[1], ev);
        st[2] = fmax(st[2], fabs((double)y_obs[j]));
        st[3] += ev * ev;
        st[4] += 1.0;
      }
    }
  }
  if (chunk_stats) {
    __shared__ double red[5][SIM_THREADS / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      st[0] = fmin(st[0], __shfl_xor(st[0], o, 64));
      st[1] = fmax(st[1], __shfl_xor(st[1], o, 64));
      st[2] = fmax(st[2], __shfl_xor(st[2], o, 64));
      st[3] += __shfl_xor(st[3], o, 64);
      st[4] += __shfl_xor(st[4], o, 64);
    }
    if (lane == 0)
      for (int k = 0; k < 5; ++k) red[k][wave] = st[k];
    __syncthreads();
    if (threadIdx.x == 0) {
      double r[5] = {red[0][0], red[1][0], red[2][0], red[3][0], red[4][0]};
      for (int w = 1; w < SIM_THREADS / 64; ++w) {
        r[0] = fmin(r[0], red[0][w]);
        r[1] = fmax(r[1], red[1][w]);
        r[2] = fmax(r[2], red[2][w]);
        r[3] += red[3][w];
        r[4] += red[4][w];
      }
      for (int k = 0; k < 5; ++k) chunk_stats[5 * (long long)wi + k] = r[k];
    }
  }
}

// LDS-staged forward pass: one workgroup per 16x16 tile of a patch.  The
// workgroup copies the voxel box of the tile's supports into LDS with row-
// contiguous (coalesced) loads, then every lane walks its sample's support in
// LDS.  Tiles whose box exceeds the reserved LDS walk the volume in global
// memory instead.  Tiles are dealt to the XCDs in granules of neighbouring
// tiles (xcd_work), keeping overlapping tiles in the same L2.
__global__ void __launch_bounds__(SIM_THREADS)
k_simulate_tiles(const ProbDev *__restrict__ probs, const PatchDev *__restrict__ patches,
                 const int *__restrict__ tile_off, int M, int tile_w, int tile_h, int n_tiles,
                 const GeoF *__restrict__ geo, const float *__restrict__ invz,
                 const float *__restrict__ X, const float *__restrict__ y_obs,
                 float *__restrict__ y_sim, float *__restrict__ resid, int lds_cap, int granule) {
  extern __shared__ float xs[];
  const int t = xcd_work(blockIdx.x, granule);
  if (t >= n_tiles) return;
  const TileWork tw = tile_at(tile_off, M, patches, tile_w, tile_h, t);
  const PatchDev pt = patches[tw.patch];
  const ProbDev pr = probs[pt.problem];
  const GeoF &g = geo[tw.patch];
  const float *Xp = X + pr.vol_off;
  int lo[3], hi[3];
  const int cnt = tile_box(g, pr, pt, tw, lo, hi);
  const bool staged = cnt > 0 && cnt <= lds_cap;
  const int dx = hi[0] - lo[0] + 1, dy = hi[1] - lo[1] + 1;
  if (staged) {
    // the box as one flat index range: consecutive lanes take consecutive x
    // of a row and continue into the next row, so no lane idles on short rows
    const float *src0 = Xp + ((long long)lo[2] * pr.ny + lo[1]) * pr.nx + lo[0];
    const long long zstride = (long long)pr.ny * pr.nx;
    for (int e = threadIdx.x; e < cnt; e += SIM_THREADS) {
      const int r = e / dx, x = e - r * dx;
      const int yy = r % dy, zz = r / dy;
      xs[e] = src0[zz * zstride + (long long)yy * pr.nx + x];
    }
    __syncthreads();
  }
  const int tid = threadIdx.x;
  if (tid >= tw.tw * tw.th) return;
  const int lu = tw.u0 + tid % tw.tw, lv = tw.v0 + tid / tw.tw;
  const long long j = pt.off + (long long)lv * pt.w + lu;
  const float iz = invz[j];
  float yh = 0.f;
  if (iz > 0.f) {
    int b[3];
    float f[3];
    sample_centre(g, pr, pt.x0 + lu, pt.y0 + lv, pt.slice, b, f);
    float z = 0.f, acc = 0.f;
    if (staged) {
      const float *Xb = xs + ((b[2] - lo[2]) * dy + (b[1] - lo[1])) * dx + (b[0] - lo[0]);
      psf_walk_s<float, GeoF, true>(g, lo, hi, b, f, Xb, dx, dx * dy, z, acc);
    } else {
      psf_walk<float, GeoF, true>(g, pr, b, f, Xp, z, acc);
    }
    yh = acc * iz;
  }
  if (y_sim) y_sim[j] = yh;
  if (resid) resid[j] = iz > 0.f ? y_obs[j] - yh : 0.f;
}

// y-fastest copy of every problem's volume: XT[(z nx + x) ny + y] =
// X[(z ny + y) nx + x], by 64 x 64 tiles through LDS (rows of both arrays
// read and written whole).
constexpr int XT_TILE = 64;
__global__ void __launch_bounds__(256) k_transpose_xy(const float *__restrict__ X,
                                                      float *__restrict__ XT, int nx, int ny) {
  __shared__ float t[XT_TILE][XT_TILE + 1];
  const int x0 = blockIdx.x * XT_TILE, y0 = blockIdx.y * XT_TILE;
  const long long zo = (long long)blockIdx.z * nx * ny;
  const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
  for (int r = r0; r < XT_TILE; r += 4) {
    const int x = x0 + c, y = y0 + r;
    if (x < nx && y < ny) t[r][c] = X[zo + (long long)y * nx + x];
  }
  __syncthreads();
  for (int r = r0; r < XT_TILE; r += 4) {
    const int y = y0 + c, x = x0 + r;
    if (x < nx && y < ny) XT[zo + (long long)x * ny + y] = t[c][r];
  }
}

// Fills p->d_xt from X when the plan has patches that read it; returns the
// copy (or nullptr).
static const float *volume_xt(const pvr_plan *p, const float *X, hipStream_t stream) {
  if (!p->any_xt) return nullptr;
  for (int b = 0; b < p->P; ++b) {
    const ProbDev &pr = p->h_prob[b];
    const dim3 grid((pr.nx + XT_TILE - 1) / XT_TILE, (pr.ny + XT_TILE - 1) / XT_TILE, pr.nz);
    hipLaunchKernelGGL(k_transpose_xy, grid, dim3(256), 0, stream, X + pr.vol_off,
                       p->d_xt + pr.vol_off, pr.nx, pr.ny);
  }
  return p->d_xt;
}

template <typename T>
static pvr_status simulate_impl(const pvr_plan *p, const T *X, const T *y_obs, T *y_sim, T *resid,
                                const T *invz, hipStream_t stream) {
  if (!X) return fail(PVR_EINVAL, "pvr_simulate: X is NULL");
  if (resid && !y_obs) return fail(PVR_EINVAL, "pvr_simulate: resid requires y_obs");
  if (!y_sim && !resid) return PVR_OK;
  if (sizeof(T) == 4 && p->use_tiles && p->lds_box > 0 && p->psf == PVR_PSF_GAUSSIAN) {
    hipEvent_t *ev = timing_slot(p, PVR_KERNEL_SIMULATE);
    if (ev) HIP_TRY(hipEventRecord(ev[0], stream));
    hipLaunchKernelGGL(k_simulate_tiles, dim3(xcd_blocks(p->n_tiles, p->sim_granule)), dim3(SIM_THREADS),
                       (size_t)p->lds_box * sizeof(float), stream, p->d_prob, p->d_patch,
                       p->d_tile_off, p->M, p->tile_w, p->tile_h, p->n_tiles, p->d_geof,
                       (const float *)invz,
                       (const float *)X, (const float *)y_obs, (float *)y_sim, (float *)resid,
                       p->lds_box, p->sim_granule);
    HIP_TRY(hipGetLastError());
    if (ev) HIP_TRY(hipEventRecord(ev[1], stream));
    const_cast<pvr_plan *>(p)->stats_valid = false;
    return PVR_OK;
  }
  double *stats = (sizeof(T) == 4 && resid) ? p->d_chunk_stats : nullptr;
  hipEvent_t *ev = timing_slot(p, PVR_KERNEL_SIMULATE);
  if (ev) HIP_TRY(hipEventRecord(ev[0], stream));
  const T *XT = nullptr;
  if constexpr (sizeof(T) == 4) {
    XT = volume_xt(p, X, stream);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_simulate<T>, dim3(xcd_blocks(p->n_sim_blocks, p->sim_granule)),
                     dim3(SIM_THREADS), 0, stream, p->d_prob,
                     p->d_patch, p->d_sim_blocks,
                     (const typename GeoOf<T>::type *)(sizeof(T) == 4 ? (const void *)p->d_geof
                                                                      : (const void *)p->d_geod),
                     invz, X, XT, y_obs, y_sim, resid, stats, p->n_sim_blocks, p->sim_granule);
  HIP_TRY(hipGetLastError());
  if (ev) HIP_TRY(hipEventRecord(ev[1], stream));
  // the residual statistics describe these buffers until the next build
  pvr_plan *mp = const_cast<pvr_plan *>(p);
  mp->rq_fresh = false;  // the residuals may have changed
  mp->stats_valid = stats != nullptr;
  mp->stats_resid = resid;
  mp->stats_y = y_obs;
  return PVR_OK;
}

extern "C" pvr_status pvr_simulate(const pvr_plan *p, const float *X, const float *y_obs,
                                   float *y_sim, float *resid, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_simulate", X, 4);
  PVR_ALIGNED("pvr_simulate", y_obs, 4);
  PVR_ALIGNED("pvr_simulate", y_sim, 4);
  PVR_ALIGNED("pvr_simulate", resid, 4);
  if (!p) return fail(PVR_EINVAL, "pvr_simulate: plan is NULL");
  if (!p->built) return fail(PVR_EINVAL, "pvr_simulate: plan has not been built");
  PVR_TRY_STATUS(debug_finite(p, "pvr_simulate", "X", X, p->V, stream));
  PVR_TRY_STATUS(debug_finite(p, "pvr_simulate", "y_obs", y_obs, p->N, stream));
  return simulate_impl<float>(p, X, y_obs, y_sim, resid, p->d_invz, stream);
  PVR_API_END();
}

extern "C" pvr_status pvr_simulate_f64(const pvr_plan *p, const double *X, const double *y_obs,
                                       double *y_sim, double *resid, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_simulate_f64", X, 8);
  PVR_ALIGNED("pvr_simulate_f64", y_obs, 8);
  PVR_ALIGNED("pvr_simulate_f64", y_sim, 8);
  PVR_ALIGNED("pvr_simulate_f64", resid, 8);
  if (!p) return fail(PVR_EINVAL, "pvr_simulate_f64: plan is NULL");
  if (!p->built || !p->built64)
    return fail(PVR_EINVAL, "pvr_simulate_f64: plan needs pvr_plan_build_f64 on a workspace "
                            "attached with PVR_WS_F64");
  PVR_TRY_STATUS(debug_finite(p, "pvr_simulate_f64", "X", X, p->V, stream));
  PVR_TRY_STATUS(debug_finite(p, "pvr_simulate_f64", "y_obs", y_obs, p->N, stream));
  return simulate_impl<double>(p, X, y_obs, y_sim, resid, p->d_invz64, stream);
  PVR_API_END();
}

// ---------------------------------------------------------------------------
// registration
// ---------------------------------------------------------------------------
constexpr int REG_THREADS = 256;

// Sum of N doubles over the workgroup (fixed order: wave butterflies, then
// the 4 wave results in order).
template <int N>
__device__ __forceinline__ void block_sum(double v[N], double (*lds)[REG_THREADS / 64]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double x = v[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) lds[q][wave] = x;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double x = 0;
#pragma unroll
    for (int w = 0; w < REG_THREADS / 64; ++w) x += lds[q][w];
    v[q] = x;
  }
  __syncthreads();
}

// Copy of a workgroup-uniform struct held in LDS into scalar registers: every
// 32-bit word passes through readfirstlane, so the walks read the constants
// from SGPRs instead of holding a VGPR copy per lane.
template <typename S>
__device__ __forceinline__ S wave_uniform(const S &src) {
  static_assert(sizeof(S) % 4 == 0, "uniform copy works on 32-bit words");
  S dst;
  const uint32_t *a = reinterpret_cast<const uint32_t *>(&src);
  uint32_t *d = reinterpret_cast<uint32_t *>(&dst);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(S) / 4); ++i) d[i] = __builtin_amdgcn_readfirstlane(a[i]);
  return dst;
}

struct RegShared {
  GeoF g;
  GradConst gc;     // exact-gradient constants of the evaluated transform
  GradMom gm;
  double red[24][REG_THREADS / 64];
  // optimiser state (uniform across the workgroup; kept out of registers)
  double th[6];     // transform evaluated next
  double q[6];      // current point, scaled variables
  double grad[6];
  double sc[6];
  double fval;      // result of the last evaluation
  // work done, for the kernel's roofline: evaluations and samples walked
  // (plain, exact gradient); written by lane 0 only
  double walked[2];
  int evals[2];
};

// NCC of the patch against its simulation at sh.th (valid samples only);
// every lane returns the same value.
template <bool XT, int PSF = PVR_PSF_GAUSSIAN>
__device__ double reg_eval(RegShared &sh, const ProbDev &pr, const StackDev &st, const PatchDev &pt,
                           double k, __amdgpu_buffer_rsrc_t xr, unsigned nbytes,
                           const float *__restrict__ y,
                           const uint8_t *__restrict__ mask) {
  if (threadIdx.x == 0) {
    GeoD gd;
    int bb[6];
    make_geometry<PSF>(pr, st, pt, sh.th, k, gd, sh.g, bb);
  }
  __syncthreads();
  const GeoF g = wave_uniform(sh.g);
  double acc6[6] = {0, 0, 0, 0, 0, 0};
  const int n = pt.w * pt.h;
  for (int l = threadIdx.x; l < n; l += REG_THREADS) {
    const long long j = pt.off + l;
    if (mask && !mask[j]) continue;
    const int u = pt.x0 + l % pt.w, v = pt.y0 + l / pt.w;
    int b[3];
    float f[3];
    if (!sample_centre(g, pr, u, v, pt.slice, b, f)) continue;
    float z = 0.f;
    float a;
    if constexpr (PSF == PVR_PSF_SINC)
      a = g.perm[2] == (XT ? 1 : 0)
              ? psf_walk_sinc<float, GeoF, true, 1, XT>(g, pr, b, f, xr, nbytes, &z)
              : psf_walk_sinc<float, GeoF, true, 2, XT>(g, pr, b, f, xr, nbytes, &z);
    else
      a = g.perm[2] == (XT ? 1 : 0)
              ? psf_walk_fwd<float, GeoF, true, 1, XT>(g, pr, b, f, xr, nbytes, &z)
              : psf_walk_fwd<float, GeoF, true, 2, XT>(g, pr, b, f, xr, nbytes, &z);
    if (!(z > 0.f)) continue;
    const double yh = (double)(a / z), yo = (double)y[j];
    acc6[0] += 1.0;
    acc6[1] += yo;
    acc6[2] += yo * yo;
    acc6[3] += yh;
    acc6[4] += yh * yh;
    acc6[5] += yo * yh;
  }
  block_sum<6>(acc6, sh.red);
  const double cnt = acc6[0];
  if (threadIdx.x == 0) {
    sh.walked[0] += cnt;
    sh.evals[0] += 1;
  }
  if (!(cnt > 0)) return 0.0;
  const double my = acc6[1] / cnt, mh = acc6[3] / cnt;
  const double vy = acc6[2] / cnt - my * my, vh = acc6[4] / cnt - mh * mh;
  const double cv = acc6[5] / cnt - my * mh;
  if (!(vy > 1e-12 * my * my) || !(vh > 1e-12 * mh * mh) || !(vy > 0) || !(vh > 0)) return 0.0;
  return cv / sqrt(vy * vh);
}

// NCC of the patch at sh.th and its exact gradient with respect to the six
// parameters of sh.th.  One walk per valid sample gives y_hat and, through
// the moments of pvr_grad.h, d y_hat / d theta = sum_i (X_i - y_hat) dg_i / Z;
// with n valid samples, S_a = sum (y - mean y)^2 and S_b = sum (y_hat -
// mean y_hat)^2,
//   d NCC / d theta = sum_j [(y_j - mean y) / sqrt(S_a S_b)
//                            - NCC (y_hat_j - mean y_hat) / S_b] d y_hat_j,
// which needs only the per-patch sums of d y_hat, y d y_hat and
// y_hat d y_hat beside the six NCC sums.  Every lane returns the same values.
template <bool XT>
__device__ double reg_eval_exact(RegShared &sh, const ProbDev &pr, const StackDev &st,
                                 const PatchDev &pt, double k, __amdgpu_buffer_rsrc_t xr,
                                 unsigned nbytes, const float *__restrict__ y,
                                 const uint8_t *__restrict__ mask, double gth[6]) {
  if (threadIdx.x == 0) {
    GeoD gd;
    int bb[6];
    make_geometry(pr, st, pt, sh.th, k, gd, sh.g, bb);
    make_grad_const(pr, st, pt, sh.th, sh.gc);
    make_grad_mom(sh.gc, gd.perm, sh.gm);
  }
  __syncthreads();
  const GeoF g = wave_uniform(sh.g);
  double acc[24];
#pragma unroll
  for (int q = 0; q < 24; ++q) acc[q] = 0.0;
  const int n = pt.w * pt.h;
  for (int l = threadIdx.x; l < n; l += REG_THREADS) {
    const long long j = pt.off + l;
    if (mask && !mask[j]) continue;
    const int u = pt.x0 + l % pt.w, v = pt.y0 + l / pt.w;
    int b[3];
    float f[3];
    if (!sample_centre(g, pr, u, v, pt.slice, b, f)) continue;
    float xb, a, z, mx[9], me[9];
    if (g.perm[2] == (XT ? 1 : 0))
      psf_walk_grad<1, XT>(g, pr, b, f, xr, nbytes, xb, a, z, mx, me);
    else
      psf_walk_grad<2, XT>(g, pr, b, f, xr, nbytes, xb, a, z, mx, me);
    if (!(z > 0.f)) continue;
    const float iz = 1.f / z;
    const float dl = a * iz;  // y_hat - X_b
    const float yhf = xb + dl;
    float m[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) m[c] = fma(-dl, me[c], mx[c]);
    // q = x_j - (c + t)
    double xv[3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
      xv[r] = fma(g.H[4 * r], (double)u,
                  fma(g.H[4 * r + 1], (double)v, fma(g.H[4 * r + 2], (double)pt.slice, g.H[4 * r + 3])));
    float qt[3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
      qt[r] = (float)(sh.gc.Vl[3 * r] * xv[0] + sh.gc.Vl[3 * r + 1] * xv[1] +
                      sh.gc.Vl[3 * r + 2] * xv[2] + sh.gc.v2w_o[r] - sh.gc.ct[r]);
    float a6[6];
    grad_from_moments(sh.gm, m, qt, a6);
    const double yh = (double)yhf, yo = (double)y[j];
    acc[0] += 1.0;
    acc[1] += yo;
    acc[2] += yo * yo;
    acc[3] += yh;
    acc[4] += yh * yh;
    acc[5] += yo * yh;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double d = (double)(a6[c] * iz);
      acc[6 + c] += d;
      acc[12 + c] += yo * d;
      acc[18 + c] += yh * d;
    }
  }
  block_sum<24>(acc, sh.red);
#pragma unroll
  for (int c = 0; c < 6; ++c) gth[c] = 0.0;
  const double cnt = acc[0];
  if (threadIdx.x == 0) {
    sh.walked[1] += cnt;
    sh.evals[1] += 1;
  }
  if (!(cnt > 0)) return 0.0;
  const double my = acc[1] / cnt, mh = acc[3] / cnt;
  const double vy = acc[2] / cnt - my * my, vh = acc[4] / cnt - mh * mh;
  const double cv = acc[5] / cnt - my * mh;
  if (!(vy > 1e-12 * my * my) || !(vh > 1e-12 * mh * mh) || !(vy > 0) || !(vh > 0)) return 0.0;
  const double ncc = cv / sqrt(vy * vh);
  const double sab = cnt * sqrt(vy * vh), sb = cnt * vh;
#pragma unroll
  for (int c = 0; c < 6; ++c)
    gth[c] = (acc[12 + c] - my * acc[6 + c]) / sab - ncc * (acc[18 + c] - mh * acc[6 + c]) / sb;
  return ncc;
}

// One workgroup per patch; the optimiser's control flow is uniform (every
// lane sees the same reduced NCC values), its state lives in LDS.  EXACT
// selects the exact gradient (one reg_eval_exact) over central differences
// (twelve reg_eval); XT the y-fastest volume copy (patches of layout 1); PSF
// the plan's PSF (the exact gradient is written for the Gaussian only).
template <bool EXACT, bool XT, int PSF>
__device__ __forceinline__ void register_patch(
    RegShared &sh, const ProbDev *__restrict__ probs, const StackDev *__restrict__ stacks,
    const PatchDev *__restrict__ patches, const float *__restrict__ Xv,
    const float *__restrict__ y, const uint8_t *__restrict__ mask, float *__restrict__ theta,
    float *__restrict__ ncc_out, const uint8_t *__restrict__ reg, const pvr_reg_params &prm,
    double k, unsigned long long *__restrict__ stats) {
  const int s = blockIdx.x;
  const PatchDev pt = patches[s];
  const ProbDev pr = probs[pt.problem];
  const StackDev st = stacks[pt.stack];
  const unsigned nbytes = (unsigned)(pr.nx * pr.ny * pr.nz) * (unsigned)sizeof(float);
  const __amdgpu_buffer_rsrc_t xr = raw_buffer(Xv + pr.vol_off, nbytes);
  // observed standard deviation over unmasked samples
  double sy[6] = {0, 0, 0, 0, 0, 0};
  const int n = pt.w * pt.h;
  for (int l = threadIdx.x; l < n; l += REG_THREADS) {
    const long long j = pt.off + l;
    if (mask && !mask[j]) continue;
    const double yo = y[j];
    sy[0] += 1.0;
    sy[1] += yo;
    sy[2] += yo * yo;
  }
  block_sum<6>(sy, sh.red);
  double sd = 0;
  if (sy[0] > 0) {
    const double m = sy[1] / sy[0];
    sd = sqrt(fmax(sy[2] / sy[0] - m * m, 0.0));
  }
  if (threadIdx.x == 0) {
    sh.walked[0] = sh.walked[1] = 0.0;
    sh.evals[0] = sh.evals[1] = 0;
    const double su = st.spacing[0], sv = st.spacing[1];
    double rho = 0.5 * sqrt((pt.w - 1) * (pt.w - 1) * su * su + (pt.h - 1) * (pt.h - 1) * sv * sv);
    rho = rho < 1.0 ? 1.0 : rho;
    for (int a = 0; a < 6; ++a) {
      sh.th[a] = (double)theta[6 * s + a];
      sh.sc[a] = a < 3 ? rho : 1.0;
      sh.q[a] = sh.th[a] * sh.sc[a];
    }
  }
  __syncthreads();
  double f0 = reg_eval<XT, PSF>(sh, pr, st, pt, k, xr, nbytes, y, mask);
  const bool do_reg = (reg ? reg[s] != 0 : true) && sd >= prm.min_std && prm.max_iter > 0;
  if (do_reg) {
    double delta = prm.step0;
    bool have_grad = false, moved = false;
    for (int it = 0; it < prm.max_iter; ++it) {
      if (delta < prm.step_min) break;
      if constexpr (EXACT) static_assert(PSF == PVR_PSF_GAUSSIAN, "exact gradient: Gaussian PSF only");
      if (!have_grad && EXACT) {
        __syncthreads();
        if (threadIdx.x == 0)
          for (int b = 0; b < 6; ++b) sh.th[b] = sh.q[b] / sh.sc[b];
        double gth[6];
        reg_eval_exact<XT>(sh, pr, st, pt, k, xr, nbytes, y, mask, gth);
        if (threadIdx.x == 0)
          for (int a = 0; a < 6; ++a) sh.grad[a] = gth[a] / sh.sc[a];
        have_grad = true;
      } else if (!have_grad) {
        for (int a = 0; a < 6; ++a) {
          double fp, fm;
          __syncthreads();
          if (threadIdx.x == 0) {
            for (int b = 0; b < 6; ++b) sh.th[b] = sh.q[b] / sh.sc[b];
            sh.th[a] = (sh.q[a] + prm.fd_h) / sh.sc[a];
          }
          fp = reg_eval<XT, PSF>(sh, pr, st, pt, k, xr, nbytes, y, mask);
          __syncthreads();
          if (threadIdx.x == 0) sh.th[a] = (sh.q[a] - prm.fd_h) / sh.sc[a];
          fm = reg_eval<XT, PSF>(sh, pr, st, pt, k, xr, nbytes, y, mask);
          if (threadIdx.x == 0) sh.grad[a] = (fp - fm) / (2.0 * prm.fd_h);
        }
        have_grad = true;
      }
      __syncthreads();
      double gn = 0;
      for (int a = 0; a < 6; ++a) gn += sh.grad[a] * sh.grad[a];
      gn = sqrt(gn);
      if (!(gn > 0)) break;
      __syncthreads();
      if (threadIdx.x == 0)
        for (int a = 0; a < 6; ++a) sh.th[a] = (sh.q[a] + delta * sh.grad[a] / gn) / sh.sc[a];
      const double ft = reg_eval<XT, PSF>(sh, pr, st, pt, k, xr, nbytes, y, mask);
      if (ft > f0) {
        __syncthreads();
        if (threadIdx.x == 0)
          for (int a = 0; a < 6; ++a) sh.q[a] = sh.q[a] + delta * sh.grad[a] / gn;
        f0 = ft;
        have_grad = false;
        moved = true;
        delta = fmin(2.0 * delta, prm.step0);
      } else {
        delta *= 0.5;
      }
    }
    __syncthreads();
    if (moved && threadIdx.x == 0) {
      for (int a = 0; a < 6; ++a) theta[6 * s + a] = (float)(sh.q[a] / sh.sc[a]);
    }
  }
  if (ncc_out && threadIdx.x == 0) ncc_out[s] = (float)f0;
  if (threadIdx.x == 0) {
    atomicAdd(&stats[0], (unsigned long long)sh.evals[0]);
    atomicAdd(&stats[1], (unsigned long long)sh.walked[0]);
    atomicAdd(&stats[2], (unsigned long long)sh.evals[1]);
    atomicAdd(&stats[3], (unsigned long long)sh.walked[1]);
  }
}

// The optimiser of register_patch for the patches of one volume layout (the
// others return at once): one launch per layout keeps the register use of a
// single optimiser, and the two launches run on two streams, so that the
// patches of one layout fill the other launch's tail (patch costs differ by
// two orders of magnitude: a flat patch takes one evaluation).  The central-difference optimiser with the Gaussian PSF
// is held to 128 registers (4 waves per SIMD): its few spills cost less than
// the waves gained (1.16 -> 1.09 s for the registration passes of a 256^3
// four-stack reconstruction); the exact-gradient and sinc variants keep their
// allocation (at 128 registers they spill heavily and run slower; an
// explicit two-wave minimum changed their code and cost the exact one 12 %).
template <bool EXACT, bool XT, int PSF>
__global__ void __launch_bounds__(REG_THREADS, (!EXACT && PSF == PVR_PSF_GAUSSIAN) ? 4 : 1)
k_register(const ProbDev *__restrict__ probs, const StackDev *__restrict__ stacks,
           const PatchDev *__restrict__ patches, const float *__restrict__ Xv, int any_xt,
           const float *__restrict__ y, const uint8_t *__restrict__ mask,
           float *__restrict__ theta, float *__restrict__ ncc_out,
           const uint8_t *__restrict__ reg, pvr_reg_params prm, double k,
           unsigned long long *__restrict__ stats) {
  __shared__ RegShared sh;
  if ((any_xt && patches[blockIdx.x].layout == 1) != XT) return;
  register_patch<EXACT, XT, PSF>(sh, probs, stacks, patches, Xv, y, mask, theta, ncc_out, reg, prm,
                                 k, stats);
}

extern "C" pvr_status pvr_register_patches(const pvr_plan *p, const float *X, const float *y_obs,
                                           float *theta, float *ncc, const uint8_t *reg,
                                           const pvr_reg_params *prm, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_register_patches", X, 4);
  PVR_ALIGNED("pvr_register_patches", y_obs, 4);
  PVR_ALIGNED("pvr_register_patches", theta, 4);
  PVR_ALIGNED("pvr_register_patches", ncc, 4);
  if (!p || !X || !y_obs || !theta || !prm) return fail(PVR_EINVAL, "pvr_register_patches: NULL argument");
  if (!p->built) return fail(PVR_EINVAL, "pvr_register_patches: plan has not been built");
  PVR_TRY_STATUS(debug_finite(p, "pvr_register_patches", "X", X, p->V, stream));
  PVR_TRY_STATUS(debug_finite(p, "pvr_register_patches", "y_obs", y_obs, p->N, stream));
  PVR_TRY_STATUS(debug_finite(p, "pvr_register_patches", "theta", theta, 6LL * p->M, stream));
  if (prm->max_iter < 0 || !(prm->step0 > 0) || !(prm->step_min > 0) || !(prm->fd_h > 0))
    return fail(PVR_EINVAL, "pvr_register_patches: invalid optimiser parameters");
  if (prm->gradient != PVR_REG_GRAD_FD && prm->gradient != PVR_REG_GRAD_EXACT)
    return fail(PVR_EINVAL, "pvr_register_patches: gradient must be PVR_REG_GRAD_FD or PVR_REG_GRAD_EXACT");
  const bool sinc = p->psf == PVR_PSF_SINC;
  if (sinc && prm->gradient == PVR_REG_GRAD_EXACT)
    return fail(PVR_EUNSUPPORTED,
                "pvr_register_patches: the exact gradient is implemented for the Gaussian PSF "
                "(use PVR_REG_GRAD_FD with the sinc PSF)");
  hipEvent_t *ev = timing_slot(p, PVR_KERNEL_REGISTER);
  if (ev) HIP_TRY(hipEventRecord(ev[0], stream));
  const float *XT = volume_xt(p, X, stream);
  HIP_TRY(hipGetLastError());
  const int any = XT != nullptr;
  // the y-fastest copy's patches run on the plan's second stream, after the
  // copy, beside the others; the join makes the call's stream wait for both
  if (any) {
    HIP_TRY(hipEventRecord(p->ev_fork, stream));
    HIP_TRY(hipStreamWaitEvent(p->side, p->ev_fork, 0));
  }
#define REG_LAUNCH(E, L, S, V, STREAM)                                                           \
  hipLaunchKernelGGL((k_register<E, L, S>), dim3(p->M), dim3(REG_THREADS), 0, STREAM, p->d_prob, \
                     p->d_stack, p->d_patch, V, any, y_obs, p->d_mask, theta, ncc, reg, *prm,     \
                     p->k, p->d_reg_stats)
  if (sinc) {
    REG_LAUNCH(false, false, PVR_PSF_SINC, X, stream);
    if (any) REG_LAUNCH(false, true, PVR_PSF_SINC, XT, p->side);
  } else if (prm->gradient == PVR_REG_GRAD_EXACT) {
    REG_LAUNCH(true, false, PVR_PSF_GAUSSIAN, X, stream);
    if (any) REG_LAUNCH(true, true, PVR_PSF_GAUSSIAN, XT, p->side);
  } else {
    REG_LAUNCH(false, false, PVR_PSF_GAUSSIAN, X, stream);
    if (any) REG_LAUNCH(false, true, PVR_PSF_GAUSSIAN, XT, p->side);
  }
#undef REG_LAUNCH
  HIP_TRY(hipGetLastError());
  if (any) {
    HIP_TRY(hipEventRecord(p->ev_join, p->side));
    HIP_TRY(hipStreamWaitEvent(stream, p->ev_join, 0));
  }
  if (ev) HIP_TRY(hipEventRecord(ev[1], stream));
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_plan_reg_stats(pvr_plan *p, int64_t out[4], hipStream_t stream) {
  PVR_API_BEGIN();
  if (!p || !out) return fail(PVR_EINVAL, "pvr_plan_reg_stats: NULL argument");
  for (int i = 0; i < 4; ++i) out[i] = 0;
  if (!p->attached) return PVR_OK;
  unsigned long long v[4];
  HIP_TRY(hipMemcpyAsync(v, p->d_reg_stats, sizeof v, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  for (int i = 0; i < 4; ++i) out[i] = (int64_t)v[i];
  launch_fill_i32((int *)p->d_reg_stats, 0, 8, stream);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}
