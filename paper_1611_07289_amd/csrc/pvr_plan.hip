// Plan creation and the motion-dependent build: per-patch geometry, per-sample
// PSF normalisers and the brick -> patch index of the gather adjoint.
#include <limits.h>
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

static pvr_status make_tiles(pvr_plan *p, int tile_w, int tile_h);

// Largest capacity of an adjoint index list (its offsets are int32).
constexpr long long INDEX_CAP_MAX = 0x7ffffff0LL;

// Upper bound, over every motion and either PSF, on the number of bricks of
// e^3 voxels (a lattice of step e voxels) that the separating-axis test of
// the index kernels lists for one patch.  A brick is listed only if its
// voxel-centre box meets each of the three slabs of the patch's pixel-frame
// support box, so its centre lies in the support box widened on every side
// by the box's largest projected half-width hb = (e - 1)/2 sum_c |V_c| (V_c
// the voxel axes in mm).  That widened box K is a rotated box with sides
// D_a (mm), and the cells of the centres inside it are disjoint and lie in K
// grown by the cell's circumradius R, so the count is at most
// (D0 D1 D2 + 2 (D0 D1 + D1 D2 + D2 D0) R + pi (D0 + D1 + D2) R^2 +
// 4/3 pi R^3) / (e^3 |det V|), the Steiner volume of the grown box over the
// cell volume.  At most `cap` (the grid's own count).
static long long pair_bound(const ProbDev &pr, const StackDev &st, const PatchDev &q, double k,
                            int e, long long cap) {
  double V[3][3], sumn = 0;
  for (int c = 0; c < 3; ++c) {
    double n2 = 0;
    for (int r = 0; r < 3; ++r) {
      V[c][r] = pr.v2w[4 * r + c];
      n2 += V[c][r] * V[c][r];
    }
    sumn += sqrt(n2);
  }
  double R = 0;
  for (int sgn = 0; sgn < 8; ++sgn) {
    double n2 = 0;
    for (int r = 0; r < 3; ++r) {
      double x = 0;
      for (int c = 0; c < 3; ++c) x += ((sgn >> c) & 1 ? -1.0 : 1.0) * V[c][r];
      n2 += x * x;
    }
    R = std::max(R, sqrt(n2));
  }
  R *= 0.5 * e;
  const double det = fabs(V[0][0] * (V[1][1] * V[2][2] - V[1][2] * V[2][1]) -
                          V[1][0] * (V[0][1] * V[2][2] - V[0][2] * V[2][1]) +
                          V[2][0] * (V[0][1] * V[1][2] - V[0][2] * V[1][1]));
  const double hb = 0.5 * (e - 1) * sumn;
  const double reach_u = std::max(k * st.sigma[0], st.wz[0]);
  const double reach_v = std::max(k * st.sigma[1], st.wz[1]);
  const double reach_n = k * st.sigma[2];
  double D[3] = {(q.w - 1) * st.spacing[0] + 2 * reach_u + 2 * hb,
                 (q.h - 1) * st.spacing[1] + 2 * reach_v + 2 * hb, 2 * reach_n + 2 * hb};
  for (double &d : D) d = d * (1 + 1e-6) + 1e-6;  // room for the test's rounding
  const double pi = 3.14159265358979323846;
  const double vol = D[0] * D[1] * D[2] + 2 * (D[0] * D[1] + D[1] * D[2] + D[2] * D[0]) * R +
                     pi * (D[0] + D[1] + D[2]) * R * R + 4.0 / 3.0 * pi * R * R * R;
  const double n = ceil(vol / (det * e * e * e)) + 1;
  return n >= (double)cap ? cap : (long long)n;
}

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
                           int M, double k, int psf, GeoD *__restrict__ gd, GeoF *__restrict__ gf,
                           int *__restrict__ bb, double *__restrict__ sbox) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= M) return;
  const PatchDev pt = patches[s];
  const StackDev st = stacks[pt.stack];
  GeoD g;
  GeoF f;
  if (psf == PVR_PSF_SINC)
    make_geometry<PVR_PSF_SINC>(probs[pt.problem], st, pt, theta + 6 * s, k, g, f, bb + 6 * s);
  else
    make_geometry<PVR_PSF_GAUSSIAN>(probs[pt.problem], st, pt, theta + 6 * s, k, g, f, bb + 6 * s);
  gd[s] = g;
  gf[s] = f;
  // voxel -> pixel map and the pixel-frame support box of the patch
  double *o = sbox + 18 * s;
  for (int q = 0; q < 12; ++q) o[q] = g.G[q];
  const bool sinc = psf == PVR_PSF_SINC;
  const double ru = sinc ? st.wz[0] / st.spacing[0] : k * st.sigma[0] / st.spacing[0],
               rv = sinc ? st.wz[1] / st.spacing[1] : k * st.sigma[1] / st.spacing[1],
               rk = k * st.sigma[2] / st.spacing[2];
  o[12] = pt.x0 - ru; o[13] = pt.x0 + pt.w - 1 + ru;
  o[14] = pt.y0 - rv; o[15] = pt.y0 + pt.h - 1 + rv;
  o[16] = pt.slice - rk; o[17] = pt.slice + rk;
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
    if (ok && g.psf == PVR_PSF_SINC) {
      const __amdgpu_buffer_rsrc_t none = raw_buffer((const T *)nullptr, 0u);
      psf_walk_sinc<T, typename GeoOf<T>::type, false>(g, pr, b, f, none, 0u, &z);
    } else if (ok) {
      psf_walk<T, typename GeoOf<T>::type, false>(g, pr, b, f, nullptr, z, acc);
    }
    ok = ok && z > (T)0;
    const T iz = ok ? (T)1 / z : (T)0;
    invz[j] = (float)iz;
    if (invz64) invz64[j] = (double)iz;
  }
}

// brick -> patch index: count, scan, fill.  Every brick scans the patches of
// its problem in order, so each list is sorted by patch (deterministic).  A
// patch is listed when the brick is inside its voxel bounding box and the
// brick's corner voxels, mapped into the patch's pixel frame, overlap the
// patch's support box on each of the three stack axes (separating-axis
// test; conservative).
__device__ __forceinline__ bool box_meets_patch(const double *__restrict__ sb, const double lo[3],
                                                const double hi[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double *g = sb + 4 * a;
    double mn = g[3], mx = g[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double p = g[c] * lo[c], q = g[c] * hi[c];
      mn += fmin(p, q);
      mx += fmax(p, q);
    }
    if (mx < sb[12 + 2 * a] || mn > sb[13 + 2 * a]) return false;
  }
  return true;
}

__device__ __forceinline__ bool brick_meets_patch(const int *__restrict__ r, const double *__restrict__ sb,
                                                  int bx, int by, int bz) {
  if (!((bx >= r[0]) & (bx <= r[3]) & (by >= r[1]) & (by <= r[4]) & (bz >= r[2]) & (bz <= r[5])))
    return false;
  const double lo[3] = {(double)(bx * BRICK), (double)(by * BRICK), (double)(bz * BRICK)};
  const double hi[3] = {lo[0] + BRICK - 1, lo[1] + BRICK - 1, lo[2] + BRICK - 1};
  return box_meets_patch(sb, lo, hi);
}

// Second level: each brick's 8 sub-bricks (SUB^3 voxels, one wavefront of the
// adjoint each) keep the patches of the brick's list that reach them.
__device__ __forceinline__ void sub_box(const ProbDev &pr, int sbi, double lo[3], double hi[3]) {
  const int bi = sbi >> 3, w = sbi & 7;
  const int local = bi - pr.brick_base;
  const int bx = local % pr.nbx, by = (local / pr.nbx) % pr.nby, bz = local / (pr.nbx * pr.nby);
  lo[0] = bx * BRICK + (w & 1) * SUB;
  lo[1] = by * BRICK + ((w >> 1) & 1) * SUB;
  lo[2] = bz * BRICK + (w >> 2) * SUB;
  for (int a = 0; a < 3; ++a) hi[a] = lo[a] + SUB - 1;
}

// One wavefront per brick: the lanes take 64 entries of the brick's list at
// a time and test each entry's patch against the 8 sub-bricks; per
// sub-brick a ballot counts the hits (k_sub_count) or places them in list
// order, which is ascending patch order (k_sub_fill).
__device__ __forceinline__ unsigned sub_mask(const ProbDev &pr, int bi,
                                             const double *__restrict__ sb) {
  unsigned m = 0;
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    double lo[3], hi[3];
    sub_box(pr, bi * 8 + w, lo, hi);
    m |= box_meets_patch(sb, lo, hi) ? 1u << w : 0u;
  }
  return m;
}

__global__ void __launch_bounds__(256)
k_sub_count(const ProbDev *__restrict__ probs, const int *__restrict__ brick_prob,
            const double *__restrict__ sbox, int nb, const int *__restrict__ off,
            const int *__restrict__ list, int *__restrict__ count) {
  const int lane = threadIdx.x & 63;
  const int bi = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (bi >= nb) return;  // uniform over the wavefront
  const ProbDev pr = probs[brick_prob[bi]];
  int c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int q0 = off[bi]; q0 < off[bi + 1]; q0 += 64) {
    const int q = q0 + lane;
    const unsigned m = q < off[bi + 1] ? sub_mask(pr, bi, sbox + 18 * list[q]) : 0u;
#pragma unroll
    for (int w = 0; w < 8; ++w) c[w] += __popcll(__ballot((m >> w) & 1u));
  }
  if (lane < 8) {
    int v = c[0];
#pragma unroll
    for (int w = 1; w < 8; ++w) v = lane == w ? c[w] : v;
    count[bi * 8 + lane] = v;
  }
}

__global__ void __launch_bounds__(256)
k_sub_fill(const ProbDev *__restrict__ probs, const int *__restrict__ brick_prob,
           const double *__restrict__ sbox, int nb, const int *__restrict__ off,
           const int *__restrict__ list, const int *__restrict__ soff,
           int *__restrict__ slist) {
  const int lane = threadIdx.x & 63;
  const int bi = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (bi >= nb) return;  // uniform over the wavefront
  const ProbDev pr = probs[brick_prob[bi]];
  const unsigned long long below = (1ull << lane) - 1ull;
  int c[8], end[8];
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    c[w] = soff[bi * 8 + w];
    end[w] = soff[bi * 8 + w + 1];  // clamped to the capacity
  }
  for (int q0 = off[bi]; q0 < off[bi + 1]; q0 += 64) {
    const int q = q0 + lane;
    const int sp = q < off[bi + 1] ? list[q] : 0;
    const unsigned m = q < off[bi + 1] ? sub_mask(pr, bi, sbox + 18 * sp) : 0u;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
      const bool h = (m >> w) & 1u;
      const unsigned long long bal = __ballot(h);
      const int pos = c[w] + __popcll(bal & below);
      if (h && pos < end[w]) slist[pos] = sp;
      c[w] += __popcll(bal);
    }
  }
}

// Union of the brick ranges of 64 consecutive patches (group G holds the
// patches 64 G .. 64 G + 63 of the whole table): a brick outside it meets
// none of them.  Empty ranges (low end above the high end) only widen it.
constexpr int PGROUP = 64;
__global__ void __launch_bounds__(256)
k_group_box(const int *__restrict__ bb, int M, int *__restrict__ gbox) {
  const int lane = threadIdx.x & 63;
  const int G = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (G * PGROUP >= M) return;  // uniform over the wavefront
  const int s = G * PGROUP + lane;
  const bool ok = s < M;
  int v[6];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    v[r] = ok ? bb[6 * s + r] : INT_MAX;
    v[3 + r] = ok ? bb[6 * s + 3 + r] : INT_MIN;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      v[r] = min(v[r], __shfl_xor(v[r], o, 64));
      v[3 + r] = max(v[3 + r], __shfl_xor(v[3 + r], o, 64));
    }
  if (lane < 6) gbox[6 * G + lane] = v[lane];
}

__device__ __forceinline__ bool brick_in_group(const int *__restrict__ gb, int bx, int by, int bz) {
  return bx >= gb[0] && bx <= gb[3] && by >= gb[1] && by <= gb[4] && bz >= gb[2] && bz <= gb[5];
}

// One wavefront per brick: over the groups that hold the brick's problem's
// patches, the lanes first test 64 group ranges at once, then the 64
// patches of each group whose range union holds the brick.  The count is a
// wave sum; the fill writes the meeting patches in ascending patch order
// (ballot prefix counts), the order that fixes the adjoint's summation
// order.
constexpr int BIN_THREADS = 256;

__global__ void __launch_bounds__(BIN_THREADS)
k_bin_count(const ProbDev *__restrict__ probs, const int *__restrict__ brick_prob,
            const int *__restrict__ bb, const int *__restrict__ gbox,
            const double *__restrict__ sbox, int nb, int *__restrict__ count) {
  const int lane = threadIdx.x & 63;
  const int bi = __builtin_amdgcn_readfirstlane(blockIdx.x * (BIN_THREADS / 64) + (threadIdx.x >> 6));
  if (bi >= nb) return;  // uniform over the wavefront
  const ProbDev pr = probs[brick_prob[bi]];
  const int local = bi - pr.brick_base;
  const int bx = local % pr.nbx, by = (local / pr.nbx) % pr.nby, bz = local / (pr.nbx * pr.nby);
  int c = 0;
  if (pr.patch_end > pr.patch_begin) {
    const int g1 = (pr.patch_end - 1) / PGROUP;
    for (int G0 = pr.patch_begin / PGROUP; G0 <= g1; G0 += 64) {
      // the lanes test 64 groups at once; the groups that hold the brick
      // are then taken in ascending order
      const int Gl = G0 + lane;
      unsigned long long hit = __ballot(Gl <= g1 && brick_in_group(gbox + 6 * Gl, bx, by, bz));
      while (hit) {
        const int G = G0 + __builtin_ctzll(hit);
        hit &= hit - 1;
        const int s = G * PGROUP + lane;
        if (s >= pr.patch_begin && s < pr.patch_end &&
            brick_meets_patch(bb + 6 * s, sbox + 18 * s, bx, by, bz))
          ++c;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if (lane == 0) count[bi] = c;
}

__global__ void __launch_bounds__(BIN_THREADS)
k_bin_fill(const ProbDev *__restrict__ probs, const int *__restrict__ brick_prob,
           const int *__restrict__ bb, const int *__restrict__ gbox,
           const double *__restrict__ sbox, int nb, const int *__restrict__ off,
           int *__restrict__ list) {
  const int lane = threadIdx.x & 63;
  const int bi = __builtin_amdgcn_readfirstlane(blockIdx.x * (BIN_THREADS / 64) + (threadIdx.x >> 6));
  if (bi >= nb) return;  // uniform over the wavefront
  const ProbDev pr = probs[brick_prob[bi]];
  const int local = bi - pr.brick_base;
  const int bx = local % pr.nbx, by = (local / pr.nbx) % pr.nby, bz = local / (pr.nbx * pr.nby);
  const unsigned long long below = (1ull << lane) - 1ull;
  int c = off[bi];
  const int end = off[bi + 1];  // the list's end, clamped to its capacity
  if (pr.patch_end > pr.patch_begin) {
    const int g1 = (pr.patch_end - 1) / PGROUP;
    for (int G0 = pr.patch_begin / PGROUP; G0 <= g1; G0 += 64) {
      const int Gl = G0 + lane;
      unsigned long long hit = __ballot(Gl <= g1 && brick_in_group(gbox + 6 * Gl, bx, by, bz));
      while (hit) {
        const int G = G0 + __builtin_ctzll(hit);
        hit &= hit - 1;
        const int s = G * PGROUP + lane;
        const bool m = s >= pr.patch_begin && s < pr.patch_end &&
                       brick_meets_patch(bb + 6 * s, sbox + 18 * s, bx, by, bz);
        const unsigned long long bal = __ballot(m);
        const int pos = c + __popcll(bal & below);
        if (m && pos < end) list[pos] = s;
        c += __popcll(bal);
      }
    }
  }
}

// Largest voxel box over the forward tiles (sizes the staged LDS).
__global__ void k_tile_boxmax(const ProbDev *__restrict__ probs, const PatchDev *__restrict__ patches,
                              const int *__restrict__ tile_off, int M, int tile_w, int tile_h,
                              int n_tiles, const GeoF *__restrict__ geo, int *__restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const TileWork tw = tile_at(tile_off, M, patches, tile_w, tile_h, t);
  const PatchDev pt = patches[tw.patch];
  int lo[3], hi[3];
  const int c = tile_box(geo[tw.patch], probs[pt.problem], pt, tw, lo, hi);
  atomicMax(out, c);
}

// Exclusive scan of count[0..n) into off[0..n], off[n] = total, in three
// passes: block sums over chunks of SCAN_CHUNK counts (each thread four
// consecutive ones), one workgroup scanning the block sums (tiles of
// SCAN_T with a carry) and writing the total, then every block scanning its
// chunk from its base.  The offsets are clamped to the list's capacity
// `cap`; a total beyond it (which the host bound on the pairs rules out)
// raises PVR_FAULT_INDEX, and the lists then keep only what fits.
constexpr int SCAN_T = 1024, SCAN_PER = 4, SCAN_CHUNK = SCAN_T * SCAN_PER;

static int scan_blocks(long long n) { return (int)((n + SCAN_CHUNK - 1) / SCAN_CHUNK); }

// inclusive scan of one value per thread across the workgroup (Hillis-Steele)
__device__ __forceinline__ long long block_incl_scan(long long v, long long *lds) {
  const int tid = threadIdx.x;
  lds[tid] = v;
  __syncthreads();
  for (int d = 1; d < SCAN_T; d <<= 1) {
    const long long u = tid >= d ? lds[tid - d] : 0;
    __syncthreads();
    lds[tid] += u;
    __syncthreads();
  }
  return lds[tid];
}

__global__ void __launch_bounds__(SCAN_T)
k_scan_sums(const int *__restrict__ count, int n, long long *__restrict__ bsum) {
  __shared__ long long lds[SCAN_T / 64];
  const int base = blockIdx.x * SCAN_CHUNK + threadIdx.x * SCAN_PER;
  long long v = 0;
#pragma unroll
  for (int q = 0; q < SCAN_PER; ++q)
    if (base + q < n) v += count[base + q];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int w = 0; w < SCAN_T / 64; ++w) t += lds[w];
    bsum[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(SCAN_T)
k_scan_top(long long *__restrict__ bsum, int nblk, int n, int *__restrict__ off,
           int *__restrict__ total, long long cap, unsigned *__restrict__ status) {
  __shared__ long long lds[SCAN_T];
  long long carry = 0;
  for (int t0 = 0; t0 < nblk; t0 += SCAN_T) {
    const int i = t0 + threadIdx.x;
    const long long v = i < nblk ? bsum[i] : 0;
    const long long incl = block_incl_scan(v, lds);
    if (i < nblk) bsum[i] = carry + incl - v;  // the block's base
    carry += lds[SCAN_T - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    off[n] = (int)min(carry, cap);
    total[0] = (int)min(carry, cap);
    if (carry > cap) atomicOr(status, PVR_FAULT_INDEX);
  }
}

__global__ void __launch_bounds__(SCAN_T)
k_scan_apply(const int *__restrict__ count, int n, const long long *__restrict__ bbase,
             int *__restrict__ off, long long cap) {
  __shared__ long long lds[SCAN_T];
  const int base = blockIdx.x * SCAN_CHUNK + threadIdx.x * SCAN_PER;
  int c[SCAN_PER];
  long long v = 0;
#pragma unroll
  for (int q = 0; q < SCAN_PER; ++q) {
    c[q] = base + q < n ? count[base + q] : 0;
    v += c[q];
  }
  long long run = bbase[blockIdx.x] + block_incl_scan(v, lds) - v;
#pragma unroll
  for (int q = 0; q < SCAN_PER; ++q)
    if (base + q < n) {
      off[base + q] = (int)min(run, cap);
      run += c[q];
    }
}

static pvr_status launch_scan(const int *count, int n, long long *scratch, int *off, int *total,
                              long long cap, unsigned *status, hipStream_t stream) {
  const int nblk = scan_blocks(n);
  hipLaunchKernelGGL(k_scan_sums, dim3(nblk), dim3(SCAN_T), 0, stream, count, n, scratch);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_T), 0, stream, scratch, nblk, n, off, total,
                     cap, status);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_scan_apply, dim3(nblk), dim3(SCAN_T), 0, stream, count, n,
                     (const long long *)scratch, off, cap);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
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
    if ((long long)g.nx * g.ny * g.nz > (1LL << 28))
      return fail(PVR_ESHAPE, "pvr_plan_create: grid %d has more than 2^28 voxels", b);
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
      if (a < 2) d.wz[a] = st.fwhm_mm[a];
    }
    for (int a = 0; a < 3; ++a)
      for (int c = a + 1; c < 3; ++c) {
        double dt = d.E[a] * d.E[c] + d.E[3 + a] * d.E[3 + c] + d.E[6 + a] * d.E[6 + c];
        if (fabs(dt) > 1e-9) return fail(PVR_ESHAPE, "pvr_plan_create: stack %d axes %d and %d are not orthogonal", s, a, c);
      }
  }
  // the adjoint's candidate grid depends on the stacks only
  p->max_hu = p->max_hv = 0;
  {
    const double sk = sqrt(KAPPA), K2 = KAPPA * cutoff_k * cutoff_k;
    for (int s = 0; s < n_stacks; ++s) {
      const StackDev &d = p->h_stack[s];
      p->max_hu = std::max(p->max_hu, cand_halfwidth(K2, sk * d.spacing[0] / d.sigma[0]));
      p->max_hv = std::max(p->max_hv, cand_halfwidth(K2, sk * d.spacing[1] / d.sigma[1]));
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
    {
      // rows of the patch run along the stack's u axis: when that is closer
      // to voxel y than to voxel x, the forward walks read the y-fastest copy
      const double *W = p->h_prob[prob].w2v, *A = st.p2w;
      double du[3];
      for (int r = 0; r < 3; ++r) du[r] = W[4 * r] * A[0] + W[4 * r + 1] * A[4] + W[4 * r + 2] * A[8];
      d.layout = fabs(du[1]) > fabs(du[0]) ? 1 : 0;
      if (d.layout) p->any_xt = true;
    }
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
    p->max_problem_patches = 0;
    for (int b = 0; b < n_problems; ++b) {
      if (pcount[b] > PVR_MAX_PROBLEM_PATCHES)
        return fail(PVR_ESHAPE, "pvr_plan_create: problem %d has more than %d patches", b,
                    PVR_MAX_PROBLEM_PATCHES);
      p->max_problem_patches = std::max(p->max_problem_patches, pcount[b]);
      p->h_prob[b].patch_begin = pb; p->h_prob[b].patch_end = pb + pcount[b];
      p->h_prob[b].sample_begin = sb; p->h_prob[b].sample_end = sb + scount[b];
      pb += pcount[b];
      sb += scount[b];
    }
  }
  {
    // forward chunks are patch-major, so every problem's chunks form a range
    int c = 0;
    for (int b = 0; b < n_problems; ++b) {
      p->h_prob[b].chunk_begin = c;
      while (c < (int)blocks.size() && blocks[c].patch < p->h_prob[b].patch_end) ++c;
      p->h_prob[b].chunk_end = c;
    }
  }
  p->h_sample_off[n_patches] = so;
  p->N = so;
  if (so > 0x7fffffffLL * 4) return fail(PVR_ESHAPE, "pvr_plan_create: too many samples");
  p->n_sim_blocks = (int)blocks.size();
  for (int s = 0; s < n_patches; ++s)
    if (patches[s].w > 32767 || patches[s].h > 32767 ||
        (long long)patches[s].w * patches[s].h > (1LL << 26))
      return fail(PVR_ESHAPE, "pvr_plan_create: patch %d too large (w, h <= 32767, w * h <= 2^26)", s);
  p->tile_w = TILE;
  p->tile_h = TILE;
  p->use_tiles = false;
  p->sim_granule = SIM_XCD_GRANULE;
  p->bp_granule = BP_XCD_GRANULE;
  p->h_tile_off = (int *)calloc(n_patches + 1, sizeof(int));
  {
    const pvr_status st = make_tiles(p, TILE, TILE);
    if (st != PVR_OK) return st;
  }
  std::vector<int> plane_prob;
  std::vector<int> plane_first(n_problems);
  p->max_nx = p->max_ny = 0;
  for (int b = 0; b < n_problems; ++b) {
    plane_first[b] = (int)plane_prob.size();
    for (int z = 0; z < p->h_prob[b].nz; ++z) plane_prob.push_back(b);
    p->max_nx = std::max(p->max_nx, p->h_prob[b].nx);
    p->max_ny = std::max(p->max_ny, p->h_prob[b].ny);
  }
  p->n_planes = (int)plane_prob.size();
  if (p->n_planes > 65535) return fail(PVR_ESHAPE, "pvr_plan_create: more than 65535 z-planes in total");
  plane_prob.insert(plane_prob.end(), plane_first.begin(), plane_first.end());
  p->h_plane_prob = (int *)malloc(sizeof(int) * plane_prob.size());
  std::copy(plane_prob.begin(), plane_prob.end(), p->h_plane_prob);
  p->h_brick_prob = (int *)malloc(sizeof(int) * (size_t)std::max(nbr, 1));
  for (int b = 0; b < n_problems; ++b)
    for (int i = 0; i < p->h_prob[b].n_bricks; ++i) p->h_brick_prob[p->h_prob[b].brick_base + i] = b;
  p->h_sim_blocks = (BlockWork *)malloc(sizeof(BlockWork) * std::max<size_t>(blocks.size(), 1));
  std::copy(blocks.begin(), blocks.end(), p->h_sim_blocks);
  // capacity of the adjoint's index: bounds over every motion, so that no
  // build needs to read a count back or to grow a list
  {
    long long bins = 0, subs = 0;
    for (int s = 0; s < n_patches; ++s) {
      const PatchDev &q = p->h_patch[s];
      const ProbDev &pr = p->h_prob[q.problem];
      const long long b = pair_bound(pr, p->h_stack[q.stack], q, cutoff_k, BRICK, pr.n_bricks);
      bins += b;
      subs += std::min(8 * b, pair_bound(pr, p->h_stack[q.stack], q, cutoff_k, SUB, 8LL * pr.n_bricks));
    }
    p->bin_cap = std::min(bins, (long long)INDEX_CAP_MAX);
    p->sub_cap = std::min(subs, (long long)INDEX_CAP_MAX);
  }
  p->device = -1;  // the device of the first workspace
  guard.release();
  *out = p;
  return PVR_OK;
  PVR_API_END();
}

// The plan's device state, in one fixed order: with a NULL base this only
// measures the workspace (the same calls size and carve it).
static size_t layout(pvr_plan *p, char *base, int flags) {
  WsCursor c{base, 0};
  const long long M = p->M, N = p->N, nb = p->n_bricks;
  p->d_prob = ws_take<ProbDev>(c, p->P);
  p->d_stack = ws_take<StackDev>(c, p->S);
  p->d_patch = ws_take<PatchDev>(c, M);
  p->d_sim_blocks = ws_take<BlockWork>(c, p->n_sim_blocks);
  p->d_tile_off = ws_take<int>(c, M + 1);
  p->d_box_max = ws_take<int>(c, 4);
  p->d_brick_prob = ws_take<int>(c, nb);
  p->d_plane_prob = ws_take<int>(c, p->n_planes + p->P);
  p->d_theta = ws_take<double>(c, 6 * M);
  p->d_geod = ws_take<GeoD>(c, M);
  p->d_geof = ws_take<GeoF>(c, M);
  p->d_bb = ws_take<int>(c, 6 * M);
  p->d_gbox = ws_take<int>(c, 6 * ((M + 63) / 64));
  p->d_scan = ws_take<long long>(c, (8 * nb + 4095) / 4096 + 1);
  p->d_sbox = ws_take<double>(c, 18 * M);
  p->d_invz = ws_take<float>(c, N);
  p->d_mask = ws_take<uint8_t>(c, N);
  p->d_active = ws_take<uint8_t>(c, M);
  p->d_bin_count = ws_take<int>(c, nb);
  p->d_bin_off = ws_take<int>(c, nb + 1);
  p->d_bin_patch = ws_take<int>(c, p->bin_cap);
  p->d_sub_count = ws_take<int>(c, 8 * nb);
  p->d_sub_off = ws_take<int>(c, 8 * nb + 1);
  p->d_sub_patch = ws_take<int>(c, p->sub_cap);
  // one guard entry (zero) before and after the N entries: the adjoint's
  // wide loads may pair a patch's first or last entry with its neighbour
  p->d_rq = ws_take<float2>(c, N + 2);
  p->d_pstat = ws_take<double>(c, 10 * M);
  p->d_pbar = ws_take<float>(c, M);
  p->d_pval = ws_take<float>(c, M);
  p->d_chunk_stats = ws_take<double>(c, 5LL * p->n_sim_blocks);
  p->d_xt = p->any_xt ? ws_take<float>(c, p->V) : nullptr;
  p->d_total = ws_take<int>(c, 4);
  p->d_reg_stats = ws_take<unsigned long long>(c, 4);
  p->d_status = ws_take<unsigned>(c, 1);
  p->d_dbg = ws_take<unsigned long long>(c, 1);
  p->d_invz64 = (flags & PVR_WS_F64) ? ws_take<double>(c, N) : nullptr;
  p->d_rq64 = (flags & PVR_WS_F64) ? ws_take<double2>(c, N + 2) : nullptr;
  return (c.off + 255) & ~(size_t)255;
}

extern "C" pvr_status pvr_plan_workspace_size(const pvr_plan *p, int32_t flags, size_t *bytes) {
  PVR_API_BEGIN();
  if (!p || !bytes) return fail(PVR_EINVAL, "pvr_plan_workspace_size: NULL argument");
  if (flags & ~PVR_WS_F64) return fail(PVR_EINVAL, "pvr_plan_workspace_size: unknown flags 0x%x", flags);
  pvr_plan q = *p;  // layout() writes pointers: measure on a copy
  *bytes = layout(&q, nullptr, flags);
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_plan_attach(pvr_plan *p, void *workspace, size_t bytes, int32_t flags,
                                      hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_plan_attach", workspace, 256);
  if (!p || !workspace) return fail(PVR_EINVAL, "pvr_plan_attach: NULL argument");
  if (flags & ~PVR_WS_F64) return fail(PVR_EINVAL, "pvr_plan_attach: unknown flags 0x%x", flags);
  {
    pvr_plan q = *p;
    const size_t need = layout(&q, nullptr, flags);
    if (bytes < need)
      return fail(PVR_ESHAPE, "pvr_plan_attach: workspace of %zu bytes, %zu needed", bytes, need);
  }
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (p->device >= 0 && dev != p->device)
    return fail(PVR_EINVAL, "pvr_plan_attach: device %d is current, the plan belongs to device %d",
                dev, p->device);
  if (p->attached) HIP_TRY(hipStreamSynchronize(stream));  // the old workspace may be in use
  if (!p->side) {
    HIP_TRY(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
  }
  p->device = dev;
  layout(p, (char *)workspace, flags);
  p->ws = workspace;
  p->ws_bytes = bytes;
  p->ws_flags = flags;
  const int M = p->M;
  HIP_TRY(hipMemcpyAsync(p->d_prob, p->h_prob, sizeof(ProbDev) * p->P, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(p->d_stack, p->h_stack, sizeof(StackDev) * p->S, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(p->d_patch, p->h_patch, sizeof(PatchDev) * M, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(p->d_sim_blocks, p->h_sim_blocks, sizeof(BlockWork) * p->n_sim_blocks,
                         hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(p->d_tile_off, p->h_tile_off, sizeof(int) * (M + 1), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(p->d_brick_prob, p->h_brick_prob, sizeof(int) * p->n_bricks,
                         hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(p->d_plane_prob, p->h_plane_prob, sizeof(int) * (p->n_planes + p->P),
                         hipMemcpyHostToDevice, stream));
  launch_fill_f32((float *)p->d_rq, 0.f, 2 * (p->N + 2), stream);
  if (p->d_rq64) launch_fill_f64((double *)p->d_rq64, 0.0, 2 * (p->N + 2), stream);
  launch_fill_i32((int *)p->d_status, 0, 1, stream);
  launch_fill_i32(p->d_total, 0, 4, stream);
  launch_fill_i32((int *)p->d_reg_stats, 0, 8, stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(stream));  // the uploads read pageable host tables of the plan
  p->attached = true;
  p->built = p->built64 = false;
  p->index_valid = false;
  p->stats_valid = false;
  p->rq_fresh = false;
  ++p->generation;
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
  out->n_bin_pairs = 0;
  if (p->attached && p->index_valid) {
    int tot[4];
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(tot, p->d_total, sizeof tot, hipMemcpyDeviceToHost));
    out->n_bin_pairs = tot[1];
  }
  out->device_bytes = p->attached ? (int64_t)p->ws_bytes : 0;
  out->bin_capacity = p->bin_cap;
  out->sub_capacity = p->sub_cap;
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

extern "C" const float *pvr_plan_inv_z(const pvr_plan *p) {
  return p && p->attached ? p->d_invz : nullptr;
}

// Forward tiles: every patch cut into tile_w x tile_h rectangles (edge tiles
// smaller), row of tiles after row of tiles; h_tile_off counts the tiles
// before each patch (a workgroup finds its tile with tile_at).
static pvr_status make_tiles(pvr_plan *p, int tile_w, int tile_h) {
  long long t = 0;
  for (int s = 0; s < p->M; ++s) {
    const PatchDev &q = p->h_patch[s];
    const int tw = std::min(q.w, tile_w), th = std::min(q.h, tile_h);
    p->h_tile_off[s] = (int)t;
    t += (long long)((q.w + tw - 1) / tw) * ((q.h + th - 1) / th);
    if (t > 0x7fffffffLL)
      return fail(PVR_ESHAPE, "forward tiles of %dx%d: more than 2^31 tiles", tile_w, tile_h);
  }
  p->h_tile_off[p->M] = (int)t;
  p->n_tiles = (int)t;
  p->tile_w = tile_w;
  p->tile_h = tile_h;
  return PVR_OK;
}

static pvr_status update_lds_box(pvr_plan *p, hipStream_t stream) {
  const int T = 256;
  launch_fill_i32(p->d_box_max, 0, 1, stream);
  hipLaunchKernelGGL(k_tile_boxmax, dim3((p->n_tiles + T - 1) / T), dim3(T), 0, stream, p->d_prob,
                     p->d_patch, p->d_tile_off, p->M, p->tile_w, p->tile_h, p->n_tiles, p->d_geof,
                     p->d_box_max);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(p->h_total + 2, p->d_box_max, sizeof(int), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  p->lds_box = std::min(p->h_total[2], LDS_BOX_MAX);
  return PVR_OK;
}

extern "C" pvr_status pvr_plan_set_psf(pvr_plan *p, int32_t kind) {
  PVR_API_BEGIN();
  if (!p) return fail(PVR_EINVAL, "pvr_plan_set_psf: plan is NULL");
  if (kind != PVR_PSF_GAUSSIAN && kind != PVR_PSF_SINC)
    return fail(PVR_EINVAL, "pvr_plan_set_psf: kind must be PVR_PSF_GAUSSIAN or PVR_PSF_SINC");
  p->psf = kind;
  // the adjoint's candidate grid follows the PSF's in-plane reach
  const double sk = sqrt(KAPPA), K2 = KAPPA * p->k * p->k;
  p->max_hu = p->max_hv = 0;
  for (int s = 0; s < p->S; ++s) {
    const StackDev &d = p->h_stack[s];
    const int hu = kind == PVR_PSF_SINC ? sinc_halfwidth(d.spacing[0] / d.wz[0])
                                        : cand_halfwidth(K2, sk * d.spacing[0] / d.sigma[0]);
    const int hv = kind == PVR_PSF_SINC ? sinc_halfwidth(d.spacing[1] / d.wz[1])
                                        : cand_halfwidth(K2, sk * d.spacing[1] / d.sigma[1]);
    p->max_hu = std::max(p->max_hu, hu);
    p->max_hv = std::max(p->max_hv, hv);
  }
  p->built = p->built64 = false;
  p->index_valid = false;
  p->stats_valid = false;
  p->rq_fresh = false;
  ++p->generation;
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_plan_set_tiles(pvr_plan *p, int32_t tile_w, int32_t tile_h,
                                         hipStream_t stream) {
  PVR_API_BEGIN();
  if (!p) return fail(PVR_EINVAL, "pvr_plan_set_tiles: plan is NULL");
  if (!p->attached) return fail(PVR_EINVAL, "pvr_plan_set_tiles: no workspace attached");
  ++p->generation;
  if (tile_w == 0 && tile_h == 0) {
    p->use_tiles = false;
    return PVR_OK;
  }
  if (tile_w <= 0 || tile_h <= 0 || tile_w * tile_h > 256)
    return fail(PVR_EINVAL, "pvr_plan_set_tiles: need 0 < tile_w * tile_h <= 256 (or 0 x 0)");
  HIP_TRY(hipStreamSynchronize(stream));  // earlier launches may still read the tile table
  const pvr_status st = make_tiles(p, tile_w, tile_h);
  if (st != PVR_OK) {
    p->use_tiles = false;
    return st;
  }
  HIP_TRY(hipMemcpyAsync(p->d_tile_off, p->h_tile_off, sizeof(int) * (p->M + 1),
                         hipMemcpyHostToDevice, stream));
  p->use_tiles = true;
  if (p->built) return update_lds_box(p, stream);
  HIP_TRY(hipStreamSynchronize(stream));
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_plan_set_granules(pvr_plan *p, int32_t sim_granule,
                                            int32_t bp_granule) {
  PVR_API_BEGIN();
  if (!p) return fail(PVR_EINVAL, "pvr_plan_set_granules: plan is NULL");
  if (sim_granule < 1 || sim_granule > 4096 || bp_granule < 1 || bp_granule > 4096)
    return fail(PVR_EINVAL, "pvr_plan_set_granules: granules must lie in [1, 4096]");
  p->sim_granule = sim_granule;
  p->bp_granule = bp_granule;
  ++p->generation;
  return PVR_OK;
  PVR_API_END();
}

// brick -> patch and sub-brick -> patch lists of the gather adjoint for the
// geometry of the last build, into lists of the capacities bounded at plan
// creation: no count is read back, nothing is synchronised.
pvr_status pvr::plan_build_index(pvr_plan *p, hipStream_t stream) {
  const int nb = p->n_bricks;
  const int nbw = (nb + BIN_THREADS / 64 - 1) / (BIN_THREADS / 64);
  hipLaunchKernelGGL(k_group_box, dim3((p->M + 255) / 256), dim3(256), 0, stream, p->d_bb, p->M,
                     p->d_gbox);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_bin_count, dim3(nbw), dim3(BIN_THREADS), 0, stream, p->d_prob,
                     p->d_brick_prob, p->d_bb, p->d_gbox, p->d_sbox, nb, p->d_bin_count);
  HIP_TRY(hipGetLastError());
  PVR_TRY_STATUS(launch_scan(p->d_bin_count, nb, p->d_scan, p->d_bin_off, p->d_total, p->bin_cap,
                             p->d_status, stream));
  hipLaunchKernelGGL(k_bin_fill, dim3(nbw), dim3(BIN_THREADS), 0, stream, p->d_prob,
                     p->d_brick_prob, p->d_bb, p->d_gbox, p->d_sbox, nb, p->d_bin_off,
                     p->d_bin_patch);
  HIP_TRY(hipGetLastError());
  const int nsb = nb * 8;
  hipLaunchKernelGGL(k_sub_count, dim3((nb + 3) / 4), dim3(256), 0, stream, p->d_prob,
                     p->d_brick_prob, p->d_sbox, nb, p->d_bin_off, p->d_bin_patch, p->d_sub_count);
  HIP_TRY(hipGetLastError());
  PVR_TRY_STATUS(launch_scan(p->d_sub_count, nsb, p->d_scan, p->d_sub_off, p->d_total + 1,
                             p->sub_cap, p->d_status, stream));
  hipLaunchKernelGGL(k_sub_fill, dim3((nb + 3) / 4), dim3(256), 0, stream, p->d_prob,
                     p->d_brick_prob, p->d_sbox, nb, p->d_bin_off, p->d_bin_patch, p->d_sub_off,
                     p->d_sub_patch);
  HIP_TRY(hipGetLastError());
  p->index_valid = true;
  ++p->generation;
  return PVR_OK;
}

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
                     p->d_patch, p->d_theta, M, p->k, p->psf, p->d_geod, p->d_geof, p->d_bb,
                     p->d_sbox);
  HIP_TRY(hipGetLastError());
  // an FP64 build also writes FP64 normalisers when the workspace has room
  // for them (PVR_WS_F64); the FP32 ones are written either way
  if (f64 && p->d_invz64) {
    hipLaunchKernelGGL(k_normalisers<double>, dim3(p->n_sim_blocks), dim3(SIM_THREADS), 0, stream,
                       p->d_prob, p->d_patch, p->d_sim_blocks, p->d_geod, p->d_mask, p->d_active,
                       p->d_invz, p->d_invz64);
  } else {
    hipLaunchKernelGGL(k_normalisers<float>, dim3(p->n_sim_blocks), dim3(SIM_THREADS), 0, stream,
                       p->d_prob, p->d_patch, p->d_sim_blocks, p->d_geof, p->d_mask, p->d_active,
                       p->d_invz, (double *)nullptr);
  }
  HIP_TRY(hipGetLastError());
  // forward-tile boxes (LDS size of the staged forward pass)
  if (p->use_tiles) {
    const pvr_status st = update_lds_box(p, stream);
    if (st != PVR_OK) return st;
  }
  p->index_valid = false;
  p->stats_valid = false;
  p->rq_fresh = false;
  p->built = true;
  p->built64 = f64 && p->d_invz64;
  ++p->generation;
  return PVR_OK;
}

extern "C" pvr_status pvr_plan_build(pvr_plan *p, const float *theta, const uint8_t *active,
                                     const uint8_t *sample_mask, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_plan_build", theta, 4);
  if (!p || !theta) return fail(PVR_EINVAL, "pvr_plan_build: NULL plan or theta");
  if (!p->attached) return fail(PVR_EINVAL, "pvr_plan_build: no workspace attached (pvr_plan_attach)");
  PVR_TRY_STATUS(debug_finite(p, "pvr_plan_build", "theta", theta, 6LL * p->M, stream));
  const int n = 6 * p->M;
  hipLaunchKernelGGL(k_theta_to_f64, dim3((n + 255) / 256), dim3(256), 0, stream, theta, p->d_theta, n);
  HIP_TRY(hipGetLastError());
  return plan_build_common(p, active, sample_mask, false, stream);
  PVR_API_END();
}

extern "C" pvr_status pvr_plan_build_f64(pvr_plan *p, const double *theta, const uint8_t *active,
                                         const uint8_t *sample_mask, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_plan_build_f64", theta, 8);
  if (!p || !theta) return fail(PVR_EINVAL, "pvr_plan_build_f64: NULL plan or theta");
  if (!p->attached) return fail(PVR_EINVAL, "pvr_plan_build_f64: no workspace attached (pvr_plan_attach)");
  PVR_TRY_STATUS(debug_finite(p, "pvr_plan_build_f64", "theta", theta, 6LL * p->M, stream));
  const int n = 6 * p->M;
  hipLaunchKernelGGL(k_copy_theta, dim3((n + 255) / 256), dim3(256), 0, stream, theta, p->d_theta, n);
  HIP_TRY(hipGetLastError());
  return plan_build_common(p, active, sample_mask, true, stream);
  PVR_API_END();
}
