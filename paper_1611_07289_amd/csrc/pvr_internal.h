// Internal declarations of the PVR HIP library (gfx950, wave64).
//
// Data held by a plan:
//   ProbDev   one per reconstruction: grid, volume / brick / patch ranges
//   StackDev  one per stack: pixel -> world affine, unit axes, PSF sigmas
//   PatchDev  one per patch: stack, slice, rectangle, sample offset
//   GeoD/GeoF one per patch, rebuilt from theta: the moved sample-centre map
//             H (pixel -> voxel coordinates), its inverse G, the constants of
//             the PSF quadratic form in voxel offsets (forward direction) and
//             in pixel offsets (adjoint direction), and the brick range the
//             patch can touch.
//
// The PSF weight of voxel v for a sample centred at x is
//   g_hat = 2^(-Q') - 2^(-K2)   if Q' <= K2, else 0,
// with Q' = kappa * sum_a (d_a / sigma_a)^2, d = F^T (v - x), kappa =
// log2(e)/2 and K2 = kappa k^2, i.e. exp(-Q/2) - exp(-k^2/2) on the support
// sum (d_a/sigma_a)^2 <= k^2 (Gaussian PSF along the moved stack axes,
// continuous at the cut-off).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pvr.h"

namespace pvr {

constexpr int BRICK = 8;            // adjoint brick edge (voxels)
constexpr int SUB = 4;              // sub-brick edge: one wavefront of the adjoint
constexpr int SIM_CHUNK = 1024;     // samples per forward workgroup
constexpr int SIM_THREADS = 256;
constexpr double KAPPA = 0.72134752044448170368;  // log2(e) / 2

struct ProbDev {
  int nx, ny, nz;
  int nbx, nby, nbz;
  int brick_base, n_bricks;
  int patch_begin, patch_end;
  int chunk_begin, chunk_end;   // forward work chunks (BlockWork) of the problem
  long long vol_off;
  long long sample_begin, sample_end;
  double v2w[12];
  double w2v[12];
};

struct StackDev {
  int problem, nx, ny, ns;
  double p2w[12];
  double E[9];        // unit axes as columns (row-major 3x3)
  double spacing[3];  // column norms of the linear part
  double sigma[3];    // PSF standard deviations (mm)
  double wz[2];       // sinc PSF: in-plane first zeros (mm) = in-plane FWHM
};

struct PatchDev {
  int stack, slice, x0, y0, w, h, problem;
  int layout;  // volume copy the forward walks read: 0 = X (x fastest), 1 = y fastest
  long long off;
};

// Motion-dependent per-patch constants, double precision.
struct GeoD {
  double H[12];   // (u, v, slice, 1) -> voxel coords of the moved centre
  double G[12];   // voxel (i, j, k, 1) -> unmoved pixel coords (u, v, s)
  // forward quadratic form Q'(w) = w^T A w in voxel offsets w, permuted so
  // that axis c (inner loop) has the longest extent; a outer, b middle.
  double Acc, Aca, Acb, Saa, Sab, Sbb, iAinv_aa, ha;
  double inv_Acc, inv_Sbb, nSab_Sbb;
  double K2, cut;           // kappa k^2 and 2^-K2
  double cu, cv, ck;        // adjoint: sqrt(kappa) * spacing / sigma
  double inv_cu, inv_cv;
  double ext[3];            // support half-extent along voxel axes (voxels)
  int perm[3];
  int bb_lo[3], bb_hi[3];   // brick range (inclusive); empty if lo > hi
  int hu, hv;               // adjoint candidate half-widths (pixels)
  int psf;                  // PVR_PSF_GAUSSIAN or PVR_PSF_SINC
  double L[9];              // sinc PSF: voxel offset -> (t_u, t_v, t_n), row-major
  double kcut;              // k (the slice profile's cut in standard deviations)
};

// The same constants in single precision for the float kernels (G stays in
// double: it maps voxel indices of up to a few hundred to pixel coordinates
// whose fractional part sets the weights).
struct GeoF {
  double H[12];
  double G[12];
  float Acc, Aca, Acb, Saa, Sab, Sbb, iAinv_aa, ha;
  float inv_Acc, inv_Sbb, nSab_Sbb;
  float K2, cut;
  float cu, cv, ck, inv_cu, inv_cv;
  float ext[3];             // support half-extent along voxel axes (voxels)
  int perm[3];
  int hu, hv;               // adjoint candidate half-widths (pixels)
  int psf;                  // PVR_PSF_GAUSSIAN or PVR_PSF_SINC
  float L[9];               // sinc PSF: voxel offset -> (t_u, t_v, t_n), row-major
  float kcut;               // k
};

template <typename T> struct GeoOf;
template <> struct GeoOf<float> { using type = GeoF; };
template <> struct GeoOf<double> { using type = GeoD; };

struct BlockWork {   // one forward workgroup: a chunk of one patch
  int patch;
  int l0;            // first local sample
};

// Workgroups are dealt to the 8 XCDs round-robin by block index, and every
// XCD has its own L2.  xcd_work regroups the work list into granules of g
// consecutive items: XCD x takes granules x, x + 8, x + 16, ..., so the items
// of a granule (neighbouring chunks of a patch, neighbouring bricks) share one
// L2 while every XCD still sees a uniform mix of the whole list.  The grid
// has xcd_blocks(n, g) blocks; items >= n are empty.  g = 1 is the plain
// round-robin order.
constexpr int N_XCD = 8;
__host__ __device__ __forceinline__ int xcd_blocks(int n, int g) {
  return (n + N_XCD * g - 1) / (N_XCD * g) * (N_XCD * g);
}
__device__ __forceinline__ int xcd_work(int b, int g) {
  const int i = b / N_XCD;
  return (i / g) * (N_XCD * g) + (b % N_XCD) * g + i % g;
}
// default granules (pvr_plan_set_granules changes them per plan; the launch
// order changes, the results do not)
constexpr int SIM_XCD_GRANULE = 4;   // forward chunks (4 of 1024 samples, one 64x64 patch)
constexpr int BP_XCD_GRANULE = 32;   // adjoint bricks (a row of a 256^3 grid's bricks)

constexpr int TILE = 16;            // forward tile edge (pixels)
constexpr int LDS_BOX_MAX = 16384;  // staged voxels per forward workgroup (64 KiB)

struct TileWork {    // one forward workgroup: a rectangle of one patch
  int patch;
  short u0, v0, tw, th;  // patch-local origin and size (tw * th <= 256)
};

// Tile t of the forward tiling (tile_w x tile_h rectangles, edge tiles
// smaller, a patch's tiles row after row): its patch is the s with
// tile_off[s] <= t < tile_off[s + 1] (binary search over the M + 1 offsets).
__device__ __forceinline__ TileWork tile_at(const int *__restrict__ tile_off, int M,
                                            const PatchDev *__restrict__ patches, int tile_w,
                                            int tile_h, int t) {
  int lo = 0, hi = M;  // tile_off[lo] <= t < tile_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (tile_off[mid] <= t) lo = mid; else hi = mid;
  }
  const PatchDev pt = patches[lo];
  const int tw = min(pt.w, tile_w), th = min(pt.h, tile_h);
  const int ntx = (pt.w + tw - 1) / tw;
  const int l = t - tile_off[lo];
  const int u0 = (l % ntx) * tw, v0 = (l / ntx) * th;
  return TileWork{lo, (short)u0, (short)v0, (short)min(tw, pt.w - u0), (short)min(th, pt.h - v0)};
}

template <typename T> __device__ __forceinline__ T fast_exp2(T x);
template <> __device__ __forceinline__ float fast_exp2<float>(float x) {
  return __builtin_amdgcn_exp2f(x);
}
template <> __device__ __forceinline__ double fast_exp2<double>(double x) {
  return exp2(x);
}

__device__ __forceinline__ int sel3(int i, int a0, int a1, int a2) {
  return i == 0 ? a0 : (i == 1 ? a1 : a2);
}
template <typename T>
__device__ __forceinline__ T sel3f(int i, T a0, T a1, T a2) {
  return i == 0 ? a0 : (i == 1 ? a1 : a2);
}

// Moved centre of pixel (u, v) of patch geometry g in voxel coordinates,
// split into the nearest voxel b and the offset f = x - b (|f| <= 1/2).
// Returns whether the centre lies in the half-open box [-1/2, n - 1/2)^3.
template <typename GEO, typename T>
__device__ __forceinline__ bool sample_centre(const GEO &g, const ProbDev &p,
                                              int u, int v, int slice,
                                              int b[3], T f[3]) {
  double x[3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
    x[r] = fma(g.H[4 * r], (double)u,
               fma(g.H[4 * r + 1], (double)v,
                   fma(g.H[4 * r + 2], (double)slice, g.H[4 * r + 3])));
  bool in = x[0] >= -0.5 && x[0] < p.nx - 0.5 && x[1] >= -0.5 &&
            x[1] < p.ny - 0.5 && x[2] >= -0.5 && x[2] < p.nz - 0.5;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    double bb = rint(x[r]);
    b[r] = (int)bb;
    f[r] = (T)(x[r] - bb);
  }
  return in;
}

// Square root for the row bounds of the walks: in FP32 the hardware square
// root (about one ulp) widened by a relative 1e-6, so a row never loses a
// voxel of the support (a voxel the wider range adds lies outside it, where
// the clamped weight 2^-Q - 2^-K2 is 0); in FP64 the IEEE square root.
template <typename T> __device__ __forceinline__ T fast_sqrt(T x);
template <> __device__ __forceinline__ float fast_sqrt<float>(float x) {
  return __builtin_amdgcn_sqrtf(x) * 1.000001f;
}
template <> __device__ __forceinline__ double fast_sqrt<double>(double x) { return sqrt(x); }

// Walk the PSF support of one sample (nearest voxel b, offset f) over the
// voxels inside the grid and return sum g_hat and sum g_hat * X.  Rows along
// the inner axis c are enumerated exactly from the quadratic form: for the
// outer offset w_a the middle range comes from the Schur complement, for each
// (w_a, w_b) the inner range from the 1D quadratic in w_c.
// clo / chi: inclusive voxel bounds the walk is clipped to (the grid, or a
// staged box inside it); Xb points at voxel b in storage with strides
// (1, sy, sz).
template <typename T, typename GEO, bool HAS_X>
__device__ __forceinline__ void psf_walk_s(const GEO &g, const int clo[3], const int chi[3],
                                           const int b[3], const T f[3], const T *Xb, int sy,
                                           int sz, T &z, T &acc) {
  const int ia = g.perm[0], ib = g.perm[1], ic = g.perm[2];
  const int st_a = sel3(ia, 1, sy, sz), st_b = sel3(ib, 1, sy, sz), st_c = sel3(ic, 1, sy, sz);
  const int b_a = sel3(ia, b[0], b[1], b[2]), b_b = sel3(ib, b[0], b[1], b[2]),
            b_c = sel3(ic, b[0], b[1], b[2]);
  const T f_a = sel3f<T>(ia, f[0], f[1], f[2]), f_b = sel3f<T>(ib, f[0], f[1], f[2]),
          f_c = sel3f<T>(ic, f[0], f[1], f[2]);
  const T K2 = (T)g.K2, cut = (T)g.cut, Acc = (T)g.Acc, Aca = (T)g.Aca,
          Acb = (T)g.Acb, Saa = (T)g.Saa, Sab = (T)g.Sab, Sbb = (T)g.Sbb,
          iAaa = (T)g.iAinv_aa, ha = (T)g.ha, iAcc = (T)g.inv_Acc,
          iSbb = (T)g.inv_Sbb, nSab = (T)g.nSab_Sbb;
  const int lo_a = max((int)ceil(f_a - ha), sel3(ia, clo[0], clo[1], clo[2]) - b_a);
  const int hi_a = min((int)floor(f_a + ha), sel3(ia, chi[0], chi[1], chi[2]) - b_a);
  const int cl_b = sel3(ib, clo[0], clo[1], clo[2]) - b_b, ch_b = sel3(ib, chi[0], chi[1], chi[2]) - b_b;
  const int cl_c = sel3(ic, clo[0], clo[1], clo[2]) - b_c, ch_c = sel3(ic, chi[0], chi[1], chi[2]) - b_c;
  for (int oa = lo_a; oa <= hi_a; ++oa) {
    const T wa = (T)oa - f_a;
    const T rem = K2 - wa * wa * iAaa;
    if (rem < (T)0) continue;
    const T wbc = nSab * wa;
    const T rb = fast_sqrt<T>(rem * iSbb);
    const int lo_b = max((int)ceil(f_b + wbc - rb), cl_b);
    const int hi_b = min((int)floor(f_b + wbc + rb), ch_b);
    const T qa = Saa * wa * wa;
    const T sa2 = (T)2 * Sab * wa;
    for (int ob = lo_b; ob <= hi_b; ++ob) {
      const T wb = (T)ob - f_b;
      const T q1 = qa + wb * (sa2 + Sbb * wb);
      const T rem2 = K2 - q1;
      if (rem2 < (T)0) continue;
      const T wcc = -(Aca * wa + Acb * wb) * iAcc;
      const T rc = fast_sqrt<T>(rem2 * iAcc);
      const int lo_c = max((int)ceil(f_c + wcc - rc), cl_c);
      const int hi_c = min((int)floor(f_c + wcc + rc), ch_c);
      T d = ((T)lo_c - f_c) - wcc;
      int off = oa * st_a + ob * st_b + lo_c * st_c;
      for (int oc = lo_c; oc <= hi_c; ++oc) {
        const T Q = fma(Acc * d, d, q1);
        T gh = fast_exp2<T>(-Q) - cut;
        gh = gh > (T)0 ? gh : (T)0;
        z += gh;
        if (HAS_X) acc = fma(gh, Xb[off], acc);
        off += st_c;
        d += (T)1;
      }
    }
  }
}

// Walk over the global volume of problem p (X points at the problem's voxel 0).
template <typename T, typename GEO, bool HAS_X>
__device__ __forceinline__ void psf_walk(const GEO &g, const ProbDev &p, const int b[3],
                                         const T f[3], const T *__restrict__ X, T &z, T &acc) {
  const T *Xb = HAS_X ? X + ((long long)b[2] * p.ny + b[1]) * p.nx + b[0] : nullptr;
  const int clo[3] = {0, 0, 0}, chi[3] = {p.nx - 1, p.ny - 1, p.nz - 1};
  psf_walk_s<T, GEO, HAS_X>(g, clo, chi, b, f, Xb, p.nx, p.nx * p.ny, z, acc);
}

// Forward-only walk (the normaliser comes from the build): sum g_hat X over
// the support of one sample, X read through a raw buffer of the problem's
// volume.  Same enumeration as psf_walk_s, tuned for the simulation:
//  * each row's loads are issued four at a time before their use, so a
//    lane keeps several volume reads in flight instead of one;
//  * a buffer load never faults, so the group of four reads past the row
//    end without an address clamp (those voxels get weight 0);
//  * the row bounds use the hardware square root, widened by a relative
//    1e-6: voxels the wider range adds lie outside the support, where
//    2^-Q - 2^-K2 <= 0 clamps to 0.
// Raw buffer over `bytes` bytes from `base` (bytes < 2^32; the count is a
// 32-bit unsigned field of the resource).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_buffer(const void *base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)bytes, 0x00020000);
}
template <typename T> __device__ __forceinline__ T load_vox(__amdgpu_buffer_rsrc_t r, unsigned off);
template <> __device__ __forceinline__ float load_vox<float>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <> __device__ __forceinline__ double load_vox<double>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
// Four voxels of a row at byte offset off, stride step.  When the row runs
// along x (step of one float) and the four lie inside the buffer, one 16-byte
// load fetches them: a lane then touches one cache line per group instead of
// issuing four loads, which matters for stacks whose pixel rows run across
// x, where the 64 lanes of a wave hit 64 different lines.
// ROW: 1 = rows run along x (one float apart), 2 = they do not, 0 = decide
// from step at run time.
template <typename T, int ROW>
__device__ __forceinline__ void load_group(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned step,
                                           unsigned nbytes, T x[4]) {
  if constexpr (sizeof(T) == 4 && ROW != 2) {
    if ((ROW == 1 || step == 4) && off + 16 <= nbytes) {
      typedef float f4 __attribute__((ext_vector_type(4)));
      const f4 v = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
      x[0] = v.x;
      x[1] = v.y;
      x[2] = v.z;
      x[3] = v.w;
      return;
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) x[k] = load_vox<T>(r, off + (unsigned)k * step);
}

// max(x, 0) for x in [-1, 1] (the output clamp of the producing instruction)
template <typename T> __device__ __forceinline__ T clamp01(T x);
template <> __device__ __forceinline__ float clamp01<float>(float x) {
  return __builtin_amdgcn_fmed3f(x, 0.f, 1.f);
}
template <> __device__ __forceinline__ double clamp01<double>(double x) { return fmax(x, 0.0); }

// WITH_Z also sums the weights (the normaliser Z over in-volume voxels).
// xr views the problem's volume (nbytes bytes), x fastest, or with XT its
// y-fastest copy ((z nx + x) ny + y).  ROW as for load_group: 1 when the inner
// axis is the fastest one of the layout (g.perm[2] == 0, or 1 with XT).
template <typename T, typename GEO, bool WITH_Z = false, int ROW = 0, bool XT = false>
__device__ __forceinline__ T psf_walk_fwd(const GEO &g, const ProbDev &p, const int b[3],
                                          const T f[3], __amdgpu_buffer_rsrc_t xr,
                                          unsigned nbytes, T *z_out = nullptr) {
  const int sx = XT ? p.ny : 1, sy = XT ? 1 : p.nx, sz = p.nx * p.ny;
  const int ia = g.perm[0], ib = g.perm[1], ic = g.perm[2];
  const int st_a = sel3(ia, sx, sy, sz), st_b = sel3(ib, sx, sy, sz), st_c = sel3(ic, sx, sy, sz);
  const int b_a = sel3(ia, b[0], b[1], b[2]), b_b = sel3(ib, b[0], b[1], b[2]),
            b_c = sel3(ic, b[0], b[1], b[2]);
  const int n_a = sel3(ia, p.nx, p.ny, p.nz), n_b = sel3(ib, p.nx, p.ny, p.nz),
            n_c = sel3(ic, p.nx, p.ny, p.nz);
  const T f_a = sel3f<T>(ia, f[0], f[1], f[2]), f_b = sel3f<T>(ib, f[0], f[1], f[2]),
          f_c = sel3f<T>(ic, f[0], f[1], f[2]);
  const T K2 = (T)g.K2, cut = (T)g.cut, Acc = (T)g.Acc, Aca = (T)g.Aca,
          Acb = (T)g.Acb, Saa = (T)g.Saa, Sab = (T)g.Sab, Sbb = (T)g.Sbb,
          iAaa = (T)g.iAinv_aa, ha = (T)g.ha, iAcc = (T)g.inv_Acc,
          iSbb = (T)g.inv_Sbb, nSab = (T)g.nSab_Sbb;
  const int lo_a = max((int)ceil(f_a - ha), -b_a);
  const int hi_a = min((int)floor(f_a + ha), n_a - 1 - b_a);
  const int cl_b = -b_b, ch_b = n_b - 1 - b_b, cl_c = -b_c, ch_c = n_c - 1 - b_c;
  const int vb = b[0] * sx + b[1] * sy + b[2] * sz;
  const unsigned step = (unsigned)st_c * (unsigned)sizeof(T);
  T acc = (T)0, z = (T)0;
  for (int oa = lo_a; oa <= hi_a; ++oa) {
    const T wa = (T)oa - f_a;
    const T rem = K2 - wa * wa * iAaa;
    if (rem < (T)0) continue;
    const T wbc = nSab * wa;
    const T rb = fast_sqrt<T>(rem * iSbb);
    const int lo_b = max((int)ceil(f_b + wbc - rb), cl_b);
    const int hi_b = min((int)floor(f_b + wbc + rb), ch_b);
    const T qa = Saa * wa * wa;
    const T sa2 = (T)2 * Sab * wa;
    for (int ob = lo_b; ob <= hi_b; ++ob) {
      const T wb = (T)ob - f_b;
      const T q1 = qa + wb * (sa2 + Sbb * wb);
      const T rem2 = K2 - q1;
      if (rem2 < (T)0) continue;
      const T wcc = -(Aca * wa + Acb * wb) * iAcc;
      const T rc = fast_sqrt<T>(rem2 * iAcc);
      const int lo_c = max((int)ceil(f_c + wcc - rc), cl_c);
      const int hi_c = min((int)floor(f_c + wcc + rc), ch_c);
      const int n = hi_c - lo_c + 1;
      T d = ((T)lo_c - f_c) - wcc;
      unsigned off = (unsigned)(vb + oa * st_a + ob * st_b + lo_c * st_c) * (unsigned)sizeof(T);
      for (int k0 = 0; k0 < n; k0 += 4) {
        T x[4];
        load_group<T, ROW>(xr, off, step, nbytes, x);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const T Q = fma(Acc * d, d, q1);
          const T gh = k0 + k < n ? clamp01<T>(fast_exp2<T>(-Q) - cut) : (T)0;
          acc = fma(gh, x[k], acc);
          if (WITH_Z) z += gh;
          d += (T)1;
        }
        off += 4 * step;
      }
    }
  }
  if (WITH_Z) *z_out = z;
  return acc;
}

// s(t) = sin(pi t) / (pi t) for |t| <= 1 as a polynomial in y = (pi t)^2.
// FP32: degree 6, the Chebyshev interpolant of s on y in [0, pi^2] (nodes
// at the zeros of T_7 mapped onto the interval) in monomial form; it differs
// from s by less than 1e-9, far below the FP32 rounding of the Horner
// evaluation (about 1.5e-7 at worst over |t| <= 1).  FP64: the Taylor series
// sum_m (-1)^m y^m / (2m + 1)! through y^11 (the first omitted term,
// pi^24 / 25!, is below 6e-14).
template <typename T> __device__ __forceinline__ T sinc_poly(T t);
template <> __device__ __forceinline__ float sinc_poly<float>(float t) {
  const float y = (3.14159265358979f * t) * (3.14159265358979f * t);
  float s = 1.3611596572093987e-10f;
  s = fmaf(s, y, -2.4728366909698707e-08f);
  s = fmaf(s, y, 2.7535800199984806e-06f);
  s = fmaf(s, y, -1.9840530876535922e-04f);
  s = fmaf(s, y, 8.3333216607570648e-03f);
  s = fmaf(s, y, -1.6666665673255920e-01f);
  return fmaf(s, y, 1.0f);
}
template <> __device__ __forceinline__ double sinc_poly<double>(double t) {
  const double y = (3.141592653589793 * t) * (3.141592653589793 * t);
  double s = -3.8681701706306841e-23;             // -1 / 23!
  s = fma(s, y, 1.9572941063391263e-20);          //  1 / 21!
  s = fma(s, y, -8.2206352466243295e-18);         // -1 / 19!
  s = fma(s, y, 2.8114572543455208e-15);          //  1 / 17!
  s = fma(s, y, -7.6471637318198164e-13);         // -1 / 15!
  s = fma(s, y, 1.6059043836821613e-10);          //  1 / 13!
  s = fma(s, y, -2.5052108385441720e-08);         // -1 / 11!
  s = fma(s, y, 2.7557319223985893e-06);          //  1 / 9!
  s = fma(s, y, -1.9841269841269841e-04);         // -1 / 7!
  s = fma(s, y, 8.3333333333333333e-03);          //  1 / 5!
  s = fma(s, y, -1.6666666666666667e-01);         // -1 / 3!
  return fma(s, y, 1.0);
}

// Walk the support box of one sample for the sinc PSF (PVR_PSF_SINC): with
// t = L (voxel - centre), the support is |t_u| < 1, |t_v| < 1, |t_n| <= k.
// The outer axes a, b run over the box's voxel extents; along the inner axis
// c each row's range is the intersection of the three slabs (exact, then
// widened by 1e-4 voxel; the weight decides membership voxel by voxel).  The
// row's voxels are loaded four at a time (load_group; ROW and XT as for
// psf_walk_fwd).  Returns sum g_hat X (WITH_X) and sum g_hat in *z_out, over
// in-grid voxels.
template <typename T, typename GEO, bool WITH_X, int ROW = 0, bool XT = false>
__device__ __forceinline__ T psf_walk_sinc(const GEO &g, const ProbDev &p, const int b[3],
                                           const T f[3], __amdgpu_buffer_rsrc_t xr,
                                           unsigned nbytes, T *z_out) {
  const int sx = XT ? p.ny : 1, sy = XT ? 1 : p.nx, sz = p.nx * p.ny;
  const int ia = g.perm[0], ib = g.perm[1], ic = g.perm[2];
  const int st_a = sel3(ia, sx, sy, sz), st_b = sel3(ib, sx, sy, sz), st_c = sel3(ic, sx, sy, sz);
  const int b_a = sel3(ia, b[0], b[1], b[2]), b_b = sel3(ib, b[0], b[1], b[2]),
            b_c = sel3(ic, b[0], b[1], b[2]);
  const int n_a = sel3(ia, p.nx, p.ny, p.nz), n_b = sel3(ib, p.nx, p.ny, p.nz),
            n_c = sel3(ic, p.nx, p.ny, p.nz);
  const T f_a = sel3f<T>(ia, f[0], f[1], f[2]), f_b = sel3f<T>(ib, f[0], f[1], f[2]),
          f_c = sel3f<T>(ic, f[0], f[1], f[2]);
  T La[3], Lb[3], Lc[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    La[i] = (T)g.L[3 * i + ia];
    Lb[i] = (T)g.L[3 * i + ib];
    Lc[i] = (T)g.L[3 * i + ic];
  }
  const T Bd[3] = {(T)1, (T)1, (T)g.kcut};
  // the slab bounds along the inner axis scale by 1 / Lc: one division per
  // axis and sample instead of two per axis and row (the bounds are widened
  // below, so a last-place difference never drops a voxel of the support)
  T iLc[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) iLc[i] = fabs(Lc[i]) > (T)1e-20 ? (T)1 / Lc[i] : (T)0;
  const T cut = (T)g.cut, kap = (T)KAPPA;
  const T ea = (T)g.ext[ia], eb = (T)g.ext[ib];
  const int lo_a = max((int)ceil(f_a - ea), -b_a);
  const int hi_a = min((int)floor(f_a + ea), n_a - 1 - b_a);
  const int lo_b = max((int)ceil(f_b - eb), -b_b);
  const int hi_b = min((int)floor(f_b + eb), n_b - 1 - b_b);
  const int vb = b[0] * sx + b[1] * sy + b[2] * sz;
  const unsigned step = (unsigned)st_c * (unsigned)sizeof(T);
  T acc = (T)0, z = (T)0;
  for (int oa = lo_a; oa <= hi_a; ++oa) {
    const T wa = (T)oa - f_a;
    for (int ob = lo_b; ob <= hi_b; ++ob) {
      const T wb = (T)ob - f_b;
      T r[3];
      T lo = (T)-1e30, hi = (T)1e30;
      bool empty = false;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        r[i] = La[i] * wa + Lb[i] * wb;
        if (fabs(Lc[i]) > (T)1e-20) {
          const T t1 = (-Bd[i] - r[i]) * iLc[i], t2 = (Bd[i] - r[i]) * iLc[i];
          lo = fmax(lo, fmin(t1, t2));
          hi = fmin(hi, fmax(t1, t2));
        } else if (fabs(r[i]) > Bd[i]) {
          empty = true;
        }
      }
      if (empty || !(lo <= hi)) continue;
      const int lo_c = max((int)ceil(f_c + lo - (T)1e-4), -b_c);
      const int hi_c = min((int)floor(f_c + hi + (T)1e-4), n_c - 1 - b_c);
      const int n = hi_c - lo_c + 1;
      const T wc0 = (T)lo_c - f_c;
      T t0 = fma(Lc[0], wc0, r[0]), t1 = fma(Lc[1], wc0, r[1]), t2 = fma(Lc[2], wc0, r[2]);
      unsigned off = (unsigned)(vb + oa * st_a + ob * st_b + lo_c * st_c) * (unsigned)sizeof(T);
      for (int k0 = 0; k0 < n; k0 += 4) {
        T x[4];
        if (WITH_X) load_group<T, ROW>(xr, off, step, nbytes, x);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          T gz = fast_exp2<T>(-kap * t2 * t2) - cut;
          gz = gz > (T)0 ? gz : (T)0;
          const bool in = k0 + k < n && fabs(t0) < (T)1 && fabs(t1) < (T)1;
          const T gh = in ? sinc_poly<T>(t0) * sinc_poly<T>(t1) * gz : (T)0;
          if (WITH_X) acc = fma(gh, x[k], acc);
          z += gh;
          t0 += Lc[0];
          t1 += Lc[1];
          t2 += Lc[2];
        }
        off += 4 * step;
      }
    }
  }
  *z_out = z;
  return acc;
}

// Voxel box (inclusive, clipped to the grid, padded by one voxel) that holds
// the PSF supports of every sample of a tile: the tile's corner centres
// bound all its centres (the pixel -> voxel map is affine), and a support
// reaches ext voxels from its centre along each axis.  Returns the number of
// voxels (0 if the box is empty).
template <typename GEO>
__device__ __forceinline__ int tile_box(const GEO &g, const ProbDev &pr, const PatchDev &pt,
                                        const TileWork &tw, int lo[3], int hi[3]) {
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double u = pt.x0 + tw.u0 + ((q & 1) ? tw.tw - 1 : 0);
    const double v = pt.y0 + tw.v0 + ((q & 2) ? tw.th - 1 : 0);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const double x = g.H[4 * r] * u + g.H[4 * r + 1] * v + g.H[4 * r + 2] * pt.slice + g.H[4 * r + 3];
      mn[r] = fmin(mn[r], x);
      mx[r] = fmax(mx[r], x);
    }
  }
  const int n[3] = {pr.nx, pr.ny, pr.nz};
  int cnt = 1;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    lo[r] = max(0, (int)floor(mn[r] - (double)g.ext[r]) - 1);
    hi[r] = min(n[r] - 1, (int)ceil(mx[r] + (double)g.ext[r]) + 1);
    cnt *= max(0, hi[r] - lo[r] + 1);
  }
  return cnt;
}

// Per-thread-slot helpers for deterministic block reductions.
template <typename T, int NT>
__device__ __forceinline__ T block_sum(T v, T *lds) {
  const int tid = threadIdx.x;
  lds[tid] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) lds[tid] = lds[tid] + lds[tid + s];
    __syncthreads();
  }
  T r = lds[0];
  __syncthreads();
  return r;
}

}  // namespace pvr

// ---------------------------------------------------------------------------
// host-side plan object
// ---------------------------------------------------------------------------
namespace pvr {
constexpr int TIMING_KERNELS = 3;
constexpr int TIMING_CAP = 256;  // event pairs per kernel between reads
struct KernelTimer {
  hipEvent_t ev[TIMING_CAP][2];
  int n;
};
}  // namespace pvr

struct pvr_plan {
  int device;
  int P, S, M;
  int max_problem_patches;
  int max_hu, max_hv;         // adjoint candidate half-widths over all stacks
  long long N, V;
  int n_bricks;
  double k;
  // host copies (the device tables are uploaded from these by pvr_plan_attach)
  pvr::ProbDev *h_prob;
  pvr::StackDev *h_stack;
  pvr::PatchDev *h_patch;
  long long *h_sample_off;   // [M+1]
  long long *h_vol_off;      // [P+1]
  pvr::BlockWork *h_sim_blocks;  // [n_sim_blocks]
  int *h_brick_prob;         // [n_bricks]
  int *h_plane_prob;         // [n_planes + P]
  int *h_tile_off;           // [M+1] tiles before each patch (current tile shape)
  int n_sim_blocks;
  // caller's device workspace (pvr_plan_attach); every d_ pointer below lies
  // inside it.  The plan allocates no device memory.
  void *ws;
  size_t ws_bytes;
  int ws_flags;              // PVR_WS_* it was sized for
  bool attached;
  // device, static
  pvr::ProbDev *d_prob;
  pvr::StackDev *d_stack;
  pvr::PatchDev *d_patch;
  pvr::BlockWork *d_sim_blocks;
  int *d_tile_off;           // [M+1]
  int n_tiles, tile_w, tile_h;
  int sim_granule, bp_granule;  // XCD granules of the forward work and the adjoint bricks
  bool use_tiles;            // forward pass staged per tile in LDS (else global walk)
  bool timing;               // record event pairs around the hot kernels
  pvr::KernelTimer *timers;  // [TIMING_KERNELS] (created on first enable)
  int *d_box_max;            // [1] largest tile box (voxels) of the last build
  int lds_box;               // LDS floats reserved per forward workgroup
  int *d_brick_prob;         // [n_bricks]
  int *d_plane_prob;         // [n_planes] problem of each z-plane, then [P] first plane
  int n_planes, max_nx, max_ny;
  // device, per build
  double *d_theta;           // [M][6]
  pvr::GeoD *d_geod;
  pvr::GeoF *d_geof;
  float *d_invz;             // [N]
  double *d_invz64;          // [N] (workspaces with PVR_WS_F64)
  uint8_t *d_mask;           // [N]
  uint8_t *d_active;         // [M]
  int *d_bb;                 // [M][6] brick range per patch
  int *d_gbox;               // [ceil(M / 64)][6] union of the ranges of 64 consecutive patches
  long long *d_scan;         // block sums of the index scans
  double *d_sbox;            // [M][18] voxel->pixel map and pixel support box
  int *d_bin_count;          // [n_bricks]
  int *d_bin_off;            // [n_bricks + 1]
  int *d_bin_patch;          // [bin_cap]
  long long bin_cap;         // host bound on brick/patch pairs over all motions
  int *d_sub_count;          // [8 n_bricks]
  int *d_sub_off;            // [8 n_bricks + 1]
  int *d_sub_patch;          // [sub_cap]
  long long sub_cap;         // host bound on sub-brick/patch pairs
  bool built, built64, index_valid;
  // scratch
  float2 *d_rq;              // [N + 2]: zero guard, N entries, zero guard
  double2 *d_rq64;           // [N + 2] likewise (workspaces with PVR_WS_F64)
  double *d_pstat;           // [M][10] per-patch EM partials
  float *d_pbar;             // [M] potentials when the caller passes none
  float *d_pval;             // [M] classification scratch (problems beyond the LDS copy)
  double *d_chunk_stats;     // [n_sim_blocks][5] residual statistics of the last simulate
  float *d_xt;               // [V] y-fastest copy of the volume (plans with layout-1 patches)
  bool any_xt;
  int psf;                   // PVR_PSF_GAUSSIAN (default) or PVR_PSF_SINC
  const void *stats_resid, *stats_y;  // ... and the buffers they describe
  bool stats_valid;
  // adjoint inputs prepared by pvr_robust_weights (PVR_EM_PREP_ADJOINT) for
  // these residual / posterior buffers, on a second stream beside the
  // patch classification
  bool rq_fresh;
  const void *rq_e, *rq_p;
  hipStream_t side;
  hipEvent_t ev_fork, ev_join;
  unsigned *d_status;        // [1] fault flags (PVR_FAULT_*), read by pvr_check
  unsigned long long *d_dbg; // [1] first offending index of a debug-mode input check
  long long generation;      // bumped whenever launches recorded earlier would go stale
  int *d_total;              // [4] index totals: brick pairs, sub-brick pairs
  unsigned long long *d_reg_stats;  // [4] registration evaluations and samples walked
                                    // (plain, then exact gradient) since the last read
  int h_total[4];            // host readback
};

// Debug mode (pvr_set_debug, or PVR_DEBUG in the environment): input checks
// of the core entry points, run on the device before their launches.
// debug_finite rejects a non-finite element of a[0, n); debug_weights also a
// negative one.  Both are no-ops outside debug mode, for a null array and
// while the stream is captured into a graph.
namespace pvr {
bool debug_on();
pvr_status debug_finite(const pvr_plan *p, const char *fn, const char *what, const float *a,
                        long long n, hipStream_t stream);
pvr_status debug_finite(const pvr_plan *p, const char *fn, const char *what, const double *a,
                        long long n, hipStream_t stream);
pvr_status debug_weights(const pvr_plan *p, const char *fn, const char *what, const float *a,
                         long long n, hipStream_t stream);
pvr_status debug_weights(const pvr_plan *p, const char *fn, const char *what, const double *a,
                         long long n, hipStream_t stream);
}  // namespace pvr
