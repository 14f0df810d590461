// Superpixel patch extraction: SLIC on every observed slice (see
// include/pvr_slic.h for the definition).  Assignment is a gather over pixel
// tiles: the centres that can reach a tile are listed in LDS, and every pixel
// keeps the least (D^2 as FP32 bits) << 32 | index over the list.  D^2 >= 0,
// so the bit patterns order like the values and the packed minimum is the
// least distance, ties to the lower index, whatever the order of the list.
// The update gathers too: one workgroup per centre sums the pixels of its
// window that carry its label.
#include <limits.h>
#include <math.h>
#include <stdint.h>

#include "pvr_internal.h"
#include "pvr_slic.h"
#include "pvr_util.h"

#include <algorithm>
#include <mutex>

using namespace pvr;

namespace {

constexpr int SLIC_T = 256;

__device__ __forceinline__ void cell_of(int k, int kx, int a, int h, int w, float &x, float &y) {
  const int i = k % kx, j = k / kx;
  x = 0.5f * (float)(i * a + min(w, (i + 1) * a) - 1);
  y = 0.5f * (float)(j * a + min(h, (j + 1) * a) - 1);
}

// window of a centre: integer pixel ranges with |x - cx| <= a, clipped to the
// image (empty when x0 > x1 or y0 > y1).  The centre is first clamped to a
// band around the image that leaves every window inside the image unchanged,
// so that any input (NaN, infinities, far-off centres) gives small integers.
__device__ __forceinline__ void window(float cx, float cy, int a, int h, int w, int &x0, int &x1,
                                       int &y0, int &y1) {
  const float fa = (float)a;
  cx = fminf(fmaxf(cx, -2.f * fa - 1.f), (float)w + 2.f * fa);
  cy = fminf(fmaxf(cy, -2.f * fa - 1.f), (float)h + 2.f * fa);
  x0 = max(0, (int)ceilf(cx - fa));
  x1 = min(w - 1, (int)floorf(cx + fa));
  y0 = max(0, (int)ceilf(cy - fa));
  y1 = min(h - 1, (int)floorf(cy + fa));
}

}  // namespace

__global__ void k_slic_init(const float *__restrict__ img, int n_img, int h, int w, int a, int kx,
                            int K, float t0, float *__restrict__ C) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n_img * K) return;
  const int im = (int)(t / K), k = (int)(t % K);
  float x, y;
  cell_of(k, kx, a, h, w, x, y);
  const int px = (int)floorf(x + 0.5f), py = (int)floorf(y + 0.5f);
  float *c = C + 4 * t;
  c[0] = x;
  c[1] = y;
  c[2] = img[((long long)im * h + py) * w + px];
  c[3] = t0;
}

// Largest distance of a centre from its grid cell's middle, per image: a
// centre whose window covers a pixel sits in a cell at most a + drift away.
__global__ void __launch_bounds__(SLIC_T)
k_slic_drift(const float *__restrict__ C, int h, int w, int a, int kx, int K,
             float *__restrict__ drift) {
  __shared__ float red[SLIC_T / 64];
  const int im = blockIdx.x;
  float d = 0.0f;
  for (int k = threadIdx.x; k < K; k += SLIC_T) {
    const float *c = C + 4 * ((long long)im * K + k);
    float gx, gy;
    cell_of(k, kx, a, h, w, gx, gy);
    const float e = fmaxf(fabsf(c[0] - gx), fabsf(c[1] - gy));
    d = (e == e) ? fmaxf(d, e) : INFINITY;  // a NaN centre widens the search to all cells
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) d = fmaxf(d, __shfl_xor(d, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = d;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < SLIC_T / 64; ++q) d = fmaxf(d, red[q]);
    drift[im] = fmaxf(d, red[0]);
  }
}

constexpr int TILE_X = 32, TILE_Y = SLIC_T / TILE_X;

struct Cand {
  float cx, cy, ci, s;
  int k;
};

// Assignment as a gather: one workgroup per TILE_X x TILE_Y pixel tile.  The
// centres whose window can reach the tile are found among the cells within
// a + drift of it and listed in LDS (a chunk of SLIC_T cells at a time), then
// every pixel takes the least packed (D^2 bits, index) over the list -- the
// same key and the same FP32 arithmetic for every (pixel, centre) pair
// whatever the order of the list.
__global__ void __launch_bounds__(SLIC_T)
k_slic_gather(const float *__restrict__ img, int h, int w, int a, int kx, int ky, int K,
              const float *__restrict__ C, const float *__restrict__ drift,
              int32_t *__restrict__ labels) {
  __shared__ Cand list[SLIC_T];
  __shared__ int n_list;
  const int im = blockIdx.y;
  const int tiles_x = (w + TILE_X - 1) / TILE_X;
  const int tx0 = (blockIdx.x % tiles_x) * TILE_X, ty0 = (blockIdx.x / tiles_x) * TILE_Y;
  const int tx1 = min(w, tx0 + TILE_X) - 1, ty1 = min(h, ty0 + TILE_Y) - 1;
  const int x = tx0 + (threadIdx.x % TILE_X), y = ty0 + (threadIdx.x / TILE_X);
  const bool inside = x <= tx1 && y <= ty1;
  const long long p = ((long long)im * h + y) * w + x;
  const float I = inside ? img[p] : 0.0f;
  // cells i whose middle (in [i a, i a + (a-1)/2]) lies within a + drift of the tile
  const float D = drift[im];
  int i0 = 0, i1 = kx - 1, j0 = 0, j1 = ky - 1;
  if (D <= 4.0f * (float)(h + w)) {
    const float r = (float)a + D + 1.0f;
    i0 = max(0, (int)floorf(((float)tx0 - r - 0.5f * (float)(a - 1)) / (float)a));
    i1 = min(kx - 1, (int)floorf(((float)tx1 + r) / (float)a));
    j0 = max(0, (int)floorf(((float)ty0 - r - 0.5f * (float)(a - 1)) / (float)a));
    j1 = min(ky - 1, (int)floorf(((float)ty1 + r) / (float)a));
  }
  const int ni = i1 - i0 + 1, ncand = (ni > 0 && j1 >= j0) ? ni * (j1 - j0 + 1) : 0;
  uint64_t best = ~0ull;
  for (int c0 = 0; c0 < ncand; c0 += SLIC_T) {
    if (threadIdx.x == 0) n_list = 0;
    __syncthreads();
    const int c = c0 + threadIdx.x;
    if (c < ncand) {
      const int k = (j0 + c / ni) * kx + i0 + c % ni;
      const float4 cc = *(const float4 *)(C + 4 * ((long long)im * K + k));
      // the window |x - cx| <= a meets the tile (one pixel of slack for rounding)
      if (cc.x - (float)a <= (float)(tx1 + 1) && cc.x + (float)a >= (float)(tx0 - 1) &&
          cc.y - (float)a <= (float)(ty1 + 1) && cc.y + (float)a >= (float)(ty0 - 1)) {
        const int slot = atomicAdd(&n_list, 1);
        list[slot] = Cand{cc.x, cc.y, cc.z, cc.w * cc.w / (float)(a * a), k};
      }
    }
    __syncthreads();
    const int n = n_list;
    for (int e = 0; e < n; ++e) {
      const Cand cd = list[e];
      const float dx = (float)x - cd.cx, dy = (float)y - cd.cy;
      if (!(fabsf(dx) <= (float)a && fabsf(dy) <= (float)a)) continue;
      const float dc = I - cd.ci;
      const float d2 = fmaf(dc, dc, (dx * dx + dy * dy) * cd.s);
      const uint64_t key = ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)cd.k;
      best = key < best ? key : best;
    }
    __syncthreads();
  }
  if (inside) labels[p] = best == ~0ull ? -1 : (int32_t)(best & 0xffffffffu);
}

// Update: one workgroup per centre over its window, one pass: count, FP64
// sums of x, y and I, and the extreme intensities (max |I - mean| is reached
// at one of them).  Waves take rows, lanes consecutive pixels of a row.
__global__ void __launch_bounds__(SLIC_T)
k_slic_update(const float *__restrict__ img, int h, int w, int a, int K,
              const int32_t *__restrict__ labels, float t_min, float *__restrict__ C) {
  __shared__ double lds[4][SLIC_T / 64];
  __shared__ float lim[2][SLIC_T / 64];
  const int im = blockIdx.y, k = blockIdx.x;
  float *c = C + 4 * ((long long)im * K + k);
  int x0, x1, y0, y1;
  window(c[0], c[1], a, h, w, x0, x1, y0, y1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long base = (long long)im * h * w;
  double s[4] = {0, 0, 0, 0};  // count, sum x, sum y, sum I
  float imax = -INFINITY, imin = INFINITY;
  for (int y = y0 + wave; y <= y1; y += SLIC_T / 64) {
    const long long row = base + (long long)y * w;
    for (int x = x0 + lane; x <= x1; x += 64) {
      if (labels[row + x] == k) {
        const float I = img[row + x];
        s[0] += 1.0;
        s[1] += (double)x;
        s[2] += (double)y;
        s[3] += (double)I;
        imax = fmaxf(imax, I);
        imin = fminf(imin, I);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double v = s[r];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) lds[r][wave] = v;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    imax = fmaxf(imax, __shfl_xor(imax, o, 64));
    imin = fminf(imin, __shfl_xor(imin, o, 64));
  }
  if (lane == 0) {
    lim[0][wave] = imax;
    lim[1][wave] = imin;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      t[r] = 0.0;
      for (int q = 0; q < SLIC_T / 64; ++q) t[r] += lds[r][q];
    }
    if (!(t[0] > 0)) return;  // no pixels: the centre stays
    for (int q = 0; q < SLIC_T / 64; ++q) {
      imax = fmaxf(imax, lim[0][q]);
      imin = fminf(imin, lim[1][q]);
    }
    const double mi = t[3] / t[0];
    const double dev = fmax((double)imax - mi, mi - (double)imin);
    c[0] = (float)(t[1] / t[0]);
    c[1] = (float)(t[2] / t[0]);
    c[2] = (float)mi;
    c[3] = (float)fmax(dev, (double)t_min);
  }
}

static pvr_status check_sizes(const char *fn, int n_img, int h, int w, int a) {
  // a = 0: no centre grid to check (pack)
  if (n_img <= 0 || h <= 0 || w <= 0 || a < 0) return fail(PVR_EINVAL, "%s: sizes must be positive", fn);
  if ((long long)n_img * h * w > (1LL << 31)) return fail(PVR_ESHAPE, "%s: more than 2^31 pixels", fn);
  if (h > (1 << 20) || w > (1 << 20)) return fail(PVR_ESHAPE, "%s: a side beyond 2^20 pixels", fn);
  const long long K = a > 0 ? (long long)((h + a - 1) / a) * ((w + a - 1) / a) : 0;
  if (K > (1 << 20)) return fail(PVR_ESHAPE, "%s: more than 2^20 centres per image", fn);
  if ((long long)n_img > 65535) return fail(PVR_ESHAPE, "%s: more than 65535 images", fn);
  return PVR_OK;
}

extern "C" int64_t pvr_slic_centres(int32_t h, int32_t w, int32_t a) {
  if (h <= 0 || w <= 0 || a <= 0) return 0;
  return (int64_t)((h + a - 1) / a) * ((w + a - 1) / a);
}

extern "C" pvr_status pvr_slic_init(const float *img, int32_t n_img, int32_t h, int32_t w,
                                    int32_t a, float t0, float *centres, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_slic_init", img, 4);
  PVR_ALIGNED("pvr_slic_init", centres, 16);
  if (!img || !centres) return fail(PVR_EINVAL, "pvr_slic_init: NULL argument");
  if (a <= 0 || a > (1 << 20)) return fail(PVR_EINVAL, "pvr_slic_init: a must be in [1, 2^20]");
  pvr_status st = check_sizes("pvr_slic_init", n_img, h, w, a);
  if (st != PVR_OK) return st;
  const int kx = (w + a - 1) / a, K = kx * ((h + a - 1) / a);
  const long long n = (long long)n_img * K;
  hipLaunchKernelGGL(k_slic_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, img,
                     n_img, h, w, a, kx, K, t0, centres);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_slic_assign(const float *img, int32_t n_img, int32_t h, int32_t w,
                                      int32_t a, const float *centres, uint64_t *ws,
                                      int32_t *labels, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_slic_assign", img, 4);
  PVR_ALIGNED("pvr_slic_assign", centres, 16);
  PVR_ALIGNED("pvr_slic_assign", ws, 8);
  PVR_ALIGNED("pvr_slic_assign", labels, 4);
  if (!img || !centres || !ws || !labels) return fail(PVR_EINVAL, "pvr_slic_assign: NULL argument");
  if (a <= 0 || a > (1 << 20)) return fail(PVR_EINVAL, "pvr_slic_assign: a must be in [1, 2^20]");
  pvr_status st = check_sizes("pvr_slic_assign", n_img, h, w, a);
  if (st != PVR_OK) return st;
  const int kx = (w + a - 1) / a, ky = (h + a - 1) / a, K = kx * ky;
  float *drift = (float *)ws;  // n_img floats
  hipLaunchKernelGGL(k_slic_drift, dim3(n_img), dim3(SLIC_T), 0, stream, centres, h, w, a, kx, K,
                     drift);
  const long long tiles = (long long)((w + TILE_X - 1) / TILE_X) * ((h + TILE_Y - 1) / TILE_Y);
  hipLaunchKernelGGL(k_slic_gather, dim3((unsigned)tiles, n_img), dim3(SLIC_T), 0, stream, img, h,
                     w, a, kx, ky, K, centres, drift, labels);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_slic_update(const float *img, int32_t n_img, int32_t h, int32_t w,
                                      int32_t a, const int32_t *labels, float t_min,
                                      float *centres, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_slic_update", img, 4);
  PVR_ALIGNED("pvr_slic_update", labels, 4);
  PVR_ALIGNED("pvr_slic_update", centres, 16);
  if (!img || !labels || !centres) return fail(PVR_EINVAL, "pvr_slic_update: NULL argument");
  if (a <= 0 || a > (1 << 20)) return fail(PVR_EINVAL, "pvr_slic_update: a must be in [1, 2^20]");
  pvr_status st = check_sizes("pvr_slic_update", n_img, h, w, a);
  if (st != PVR_OK) return st;
  const int K = ((w + a - 1) / a) * ((h + a - 1) / a);
  hipLaunchKernelGGL(k_slic_update, dim3(K, n_img), dim3(SLIC_T), 0, stream, img, h, w, a, K,
                     labels, t_min, centres);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_slic(const float *img, int32_t n_img, int32_t h, int32_t w, int32_t a,
                               float t0, float t_min, int32_t iters, uint64_t *ws,
                               float *centres, int32_t *labels, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_slic", img, 4);
  PVR_ALIGNED("pvr_slic", centres, 16);
  PVR_ALIGNED("pvr_slic", ws, 8);
  PVR_ALIGNED("pvr_slic", labels, 4);
  if (iters < 0) return fail(PVR_EINVAL, "pvr_slic: iters < 0");
  pvr_status st = pvr_slic_init(img, n_img, h, w, a, t0, centres, stream);
  for (int it = 0; st == PVR_OK && it < iters; ++it) {
    st = pvr_slic_assign(img, n_img, h, w, a, centres, ws, labels, stream);
    if (st == PVR_OK) st = pvr_slic_update(img, n_img, h, w, a, labels, t_min, centres, stream);
  }
  if (st == PVR_OK) st = pvr_slic_assign(img, n_img, h, w, a, centres, ws, labels, stream);
  return st;
  PVR_API_END();
}

// ---------------------------------------------------------------------------
// Superpixel patches: dilated bounding boxes and the packed samples.

__global__ void __launch_bounds__(SLIC_T)
k_slic_boxes(const int32_t *__restrict__ labels, int h, int w, int a, int K,
             const float *__restrict__ C, int gamma, int32_t *__restrict__ boxes) {
  __shared__ int red[4][SLIC_T / 64];
  const int im = blockIdx.y, k = blockIdx.x;
  const float *c = C + 4 * ((long long)im * K + k);
  int x0, x1, y0, y1;
  window(c[0], c[1], a, h, w, x0, x1, y0, y1);
  const int ww = x1 - x0 + 1, n = (ww > 0 && y1 >= y0) ? ww * (y1 - y0 + 1) : 0;
  const long long base = (long long)im * h * w;
  int b[4] = {INT_MAX, INT_MAX, INT_MIN, INT_MIN};  // min x, min y, max x, max y
  for (int q = threadIdx.x; q < n; q += SLIC_T) {
    const int x = x0 + q % ww, y = y0 + q / ww;
    if (labels[base + (long long)y * w + x] == k) {
      b[0] = min(b[0], x); b[1] = min(b[1], y);
      b[2] = max(b[2], x); b[3] = max(b[3], y);
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    b[0] = min(b[0], __shfl_xor(b[0], o, 64));
    b[1] = min(b[1], __shfl_xor(b[1], o, 64));
    b[2] = max(b[2], __shfl_xor(b[2], o, 64));
    b[3] = max(b[3], __shfl_xor(b[3], o, 64));
  }
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) red[r][wave] = b[r];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < SLIC_T / 64; ++q) {
      b[0] = min(b[0], red[0][q]); b[1] = min(b[1], red[1][q]);
      b[2] = max(b[2], red[2][q]); b[3] = max(b[3], red[3][q]);
    }
    int32_t *o = boxes + 4 * ((long long)im * K + k);
    if (b[2] < b[0]) {
      o[0] = o[1] = o[2] = o[3] = 0;
    } else {
      const int bx0 = max(0, b[0] - gamma), by0 = max(0, b[1] - gamma);
      const int bx1 = min(w - 1, b[2] + gamma), by1 = min(h - 1, b[3] + gamma);
      o[0] = bx0; o[1] = by0; o[2] = bx1 - bx0 + 1; o[3] = by1 - by0 + 1;
    }
  }
}

struct PackDesc {
  int32_t img, label, x0, y0, bw, bh;
  long long off;
};

constexpr int PACK_MAX_PIXELS = 65536;

// One workgroup per patch.  The label's indicator over the box sits in LDS as
// bit 0 of a byte; a sliding-window count along the rows gives the row
// dilation (bit 1), the same along the columns of bit 1 the square dilation
// (bit 2).
__global__ void __launch_bounds__(SLIC_T)
k_slic_pack(const float *__restrict__ img, const int32_t *__restrict__ labels, int h, int w,
            int gamma, const PackDesc *__restrict__ tab, float *__restrict__ y,
            uint8_t *__restrict__ mask) {
  extern __shared__ uint8_t bits[];
  const PackDesc d = tab[blockIdx.x];
  const int bw = d.bw, bh = d.bh, n = bw * bh;
  const long long base = (long long)d.img * h * w;
  for (int q = threadIdx.x; q < n; q += SLIC_T) {
    const long long p = base + (long long)(d.y0 + q / bw) * w + d.x0 + q % bw;
    bits[q] = labels[p] == d.label ? 1 : 0;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < bh; r += SLIC_T) {
    uint8_t *row = bits + r * bw;
    int cnt = 0;
    for (int x = 0; x < min(gamma, bw); ++x) cnt += row[x] & 1;
    for (int x = 0; x < bw; ++x) {
      if (x + gamma < bw) cnt += row[x + gamma] & 1;
      if (x - gamma - 1 >= 0) cnt -= row[x - gamma - 1] & 1;
      if (cnt > 0) row[x] |= 2;
    }
  }
  __syncthreads();
  for (int col = threadIdx.x; col < bw; col += SLIC_T) {
    uint8_t *cp = bits + col;
    int cnt = 0;
    for (int yy = 0; yy < min(gamma, bh); ++yy) cnt += (cp[yy * bw] >> 1) & 1;
    for (int yy = 0; yy < bh; ++yy) {
      if (yy + gamma < bh) cnt += (cp[(yy + gamma) * bw] >> 1) & 1;
      if (yy - gamma - 1 >= 0) cnt -= (cp[(yy - gamma - 1) * bw] >> 1) & 1;
      if (cnt > 0) cp[yy * bw] |= 4;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < n; q += SLIC_T) {
    const long long p = base + (long long)(d.y0 + q / bw) * w + d.x0 + q % bw;
    y[d.off + q] = img[p];
    mask[d.off + q] = (bits[q] >> 2) & 1;
  }
}

extern "C" pvr_status pvr_slic_boxes(const int32_t *labels, int32_t n_img, int32_t h, int32_t w,
                                     int32_t a, const float *centres, int32_t gamma,
                                     int32_t *boxes, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_slic_boxes", labels, 4);
  PVR_ALIGNED("pvr_slic_boxes", centres, 16);
  PVR_ALIGNED("pvr_slic_boxes", boxes, 4);
  if (!labels || !centres || !boxes) return fail(PVR_EINVAL, "pvr_slic_boxes: NULL argument");
  if (gamma < 0) return fail(PVR_EINVAL, "pvr_slic_boxes: gamma < 0");
  if (a <= 0 || a > (1 << 20)) return fail(PVR_EINVAL, "pvr_slic_boxes: a must be in [1, 2^20]");
  pvr_status st = check_sizes("pvr_slic_boxes", n_img, h, w, a);
  if (st != PVR_OK) return st;
  const int K = ((w + a - 1) / a) * ((h + a - 1) / a);
  hipLaunchKernelGGL(k_slic_boxes, dim3(K, n_img), dim3(SLIC_T), 0, stream, labels, h, w, a, K,
                     centres, gamma, boxes);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}

// Checks the host table of pvr_slic_pack and returns the largest box (pixels,
// the kernel's LDS bytes).
static pvr_status pack_check(const char *fn, int32_t n_img, int32_t h, int32_t w, int32_t M,
                             const int32_t *table, int *most) {
  *most = 0;
  for (int s = 0; s < M; ++s) {
    const int32_t *t = table + 6 * (size_t)s;
    if (t[0] < 0 || t[0] >= n_img || t[4] <= 0 || t[5] <= 0 || t[2] < 0 || t[3] < 0 ||
        t[2] > w - t[4] || t[3] > h - t[5])
      return fail(PVR_ESHAPE, "%s: patch %d (image %d, box %d,%d %dx%d) leaves its image", fn, s,
                  t[0], t[2], t[3], t[4], t[5]);
    if ((long long)t[4] * t[5] > PACK_MAX_PIXELS)
      return fail(PVR_ESHAPE, "%s: patch %d holds %lld pixels (at most %d)", fn, s,
                  (long long)t[4] * t[5], PACK_MAX_PIXELS);
    *most = std::max(*most, t[4] * t[5]);
  }
  return PVR_OK;
}

// Writes the M descriptors (with their sample offsets) into the device table
// `dtab` through a host staging array on the stack, one synchronised copy per
// PACK_STAGE descriptors, then launches the packing.  No memory is allocated.
constexpr int PACK_STAGE = 1024;

static pvr_status pack_launch(const float *img, const int32_t *labels, int32_t h, int32_t w,
                              int32_t gamma, int32_t M, const int32_t *table, int most,
                              PackDesc *dtab, float *y, uint8_t *mask, hipStream_t stream) {
  PackDesc stage[PACK_STAGE];
  long long off = 0;
  for (int s0 = 0; s0 < M; s0 += PACK_STAGE) {
    const int n = std::min(PACK_STAGE, M - s0);
    for (int i = 0; i < n; ++i) {
      const int32_t *t = table + 6 * (size_t)(s0 + i);
      stage[i] = PackDesc{t[0], t[1], t[2], t[3], t[4], t[5], off};
      off += (long long)t[4] * t[5];
    }
    HIP_TRY(hipMemcpyAsync(dtab + s0, stage, sizeof(PackDesc) * (size_t)n, hipMemcpyHostToDevice,
                           stream));
    HIP_TRY(hipStreamSynchronize(stream));  // the stage is reused / leaves scope
  }
  hipLaunchKernelGGL(k_slic_pack, dim3(M), dim3(SLIC_T), (size_t)most, stream, img, labels, h, w,
                     gamma, (const PackDesc *)dtab, y, mask);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
}

extern "C" size_t pvr_slic_pack_workspace(int32_t M) {
  return M > 0 ? sizeof(PackDesc) * (size_t)M : 0;
}

extern "C" pvr_status pvr_slic_pack(const float *img, const int32_t *labels, int32_t n_img,
                                    int32_t h, int32_t w, int32_t gamma, int32_t M,
                                    const int32_t *table, void *workspace, size_t workspace_bytes,
                                    float *y, uint8_t *mask, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_slic_pack", img, 4);
  PVR_ALIGNED("pvr_slic_pack", labels, 4);
  PVR_ALIGNED("pvr_slic_pack", y, 4);
  PVR_ALIGNED("pvr_slic_pack", workspace, 16);
  if (!img || !labels || !table || (M > 0 && (!y || !mask || !workspace)))
    return fail(PVR_EINVAL, "pvr_slic_pack: NULL argument");
  if (gamma < 0 || M < 0) return fail(PVR_EINVAL, "pvr_slic_pack: gamma < 0 or M < 0");
  pvr_status st = check_sizes("pvr_slic_pack", n_img, h, w, 0);
  if (st != PVR_OK) return st;
  if (M == 0) return PVR_OK;
  if (workspace_bytes < pvr_slic_pack_workspace(M))
    return fail(PVR_ESHAPE, "pvr_slic_pack: workspace of %zu bytes, %zu needed for %d patches",
                workspace_bytes, pvr_slic_pack_workspace(M), M);
  int most = 0;
  st = pack_check("pvr_slic_pack", n_img, h, w, M, table, &most);
  if (st != PVR_OK) return st;
  return pack_launch(img, labels, h, w, gamma, M, table, most, (PackDesc *)workspace, y, mask,
                     stream);
  PVR_API_END();
}

// ---------------------------------------------------------------------------
// pvr_slic_pack_noalloc: the same packing for callers that cannot allocate
// device memory.  The descriptor table lives in `scratch`, a file-scope
// device array of PVR_SLIC_PACK_NOALLOC_MAX entries; every device holds its
// own copy, whose address is looked up once per device.  In host code the
// array's name is only a host-side stand-in: the kernels receive the looked
// up device address.
// ---------------------------------------------------------------------------
static __device__ __align__(256) PackDesc scratch[PVR_SLIC_PACK_NOALLOC_MAX];

namespace {
constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
PackDesc *g_scratch_ptr[SCRATCH_DEVICES];  // device address of `scratch` per device
}  // namespace

static pvr_status scratch_on_current_device(PackDesc **out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_DEVICES)
    return fail(PVR_EUNSUPPORTED, "pvr_slic_pack_noalloc: device %d beyond %d", dev, SCRATCH_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(PVR_EHIP, "pvr_slic_pack_noalloc: no device address for the table");
    g_scratch_ptr[dev] = (PackDesc *)ptr;
  }
  *out = g_scratch_ptr[dev];
  return PVR_OK;
}

extern "C" pvr_status pvr_slic_pack_noalloc(const float *img, const int32_t *labels,
                                            int32_t n_img, int32_t h, int32_t w, int32_t gamma,
                                            int32_t M, const int32_t *table, float *y,
                                            uint8_t *mask, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_slic_pack_noalloc", img, 4);
  PVR_ALIGNED("pvr_slic_pack_noalloc", labels, 4);
  PVR_ALIGNED("pvr_slic_pack_noalloc", y, 4);
  if (!img || !labels || !table || (M > 0 && (!y || !mask)))
    return fail(PVR_EINVAL, "pvr_slic_pack_noalloc: NULL argument");
  if (gamma < 0 || M < 0) return fail(PVR_EINVAL, "pvr_slic_pack_noalloc: gamma < 0 or M < 0");
  if (M > PVR_SLIC_PACK_NOALLOC_MAX)
    return fail(PVR_ESHAPE, "pvr_slic_pack_noalloc: %d patches, at most %d", M,
                PVR_SLIC_PACK_NOALLOC_MAX);
  pvr_status st = check_sizes("pvr_slic_pack_noalloc", n_img, h, w, 0);
  if (st != PVR_OK) return st;
  if (M == 0) return PVR_OK;
  int most = 0;
  st = pack_check("pvr_slic_pack_noalloc", n_img, h, w, M, table, &most);
  if (st != PVR_OK) return st;
  PackDesc *tab = nullptr;
  st = scratch_on_current_device(&tab);
  if (st != PVR_OK) return st;
  st = pack_launch(img, labels, h, w, gamma, M, table, most, tab, y, mask, stream);
  if (st != PVR_OK) return st;
  HIP_TRY(hipStreamSynchronize(stream));  // the device's table is free again on return
  return PVR_OK;
  PVR_API_END();
}
