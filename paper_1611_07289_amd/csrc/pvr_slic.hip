// Superpixel patch extraction: SLIC on every observed slice (see
// include/pvr_slic.h for the definition).  Assignment is a scatter from the
// centres: one workgroup per (image, centre) walks the centre's 2a x 2a window
// and takes, per pixel, the atomic minimum of (D^2 as FP32 bits) << 32 |
// index.  D^2 >= 0, so the bit patterns order like the values and the packed
// minimum is the least distance, ties to the lower index, whatever the order
// the workgroups run in.  The update gathers: one workgroup per centre sums
// the pixels of its window that carry its label.
#include <limits.h>
#include <math.h>
#include <stdint.h>

#include "pvr_internal.h"
#include "pvr_slic.h"
#include "pvr_util.h"

#include <algorithm>
#include <vector>

using namespace pvr;

namespace {

constexpr int SLIC_T = 256;

__device__ __forceinline__ void cell_of(int k, int kx, int a, int h, int w, float &x, float &y) {
  const int i = k % kx, j = k / kx;
  x = 0.5f * (float)(i * a + min(w, (i + 1) * a) - 1);
  y = 0.5f * (float)(j * a + min(h, (j + 1) * a) - 1);
}

// window of a centre: integer pixel ranges with |x - cx| <= a, clipped
__device__ __forceinline__ void window(float cx, float cy, int a, int h, int w, int &x0, int &x1,
                                       int &y0, int &y1) {
  x0 = max(0, (int)ceilf(cx - (float)a));
  x1 = min(w - 1, (int)floorf(cx + (float)a));
  y0 = max(0, (int)ceilf(cy - (float)a));
  y1 = min(h - 1, (int)floorf(cy + (float)a));
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

__global__ void k_slic_fill(uint64_t *__restrict__ s, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) s[i] = ~0ull;
}

__global__ void __launch_bounds__(SLIC_T)
k_slic_scatter(const float *__restrict__ img, int h, int w, int a, int K,
               const float *__restrict__ C, uint64_t *__restrict__ best) {
  const int im = blockIdx.y, k = blockIdx.x;
  const float *c = C + 4 * ((long long)im * K + k);
  const float cx = c[0], cy = c[1], ci = c[2], tt = c[3];
  const float s = tt * tt / (float)(a * a);
  int x0, x1, y0, y1;
  window(cx, cy, a, h, w, x0, x1, y0, y1);
  const int ww = x1 - x0 + 1, n = ww * (y1 - y0 + 1);
  if (ww <= 0 || y1 < y0) return;
  const long long base = (long long)im * h * w;
  for (int q = threadIdx.x; q < n; q += SLIC_T) {
    const int x = x0 + q % ww, y = y0 + q / ww;
    const float dx = (float)x - cx, dy = (float)y - cy;
    if (!(fabsf(dx) <= (float)a && fabsf(dy) <= (float)a)) continue;
    const long long p = base + (long long)y * w + x;
    const float dc = img[p] - ci;
    const float d2 = fmaf(dc, dc, (dx * dx + dy * dy) * s);
    const uint64_t packed = ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)k;
    atomicMin((unsigned long long *)(best + p), (unsigned long long)packed);
  }
}

__global__ void k_slic_labels(const uint64_t *__restrict__ best, long long n,
                              int32_t *__restrict__ labels) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) labels[i] = best[i] == ~0ull ? -1 : (int32_t)(best[i] & 0xffffffffu);
}

// sum of RED values over the workgroup in a fixed order
template <int RED>
__device__ __forceinline__ void block_sum_d(double v[RED], double (*lds)[SLIC_T / 64]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < RED; ++r) {
    double x = v[r];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) lds[r][wave] = x;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RED; ++r) {
    double x = 0;
#pragma unroll
    for (int q = 0; q < SLIC_T / 64; ++q) x += lds[r][q];
    v[r] = x;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(SLIC_T)
k_slic_update(const float *__restrict__ img, int h, int w, int a, int K,
              const int32_t *__restrict__ labels, float t_min, float *__restrict__ C) {
  __shared__ double lds[4][SLIC_T / 64];
  const int im = blockIdx.y, k = blockIdx.x;
  float *c = C + 4 * ((long long)im * K + k);
  const float cx = c[0], cy = c[1];
  int x0, x1, y0, y1;
  window(cx, cy, a, h, w, x0, x1, y0, y1);
  const int ww = x1 - x0 + 1, n = (ww > 0 && y1 >= y0) ? ww * (y1 - y0 + 1) : 0;
  const long long base = (long long)im * h * w;
  double s[4] = {0, 0, 0, 0};  // count, sum x, sum y, sum I
  for (int q = threadIdx.x; q < n; q += SLIC_T) {
    const int x = x0 + q % ww, y = y0 + q / ww;
    const long long p = base + (long long)y * w + x;
    if (labels[p] == k) {
      s[0] += 1.0;
      s[1] += (double)x;
      s[2] += (double)y;
      s[3] += (double)img[p];
    }
  }
  block_sum_d<4>(s, lds);
  if (!(s[0] > 0)) return;  // uniform: every lane holds the same sums
  const double mi = s[3] / s[0];
  double m[1] = {0.0};
  for (int q = threadIdx.x; q < n; q += SLIC_T) {
    const int x = x0 + q % ww, y = y0 + q / ww;
    const long long p = base + (long long)y * w + x;
    if (labels[p] == k) m[0] = fmax(m[0], fabs((double)img[p] - mi));
  }
  // maximum over the workgroup (order-independent)
  {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double x = m[0];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
    if (lane == 0) lds[0][wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = lds[0][0];
      for (int q = 1; q < SLIC_T / 64; ++q) t = fmax(t, lds[0][q]);
      c[0] = (float)(s[1] / s[0]);
      c[1] = (float)(s[2] / s[0]);
      c[2] = (float)mi;
      c[3] = (float)fmax(t, (double)t_min);
    }
  }
}

static pvr_status check_sizes(const char *fn, int n_img, int h, int w, int a) {
  // a = 0: no centre grid to check (pack)
  if (n_img <= 0 || h <= 0 || w <= 0 || a < 0) return fail(PVR_EINVAL, "%s: sizes must be positive", fn);
  if ((long long)n_img * h * w > (1LL << 31)) return fail(PVR_ESHAPE, "%s: more than 2^31 pixels", fn);
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
  if (!img || !centres) return fail(PVR_EINVAL, "pvr_slic_init: NULL argument");
  if (a <= 0) return fail(PVR_EINVAL, "pvr_slic_init: a must be positive");
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
                                      int32_t a, const float *centres, uint64_t *scratch,
                                      int32_t *labels, hipStream_t stream) {
  PVR_API_BEGIN();
  if (!img || !centres || !scratch || !labels) return fail(PVR_EINVAL, "pvr_slic_assign: NULL argument");
  if (a <= 0) return fail(PVR_EINVAL, "pvr_slic_assign: a must be positive");
  pvr_status st = check_sizes("pvr_slic_assign", n_img, h, w, a);
  if (st != PVR_OK) return st;
  const int K = ((w + a - 1) / a) * ((h + a - 1) / a);
  const long long n = (long long)n_img * h * w;
  const unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_slic_fill, dim3(g), dim3(256), 0, stream, scratch, n);
  hipLaunchKernelGGL(k_slic_scatter, dim3(K, n_img), dim3(SLIC_T), 0, stream, img, h, w, a, K,
                     centres, scratch);
  hipLaunchKernelGGL(k_slic_labels, dim3(g), dim3(256), 0, stream, scratch, n, labels);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_slic_update(const float *img, int32_t n_img, int32_t h, int32_t w,
                                      int32_t a, const int32_t *labels, float t_min,
                                      float *centres, hipStream_t stream) {
  PVR_API_BEGIN();
  if (!img || !labels || !centres) return fail(PVR_EINVAL, "pvr_slic_update: NULL argument");
  if (a <= 0) return fail(PVR_EINVAL, "pvr_slic_update: a must be positive");
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
                               float t0, float t_min, int32_t iters, uint64_t *scratch,
                               float *centres, int32_t *labels, hipStream_t stream) {
  PVR_API_BEGIN();
  if (iters < 0) return fail(PVR_EINVAL, "pvr_slic: iters < 0");
  pvr_status st = pvr_slic_init(img, n_img, h, w, a, t0, centres, stream);
  for (int it = 0; st == PVR_OK && it < iters; ++it) {
    st = pvr_slic_assign(img, n_img, h, w, a, centres, scratch, labels, stream);
    if (st == PVR_OK) st = pvr_slic_update(img, n_img, h, w, a, labels, t_min, centres, stream);
  }
  if (st == PVR_OK) st = pvr_slic_assign(img, n_img, h, w, a, centres, scratch, labels, stream);
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
  if (!labels || !centres || !boxes) return fail(PVR_EINVAL, "pvr_slic_boxes: NULL argument");
  if (gamma < 0) return fail(PVR_EINVAL, "pvr_slic_boxes: gamma < 0");
  if (a <= 0) return fail(PVR_EINVAL, "pvr_slic_boxes: a must be positive");
  pvr_status st = check_sizes("pvr_slic_boxes", n_img, h, w, a);
  if (st != PVR_OK) return st;
  const int K = ((w + a - 1) / a) * ((h + a - 1) / a);
  hipLaunchKernelGGL(k_slic_boxes, dim3(K, n_img), dim3(SLIC_T), 0, stream, labels, h, w, a, K,
                     centres, gamma, boxes);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_slic_pack(const float *img, const int32_t *labels, int32_t n_img,
                                    int32_t h, int32_t w, int32_t gamma, int32_t M,
                                    const int32_t *table, float *y, uint8_t *mask,
                                    hipStream_t stream) {
  PVR_API_BEGIN();
  if (!img || !labels || !table || (M > 0 && (!y || !mask)))
    return fail(PVR_EINVAL, "pvr_slic_pack: NULL argument");
  if (gamma < 0 || M < 0) return fail(PVR_EINVAL, "pvr_slic_pack: gamma < 0 or M < 0");
  pvr_status st = check_sizes("pvr_slic_pack", n_img, h, w, 0);
  if (st != PVR_OK) return st;
  if (M == 0) return PVR_OK;
  std::vector<PackDesc> d(M);
  long long off = 0;
  int most = 0;
  for (int s = 0; s < M; ++s) {
    const int32_t *t = table + 6 * (size_t)s;
    if (t[0] < 0 || t[0] >= n_img || t[4] <= 0 || t[5] <= 0 || t[2] < 0 || t[3] < 0 ||
        t[2] > w - t[4] || t[3] > h - t[5])
      return fail(PVR_ESHAPE, "pvr_slic_pack: patch %d (image %d, box %d,%d %dx%d) leaves its image",
                  s, t[0], t[2], t[3], t[4], t[5]);
    if ((long long)t[4] * t[5] > PACK_MAX_PIXELS)
      return fail(PVR_ESHAPE, "pvr_slic_pack: patch %d holds %lld pixels (at most %d)", s,
                  (long long)t[4] * t[5], PACK_MAX_PIXELS);
    d[s] = PackDesc{t[0], t[1], t[2], t[3], t[4], t[5], off};
    off += (long long)t[4] * t[5];
    most = std::max(most, t[4] * t[5]);
  }
  PackDesc *dd = nullptr;
  HIP_TRY(hipMalloc((void **)&dd, sizeof(PackDesc) * (size_t)M));
  hipError_t e = hipMemcpyAsync(dd, d.data(), sizeof(PackDesc) * (size_t)M,
                                hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_slic_pack, dim3(M), dim3(SLIC_T), (size_t)most, stream, img, labels, h,
                       w, gamma, dd, y, mask);
    e = hipGetLastError();
  }
  const hipError_t e2 = hipStreamSynchronize(stream);
  (void)hipFree(dd);
  HIP_TRY(e);
  HIP_TRY(e2);
  return PVR_OK;
  PVR_API_END();
}
