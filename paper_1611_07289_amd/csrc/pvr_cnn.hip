// Learned registration initialiser: a small 2D CNN that maps a pair
// (observed patch, patch simulated from the current volume) to a 6-DoF rigid
// correction.  Hand-written training and inference kernels for gfx950:
// convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 (BF16 operands,
// FP32 accumulation); pooling, head, loss and Adam run in FP32.
//
// Layouts: activations NHWC BF16 ([B][H][W][C]); conv weights BF16
// [Cout][3][3][Cin] for the forward pass and [3][3][Cin][Cout] for the data
// gradient, FP32 master copies [Cout][3][3][Cin]; gradients FP32.
//
// MFMA 16x16x32 lane layout (lane l, i = 0..7 for operands, 0..3 for the
// result): A row l%16, k = 8*(l/16)+i; B column l%16, k = 8*(l/16)+i;
// D column l%16, row 4*(l/16)+i.
#include <math.h>
#include <stdint.h>

#include "pvr_cnn.h"
#include "pvr_internal.h"
#include "pvr_util.h"

using namespace pvr;

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16) | ((u & 0xffff) ? 0x40 : 0);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

union V8 {
  uint4 u;
  bf16x8 v;
  uint16_t h[8];
};

__device__ __forceinline__ bf16x8 load8(const uint16_t *p) {
  V8 t;
  t.u = *reinterpret_cast<const uint4 *>(p);
  return t.v;
}
__device__ __forceinline__ bf16x8 zero8() {
  V8 t;
  t.u = make_uint4(0, 0, 0, 0);
  return t.v;
}

constexpr int CT = 256;  // threads per conv workgroup (4 waves)

}  // namespace

// ---------------------------------------------------------------------------
// forward: out = relu(conv3x3(in, W, stride S, pad 1) + bias)
// one wave = 32 output pixels x COUT channels
// ---------------------------------------------------------------------------
template <int CIN, int COUT, int S>
__global__ void __launch_bounds__(CT)
k_conv_fwd(const uint16_t *__restrict__ in, const uint16_t *__restrict__ W,
           const float *__restrict__ bias, uint16_t *__restrict__ out, int B, int H, int Wd,
           int relu) {
  constexpr int NT = COUT / 16;
  const int Ho = (H - 1) / S + 1, Wo = (Wd - 1) / S + 1;
  const long long P = (long long)B * Ho * Wo;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long pbase = ((long long)blockIdx.x * 4 + wave) * 32;
  if (pbase >= P) return;
  int pb[2], py[2], px[2];
  bool pv[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const long long p = pbase + mt * 16 + (lane & 15);
    pv[mt] = p < P;
    const long long pp = pv[mt] ? p : 0;
    pb[mt] = (int)(pp / (Ho * Wo));
    const int r = (int)(pp % (Ho * Wo));
    py[mt] = r / Wo;
    px[mt] = r % Wo;
  }
  f32x4 acc[2][NT];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = (f32x4){0.f, 0.f, 0.f, 0.f};
  const int kq = lane >> 4;  // which 8-wide k group
  if (CIN >= 32) {
    constexpr int CB = CIN / 32;
    for (int t = 0; t < 9 * CB; ++t) {
      const int tap = t / CB, cb = t % CB;
      const int ky = tap / 3, kx = tap % 3;
      const int ci0 = cb * 32 + 8 * kq;
      bf16x8 a[2];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        const int iy = py[mt] * S + ky - 1, ix = px[mt] * S + kx - 1;
        if (pv[mt] && iy >= 0 && iy < H && ix >= 0 && ix < Wd)
          a[mt] = load8(in + (((long long)pb[mt] * H + iy) * Wd + ix) * CIN + ci0);
        else
          a[mt] = zero8();
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int co = nt * 16 + (lane & 15);
        const bf16x8 b = load8(W + (long long)co * 9 * CIN + tap * CIN + ci0);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b, acc[mt][nt], 0, 0, 0);
      }
    }
  } else {
    // CIN < 32: the whole K = 9*CIN (<= 32) in one step, zero padded
    constexpr int K = 9 * CIN;
    bf16x8 a[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      V8 t;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = 8 * kq + i;
        uint16_t v = 0;
        if (k < K && pv[mt]) {
          const int tap = k / CIN, ci = k % CIN;
          const int iy = py[mt] * S + tap / 3 - 1, ix = px[mt] * S + tap % 3 - 1;
          if (iy >= 0 && iy < H && ix >= 0 && ix < Wd)
            v = in[(((long long)pb[mt] * H + iy) * Wd + ix) * CIN + ci];
        }
        t.h[i] = v;
      }
      a[mt] = t.v;
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int co = nt * 16 + (lane & 15);
      V8 t;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = 8 * kq + i;
        t.h[i] = k < K ? W[co * K + k] : (uint16_t)0;
      }
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], t.v, acc[mt][nt], 0, 0, 0);
    }
  }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int co = nt * 16 + (lane & 15);
      const float bb = bias[co];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long long p = pbase + mt * 16 + 4 * kq + i;
        if (p < P) {
          float v = acc[mt][nt][i] + bb;
          if (relu) v = v > 0.f ? v : 0.f;
          out[p * COUT + co] = f2bf(v);
        }
      }
    }
}

// ---------------------------------------------------------------------------
// data gradient: gin = conv^T(gpre), gpre = gout * [out > 0]
// M = input pixels, N = CIN, K = 9 * COUT; Wt = [3][3][CIN][COUT]
// ---------------------------------------------------------------------------
template <int CIN, int COUT, int S>
__global__ void __launch_bounds__(CT)
k_conv_dgrad(const uint16_t *__restrict__ gout, const uint16_t *__restrict__ out,
             const uint16_t *__restrict__ Wt, uint16_t *__restrict__ gin, int B, int H, int Wd) {
  constexpr int NT = CIN / 16;
  constexpr int CB = COUT / 32;
  const int Ho = (H - 1) / S + 1, Wo = (Wd - 1) / S + 1;
  const long long P = (long long)B * H * Wd;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long pbase = ((long long)blockIdx.x * 4 + wave) * 32;
  if (pbase >= P) return;
  int pb[2], py[2], px[2];
  bool pv[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const long long p = pbase + mt * 16 + (lane & 15);
    pv[mt] = p < P;
    const long long pp = pv[mt] ? p : 0;
    pb[mt] = (int)(pp / (H * Wd));
    const int r = (int)(pp % (H * Wd));
    py[mt] = r / Wd;
    px[mt] = r % Wd;
  }
  f32x4 acc[2][NT];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = (f32x4){0.f, 0.f, 0.f, 0.f};
  const int kq = lane >> 4;
  for (int t = 0; t < 9 * CB; ++t) {
    const int tap = t / CB, cb = t % CB;
    const int ky = tap / 3, kx = tap % 3;
    const int co0 = cb * 32 + 8 * kq;
    bf16x8 a[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const int ny = py[mt] + 1 - ky, nx = px[mt] + 1 - kx;  // = oy * S
      bool ok = pv[mt] && ny >= 0 && nx >= 0 && (ny % S) == 0 && (nx % S) == 0;
      const int oy = ny / S, ox = nx / S;
      ok = ok && oy < Ho && ox < Wo;
      if (ok) {
        const long long o = (((long long)pb[mt] * Ho + oy) * Wo + ox) * COUT + co0;
        V8 g, y;
        g.u = *reinterpret_cast<const uint4 *>(gout + o);
        y.u = *reinterpret_cast<const uint4 *>(out + o);
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (!(bf2f(y.h[i]) > 0.f)) g.h[i] = 0;
        a[mt] = g.v;
      } else {
        a[mt] = zero8();
      }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int ci = nt * 16 + (lane & 15);
      const bf16x8 b = load8(Wt + ((long long)tap * CIN + ci) * COUT + co0);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b, acc[mt][nt], 0, 0, 0);
    }
  }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int ci = nt * 16 + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long long p = pbase + mt * 16 + 4 * kq + i;
        if (p < P) gin[p * CIN + ci] = f2bf(acc[mt][nt][i]);
      }
    }
}

// ---------------------------------------------------------------------------
// weight gradient: dW[co][tap][ci] = sum_p gpre[p][co] in[p @ tap][ci]
// One workgroup = one chunk of WCH output pixels and one tap (all taps when
// CIN < 32: K columns = (tap, ci) flattened, padded to a multiple of 16).
// Partial sums per chunk go to part[chunk][...]; a second kernel adds the
// chunks in order (deterministic).
// ---------------------------------------------------------------------------
constexpr int WCH = 1024;

template <int CIN>
struct WCols {
  static constexpr int n = CIN >= 32 ? CIN : ((9 * CIN + 15) / 16) * 16;
};

template <int CIN, int COUT, int S>
__global__ void __launch_bounds__(CT)
k_conv_wgrad(const uint16_t *__restrict__ gout, const uint16_t *__restrict__ out,
             const uint16_t *__restrict__ in, float *__restrict__ part,
             float *__restrict__ bpart, int B, int H, int Wd) {
  constexpr int NC = WCols<CIN>::n;      // columns of this workgroup's dW block
  constexpr int TM = COUT / 16, TN = NC / 16;
  constexpr int TILES = TM * TN;
  constexpr int TPW = (TILES + 3) / 4;   // tiles per wave
  __shared__ uint16_t Lg[32][COUT + 8];  // gpre tile (pixel-major), padded rows
  __shared__ uint16_t Li[32][NC + 8];    // input tile at this tap
  const int Ho = (H - 1) / S + 1, Wo = (Wd - 1) / S + 1;
  const long long P = (long long)B * Ho * Wo;
  const int chunk = blockIdx.x;
  const int tap = CIN >= 32 ? blockIdx.y : 0;
  const int ky = tap / 3, kx = tap % 3;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, kq = lane >> 4;
  f32x4 acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) acc[q] = (f32x4){0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;  // bias gradient partial (thread < COUT), tap 0 only
  const long long p0 = (long long)chunk * WCH;
  for (int step = 0; step < WCH / 32; ++step) {
    const long long ps = p0 + step * 32;
    if (ps >= P) break;
    // stage gpre: 32 pixels x COUT
    for (int e = threadIdx.x; e < 32 * COUT; e += CT) {
      const int r = e / COUT, c = e % COUT;
      const long long p = ps + r;
      uint16_t v = 0;
      if (p < P) {
        const uint16_t y = out[p * COUT + c];
        if (bf2f(y) > 0.f) v = gout[p * COUT + c];
      }
      Lg[r][c] = v;
    }
    // stage the input: 32 pixels x NC columns
    for (int e = threadIdx.x; e < 32 * NC; e += CT) {
      const int r = e / NC, c = e % NC;
      const long long p = ps + r;
      uint16_t v = 0;
      if (p < P) {
        const int b = (int)(p / (Ho * Wo));
        const int rr = (int)(p % (Ho * Wo));
        const int oy = rr / Wo, ox = rr % Wo;
        int ci = c, tky = ky, tkx = kx;
        bool okc = true;
        if (CIN < 32) {
          okc = c < 9 * CIN;
          const int t2 = c / CIN;
          ci = c % CIN;
          tky = t2 / 3;
          tkx = t2 % 3;
        }
        const int iy = oy * S + tky - 1, ix = ox * S + tkx - 1;
        if (okc && iy >= 0 && iy < H && ix >= 0 && ix < Wd)
          v = in[(((long long)b * H + iy) * Wd + ix) * CIN + ci];
      }
      Li[r][c] = v;
    }
    __syncthreads();
    if (tap == 0 && threadIdx.x < COUT) {
      for (int r = 0; r < 32; ++r) bsum += bf2f(Lg[r][threadIdx.x]);
    }
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int tile = wave * TPW + q;
      if (tile < TILES) {
        const int tm = tile / TN, tn = tile % TN;
        V8 a, b;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          a.h[i] = Lg[8 * kq + i][tm * 16 + (lane & 15)];
          b.h[i] = Li[8 * kq + i][tn * 16 + (lane & 15)];
        }
        acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc[q], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // partial block: part[chunk][tap][co][col]
  const int taps = CIN >= 32 ? 9 : 1;
  float *dst = part + ((long long)chunk * taps + tap) * COUT * NC;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int tile = wave * TPW + q;
    if (tile < TILES) {
      const int tm = tile / TN, tn = tile % TN;
#pragma unroll
      for (int i = 0; i < 4; ++i) dst[(tm * 16 + 4 * kq + i) * NC + tn * 16 + (lane & 15)] = acc[q][i];
    }
  }
  if (tap == 0 && threadIdx.x < COUT) bpart[(long long)chunk * COUT + threadIdx.x] = bsum;
}

// dW[co][tap][ci] (FP32, layout of the master weights) = sum over chunks.
template <int CIN, int COUT>
__global__ void k_wgrad_reduce(const float *__restrict__ part, const float *__restrict__ bpart,
                               int n_chunks, float *__restrict__ dW, float *__restrict__ db) {
  constexpr int NC = WCols<CIN>::n;
  constexpr int taps = CIN >= 32 ? 9 : 1;
  const int K = 9 * CIN;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < COUT * K) {
    const int co = idx / K, k = idx % K;
    const int tap = CIN >= 32 ? k / CIN : 0;
    const int col = CIN >= 32 ? k % CIN : k;
    double s = 0;
    for (int c = 0; c < n_chunks; ++c)
      s += part[(((long long)c * taps + tap) * COUT + co) * NC + col];
    dW[idx] = (float)s;
  }
  if (idx < COUT) {
    double s = 0;
    for (int c = 0; c < n_chunks; ++c) s += bpart[(long long)c * COUT + idx];
    db[idx] = (float)s;
  }
}

// ---------------------------------------------------------------------------
// pair packing: channel 0 = observed patch, channel 1 = simulated patch, each
// normalised to zero mean / unit variance over the patch's valid samples
// (invalid samples 0).  One workgroup per pair; patches are 64 x 64.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_pack_pairs(const PatchDev *__restrict__ patches, const int *__restrict__ ids,
             const float *__restrict__ invz, const float *__restrict__ y,
             const float *__restrict__ ys, uint16_t *__restrict__ outp, int side) {
  __shared__ double red[5][4];
  const int bi = blockIdx.x;
  const PatchDev pt = patches[ids[bi]];
  const int n = side * side;
  double a[5] = {0, 0, 0, 0, 0};
  for (int l = threadIdx.x; l < n; l += 256) {
    const long long j = pt.off + l;
    if (invz[j] > 0.f) {
      const double u = y[j], v = ys[j];
      a[0] += 1; a[1] += u; a[2] += u * u; a[3] += v; a[4] += v * v;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double x = a[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) red[k][wave] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 5; ++k) a[k] = red[k][0] + red[k][1] + red[k][2] + red[k][3];
  const double c = a[0] > 0 ? a[0] : 1.0;
  const double m0 = a[1] / c, m1 = a[3] / c;
  const double s0 = sqrt(fmax(a[2] / c - m0 * m0, 0.0)) + 1e-3;
  const double s1 = sqrt(fmax(a[4] / c - m1 * m1, 0.0)) + 1e-3;
  for (int l = threadIdx.x; l < n; l += 256) {
    const long long j = pt.off + l;
    float u = 0.f, v = 0.f;
    if (invz[j] > 0.f) {
      u = (float)((y[j] - m0) / s0);
      v = (float)((ys[j] - m1) / s1);
    }
    const long long o = ((long long)bi * n + l) * 2;
    outp[o] = f2bf(u);
    outp[o + 1] = f2bf(v);
  }
}

// ---------------------------------------------------------------------------
// head: fully connected layer from the whole last feature map (hw positions
// x 64 channels, so the weights can depend on position) to 6 outputs,
// weighted squared loss and its gradients.  One workgroup of 256 lanes per
// sample; lane t owns the flattened inputs t, t + 256, ...
// ---------------------------------------------------------------------------
constexpr int HEAD_THREADS = 256;

__global__ void __launch_bounds__(HEAD_THREADS)
k_head(const uint16_t *__restrict__ act, int n_in, const float *__restrict__ Wfc,
       const float *__restrict__ bfc, const float *__restrict__ target,
       const float *__restrict__ lw, float *__restrict__ pred, float *__restrict__ loss_part,
       float *__restrict__ dp_out, uint16_t *__restrict__ gact, float inv_batch) {
  __shared__ float red[6][HEAD_THREADS / 64];
  __shared__ float dp[6];
  const int b = blockIdx.x, t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const uint16_t *a = act + (long long)b * n_in;
  float s[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int e = t; e < n_in; e += HEAD_THREADS) {
    const float x = bf2f(a[e]);
#pragma unroll
    for (int k = 0; k < 6; ++k) s[k] = fmaf(x, Wfc[e * 6 + k], s[k]);
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    float x = s[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) red[k][wave] = x;
  }
  __syncthreads();
  if (t < 6) {
    float o = bfc[t];
    for (int w = 0; w < HEAD_THREADS / 64; ++w) o += red[t][w];
    pred[b * 6 + t] = o;
    if (target) {
      const float d = o - target[b * 6 + t];
      dp[t] = lw[t] * d * inv_batch;
      dp_out[b * 6 + t] = dp[t];
      loss_part[b * 6 + t] = 0.5f * lw[t] * d * d * inv_batch;
    }
  }
  if (!target) return;
  __syncthreads();
  // dL/dact[e] = sum_k Wfc[e][k] dp[k]
  for (int e = t; e < n_in; e += HEAD_THREADS) {
    float g = 0.f;
#pragma unroll
    for (int k = 0; k < 6; ++k) g = fmaf(Wfc[e * 6 + k], dp[k], g);
    gact[(long long)b * n_in + e] = f2bf(g);
  }
}

// dL/dWfc[e][k] = sum_b act[b][e] dp[b][k] (samples in order), dL/dbfc[k] =
// sum_b dp[b][k]; one lane per input e (lanes n_in.. n_in + 5 take the bias).
__global__ void k_head_wgrad(const uint16_t *__restrict__ act, const float *__restrict__ dp,
                             int B, int n_in, float *__restrict__ dW, float *__restrict__ db) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n_in) {
    float g[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int b = 0; b < B; ++b) {
      const float x = bf2f(act[(long long)b * n_in + e]);
#pragma unroll
      for (int k = 0; k < 6; ++k) g[k] = fmaf(x, dp[b * 6 + k], g[k]);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) dW[e * 6 + k] = g[k];
  } else if (e < n_in + 6) {
    const int k = e - n_in;
    float g = 0.f;
    for (int b = 0; b < B; ++b) g += dp[b * 6 + k];
    db[k] = g;
  }
}

// sum of per-sample partials (fixed order)
__global__ void k_sum_rows(const float *__restrict__ part, int rows, int cols,
                           float *__restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0;
  for (int r = 0; r < rows; ++r) s += part[(long long)r * cols + c];
  out[c] = (float)s;
}

// ---------------------------------------------------------------------------
// Adam on FP32 master weights, refreshing the BF16 copies (forward layout
// [Cout][9][Cin] and, for conv layers, the transposed [9][Cin][Cout]).
// ---------------------------------------------------------------------------
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2, uint16_t *__restrict__ wb, uint16_t *__restrict__ wt,
                       int cout, int cin) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  if (wb) wb[i] = f2bf(wi);
  if (wt) {
    const int co = i / (9 * cin), k = i % (9 * cin);
    const int tap = k / cin, ci = k % cin;
    wt[((long long)tap * cin + ci) * cout + co] = f2bf(wi);
  }
}

__global__ void k_to_bf16(const float *__restrict__ w, int n, uint16_t *__restrict__ wb,
                          uint16_t *__restrict__ wt, int cout, int cin) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float wi = w[i];
  if (wb) wb[i] = f2bf(wi);
  if (wt) {
    const int co = i / (9 * cin), k = i % (9 * cin);
    const int tap = k / cin, ci = k % cin;
    wt[((long long)tap * cin + ci) * cout + co] = f2bf(wi);
  }
}

// ---------------------------------------------------------------------------
// host entry points
// ---------------------------------------------------------------------------
#define CONV_CASES(X)  \
  X(2, 32, 1)          \
  X(32, 32, 2)         \
  X(32, 64, 1)         \
  X(64, 64, 2)         \
  X(64, 64, 1)         \
  X(32, 32, 1)         \
  X(64, 32, 1)

static int out_size(int n, int s) { return (n - 1) / s + 1; }

extern "C" pvr_status pvr_cnn_conv_fwd(const uint16_t *in, const uint16_t *w, const float *bias,
                                       uint16_t *out, int32_t B, int32_t H, int32_t W,
                                       int32_t cin, int32_t cout, int32_t stride, int32_t relu,
                                       hipStream_t stream) {
  PVR_API_BEGIN();
  if (!in || !w || !bias || !out || B <= 0 || H <= 0 || W <= 0)
    return fail(PVR_EINVAL, "pvr_cnn_conv_fwd: invalid argument");
  const long long P = (long long)B * out_size(H, stride) * out_size(W, stride);
  const dim3 grid((unsigned)((P + 127) / 128));
#define LAUNCH(CI, CO, ST)                                                                     \
  if (cin == CI && cout == CO && stride == ST) {                                               \
    hipLaunchKernelGGL((k_conv_fwd<CI, CO, ST>), grid, dim3(CT), 0, stream, in, w, bias, out, \
                       B, H, W, relu);                                                         \
    HIP_TRY(hipGetLastError());                                                                \
    return PVR_OK;                                                                             \
  }
  CONV_CASES(LAUNCH)
#undef LAUNCH
  return fail(PVR_EUNSUPPORTED, "pvr_cnn_conv_fwd: no kernel for cin %d cout %d stride %d", cin,
              cout, stride);
  PVR_API_END();
}

extern "C" pvr_status pvr_cnn_conv_dgrad(const uint16_t *gout, const uint16_t *out,
                                         const uint16_t *wt, uint16_t *gin, int32_t B, int32_t H,
                                         int32_t W, int32_t cin, int32_t cout, int32_t stride,
                                         hipStream_t stream) {
  PVR_API_BEGIN();
  if (!gout || !out || !wt || !gin || B <= 0) return fail(PVR_EINVAL, "pvr_cnn_conv_dgrad: invalid argument");
  const long long P = (long long)B * H * W;
  const dim3 grid((unsigned)((P + 127) / 128));
#define LAUNCH(CI, CO, ST)                                                                       \
  if (cin == CI && cout == CO && stride == ST && CI >= 16) {                                     \
    hipLaunchKernelGGL((k_conv_dgrad<(CI >= 16 ? CI : 16), CO, ST>), grid, dim3(CT), 0, stream, \
                       gout, out, wt, gin, B, H, W);                                             \
    HIP_TRY(hipGetLastError());                                                                  \
    return PVR_OK;                                                                               \
  }
  CONV_CASES(LAUNCH)
#undef LAUNCH
  return fail(PVR_EUNSUPPORTED, "pvr_cnn_conv_dgrad: no kernel for cin %d cout %d stride %d", cin,
              cout, stride);
  PVR_API_END();
}

extern "C" int64_t pvr_cnn_wgrad_scratch(int32_t B, int32_t H, int32_t W, int32_t cin,
                                         int32_t cout, int32_t stride) {
  const long long P = (long long)B * out_size(H, stride) * out_size(W, stride);
  const long long chunks = (P + WCH - 1) / WCH;
  const int nc = cin >= 32 ? cin : ((9 * cin + 15) / 16) * 16;
  const int taps = cin >= 32 ? 9 : 1;
  return (chunks * taps * cout * nc + chunks * cout) * (long long)sizeof(float);
}

extern "C" pvr_status pvr_cnn_conv_wgrad(const uint16_t *gout, const uint16_t *out,
                                         const uint16_t *in, float *scratch, float *dw, float *db,
                                         int32_t B, int32_t H, int32_t W, int32_t cin,
                                         int32_t cout, int32_t stride, hipStream_t stream) {
  PVR_API_BEGIN();
  if (!gout || !out || !in || !scratch || !dw || !db || B <= 0)
    return fail(PVR_EINVAL, "pvr_cnn_conv_wgrad: invalid argument");
  const long long P = (long long)B * out_size(H, stride) * out_size(W, stride);
  const int chunks = (int)((P + WCH - 1) / WCH);
  const int nc = cin >= 32 ? cin : ((9 * cin + 15) / 16) * 16;
  const int taps = cin >= 32 ? 9 : 1;
  float *part = scratch;
  float *bpart = scratch + (long long)chunks * taps * cout * nc;
  const int nred = cout * 9 * cin;
#define LAUNCH(CI, CO, ST)                                                                       \
  if (cin == CI && cout == CO && stride == ST) {                                                 \
    hipLaunchKernelGGL((k_conv_wgrad<CI, CO, ST>), dim3(chunks, taps), dim3(CT), 0, stream, gout, \
                       out, in, part, bpart, B, H, W);                                           \
    HIP_TRY(hipGetLastError());                                                                  \
    hipLaunchKernelGGL((k_wgrad_reduce<CI, CO>), dim3((nred + 255) / 256), dim3(256), 0, stream, \
                       part, bpart, chunks, dw, db);                                             \
    HIP_TRY(hipGetLastError());                                                                  \
    return PVR_OK;                                                                               \
  }
  CONV_CASES(LAUNCH)
#undef LAUNCH
  return fail(PVR_EUNSUPPORTED, "pvr_cnn_conv_wgrad: no kernel for cin %d cout %d stride %d", cin,
              cout, stride);
  PVR_API_END();
}

extern "C" pvr_status pvr_cnn_pack_pairs(const pvr_plan *p, const int32_t *patch_ids, int32_t B,
                                         const float *y_obs, const float *y_sim, uint16_t *out,
                                         hipStream_t stream) {
  PVR_API_BEGIN();
  if (!p || !patch_ids || !y_obs || !y_sim || !out || B <= 0)
    return fail(PVR_EINVAL, "pvr_cnn_pack_pairs: invalid argument");
  if (!p->built) return fail(PVR_EINVAL, "pvr_cnn_pack_pairs: plan has not been built");
  for (int s = 0; s < p->M; ++s)
    if (p->h_patch[s].w != PVR_CNN_SIDE || p->h_patch[s].h != PVR_CNN_SIDE)
      return fail(PVR_ESHAPE, "pvr_cnn_pack_pairs: patch %d is not %dx%d", s, PVR_CNN_SIDE,
                  PVR_CNN_SIDE);
  hipLaunchKernelGGL(k_pack_pairs, dim3(B), dim3(256), 0, stream, p->d_patch, patch_ids, p->d_invz,
                     y_obs, y_sim, out, PVR_CNN_SIDE);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_cnn_head(const uint16_t *act, int32_t B, int32_t hw, const float *wfc,
                                   const float *bfc, const float *target, const float *loss_w,
                                   float *pred, float *loss, uint16_t *gact, float *dwfc,
                                   float *dbfc, float *scratch, hipStream_t stream) {
  PVR_API_BEGIN();
  if (!act || !wfc || !bfc || !pred || B <= 0 || hw <= 0) return fail(PVR_EINVAL, "pvr_cnn_head: invalid argument");
  if ((long long)hw * 64 > (1 << 24)) return fail(PVR_ESHAPE, "pvr_cnn_head: hw too large");
  if (target && (!loss_w || !loss || !gact || !dwfc || !dbfc || !scratch))
    return fail(PVR_EINVAL, "pvr_cnn_head: training needs loss weights, outputs and scratch");
  const int n_in = hw * 64;
  float *lp = scratch, *dp = scratch ? scratch + (long long)B * 6 : nullptr;
  hipLaunchKernelGGL(k_head, dim3(B), dim3(HEAD_THREADS), 0, stream, act, n_in, wfc, bfc, target,
                     loss_w, pred, lp, dp, gact, 1.0f / B);
  HIP_TRY(hipGetLastError());
  if (target) {
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(64), 0, stream, lp, B * 6, 1, loss);
    hipLaunchKernelGGL(k_head_wgrad, dim3((n_in + 6 + 255) / 256), dim3(256), 0, stream, act, dp,
                       B, n_in, dwfc, dbfc);
    HIP_TRY(hipGetLastError());
  }
  return PVR_OK;
  PVR_API_END();
}

extern "C" int64_t pvr_cnn_head_scratch(int32_t B) {
  return (long long)B * 12 * (long long)sizeof(float);
}

extern "C" pvr_status pvr_cnn_adam(float *w, const float *g, float *m, float *v, int32_t n,
                                   float lr, float beta1, float beta2, float eps, int32_t step,
                                   uint16_t *w_bf16, uint16_t *wt_bf16, int32_t cout, int32_t cin,
                                   hipStream_t stream) {
  PVR_API_BEGIN();
  if (!w || !m || !v || n <= 0 || step < 0) return fail(PVR_EINVAL, "pvr_cnn_adam: invalid argument");
  if (wt_bf16 && (cout <= 0 || cin <= 0 || cout * 9 * cin != n))
    return fail(PVR_EINVAL, "pvr_cnn_adam: transposed copy needs n = cout * 9 * cin");
  if (step == 0) {
    hipLaunchKernelGGL(k_to_bf16, dim3((n + 255) / 256), dim3(256), 0, stream, w, n, w_bf16,
                       wt_bf16, cout, cin);
  } else {
    if (!g) return fail(PVR_EINVAL, "pvr_cnn_adam: gradient is NULL");
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, stream, w, g, m, v, n, lr,
                       beta1, beta2, eps, c1, c2, w_bf16, wt_bf16, cout, cin);
  }
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}
