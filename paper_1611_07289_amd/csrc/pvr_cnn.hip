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
//
// Implicit GEMM with the weights as the A operand (M = COUT) and the
// gathered input as B (N = output pixels), K = 9 CIN, so that each lane ends
// with four consecutive channels of one pixel and stores them as one 8-byte
// word: no LDS staging of the output and no barrier inside the tile loop.
// The layer's weights are staged once per workgroup into LDS, rows of K padded
// by 8 elements; the workgroup (16 waves) then loops over tiles of 256 output
// pixels, one 16-pixel MFMA column block per wave, so each weight is read from
// memory once per workgroup.  The B operand is gathered from global memory, 8
// channels (16 bytes) of one input pixel per lane per tap, zero outside the
// image; all taps are loaded before the first MFMA so that their latencies
// overlap.
// ---------------------------------------------------------------------------
constexpr int FW_THREADS = 1024;                       // 16 waves share the staged weights
constexpr int FW_TILE = (FW_THREADS / 64) * 16;       // 16 output pixels per wave

template <int CIN, int COUT>
struct FwdShape {
  static constexpr int K = 9 * CIN;
  static constexpr int KP = K < 32 ? 32 : K;  // K padded to one MFMA step when CIN < 32
  static constexpr int LS = KP + 8;           // LDS row stride (elements), 16-byte rows
  static constexpr int LDS_BYTES = COUT * LS * 2;
};

// bias, ReLU, BF16: lane (kq, r16) holds channels nt*16 + 4kq .. +3 of
// pixel p, one 8-byte store per 16-channel block
template <int COUT, int NT>
__device__ __forceinline__ void conv_store(uint16_t *__restrict__ out, long long p, int kq,
                                           const f32x4 (&acc)[NT], const float (&bb)[NT][4],
                                           int relu) {
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    uint16_t h4[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float v = acc[nt][i] + bb[nt][i];
      if (relu) v = v > 0.f ? v : 0.f;
      h4[i] = f2bf(v);
    }
    const uint2 wv = make_uint2((uint32_t)h4[0] | ((uint32_t)h4[1] << 16),
                                (uint32_t)h4[2] | ((uint32_t)h4[3] << 16));
    *reinterpret_cast<uint2 *>(out + p * COUT + nt * 16 + 4 * kq) = wv;
  }
}

template <int CIN, int COUT, int S>
__global__ void __launch_bounds__(FW_THREADS)
k_conv_fwd(const uint16_t *__restrict__ in, const uint16_t *__restrict__ W,
           const float *__restrict__ bias, uint16_t *__restrict__ out, int B, int H, int Wd,
           int relu) {
  using SH = FwdShape<CIN, COUT>;
  constexpr int NT = COUT / 16, K = SH::K, KP = SH::KP, LS = SH::LS;
  __shared__ __attribute__((aligned(16))) uint16_t Wl[COUT * LS];
  if constexpr (K % 8 == 0) {
    for (int e = threadIdx.x; e < COUT * (K / 8); e += FW_THREADS) {
      const int co = e / (K / 8), k8 = e % (K / 8);
      *reinterpret_cast<uint4 *>(&Wl[co * LS + 8 * k8]) =
          *reinterpret_cast<const uint4 *>(W + (long long)co * K + 8 * k8);
    }
  } else {
    for (int e = threadIdx.x; e < COUT * KP; e += FW_THREADS) {
      const int co = e / KP, k = e % KP;
      Wl[co * LS + k] = k < K ? W[co * K + k] : (uint16_t)0;
    }
  }
  __syncthreads();
  const int Ho = (H - 1) / S + 1, Wo = (Wd - 1) / S + 1;
  const long long P = (long long)B * Ho * Wo;
  const long long n_tiles = (P + FW_TILE - 1) / FW_TILE;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kq = lane >> 4, r16 = lane & 15;
  float bb[NT][4];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i) bb[nt][i] = bias[nt * 16 + 4 * kq + i];
  // U tiles per wave and pass, their loads all issued before the first MFMA
  // (2 and 4 were measured no faster than 1 on the 64x64 layers)
  constexpr int U = 1;
  for (long long t0 = blockIdx.x; t0 < n_tiles; t0 += (long long)U * gridDim.x) {
    long long pu[U];
    bool act[U], pv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long tile = t0 + (long long)u * gridDim.x;
      const long long pbase = tile * FW_TILE + wave * 16;
      act[u] = tile < n_tiles && pbase < P;  // wave-uniform
      pu[u] = pbase + r16;
      pv[u] = act[u] && pu[u] < P;
    }
    if constexpr (CIN >= 32) {
      constexpr int CB = CIN / 32, T = 9 * CB;
      bf16x8 a[U][T];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long pp = pv[u] ? pu[u] : 0;
        const int pb = (int)(pp / (Ho * Wo));
        const int rr = (int)(pp % (Ho * Wo));
        const int py = rr / Wo, px = rr % Wo;
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const int tap = t / CB, cb = t % CB;
          const int iy = py * S + tap / 3 - 1, ix = px * S + tap % 3 - 1;
          if (pv[u] && iy >= 0 && iy < H && ix >= 0 && ix < Wd)
            a[u][t] = load8(in + (((long long)pb * H + iy) * Wd + ix) * CIN + cb * 32 + 8 * kq);
          else
            a[u][t] = zero8();
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!act[u]) continue;
        f32x4 acc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const int tap = t / CB, cb = t % CB;
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const bf16x8 w = *reinterpret_cast<const bf16x8 *>(
                &Wl[(nt * 16 + r16) * LS + tap * CIN + cb * 32 + 8 * kq]);
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, a[u][t], acc[nt], 0, 0, 0);
          }
        }
        if (pv[u]) conv_store<COUT, NT>(out, pu[u], kq, acc, bb, relu);
      }
    } else {
      // K = 9 CIN <= 32: the whole K in one step, zero padded
      V8 ta[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long pp = pv[u] ? pu[u] : 0;
        const int pb = (int)(pp / (Ho * Wo));
        const int rr = (int)(pp % (Ho * Wo));
        const int py = rr / Wo, px = rr % Wo;
        if constexpr (CIN == 2) {
          // lane group kq holds taps 4 kq .. 4 kq + 3, both channels (one dword each)
          uint32_t d[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int tap = 4 * kq + j;
            const int iy = py * S + tap / 3 - 1, ix = px * S + tap % 3 - 1;
            d[j] = (pv[u] && tap < 9 && iy >= 0 && iy < H && ix >= 0 && ix < Wd)
                       ? *reinterpret_cast<const uint32_t *>(in + (((long long)pb * H + iy) * Wd + ix) * 2)
                       : 0u;
          }
          ta[u].u = make_uint4(d[0], d[1], d[2], d[3]);
        } else {
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int k = 8 * kq + i;
            uint16_t v = 0;
            if (k < K && pv[u]) {
              const int tap = k / CIN, ci = k % CIN;
              const int iy = py * S + tap / 3 - 1, ix = px * S + tap % 3 - 1;
              if (iy >= 0 && iy < H && ix >= 0 && ix < Wd)
                v = in[(((long long)pb * H + iy) * Wd + ix) * CIN + ci];
            }
            ta[u].h[i] = v;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!act[u]) continue;
        f32x4 acc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const bf16x8 w = *reinterpret_cast<const bf16x8 *>(&Wl[(nt * 16 + r16) * LS + 8 * kq]);
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, ta[u].v, (f32x4){0.f, 0.f, 0.f, 0.f},
                                                            0, 0, 0);
        }
        if (pv[u]) conv_store<COUT, NT>(out, pu[u], kq, acc, bb, relu);
      }
    }
  }
}

// Persistent grid: as many workgroups as fit on the chip at once with the
// layer's LDS, at most one per tile.
static unsigned persistent_grid(long long n_tiles, int lds_bytes) {
  int per_cu = (150 * 1024) / (lds_bytes > 0 ? lds_bytes : 1);
  per_cu = per_cu < 1 ? 1 : (per_cu > 2 ? 2 : per_cu);  // 1024-thread workgroups
  const long long cap = 256LL * per_cu;
  return (unsigned)(n_tiles < cap ? n_tiles : cap);
}

// ---------------------------------------------------------------------------
// data gradient: gin = conv^T(gpre), gpre = gout * [out > 0]
// M = input pixels, N = CIN, K = 9 * COUT; Wt = [3][3][CIN][COUT], staged
// into LDS as rows of K per input channel; tiles and persistence as the
// forward pass.
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
struct DgradShape {
  static constexpr int K = 9 * COUT;
  static constexpr int LS = K + 8;
  static constexpr int LDS_BYTES = CIN * LS * 2;
};

template <int CIN, int COUT, int S>
__global__ void __launch_bounds__(FW_THREADS)
k_conv_dgrad(const uint16_t *__restrict__ gout, const uint16_t *__restrict__ out,
             const uint16_t *__restrict__ Wt, uint16_t *__restrict__ gin, int B, int H, int Wd) {
  using SH = DgradShape<CIN, COUT>;
  constexpr int NT = CIN / 16;
  constexpr int CB = COUT / 32, T = 9 * CB;
  constexpr int LS = SH::LS;
  __shared__ __attribute__((aligned(16))) uint16_t Wl[CIN * LS];
  for (int e = threadIdx.x; e < 9 * CIN * (COUT / 8); e += FW_THREADS) {
    const int co8 = e % (COUT / 8), r = e / (COUT / 8);  // r = tap * CIN + ci
    const int tap = r / CIN, ci = r % CIN;
    *reinterpret_cast<uint4 *>(&Wl[ci * LS + tap * COUT + 8 * co8]) =
        *reinterpret_cast<const uint4 *>(Wt + (long long)r * COUT + 8 * co8);
  }
  __syncthreads();
  const int Ho = (H - 1) / S + 1, Wo = (Wd - 1) / S + 1;
  const long long P = (long long)B * H * Wd;
  const long long n_tiles = (P + FW_TILE - 1) / FW_TILE;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kq = lane >> 4, r16 = lane & 15;
  for (long long tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const long long pbase = tile * FW_TILE + wave * 16;
    if (pbase >= P) continue;  // wave-uniform; no barrier below
    const long long p = pbase + r16;
    const bool pv = p < P;
    const long long pp = pv ? p : 0;
    const int pb = (int)(pp / (H * Wd));
    const int rr = (int)(pp % (H * Wd));
    const int py = rr / Wd, px = rr % Wd;
    f32x4 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = (f32x4){0.f, 0.f, 0.f, 0.f};
    bf16x8 a[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int tap = t / CB, cb = t % CB;
      const int ny = py + 1 - tap / 3, nx = px + 1 - tap % 3;  // = oy * S
      bool ok = pv && ny >= 0 && nx >= 0 && (ny % S) == 0 && (nx % S) == 0;
      const int oy = ny / S, ox = nx / S;
      ok = ok && oy < Ho && ox < Wo;
      if (ok) {
        const long long o = (((long long)pb * Ho + oy) * Wo + ox) * COUT + cb * 32 + 8 * kq;
        V8 g, y;
        g.u = *reinterpret_cast<const uint4 *>(gout + o);
        y.u = *reinterpret_cast<const uint4 *>(out + o);
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (!(bf2f(y.h[i]) > 0.f)) g.h[i] = 0;
        a[t] = g.v;
      } else {
        a[t] = zero8();
      }
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int tap = t / CB, cb = t % CB;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(
            &Wl[(nt * 16 + r16) * LS + tap * COUT + cb * 32 + 8 * kq]);
        // weights as the A operand (M = CIN): lane (kq, r16) ends with input
        // channels nt*16 + 4kq .. +3 of pixel p
        acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, a[t], acc[nt], 0, 0, 0);
      }
    }
    if (pv) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const uint2 wv = make_uint2((uint32_t)f2bf(acc[nt][0]) | ((uint32_t)f2bf(acc[nt][1]) << 16),
                                    (uint32_t)f2bf(acc[nt][2]) | ((uint32_t)f2bf(acc[nt][3]) << 16));
        *reinterpret_cast<uint2 *>(gin + p * CIN + nt * 16 + 4 * kq) = wv;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// weight gradient: dW[co][tap][ci] = sum_p gpre[p][co] in[p @ tap][ci]
// GEMM with M = COUT, N = taps x NC columns (tap, input channel; when
// CIN < 32 the columns are (tap, ci) flattened and padded to 32 with one
// "tap"), K = output pixels.  One workgroup (16 waves) takes a chunk of
// pixels and every (co, tap, ci) tile.  Per step, each of KSPLIT wave groups
// stages 32 pixels into LDS, transposed so that both MFMA operands are
// 16-byte reads of 8 consecutive pixels: G[co][px] (gpre, with the ReLU mask)
// and I[tap][column][px] (the input at every tap, zero outside the image).
// The waves of a group share the group's tiles; each group writes its own
// partial block (row chunk * KSPLIT + group), which k_wgrad_reduce adds in
// order (deterministic).
// ---------------------------------------------------------------------------
template <int CIN>
struct WCols {
  static constexpr int n = CIN >= 32 ? CIN : ((9 * CIN + 15) / 16) * 16;
};

template <int CIN, int COUT>
struct WgradShape {
  static constexpr int NC = WCols<CIN>::n;
  static constexpr int TAPS = CIN >= 32 ? 9 : 1;
  static constexpr int TM = COUT / 16, TN = TAPS * NC / 16, TILES = TM * TN;
  static constexpr int KSPLIT = TILES >= 144 ? 1 : TILES >= 72 ? 2 : TILES >= 36 ? 4 : 16;
  static constexpr int WPG = 16 / KSPLIT;                 // waves per group
  static constexpr int TPW = (TILES + WPG - 1) / WPG;     // tiles per wave
  static constexpr int PS = 40;                           // LDS row stride (32 pixels + 8)
  static constexpr int G_ELEMS = COUT * PS, I_ELEMS = TAPS * NC * PS;
  static constexpr long long REC = (long long)TAPS * COUT * NC;  // floats per partial block
};

// Pixels per chunk (a multiple of 32 KSPLIT), chosen for about 256 chunks.
static long long wgrad_chunk(long long P, int ksplit) {
  const long long step = 32LL * ksplit;
  long long c = (P + 255) / 256;
  c = (c + step - 1) / step * step;
  return c < step ? step : c;
}

template <int CIN, int COUT, int S>
__global__ void __launch_bounds__(1024)
k_conv_wgrad(const uint16_t *__restrict__ gout, const uint16_t *__restrict__ out,
             const uint16_t *__restrict__ in, float *__restrict__ part,
             float *__restrict__ bpart, int B, int H, int Wd, long long wch) {
  using SH = WgradShape<CIN, COUT>;
  constexpr int NC = SH::NC, TAPS = SH::TAPS, TN = SH::TN, TILES = SH::TILES;
  constexpr int KSPLIT = SH::KSPLIT, WPG = SH::WPG, TPW = SH::TPW, PS = SH::PS;
  __shared__ __attribute__((aligned(16))) uint16_t Gs[KSPLIT * SH::G_ELEMS];
  __shared__ __attribute__((aligned(16))) uint16_t Is[KSPLIT * SH::I_ELEMS];
  const int Ho = (H - 1) / S + 1, Wo = (Wd - 1) / S + 1;
  const long long P = (long long)B * Ho * Wo;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kq = lane >> 4, r16 = lane & 15;
  const int kg = wave / WPG, wl = wave % WPG;
  if (CIN < 32) {
    // the padding columns (tap, ci) >= 9 CIN stay zero
    for (int e = threadIdx.x; e < KSPLIT * SH::I_ELEMS; e += 1024) Is[e] = 0;
    __syncthreads();
  }
  f32x4 acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) acc[q] = (f32x4){0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;  // bias partial of (group kg, channel wl * 64 + lane) when < COUT
  const long long p0 = (long long)blockIdx.x * wch;
  const long long p1 = p0 + wch < P ? p0 + wch : P;
  for (long long ps = p0; ps < p1; ps += 32 * KSPLIT) {
    // stage gpre (masked by the ReLU) transposed: Gs[g][co][px]
    for (int e = threadIdx.x; e < KSPLIT * 32 * (COUT / 8); e += 1024) {
      const int c8 = e % (COUT / 8), r = e / (COUT / 8);  // r = g * 32 + px
      const int g = r / 32, px = r % 32;
      const long long p = ps + r;
      V8 gv;
      gv.u = make_uint4(0, 0, 0, 0);
      if (p < p1) {
        V8 y;
        gv.u = *reinterpret_cast<const uint4 *>(gout + p * COUT + 8 * c8);
        y.u = *reinterpret_cast<const uint4 *>(out + p * COUT + 8 * c8);
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (!(bf2f(y.h[i]) > 0.f)) gv.h[i] = 0;
      }
      uint16_t *dst = Gs + g * SH::G_ELEMS + (8 * c8) * PS + px;
#pragma unroll
      for (int i = 0; i < 8; ++i) dst[i * PS] = gv.h[i];
    }
    // stage the input at every tap transposed: Is[g][tap][col][px]
    if constexpr (CIN >= 32) {
      for (int e = threadIdx.x; e < KSPLIT * 9 * 32 * (CIN / 8); e += 1024) {
        const int c8 = e % (CIN / 8), r = e / (CIN / 8);  // r = (g * 9 + tap) * 32 + px
        const int px = r % 32, gt = r / 32;
        const int tap = gt % 9, g = gt / 9;
        const long long p = ps + g * 32 + px;
        V8 iv;
        iv.u = make_uint4(0, 0, 0, 0);
        if (p < p1) {
          const int b = (int)(p / (Ho * Wo));
          const int rr = (int)(p % (Ho * Wo));
          const int iy = (rr / Wo) * S + tap / 3 - 1, ix = (rr % Wo) * S + tap % 3 - 1;
          if (iy >= 0 && iy < H && ix >= 0 && ix < Wd)
            iv.u = *reinterpret_cast<const uint4 *>(in + (((long long)b * H + iy) * Wd + ix) * CIN + 8 * c8);
        }
        uint16_t *dst = Is + g * SH::I_ELEMS + (tap * NC + 8 * c8) * PS + px;
#pragma unroll
        for (int i = 0; i < 8; ++i) dst[i * PS] = iv.h[i];
      }
    } else {
      for (int e = threadIdx.x; e < KSPLIT * 32 * 9; e += 1024) {
        const int tap = e % 9, r = e / 9;  // r = g * 32 + px
        const int g = r / 32, px = r % 32;
        const long long p = ps + r;
        uint16_t v[CIN];
#pragma unroll
        for (int c = 0; c < CIN; ++c) v[c] = 0;
        if (p < p1) {
          const int b = (int)(p / (Ho * Wo));
          const int rr = (int)(p % (Ho * Wo));
          const int iy = (rr / Wo) * S + tap / 3 - 1, ix = (rr % Wo) * S + tap % 3 - 1;
          if (iy >= 0 && iy < H && ix >= 0 && ix < Wd)
#pragma unroll
            for (int c = 0; c < CIN; ++c) v[c] = in[(((long long)b * H + iy) * Wd + ix) * CIN + c];
        }
#pragma unroll
        for (int c = 0; c < CIN; ++c) Is[g * SH::I_ELEMS + (tap * CIN + c) * PS + px] = v[c];
      }
    }
    __syncthreads();
    {
      const int co = wl * 64 + lane;
      if (co < COUT) {
        const uint16_t *gr = Gs + kg * SH::G_ELEMS + co * PS;
        for (int px = 0; px < 32; ++px) bsum += bf2f(gr[px]);
      }
    }
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int t = wl * TPW + q;
      if (t < TILES) {
        const int tm = t / TN, tn = t % TN;
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(
            Gs + kg * SH::G_ELEMS + (tm * 16 + r16) * PS + 8 * kq);
        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(
            Is + kg * SH::I_ELEMS + (tn * 16 + r16) * PS + 8 * kq);
        acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[q], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // partial block of this group: part[row][tap][co][col], row = chunk * KSPLIT + group
  const long long row = (long long)blockIdx.x * KSPLIT + kg;
  float *dst = part + row * SH::REC;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int t = wl * TPW + q;
    if (t < TILES) {
      const int tm = t / TN, tn = t % TN;
      const int tap = tn / (NC / 16), col = (tn % (NC / 16)) * 16 + r16;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        dst[((long long)tap * COUT + tm * 16 + 4 * kq + i) * NC + col] = acc[q][i];
    }
  }
  {
    const int co = wl * 64 + lane;
    if (co < COUT) bpart[row * COUT + co] = bsum;
  }
}

// dW[co][tap][ci] (FP32, layout of the master weights) and db[co] = sums over
// the partial blocks (rows).  A workgroup of 16 waves takes 64 consecutive
// outputs (one per lane, coalesced loads) and a range of up to RED_ROWS rows;
// wave g sums rows g, g + 16, ... of the range in order (FP64) and the 16
// partial sums are added in wave order.  With one range the result is
// written directly; with several, each range's sums go to `partial` and
// k_wgrad_finish adds them in range order: the result does not depend on the
// launch.  Outputs past COUT * 9 CIN are the bias entries (row stride COUT).
constexpr int RED_WAVES = 16;
constexpr int RED_ROWS = 256;

template <int CIN, int COUT>
__global__ void __launch_bounds__(RED_WAVES * 64)
k_wgrad_reduce(const float *__restrict__ part, const float *__restrict__ bpart, int n_rows,
               float *__restrict__ dW, float *__restrict__ db, double *__restrict__ partial) {
  constexpr int NC = WCols<CIN>::n;
  constexpr int taps = CIN >= 32 ? 9 : 1;
  constexpr int K = 9 * CIN;
  constexpr int NRED = COUT * K + COUT;
  constexpr long long REC = (long long)taps * COUT * NC;
  __shared__ double red[RED_WAVES][64];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int idx = blockIdx.x * 64 + lane;
  const int r0 = blockIdx.y * RED_ROWS;
  const int r1 = n_rows < r0 + RED_ROWS ? n_rows : r0 + RED_ROWS;
  double sum = 0;
  if (idx < COUT * K) {
    const int co = idx / K, k = idx % K;
    const int tap = CIN >= 32 ? k / CIN : 0;
    const int col = CIN >= 32 ? k % CIN : k;
    const float *src = part + ((long long)tap * COUT + co) * NC + col;
    for (int c = r0 + g; c < r1; c += RED_WAVES) sum += src[c * REC];
  } else if (idx < NRED) {
    const float *src = bpart + (idx - COUT * K);
    for (int c = r0 + g; c < r1; c += RED_WAVES) sum += src[(long long)c * COUT];
  }
  red[g][lane] = sum;
  __syncthreads();
  if (g == 0 && idx < NRED) {
    double t = 0;
    for (int w = 0; w < RED_WAVES; ++w) t += red[w][lane];
    if (gridDim.y > 1) partial[(long long)blockIdx.y * NRED + idx] = t;
    else if (idx < COUT * K) dW[idx] = (float)t;
    else db[idx - COUT * K] = (float)t;
  }
}

__global__ void k_wgrad_finish(const double *__restrict__ partial, int ranges, int n_w, int nred,
                               float *__restrict__ dW, float *__restrict__ db) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nred) return;
  double t = 0;
  for (int r = 0; r < ranges; ++r) t += partial[(long long)r * nred + idx];
  if (idx < n_w) dW[idx] = (float)t;
  else db[idx - n_w] = (float)t;
}

// ---------------------------------------------------------------------------
// pair packing: channel 0 = observed patch, channel 1 = simulated patch, each
// normalised to zero mean / unit variance over the patch's valid samples
// (invalid samples 0).  One workgroup per pair; patches are 64 x 64.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_pack_pairs(const PatchDev *__restrict__ patches, const int *__restrict__ ids,
             const float *__restrict__ invz, const float *__restrict__ y,
             const float *__restrict__ ys, uint16_t *__restrict__ outp, int side, int M) {
  __shared__ double red[5][4];
  const int bi = blockIdx.x;
  const int n = side * side;
  const int id = ids[bi];
  if (id < 0 || id >= M) {  // not a patch of the plan: an all-zero pair (uniform per workgroup)
    uint32_t *o32 = reinterpret_cast<uint32_t *>(outp) + (long long)bi * n;
    for (int l = threadIdx.x; l < n; l += 256) o32[l] = 0u;
    return;
  }
  const PatchDev pt = patches[id];
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
  const double r0 = 1.0 / s0, r1 = 1.0 / s1;
  uint32_t *o32 = reinterpret_cast<uint32_t *>(outp) + (long long)bi * n;
  for (int l = threadIdx.x; l < n; l += 256) {
    const long long j = pt.off + l;
    float u = 0.f, v = 0.f;
    if (invz[j] > 0.f) {
      u = (float)((y[j] - m0) * r0);
      v = (float)((ys[j] - m1) * r1);
    }
    o32[l] = (uint32_t)f2bf(u) | ((uint32_t)f2bf(v) << 16);  // both channels of pixel l
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

// dL/dWfc[e][k] = sum_b act[b][e] dp[b][k], dL/dbfc[k] = sum_b dp[b][k].  A
// workgroup of 16 waves takes 64 inputs e (one per lane; the last lanes past
// n_in take the bias); wave g sums the samples b = g, g + 16, ... in order and
// the 16 partial sums are added in wave order (fixed summation order).
__global__ void __launch_bounds__(RED_WAVES * 64)
k_head_wgrad(const uint16_t *__restrict__ act, const float *__restrict__ dp, int B, int n_in,
             float *__restrict__ dW, float *__restrict__ db) {
  __shared__ float red[RED_WAVES][64][6];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (e < n_in) {
    for (int b = g; b < B; b += RED_WAVES) {
      const float x = bf2f(act[(long long)b * n_in + e]);
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[k] = fmaf(x, dp[b * 6 + k], acc[k]);
    }
  } else if (e < n_in + 6) {
    const int k = e - n_in;
    for (int b = g; b < B; b += RED_WAVES) acc[0] += dp[b * 6 + k];
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) red[g][lane][k] = acc[k];
  __syncthreads();
  if (g == 0) {
    float t[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int w = 0; w < RED_WAVES; ++w)
#pragma unroll
      for (int k = 0; k < 6; ++k) t[k] += red[w][lane][k];
    if (e < n_in) {
#pragma unroll
      for (int k = 0; k < 6; ++k) dW[e * 6 + k] = t[k];
    } else if (e < n_in + 6) {
      db[e - n_in] = t[0];
    }
  }
}

// sum of per-sample partials (fixed order)
// out[0] = sum of x[0..n) by one workgroup: thread t sums t, t + 1024, ...
// in order (FP64), then a fixed tree over the threads.
__global__ void __launch_bounds__(1024) k_sum_all(const float *__restrict__ x, int n,
                                                  float *__restrict__ out) {
  __shared__ double red[1024];
  double s = 0;
  for (int i = threadIdx.x; i < n; i += 1024) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)red[0];
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
  PVR_ALIGNED("pvr_cnn_conv_fwd", in, 16);
  PVR_ALIGNED("pvr_cnn_conv_fwd", w, 16);
  PVR_ALIGNED("pvr_cnn_conv_fwd", bias, 4);
  PVR_ALIGNED("pvr_cnn_conv_fwd", out, 16);
  if (!in || !w || !bias || !out || B <= 0 || H <= 0 || W <= 0)
    return fail(PVR_EINVAL, "pvr_cnn_conv_fwd: invalid argument");
  const long long P = (long long)B * out_size(H, stride) * out_size(W, stride);
  const long long n_tiles = (P + FW_TILE - 1) / FW_TILE;
#define LAUNCH(CI, CO, ST)                                                                     \
  if (cin == CI && cout == CO && stride == ST) {                                               \
    const dim3 grid(persistent_grid(n_tiles, FwdShape<CI, CO>::LDS_BYTES));                    \
    hipLaunchKernelGGL((k_conv_fwd<CI, CO, ST>), grid, dim3(FW_THREADS), 0, stream, in, w,     \
                       bias, out, B, H, W, relu);                                              \
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
  PVR_ALIGNED("pvr_cnn_conv_dgrad", gout, 16);
  PVR_ALIGNED("pvr_cnn_conv_dgrad", out, 16);
  PVR_ALIGNED("pvr_cnn_conv_dgrad", wt, 16);
  PVR_ALIGNED("pvr_cnn_conv_dgrad", gin, 16);
  if (!gout || !out || !wt || !gin || B <= 0) return fail(PVR_EINVAL, "pvr_cnn_conv_dgrad: invalid argument");
  const long long P = (long long)B * H * W;
  const long long n_tiles = (P + FW_TILE - 1) / FW_TILE;
#define LAUNCH(CI, CO, ST)                                                                       \
  if (cin == CI && cout == CO && stride == ST && CI >= 16) {                                     \
    constexpr int CIX = CI >= 16 ? CI : 16;                                                      \
    const dim3 grid(persistent_grid(n_tiles, DgradShape<CIX, CO>::LDS_BYTES));                   \
    hipLaunchKernelGGL((k_conv_dgrad<CIX, CO, ST>), grid, dim3(FW_THREADS), 0, stream,           \
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

// Rows (partial blocks) of the weight-gradient scratch for a layer shape.
template <int CIN, int COUT>
static long long wgrad_rows(long long P, long long *wch) {
  using SH = WgradShape<CIN, COUT>;
  const long long c = wgrad_chunk(P, SH::KSPLIT);
  if (wch) *wch = c;
  return (P + c - 1) / c * SH::KSPLIT;
}

extern "C" int64_t pvr_cnn_wgrad_scratch(int32_t B, int32_t H, int32_t W, int32_t cin,
                                         int32_t cout, int32_t stride) {
  const long long P = (long long)B * out_size(H, stride) * out_size(W, stride);
#define SCR(CI, CO, ST)                                                                  \
  if (cin == CI && cout == CO) {                                                         \
    using SH = WgradShape<CI, CO>;                                                       \
    const long long rows = wgrad_rows<CI, CO>(P, nullptr);                               \
    const long long ranges = (rows + RED_ROWS - 1) / RED_ROWS;                            \
    return rows * (SH::REC + CO) * (long long)sizeof(float) +                            \
           (ranges > 1 ? ranges * (9LL * CI * CO + CO) * (long long)sizeof(double) : 0); \
  }
  CONV_CASES(SCR)
#undef SCR
  return 0;
}

extern "C" pvr_status pvr_cnn_conv_wgrad(const uint16_t *gout, const uint16_t *out,
                                         const uint16_t *in, float *scratch, float *dw, float *db,
                                         int32_t B, int32_t H, int32_t W, int32_t cin,
                                         int32_t cout, int32_t stride, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_cnn_conv_wgrad", gout, 16);
  PVR_ALIGNED("pvr_cnn_conv_wgrad", out, 16);
  PVR_ALIGNED("pvr_cnn_conv_wgrad", in, 16);
  PVR_ALIGNED("pvr_cnn_conv_wgrad", scratch, 16);
  PVR_ALIGNED("pvr_cnn_conv_wgrad", dw, 4);
  PVR_ALIGNED("pvr_cnn_conv_wgrad", db, 4);
  if (!gout || !out || !in || !scratch || !dw || !db || B <= 0)
    return fail(PVR_EINVAL, "pvr_cnn_conv_wgrad: invalid argument");
  const long long P = (long long)B * out_size(H, stride) * out_size(W, stride);
  const int nred = cout * 9 * cin + cout;  // weights, then biases
#define LAUNCH(CI, CO, ST)                                                                       \
  if (cin == CI && cout == CO && stride == ST) {                                                 \
    using SH = WgradShape<CI, CO>;                                                               \
    long long wch = 0;                                                                           \
    const long long rows = wgrad_rows<CI, CO>(P, &wch);                                          \
    const int chunks = (int)(rows / SH::KSPLIT);                                                 \
    float *part = scratch;                                                                       \
    float *bpart = scratch + rows * SH::REC;                                                     \
    hipLaunchKernelGGL((k_conv_wgrad<CI, CO, ST>), dim3(chunks), dim3(1024), 0, stream, gout,    \
                       out, in, part, bpart, B, H, W, wch);                                      \
    HIP_TRY(hipGetLastError());                                                                  \
    const int ranges = (int)((rows + RED_ROWS - 1) / RED_ROWS);                                  \
    double *partial = ranges > 1 ? (double *)(bpart + rows * CO) : nullptr;                      \
    hipLaunchKernelGGL((k_wgrad_reduce<CI, CO>), dim3((nred + 63) / 64, ranges),                 \
                       dim3(RED_WAVES * 64), 0, stream, part, bpart, (int)rows, dw, db, partial); \
    HIP_TRY(hipGetLastError());                                                                  \
    if (ranges > 1) {                                                                            \
      hipLaunchKernelGGL(k_wgrad_finish, dim3((nred + 255) / 256), dim3(256), 0, stream, partial, \
                         ranges, nred - CO, nred, dw, db);                                       \
      HIP_TRY(hipGetLastError());                                                                \
    }                                                                                            \
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
  PVR_ALIGNED("pvr_cnn_pack_pairs", patch_ids, 4);
  PVR_ALIGNED("pvr_cnn_pack_pairs", y_obs, 4);
  PVR_ALIGNED("pvr_cnn_pack_pairs", y_sim, 4);
  PVR_ALIGNED("pvr_cnn_pack_pairs", out, 4);
  if (!p || !patch_ids || !y_obs || !y_sim || !out || B <= 0)
    return fail(PVR_EINVAL, "pvr_cnn_pack_pairs: invalid argument");
  if (!p->built) return fail(PVR_EINVAL, "pvr_cnn_pack_pairs: plan has not been built");
  for (int s = 0; s < p->M; ++s)
    if (p->h_patch[s].w != PVR_CNN_SIDE || p->h_patch[s].h != PVR_CNN_SIDE)
      return fail(PVR_ESHAPE, "pvr_cnn_pack_pairs: patch %d is not %dx%d", s, PVR_CNN_SIDE,
                  PVR_CNN_SIDE);
  hipLaunchKernelGGL(k_pack_pairs, dim3(B), dim3(256), 0, stream, p->d_patch, patch_ids, p->d_invz,
                     y_obs, y_sim, out, PVR_CNN_SIDE, p->M);
  HIP_TRY(hipGetLastError());
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_cnn_head(const uint16_t *act, int32_t B, int32_t hw, const float *wfc,
                                   const float *bfc, const float *target, const float *loss_w,
                                   float *pred, float *loss, uint16_t *gact, float *dwfc,
                                   float *dbfc, float *scratch, hipStream_t stream) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_cnn_head", act, 16);
  PVR_ALIGNED("pvr_cnn_head", wfc, 4);
  PVR_ALIGNED("pvr_cnn_head", bfc, 4);
  PVR_ALIGNED("pvr_cnn_head", target, 4);
  PVR_ALIGNED("pvr_cnn_head", loss_w, 4);
  PVR_ALIGNED("pvr_cnn_head", pred, 4);
  PVR_ALIGNED("pvr_cnn_head", loss, 4);
  PVR_ALIGNED("pvr_cnn_head", gact, 16);
  PVR_ALIGNED("pvr_cnn_head", dwfc, 4);
  PVR_ALIGNED("pvr_cnn_head", dbfc, 4);
  PVR_ALIGNED("pvr_cnn_head", scratch, 16);
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
    hipLaunchKernelGGL(k_sum_all, dim3(1), dim3(1024), 0, stream, lp, B * 6, loss);
    hipLaunchKernelGGL(k_head_wgrad, dim3((n_in + 6 + 63) / 64), dim3(RED_WAVES * 64), 0, stream,
                       act, dp, B, n_in, dwfc, dbfc);
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
  PVR_ALIGNED("pvr_cnn_adam", w, 4);
  PVR_ALIGNED("pvr_cnn_adam", g, 4);
  PVR_ALIGNED("pvr_cnn_adam", m, 4);
  PVR_ALIGNED("pvr_cnn_adam", v, 4);
  PVR_ALIGNED("pvr_cnn_adam", w_bf16, 16);
  PVR_ALIGNED("pvr_cnn_adam", wt_bf16, 16);
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
