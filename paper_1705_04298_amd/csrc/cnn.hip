// Learned initial extension: a 7-layer 3x3 CNN in BF16 on MFMA (FP32 accumulate).
//
// Activations are NHWC bf16 ([B][N][N][C], C = 8, 16 or 32; padded channels are 0).
// A convolution is an implicit GEMM: M = pixels, N = output channels,
// K = (tap, input channel), tap-major, so that 8 consecutive K values of one
// lane are 8 consecutive channels of one neighbour pixel (one 16-byte load).
// v_mfma_f32_16x16x32_bf16 operand layout (lane l of 64):
//   A (16 x 32): row l % 16, k = 8 (l / 16) .. + 7
//   B (32 x 16): column l % 16, k = 8 (l / 16) .. + 7
//   C (16 x 16): column l % 16, rows 4 (l / 16) .. + 3
// Backward-data is the same kernel on the output gradient with the weights
// transposed and the taps flipped; the weight gradient is a GEMM over pixels,
// staged through LDS in channel-major (transposed) form.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <utility>

#include "cnn.h"
#include "lds_limit.h"

namespace fwr {
namespace cnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

__device__ __forceinline__ bf16x8 load8(const uint16_t *p) {
  const uint4 v = *reinterpret_cast<const uint4 *>(p);
  return __builtin_bit_cast(bf16x8, v);
}
__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

template <int CIN>
constexpr int kpad() { return ((9 * CIN + 31) / 32) * 32; }

#ifndef FWR_CNN_TILE_ROWS
#define FWR_CNN_TILE_ROWS 4
#endif
constexpr int kTileRows = FWR_CNN_TILE_ROWS;  // output rows per step of the convolution
constexpr int kSegTiles = 5;  // consecutive row tiles of one frame per work item
#ifndef FWR_CNN_PIX_PAD
#define FWR_CNN_PIX_PAD 8
#endif
constexpr int kPixPad = FWR_CNN_PIX_PAD;  // bf16 padding of a staged pixel vector

// ------------------------------------------------------------------ forward / backward-data
// A work item is a segment of kSegTiles row tiles (kTileRows output rows each) of one frame,
// walked top to bottom.  The (kTileRows + 2) x (N + 2) input halo (zeros outside the frame)
// lives in LDS as a ring of kTileRows + 2 rows: grid row y sits in ring row (y + 1) mod
// (kTileRows + 2), so a tile keeps the two rows it shares with the previous one and loads only
// kTileRows new rows; an input row is fetched from memory once per segment (plus the two halo
// rows at its start) instead of once per tap or once per tile.  Pixel vectors are padded by
// 8 bf16 so that the 16 pixels of an A operand fall on different LDS banks.  The weights
// (B operands) stay in registers; each wave takes every 4th 16-pixel M tile of the tile.
// MODE 0: y = relu(conv + bias) -> bf16 NHWC [.., 32]
// MODE 1: y = (conv + bias) * out_scale for channels 0, 1 -> fp32 planar [B][2][N][N]
// MODE 2: y = conv * (act[p][c] > 0) -> bf16 NHWC [.., COUT] (gradient through the ReLU)
template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void conv_kernel(const uint16_t *__restrict__ x, const uint16_t *__restrict__ wt,
                                                   const float *__restrict__ bias, void *out,
                                                   const uint16_t *__restrict__ act, int N, int nitems,
                                                   float out_scale) {
  // C^T = W^T X^T per 16-pixel tile: A = weights (16 output channels x 32 k), B = activations
  // (32 k x 16 pixels), so lane l ends with channels 4 (l / 16) .. + 3 of pixel l % 16.
  // Persistent: the weights are loaded once; the workgroup walks the work items
  // blockIdx.x, blockIdx.x + gridDim.x, ...
  constexpr int K = kpad<CIN>(), KCH = K / 32, MT = COUT / 16, CP = CIN + kPixPad, CH = CIN / 8;
  constexpr int PIX_STEP = 256 / CH;  // halo pixels staged per pass of the workgroup
  extern __shared__ __attribute__((aligned(16))) uint16_t halo[];  // ring [kTileRows + 2][N + 2][CP]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  bf16x8 aw[KCH][MT];
#pragma unroll
  for (int kc = 0; kc < KCH; ++kc)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) aw[kc][mt] = load8(wt + (size_t)(mt * 16 + col) * K + kc * 32 + 8 * kq);
  float bv[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) bv[mt][i] = MODE == 2 ? 0.f : bias[mt * 16 + 4 * kq + i];
  const int tiles = (N + kTileRows - 1) / kTileRows, segs = (tiles + kSegTiles - 1) / kSegTiles;
  constexpr int RING = kTileRows + 2;
  const int W = N + 2, hpix = RING * W;
  const size_t NN = (size_t)N * N;
  const int c8 = threadIdx.x % CH;
#pragma unroll 1
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
  const int f = item / segs, seg = item - f * segs;
  const int kt0 = seg * kSegTiles, kt1 = kt0 + kSegTiles < tiles ? kt0 + kSegTiles : tiles;
  const uint16_t *xf = x + (size_t)f * NN * CIN;
#pragma unroll 1
  for (int tile_k = kt0; tile_k < kt1; ++tile_k) {
    const int y0 = tile_k * kTileRows;
    const int rows = N - y0 < kTileRows ? N - y0 : kTileRows;
    const int base = y0 % RING;  // ring row of halo row 0 (grid row y0 - 1)
    auto ring = [&](int j) { return base + j >= RING ? base + j - RING : base + j; };
    __syncthreads();  // the previous tile's LDS reads are done
    // halo rows j (grid row y0 - 1 + j) from jlo on: all of them at the segment's first tile, the
    // kTileRows new ones after it.  Pixel q = (j, xx + 1): walk q = jlo W + threadIdx.x / CH +
    // PIX_STEP u, loads first, then the stores into ring row ring(j)
    {
      const int jlo = tile_k == kt0 ? 0 : 2;
      int q = jlo * W + threadIdx.x / CH, r = jlo, xc = threadIdx.x / CH;
      while (xc >= W) {
        xc -= W;
        ++r;
      }
      constexpr int BATCH = 8;
      for (; q < hpix; ) {
        uint4 v[BATCH];
        int qs[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
          const int yy = y0 + r - 1, xx = xc - 1;
          qs[u] = q < hpix ? ring(r) * W + xc : -1;
          v[u] = make_uint4(0u, 0u, 0u, 0u);
          if (q < hpix && yy >= 0 && yy < N && xx >= 0 && xx < N)
            v[u] = *reinterpret_cast<const uint4 *>(xf + ((size_t)yy * N + xx) * CIN + 8 * c8);
          q += PIX_STEP;
          xc += PIX_STEP;
          while (xc >= W) {
            xc -= W;
            ++r;
          }
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u)
          if (qs[u] >= 0) *reinterpret_cast<uint4 *>(halo + (size_t)qs[u] * CP + 8 * c8) = v[u];
      }
    }
    __syncthreads();
    const int npix = rows * N;  // output pixels of the tile
    const size_t gbase = (size_t)f * NN + (size_t)y0 * N;
    int r0 = 0, x0 = wave * 16;  // (row, column) of the first pixel of tile pt, pt = wave, wave + 4, ...
    while (x0 >= N) {
      x0 -= N;
      ++r0;
    }
#pragma unroll 1
    for (int pt = wave; pt * 16 < npix; pt += 4) {
      const int pl = pt * 16 + col;  // this lane's pixel (B column, C column)
      int r = r0, xx = x0 + col;     // 16 <= N: at most one wrap within a tile
      if (xx >= N) {
        xx -= N;
        ++r;
      }
      if (pl >= npix) {  // past the tile: a valid LDS read, result discarded
        r = rows - 1;
        xx = N - 1;
      }
      x0 += 64;  // next tile of this wave: 64 pixels on
      while (x0 >= N) {
        x0 -= N;
        ++r0;
      }
      f32x4 acc[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
      // LDS offsets of the pixel's three input rows (ring rows of halo rows r, r + 1, r + 2)
      const int ro0 = (ring(r) * W + xx) * CP, ro1 = (ring(r + 1) * W + xx) * CP, ro2 = (ring(r + 2) * W + xx) * CP;
#pragma unroll
      for (int kc = 0; kc < KCH; ++kc) {
        const int k0 = kc * 32 + 8 * kq;
        const int t = k0 / CIN, c0 = k0 - t * CIN;
        const int tr = t / 3, ro = tr == 0 ? ro0 : (tr == 1 ? ro1 : ro2);
        bf16x8 b = zero8();
        if (t < 9) b = *reinterpret_cast<const bf16x8 *>(halo + ro + (t % 3) * CP + c0);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[kc][mt], b, acc[mt], 0, 0, 0);
      }
      if (pl >= npix) continue;
      const size_t q = gbase + pl;
      if constexpr (MODE == 1) {
        if (kq == 0) {  // channels 0, 1 of this pixel
          const size_t fq = q / NN, rq = q - fq * NN;
          float *o = static_cast<float *>(out);
          o[(fq * 2 + 0) * NN + rq] = (acc[0][0] + bv[0][0]) * out_scale;
          o[(fq * 2 + 1) * NN + rq] = (acc[0][1] + bv[0][1]) * out_scale;
        }
      } else {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int c = mt * 16 + 4 * kq;  // first of the lane's four channels
          f32x2 v01, v23;
          if constexpr (MODE == 0) {
            v01 = f32x2{fmaxf(acc[mt][0] + bv[mt][0], 0.f), fmaxf(acc[mt][1] + bv[mt][1], 0.f)};
            v23 = f32x2{fmaxf(acc[mt][2] + bv[mt][2], 0.f), fmaxf(acc[mt][3] + bv[mt][3], 0.f)};
          } else {
            const uint2 m = *reinterpret_cast<const uint2 *>(act + q * COUT + c);
            v01 = f32x2{bf2f(uint16_t(m.x)) > 0.f ? acc[mt][0] : 0.f, bf2f(uint16_t(m.x >> 16)) > 0.f ? acc[mt][1] : 0.f};
            v23 = f32x2{bf2f(uint16_t(m.y)) > 0.f ? acc[mt][2] : 0.f, bf2f(uint16_t(m.y >> 16)) > 0.f ? acc[mt][3] : 0.f};
          }
          const uint2 packed = make_uint2(__builtin_bit_cast(uint32_t, __builtin_convertvector(v01, bf16x2)),
                                          __builtin_bit_cast(uint32_t, __builtin_convertvector(v23, bf16x2)));
          *reinterpret_cast<uint2 *>(static_cast<uint16_t *>(out) + q * COUT + c) = packed;
        }
      }
    }
  }
  }
}

template <int CIN>
constexpr size_t halo_bytes(int N) { return size_t(kTileRows + 2) * (N + 2) * (CIN + kPixPad) * 2; }

// ------------------------------------------------------------------ weight gradient
// dW[co][t*CIN + ci] += sum_p dz[p][co] x[p + off(t)][ci]; one block per frame, 32-pixel chunks.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void wgrad_kernel(const uint16_t *__restrict__ x, const uint16_t *__restrict__ dz,
                                                    float *__restrict__ dw, float *__restrict__ db, int N) {
  constexpr int NCOL = 9 * CIN, MT = COUT / 16, NTT = (NCOL + 15) / 16, TILES = MT * NTT;
  constexpr int PER_WAVE = (TILES + 3) / 4;
  __shared__ __attribute__((aligned(16))) uint16_t dzt[COUT][32 + 8];      // [co][pixel]
  __shared__ __attribute__((aligned(16))) uint16_t xt[NTT * 16][32 + 8];   // [(t, ci)][pixel], rows >= NCOL zero
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, t = threadIdx.x;
  const int col = lane & 15, kq = lane >> 4;
  const int f = blockIdx.x, NN = N * N;
  const uint16_t *xf = x + (size_t)f * NN * CIN;
  const uint16_t *dzf = dz + (size_t)f * NN * COUT;
  f32x4 acc[PER_WAVE];
#pragma unroll
  for (int i = 0; i < PER_WAVE; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;  // bias gradient partial of channel t (t < COUT)
  for (int i = t; i < (NTT * 16 - NCOL) * 40; i += 256) xt[NCOL + i / 40][i % 40] = 0;
  for (int p0 = 0; p0 < NN; p0 += 32) {
    __syncthreads();
    for (int i = t; i < 32 * COUT; i += 256) {
      const int pp = i / COUT, c = i - pp * COUT;
      dzt[c][pp] = dzf[(size_t)(p0 + pp) * COUT + c];
    }
    for (int i = t; i < 32 * NCOL; i += 256) {
      const int pp = i / NCOL, r = i - pp * NCOL, tap = r / CIN, c = r - tap * CIN;
      const int p = p0 + pp, y = p / N, xx = p - y * N;
      const int yy = y + tap / 3 - 1, xs = xx + tap % 3 - 1;
      xt[r][pp] = (yy >= 0 && yy < N && xs >= 0 && xs < N) ? xf[((size_t)yy * N + xs) * CIN + c] : uint16_t(0);
    }
    __syncthreads();
    if (t < COUT)
      for (int pp = 0; pp < 32; ++pp) bsum += bf2f(dzt[t][pp]);
#pragma unroll
    for (int i = 0; i < PER_WAVE; ++i) {
      const int tile = wave * PER_WAVE + i;
      if (tile < TILES) {
        const int mt = tile / NTT, nt = tile - mt * NTT;
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&dzt[mt * 16 + col][8 * kq]);
        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&xt[nt * 16 + col][8 * kq]);
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < PER_WAVE; ++i) {
    const int tile = wave * PER_WAVE + i;
    if (tile < TILES) {
      const int mt = tile / NTT, nt = tile - mt * NTT;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int co = mt * 16 + 4 * kq + r, k = nt * 16 + col;
        if (k < NCOL) atomicAdd(&dw[(size_t)co * NCOL + k], acc[i][r]);
      }
    }
  }
  if (t < COUT) atomicAdd(&db[t], bsum);
}

// ------------------------------------------------------------------ features, loss, Adam
// feat[b][m][n][0..7] = (s0x * scale, s0y * scale, P, 0, ...) on the N x N grid
__global__ void features_kernel(const float *__restrict__ slopes, const uint8_t *__restrict__ mask,
                                uint16_t *__restrict__ feat, int B, int n, int N, float scale) {
  const size_t total = (size_t)B * N * N;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int b = int(i / ((size_t)N * N));
  const int rem = int(i - (size_t)b * N * N), m = rem / N, c = rem - m * N, o = (N - n) / 2;
  float sx = 0.f, sy = 0.f, pv = 0.f;
  const int ii = m - o, jj = c - o;
  if (ii >= 0 && ii < n && jj >= 0 && jj < n && mask[ii * n + jj]) {
    const float *sb = slopes + (size_t)b * 2 * n * n;
    sx = sb[ii * n + jj] * scale;
    sy = sb[n * n + ii * n + jj] * scale;
    pv = 1.f;
  }
  uint16_t *fp = feat + i * 8;
  fp[0] = f2bf(sx);
  fp[1] = f2bf(sy);
  fp[2] = f2bf(pv);
#pragma unroll
  for (int k = 3; k < 8; ++k) fp[k] = 0;
}

// dz7[p][c] = 2 (pred_raw - target * scale) * outside / count  (c < 2; channels 2..15 zero);
// pred is in slope units (pred_raw / scale); loss accumulates sum(diff^2) / count
__global__ void loss_grad_kernel(const float *__restrict__ pred, const float *__restrict__ target,
                                 const uint8_t *__restrict__ mask, uint16_t *__restrict__ dz7,
                                 float *__restrict__ loss, int B, int n, int N, float scale, float inv_count) {
  const size_t total = (size_t)B * N * N;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (i < total) {
    const int b = int(i / ((size_t)N * N));
    const int rem = int(i - (size_t)b * N * N), m = rem / N, c = rem - m * N, o = (N - n) / 2;
    const int ii = m - o, jj = c - o;
    const bool inside = ii >= 0 && ii < n && jj >= 0 && jj < n && mask[ii * n + jj];
    uint16_t *g = dz7 + i * 16;
#pragma unroll
    for (int k = 0; k < 16; ++k) g[k] = 0;
    if (!inside) {
#pragma unroll
      for (int ch = 0; ch < 2; ++ch) {
        const size_t idx = ((size_t)b * 2 + ch) * N * N + rem;
        const float d = (pred[idx] - target[idx]) * scale;
        l += d * d;
        g[ch] = f2bf(2.f * d * inv_count);
      }
    }
  }
  // wave reduction then one atomic per wave
  for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(loss, l * inv_count);
}

// The same loss, with its gradient with respect to the prediction in slope units written as a
// float map: grad = 2 scale^2 (pred - target) / count outside the pupil, 0 inside.
__global__ void loss_grad_map_kernel(const float *__restrict__ pred, const float *__restrict__ target,
                                     const uint8_t *__restrict__ mask, float *__restrict__ grad,
                                     float *__restrict__ loss, int B, int n, int N, float scale, float inv_count) {
  const size_t total = (size_t)B * N * N;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (i < total) {
    const int b = int(i / ((size_t)N * N));
    const int rem = int(i - (size_t)b * N * N), m = rem / N, c = rem - m * N, o = (N - n) / 2;
    const int ii = m - o, jj = c - o;
    const bool inside = ii >= 0 && ii < n && jj >= 0 && jj < n && mask[ii * n + jj];
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
      const size_t idx = ((size_t)b * 2 + ch) * N * N + rem;
      const float d = inside ? 0.f : (pred[idx] - target[idx]) * scale;
      l += d * d;
      grad[idx] = 2.f * d * scale * inv_count;
    }
  }
  for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(loss, l * inv_count);
}

// dz7 (the gradient at the last layer's output, bf16, 16 channels) from a gradient with respect to
// the prediction in slope units: the prediction is that output divided by the input scale.
__global__ void grad_in_kernel(const float *__restrict__ grad, uint16_t *__restrict__ dz7, int B, int N,
                               float inv_scale) {
  const size_t total = (size_t)B * N * N;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const size_t NN = (size_t)N * N, b = i / NN, rem = i - b * NN;
  uint16_t *g = dz7 + i * 16;
  g[0] = f2bf(grad[(b * 2 + 0) * NN + rem] * inv_scale);
  g[1] = f2bf(grad[(b * 2 + 1) * NN + rem] * inv_scale);
#pragma unroll
  for (int k = 2; k < 16; ++k) g[k] = 0;
}

// Adam on FP32 master weights (kernel layout [co][t][ci]), then the bf16 copies:
// wt [co][kpad] for the forward pass, wtb [ci][t' * COUTS + co] (taps flipped) for backward-data.
__global__ void adam_kernel(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m1,
                            float *__restrict__ m2, int count, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  w[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

// master weights (fp32 [cout_s][9][cin_s], padded channels 0) -> bf16 forward layout
// wt [cout_s][kpad_f] (k = t * cin_s + ci) and flipped backward-data layout
// wtb [cin_s][kpad_b] (k = t' * cout_s + co, weight w[co][8 - t'][ci])
__global__ void pack_kernel(const float *__restrict__ w, uint16_t *__restrict__ wt, uint16_t *__restrict__ wtb,
                            int cin_s, int cout_s, int kpad_f, int kpad_b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cout_s * kpad_f) {
    const int co = i / kpad_f, k = i - co * kpad_f, t = k / cin_s, ci = k - t * cin_s;
    wt[i] = f2bf(t < 9 ? w[((size_t)co * 9 + t) * cin_s + ci] : 0.f);
  }
  if (wtb && i < cin_s * kpad_b) {
    const int ci = i / kpad_b, k = i - ci * kpad_b, t = k / cout_s, co = k - t * cout_s;
    wtb[i] = f2bf(t < 9 ? w[((size_t)co * 9 + (8 - t)) * cin_s + ci] : 0.f);
  }
}

}  // namespace cnn

// ------------------------------------------------------------------ host-side launchers
namespace cnn_launch {
using namespace cnn;

// work items of a launch: kSegTiles-tile segments of every frame
static int tiles_of(int B, int N) {
  const int tiles = (N + kTileRows - 1) / kTileRows;
  return B * ((tiles + kSegTiles - 1) / kSegTiles);
}

// persistent grid: as many workgroups as the CUs hold at once (occupancy of the kernel with
// its dynamic LDS), capped by the number of tiles; measured once per kernel and grid size in
// conv_prepare, so that launches make no device queries (they may be captured in a graph)
static std::mutex g_grid_mu;
static std::map<std::pair<const void *, int>, int> g_resident;  // (kernel, N) -> workgroups

template <typename K>
static hipError_t measure_grid(K kernel, size_t lds, int N) {
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, lds);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_grid_mu);
  g_resident[{reinterpret_cast<const void *>(kernel), N}] = (per_cu > 0 ? per_cu : 1) * prop.multiProcessorCount;
  return hipSuccess;
}

template <typename K>
static int grid_of(K kernel, int N, int ntiles) {
  int g = 256;
  {
    std::lock_guard<std::mutex> lock(g_grid_mu);
    auto it = g_resident.find({reinterpret_cast<const void *>(kernel), N});
    if (it != g_resident.end()) g = it->second;
  }
  return ntiles < g ? ntiles : g;
}

hipError_t conv_prepare(int N) {
  // the halo tile can exceed the default 64 KiB of dynamic LDS
  const void *fns[5] = {reinterpret_cast<const void *>(&conv_kernel<8, 32, 0>),
                        reinterpret_cast<const void *>(&conv_kernel<32, 32, 0>),
                        reinterpret_cast<const void *>(&conv_kernel<32, 16, 1>),
                        reinterpret_cast<const void *>(&conv_kernel<16, 32, 2>),
                        reinterpret_cast<const void *>(&conv_kernel<32, 32, 2>)};
  const size_t bytes[5] = {halo_bytes<8>(N), halo_bytes<32>(N), halo_bytes<32>(N), halo_bytes<16>(N),
                           halo_bytes<32>(N)};
  for (int i = 0; i < 5; ++i) {
    if (bytes[i] > 160 * 1024) return hipErrorInvalidValue;
    const hipError_t e = fwr::raise_dynamic_lds(fns[i], int(bytes[i]));
    if (e != hipSuccess) return e;
  }
  hipError_t e = measure_grid(conv_kernel<8, 32, 0>, bytes[0], N);
  if (e == hipSuccess) e = measure_grid(conv_kernel<32, 32, 0>, bytes[1], N);
  if (e == hipSuccess) e = measure_grid(conv_kernel<32, 16, 1>, bytes[2], N);
  if (e == hipSuccess) e = measure_grid(conv_kernel<16, 32, 2>, bytes[3], N);
  if (e == hipSuccess) e = measure_grid(conv_kernel<32, 32, 2>, bytes[4], N);
  return e;
}

hipError_t conv(int layer, const uint16_t *x, const uint16_t *wt, const float *bias, void *out, int B, int N,
                float out_scale, hipStream_t s) {
  const int nt = tiles_of(B, N);
  const dim3 blk(256);
  if (layer == 0) {
    const auto k = conv_kernel<8, 32, 0>;
    hipLaunchKernelGGL(k, dim3(grid_of(k, N, nt)), blk, halo_bytes<8>(N), s, x, wt, bias, out,
                       nullptr, N, nt, 1.f);
  } else if (layer < 6) {
    const auto k = conv_kernel<32, 32, 0>;
    hipLaunchKernelGGL(k, dim3(grid_of(k, N, nt)), blk, halo_bytes<32>(N), s, x, wt, bias, out,
                       nullptr, N, nt, 1.f);
  } else {
    const auto k = conv_kernel<32, 16, 1>;
    hipLaunchKernelGGL(k, dim3(grid_of(k, N, nt)), blk, halo_bytes<32>(N), s, x, wt, bias, out,
                       nullptr, N, nt, out_scale);
  }
  return hipGetLastError();
}

// gradient w.r.t. the input of `layer` (layer >= 1), masked by the previous layer's ReLU
hipError_t conv_bwd_data(int layer, const uint16_t *dz, const uint16_t *wtb, const uint16_t *act_prev, uint16_t *dx,
                         int B, int N, hipStream_t s) {
  const int nt = tiles_of(B, N);
  const dim3 blk(256);
  if (layer == 6) {
    const auto k = conv_kernel<16, 32, 2>;
    hipLaunchKernelGGL(k, dim3(grid_of(k, N, nt)), blk, halo_bytes<16>(N), s, dz, wtb, nullptr, dx,
                       act_prev, N, nt, 1.f);
  } else {
    const auto k = conv_kernel<32, 32, 2>;
    hipLaunchKernelGGL(k, dim3(grid_of(k, N, nt)), blk, halo_bytes<32>(N), s, dz, wtb, nullptr, dx,
                       act_prev, N, nt, 1.f);
  }
  return hipGetLastError();
}

hipError_t wgrad(int layer, const uint16_t *x, const uint16_t *dz, float *dw, float *db, int B, int N, hipStream_t s) {
  if (layer == 0)
    hipLaunchKernelGGL((wgrad_kernel<8, 32>), dim3(B), dim3(256), 0, s, x, dz, dw, db, N);
  else if (layer < 6)
    hipLaunchKernelGGL((wgrad_kernel<32, 32>), dim3(B), dim3(256), 0, s, x, dz, dw, db, N);
  else
    hipLaunchKernelGGL((wgrad_kernel<32, 16>), dim3(B), dim3(256), 0, s, x, dz, dw, db, N);
  return hipGetLastError();
}

hipError_t features(const float *slopes, const uint8_t *mask, uint16_t *feat, int B, int n, int N, float scale,
                    hipStream_t s) {
  const size_t total = (size_t)B * N * N;
  hipLaunchKernelGGL(features_kernel, dim3((total + 255) / 256), dim3(256), 0, s, slopes, mask, feat, B, n, N, scale);
  return hipGetLastError();
}

hipError_t loss_grad(const float *pred, const float *target, const uint8_t *mask, uint16_t *dz7, float *loss, int B,
                     int n, int N, float scale, float inv_count, hipStream_t s) {
  const size_t total = (size_t)B * N * N;
  hipLaunchKernelGGL(loss_grad_kernel, dim3((total + 255) / 256), dim3(256), 0, s, pred, target, mask, dz7, loss, B,
                     n, N, scale, inv_count);
  return hipGetLastError();
}

hipError_t loss_grad_map(const float *pred, const float *target, const uint8_t *mask, float *grad, float *loss, int B,
                         int n, int N, float scale, float inv_count, hipStream_t s) {
  const size_t total = (size_t)B * N * N;
  hipLaunchKernelGGL(loss_grad_map_kernel, dim3((total + 255) / 256), dim3(256), 0, s, pred, target, mask, grad, loss,
                     B, n, N, scale, inv_count);
  return hipGetLastError();
}

hipError_t grad_in(const float *grad, uint16_t *dz7, int B, int N, float inv_scale, hipStream_t s) {
  const size_t total = (size_t)B * N * N;
  hipLaunchKernelGGL(grad_in_kernel, dim3((total + 255) / 256), dim3(256), 0, s, grad, dz7, B, N, inv_scale);
  return hipGetLastError();
}

hipError_t adam(float *w, const float *g, float *m1, float *m2, int count, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3((count + 255) / 256), dim3(256), 0, s, w, g, m1, m2, count, lr, b1, b2, eps,
                     c1, c2);
  return hipGetLastError();
}

hipError_t pack(const float *w, uint16_t *wt, uint16_t *wtb, int cin_s, int cout_s, int kpad_f, int kpad_b,
                hipStream_t s) {
  const int n = cout_s * kpad_f > cin_s * kpad_b ? cout_s * kpad_f : cin_s * kpad_b;
  hipLaunchKernelGGL(pack_kernel, dim3((n + 255) / 256), dim3(256), 0, s, w, wt, wtb, cin_s, cout_s, kpad_f, kpad_b);
  return hipGetLastError();
}

}  // namespace cnn_launch
}  // namespace fwr
