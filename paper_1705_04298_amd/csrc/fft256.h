// 256-point line FFT for the multi-pass paths (grids too large for one workgroup's LDS):
// 16 threads per line, 16 x 16 decomposition through LDS.
// Stage A: thread r takes points 16a + r, DFT-16 over a, twiddle W_256^(r k1); stage B: thread k1
// takes the 16 contiguous results, DFT-16.  Position 16 k1 + k2 then holds frequency k1 + 16 k2
// (digit-reversed); the inverse undoes it.  Lines are padded by one element every 16, plus one
// (273 per line), to spread LDS banks.
#pragma once

#include "fft_lane.h"

namespace fwr {
namespace mp {

constexpr int NN = 256;
constexpr int R = 16;
constexpr int LP = NN + NN / R + 1;  // padded line length (complex); odd, so that the column
                                     // pass's transposing copies spread over the LDS banks
constexpr int THREADS = 256;

__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// Stage-A twiddle table, staged in LDS by the caller: entry 17 r + k = W_256^(r k) (k < 16, entry
// 17 r + 16 unused), so that thread r reads its 15 twiddles at one base address with immediate
// offsets, and the 16 threads of a line, reading the same k, hit 16 different bank pairs (odd row
// pitch). TW_RK entries, staged by threads t < TW_RK.
constexpr int TW_RK = 17 * 16;
__device__ __forceinline__ float2 tw_rk_entry(const float2 *tw256, int t) {
  const int r = t / 17, k = t % 17;
  return tw256[(r * k) & 255];
}
// the whole table, by the nt threads of a workgroup (t = 0..nt-1)
__device__ __forceinline__ void stage_tw_rk(float2 *tw, const float2 *tw256, int t, int nt) {
  for (int i = t; i < TW_RK; i += nt) tw[i] = tw_rk_entry(tw256, i);
}

// 256-point line FFT in LDS (L = padded line), thread r = 0..15 of the line's 16; tw: tw_rk_entry.
// The caller separates stages with workgroup barriers (all lines of a block
// are transformed together).
template <int DIR>
__device__ __forceinline__ void fft_stage_a(float2 *L, int r, const float2 *tw) {
  float2 v[R];
  if constexpr (DIR < 0) {
#pragma unroll
    for (int a = 0; a < R; ++a) v[a] = L[pad(R * a + r)];
    dft<R, -1>(v);
#pragma unroll
    for (int k = 1; k < R; ++k) v[k] = cmul(v[k], tw[17 * r + k]);
#pragma unroll
    for (int k = 0; k < R; ++k) L[pad(R * k + r)] = v[k];
  } else {
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = L[pad(R * k + r)];
#pragma unroll
    for (int k = 1; k < R; ++k) v[k] = cmul_conj(v[k], tw[17 * r + k]);
    dft<R, +1>(v);
#pragma unroll
    for (int a = 0; a < R; ++a) L[pad(R * a + r)] = v[a];
  }
}
template <int DIR>
__device__ __forceinline__ void fft_stage_b(float2 *L, int r) {
  float2 v[R];
#pragma unroll
  for (int b = 0; b < R; ++b) v[b] = L[pad(R * r + b)];
  dft<R, DIR>(v);
#pragma unroll
  for (int b = 0; b < R; ++b) L[pad(R * r + b)] = v[b];
}

// The same transform with 64 threads per line (one wave per line): quads of lanes take the
// 16-point sub-transforms (line_fft_fwd<4> / line_fft_inv<4>: in-lane DFT-4, twiddles W_16, DFT-4
// across the quad, after which lane j holds sub-frequencies k + 4 beta(j), beta = (0, 2, 1, 3)).
// The LDS positions before, between and after the two stages are those of fft_stage_a /
// fft_stage_b, so both forms leave (and expect) frequency k1 + 16 k2 at position 16 k1 + k2.
// u = thread of the line (0..63), q its quad lane constants; tw16[4 k + j] = W_16^(j k);
// twq[64 k + u] = W_256^(r f1) for u = 4 r + j, f1 = k + 4 beta(j) (the stage-A twiddles in lane
// order, so that a wave's reads are consecutive).
__device__ __host__ __forceinline__ constexpr int quad_beta(int j) { return j == 1 ? 2 : (j == 2 ? 1 : j); }

template <int DIR>
__device__ __forceinline__ void fft_quad_stage_a(float2 *L, int u, const float2 *twq, const float2 *tw16,
                                                 const QuadLane &q) {
  const int r = u >> 2, j = u & 3, fb = 4 * quad_beta(j);
  float2 v[4];
  if constexpr (DIR < 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = L[pad(R * (4 * k + j) + r)];
    line_fft_fwd<4>(v, tw16, j, q);
#pragma unroll
    for (int k = 0; k < 4; ++k) L[pad(R * (k + fb) + r)] = cmul(v[k], twq[64 * k + u]);
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = cmul_conj(L[pad(R * (k + fb) + r)], twq[64 * k + u]);
    line_fft_inv<4>(v, tw16, j, q);
#pragma unroll
    for (int k = 0; k < 4; ++k) L[pad(R * (4 * k + j) + r)] = v[k];
  }
}
template <int DIR>
__device__ __forceinline__ void fft_quad_stage_b(float2 *L, int u, const float2 *tw16, const QuadLane &q) {
  const int f1 = u >> 2, j = u & 3, gb = 4 * quad_beta(j);
  float2 v[4];
  if constexpr (DIR < 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = L[pad(R * f1 + 4 * k + j)];
    line_fft_fwd<4>(v, tw16, j, q);
#pragma unroll
    for (int k = 0; k < 4; ++k) L[pad(R * f1 + k + gb)] = v[k];
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = L[pad(R * f1 + k + gb)];
    line_fft_inv<4>(v, tw16, j, q);
#pragma unroll
    for (int k = 0; k < 4; ++k) L[pad(R * f1 + 4 * k + j)] = v[k];
  }
}
// table entries from the 256-entry table W_256^e
__device__ __forceinline__ float2 tw16_entry(const float2 *tw256, int i) { return tw256[R * (i & 3) * (i >> 2)]; }
__device__ __forceinline__ float2 twq_entry(const float2 *tw256, int i) {
  const int k = i >> 6, u = i & 63, r = u >> 2, f1 = k + 4 * quad_beta(u & 3);
  return tw256[(r * f1) & (NN - 1)];
}

// frequency held at position p of a transformed line, and the position of frequency f
__device__ __host__ __forceinline__ constexpr int freq_of(int p) { return (p >> 4) + R * (p & (R - 1)); }
__device__ __host__ __forceinline__ constexpr int pos_of(int f) { return R * (f & (R - 1)) + (f >> 4); }

}  // namespace mp
}  // namespace fwr
