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

// 256-point line FFT in LDS (L = padded line), thread r = 0..15 of the line's 16.
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
    for (int k = 1; k < R; ++k) v[k] = cmul(v[k], tw[(r * k) & (NN - 1)]);
#pragma unroll
    for (int k = 0; k < R; ++k) L[pad(R * k + r)] = v[k];
  } else {
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = L[pad(R * k + r)];
#pragma unroll
    for (int k = 1; k < R; ++k) v[k] = cmul_conj(v[k], tw[(r * k) & (NN - 1)]);
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

// frequency held at position p of a transformed line, and the position of frequency f
__device__ __host__ __forceinline__ constexpr int freq_of(int p) { return (p >> 4) + R * (p & (R - 1)); }
__device__ __host__ __forceinline__ constexpr int pos_of(int f) { return R * (f & (R - 1)) + (f >> 4); }

}  // namespace mp
}  // namespace fwr
