// Device-side synthetic frames (von Karman screens, Fried slopes, noise).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fwr {

struct GenArgs {
  float *slopes;          // [B][2][n][n]
  float *phase;           // optional [B][n+1][n+1] true node phase (NULL: not written)
  const uint8_t *mask;    // [n][n] valid subapertures (device)
  uint64_t *d_counter;    // optional device frame counter added to first_pair * 2 (advanced by B)
  uint64_t first_pair;    // frame pair index of the batch's first pair
  uint32_t seed_lo, seed_hi;
  float r0, L0, d, sigma, vk_const;
  int B, n, o;
};

bool gen_supported(int N);
hipError_t gen_launch(int N, const GenArgs &a, hipStream_t s);

// The Fried slope model applied to node phases: slopes[B][2][n][n] of phase[B][n+1][n+1], plus
// noise[B][2][n][n] when given, zero on invalid subapertures (mask[n][n] on the device).
hipError_t fried_slopes_launch(const float *phase, const float *noise, const uint8_t *mask, float *slopes, int B,
                               int n, hipStream_t s);

}  // namespace fwr
