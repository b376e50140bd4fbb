// Launch interface of the Hudgin (edge-repeating) comparison extension.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace fwr {

struct HudginArgs {
  const float *slopes;   // [B][2][n][n]
  float *out;            // [B][2][N][N]
  const int32_t *src_x;  // [N][N]: window index (i n + j) of the cell whose x slope fills this cell, -1 = 0
  const int32_t *src_y;  // [N][N]: the same for the y slopes
  int B, n, N;
};

size_t hudgin_lds_bytes(int N);
hipError_t hudgin_prepare(int N);
hipError_t hudgin_launch(const HudginArgs &a, hipStream_t s);

}  // namespace fwr
