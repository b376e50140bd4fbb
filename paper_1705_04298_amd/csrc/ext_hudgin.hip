// The comparison extension of Sec. 3.2 ("Hudgin extension"): x slopes repeated up and down the
// columns, y slopes left and right along the rows, from the nearest in-pupil cell of the line
// (the plan tabulates the source cell of every grid cell), then Eq. 5 on the extended slopes.
// One workgroup per frame; the frame's extended slopes are staged in LDS for the line sums.
#include "hudgin.h"
#include "lds_limit.h"

namespace fwr {

__global__ __launch_bounds__(256) void hudgin_kernel(HudginArgs a) {
  extern __shared__ float ex[];  // [2][N][N]: s_x then s_y
  const int f = blockIdx.x, N = a.N, NN = N * N, plane = a.n * a.n;
  const float *sf = a.slopes + (size_t)f * 2 * plane;
  float *ey = ex + NN;
  float *sums = ey + NN;  // [2][N]: row sums of s_x, column sums of s_y; then [2][N][4] partials
  // gather in chunks whose loads are all issued before the LDS stores (cells without a
  // source read cell 0 and are replaced by zeros)
  constexpr int CH = 8;
  for (int i0 = threadIdx.x; i0 < NN; i0 += CH * 256) {
    int sx[CH], sy[CH];
    float vx[CH], vy[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = i0 + u * 256;
      sx[u] = i < NN ? a.src_x[i] : -1;
      sy[u] = i < NN ? a.src_y[i] : -1;
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      vx[u] = sf[sx[u] >= 0 ? sx[u] : 0];
      vy[u] = sf[plane + (sy[u] >= 0 ? sy[u] : 0)];
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = i0 + u * 256;
      if (i < NN) {
        ex[i] = sx[u] >= 0 ? vx[u] : 0.f;
        ey[i] = sy[u] >= 0 ? vy[u] : 0.f;
      }
    }
  }
  __syncthreads();
  // fixed-order line sums: four partial sums per line (every fourth element), then combined
  float *part = sums + 2 * N;  // [2][N][4]
  for (int task = threadIdx.x; task < 8 * N; task += blockDim.x) {
    const int q = task & 3, line = (task >> 2) % N, col = task >= 4 * N;
    float acc = 0.f;
    for (int u = q; u < N; u += 4) acc += col ? ey[u * N + line] : ex[line * N + u];
    part[(col * N + line) * 4 + q] = acc;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 2 * N; t += blockDim.x)
    sums[t] = (part[4 * t] + part[4 * t + 1]) + (part[4 * t + 2] + part[4 * t + 3]);
  __syncthreads();
  float *o = a.out + (size_t)f * 2 * NN;
  for (int i = threadIdx.x; i < NN; i += blockDim.x) {
    const int m = i / N, c = i - m * N;
    o[i] = c == N - 1 ? ex[i] - sums[m] : ex[i];
    o[NN + i] = m == N - 1 ? ey[i] - sums[N + c] : ey[i];
  }
}

size_t hudgin_lds_bytes(int N) { return (size_t)(2 * N * N + 2 * N + 8 * N) * sizeof(float); }

hipError_t hudgin_prepare(int N) {
  return raise_dynamic_lds(reinterpret_cast<const void *>(&hudgin_kernel), int(hudgin_lds_bytes(N)));
}

hipError_t hudgin_launch(const HudginArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(hudgin_kernel, dim3(a.B), dim3(256), hudgin_lds_bytes(a.N), s, a);
  return hipGetLastError();
}

}  // namespace fwr
