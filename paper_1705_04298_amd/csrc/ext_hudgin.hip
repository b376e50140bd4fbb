// The comparison extension of Sec. 3.2 ("Hudgin extension"): x slopes repeated up and down the
// columns, y slopes left and right along the rows, from the nearest in-pupil cell of the line
// (the plan tabulates the source cell of every grid cell), then Eq. 5 on the extended slopes.
// One workgroup per frame; the frame's extended slopes are staged in LDS for the line sums.
#include "hudgin.h"

namespace fwr {

__global__ __launch_bounds__(256) void hudgin_kernel(HudginArgs a) {
  extern __shared__ float ex[];  // [2][N][N]: s_x then s_y
  const int f = blockIdx.x, N = a.N, NN = N * N, plane = a.n * a.n;
  const float *sf = a.slopes + (size_t)f * 2 * plane;
  float *ey = ex + NN;
  float *sums = ey + NN;  // [2][N]: row sums of s_x, column sums of s_y
  for (int i = threadIdx.x; i < NN; i += blockDim.x) {
    const int sxi = a.src_x[i], syi = a.src_y[i];
    ex[i] = sxi >= 0 ? sf[sxi] : 0.f;
    ey[i] = syi >= 0 ? sf[plane + syi] : 0.f;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < N; t += blockDim.x) {  // fixed-order line sums
    float r = 0.f, c = 0.f;
    for (int u = 0; u < N; ++u) {
      r += ex[t * N + u];
      c += ey[u * N + t];
    }
    sums[t] = r;
    sums[N + t] = c;
  }
  __syncthreads();
  float *o = a.out + (size_t)f * 2 * NN;
  for (int i = threadIdx.x; i < NN; i += blockDim.x) {
    const int m = i / N, c = i - m * N;
    o[i] = c == N - 1 ? ex[i] - sums[m] : ex[i];
    o[NN + i] = m == N - 1 ? ey[i] - sums[N + c] : ey[i];
  }
}

size_t hudgin_lds_bytes(int N) { return (size_t)(2 * N * N + 2 * N) * sizeof(float); }

hipError_t hudgin_prepare(int N) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&hudgin_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(hudgin_lds_bytes(N)));
}

hipError_t hudgin_launch(const HudginArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(hudgin_kernel, dim3(a.B), dim3(256), hudgin_lds_bytes(a.N), s, a);
  return hipGetLastError();
}

}  // namespace fwr
