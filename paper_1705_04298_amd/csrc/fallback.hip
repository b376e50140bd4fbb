// Fallback of the learned start: frames whose in-pupil residual after the network's start
// exceeds a threshold (or is not a number) are listed in ascending order, their measured slopes gathered into a
// compact batch for the plain loop, and the plain loop's phases scattered back in place.
#include "learned.h"

namespace fwr {

namespace {

constexpr int kSelThreads = 1024;

// One workgroup walks the residuals in chunks of 1024; within a chunk each wave ballots its
// flags and the list positions follow from the counts of the waves before it.
__global__ __launch_bounds__(kSelThreads) void select_kernel(const float *resid, float threshold, int B,
                                                             int32_t *idx, int32_t *count) {
  __shared__ int wave_n[kSelThreads / 64];
  __shared__ int base;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int c0 = 0; c0 < B; c0 += kSelThreads) {
    const int i = c0 + threadIdx.x;
    const bool f = i < B && !(resid[i] <= threshold);  // a NaN residual always falls back
    const uint64_t m = __ballot(f);
    if (lane == 0) wave_n[w] = __popcll(m);
    __syncthreads();
    int off = base;
    for (int k = 0; k < w; ++k) off += wave_n[k];
    if (f) idx[off + __popcll(m & ((uint64_t(1) << lane) - 1))] = i;
    __syncthreads();  // every thread has read base and the wave counts
    if (threadIdx.x == 0) {
      int t = 0;
      for (int k = 0; k < kSelThreads / 64; ++k) t += wave_n[k];
      base += t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = base;
}

template <bool GATHER>
__global__ __launch_bounds__(256) void move_kernel(const float *src, const int32_t *idx, float *dst, int per_frame) {
  const size_t from = GATHER ? (size_t)idx[blockIdx.x] : blockIdx.x;
  const size_t to = GATHER ? blockIdx.x : (size_t)idx[blockIdx.x];
  const float *s = src + from * per_frame;
  float *d = dst + to * per_frame;
  for (int i = threadIdx.x; i < per_frame; i += 256) d[i] = s[i];
}

}  // namespace

hipError_t fallback_select(const float *resid, float threshold, int B, int32_t *idx, int32_t *count,
                           hipStream_t s) {
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(kSelThreads), 0, s, resid, threshold, B, idx, count);
  return hipGetLastError();
}

hipError_t fallback_gather(const float *src, const int32_t *idx, float *dst, int count, int per_frame,
                           hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(move_kernel<true>, dim3(count), dim3(256), 0, s, src, idx, dst, per_frame);
  return hipGetLastError();
}

hipError_t fallback_scatter(const float *src, const int32_t *idx, float *dst, int count, int per_frame,
                            hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(move_kernel<false>, dim3(count), dim3(256), 0, s, src, idx, dst, per_frame);
  return hipGetLastError();
}

}  // namespace fwr
