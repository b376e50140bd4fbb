// Fallback of the learned start: frames whose in-pupil residual after the network's start
// exceeds a threshold (or is not a number) are listed in ascending order, their measured slopes gathered into a
// compact batch for the plain loop, and the plain loop's phases scattered back in place.
#include "learned.h"

#include <map>
#include <mutex>

namespace fwr {

// Fixed device workspace of the allocation-free learned call (fwr_reconstruct_learned_noalloc):
// the frame list, its length and one chunk of gathered slopes and phases (layout in learned.h).
// One copy per GPU, held until the process ends.  In host code this name is not a device
// address: the address comes from hipGetSymbolAddress (fallback_scratch) and only that is used.
static __device__ __align__(256) unsigned char scratch[FWR_NOALLOC_SCRATCH_BYTES];

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

// The same move for list positions off + blockIdx.x, for as many of them as the device-side list
// length *count allows (blocks past it exit at once): the chunks of the allocation-free call.
template <bool GATHER>
__global__ __launch_bounds__(256) void move_counted_kernel(const float *src, const int32_t *idx, const int32_t *count,
                                                           int off, float *dst, int per_frame) {
  const int j = off + int(blockIdx.x);
  if (j >= *count) return;
  const size_t from = GATHER ? (size_t)idx[j] : blockIdx.x;
  const size_t to = GATHER ? blockIdx.x : (size_t)idx[j];
  const float *s = src + from * per_frame;
  float *d = dst + to * per_frame;
  for (int i = threadIdx.x; i < per_frame; i += 256) d[i] = s[i];
}

}  // namespace

hipError_t fallback_scratch(void **ptr) {
  static std::mutex mu;
  static std::map<int, void *> addr;  // device -> address of its copy of `scratch`
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
    it = addr.emplace(dev, p).first;
  }
  *ptr = it->second;
  return hipSuccess;
}

hipError_t fallback_gather_counted(const float *src, const int32_t *idx, const int32_t *count, int off, float *dst,
                                   int blocks, int per_frame, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(move_counted_kernel<true>, dim3(blocks), dim3(256), 0, s, src, idx, count, off, dst, per_frame);
  return hipGetLastError();
}

hipError_t fallback_scatter_counted(const float *src, const int32_t *idx, const int32_t *count, int off, float *dst,
                                    int blocks, int per_frame, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(move_counted_kernel<false>, dim3(blocks), dim3(256), 0, s, src, idx, count, off, dst,
                     per_frame);
  return hipGetLastError();
}

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
