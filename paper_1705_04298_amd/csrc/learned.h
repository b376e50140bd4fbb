// Device side of the learned start's fallback, and what the reconstruction API needs to know
// of a network handle.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/fwr.h"

namespace fwr {

// Grid of a network handle and the stream it enqueues on; false for an invalid handle.
bool cnn_info(fwr_cnn_t cnn, int *n_sub, int *n_grid, int *max_batch, hipStream_t *stream);

// Ascending list of the frames i < B with resid[i] > threshold, and its length in *count
// (device memory; one workgroup).
hipError_t fallback_select(const float *resid, float threshold, int B, int32_t *idx, int32_t *count,
                           hipStream_t s);
// dst[j] = src[idx[j]] (gather) or dst[idx[j]] = src[j] (scatter), j < count, for records of
// per_frame floats.
hipError_t fallback_gather(const float *src, const int32_t *idx, float *dst, int count, int per_frame,
                           hipStream_t s);
hipError_t fallback_scatter(const float *src, const int32_t *idx, float *dst, int count, int per_frame,
                            hipStream_t s);

// Allocation-free variant.  The library's fixed device workspace (FWR_NOALLOC_SCRATCH_BYTES,
// one per GPU) on the current device: frame list int32[FWR_NOALLOC_MAX_FRAMES] at byte 0, its
// length at kNoallocCountOffset, the chunk buffers from kNoallocChunkOffset on.
constexpr size_t kNoallocCountOffset = (size_t)FWR_NOALLOC_MAX_FRAMES * sizeof(int32_t);
constexpr size_t kNoallocChunkOffset = kNoallocCountOffset + 256;
hipError_t fallback_scratch(void **ptr);
// Gather / scatter of list positions off .. off + blocks - 1 that lie below the device-side
// list length *count (the other blocks exit).
hipError_t fallback_gather_counted(const float *src, const int32_t *idx, const int32_t *count, int off, float *dst,
                                   int blocks, int per_frame, hipStream_t s);
hipError_t fallback_scatter_counted(const float *src, const int32_t *idx, const int32_t *count, int off, float *dst,
                                    int blocks, int per_frame, hipStream_t s);

}  // namespace fwr
