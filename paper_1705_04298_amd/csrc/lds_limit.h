// Dynamic-LDS limit of a kernel.  hipFuncAttributeMaxDynamicSharedMemorySize is process-wide
// state of the kernel on the current device, shared by every plan that launches it, so a plan
// must never lower it below what an earlier plan's launches ask for: the limit only grows.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

namespace fwr {

// Raise the limit of `fn` on the current device to at least `bytes` (no-op when already there).
// Inline: one table for the whole library, whichever unit calls it.
inline hipError_t raise_dynamic_lds(const void *fn, int bytes) {
  static std::mutex mu;
  static std::map<std::pair<int, const void *>, int> limit;  // (device, kernel) -> bytes set
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  auto it = limit.find({dev, fn});
  if (it != limit.end() && it->second >= bytes) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) limit[{dev, fn}] = bytes;
  return e;
}

}  // namespace fwr
