// Launch interface of the Fourier-domain (packed projector) Gerchberg kernel, used for slope
// models that have no compact real-space stencil (the lenslet-averaging model of Eq. 4).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fwr {

enum : int { kFourierPeriodic = 1, kFourierPeriodicEach = 2, kFourierExtend = 4 };

struct FourierArgs {
  const float *slopes;     // [B][2][n][n]
  float *out;              // [B][n+1][n+1], or [B][2][N][N] with kFourierExtend
  const float *start;      // optional [B][2][N][N]: start slopes outside the pupil (NULL = zeros)
  float *resid;            // optional [B]: in-pupil misfit of the last iteration
  const float *alpha;      // [4N][T]: loop coefficient of Z (real), column-phase slot k of thread t
  const float2 *beta;      // [4N][T]: loop coefficient of conj(Z(-l, -k))
  const float2 *fin_a;     // [4N][T]: final coefficient of Z
  const float2 *fin_b;     // [4N][T]: final coefficient of conj(Z(-l, -k))
  const float2 *tw_lane;   // [T][4]: W_N^(j k)
  const uint32_t *inpupil; // [4N]: bit k set when cell (m, 4k + j) of thread t = 4m + j is in the pupil
  int B, n, o, n_iter, flags;
};

bool fourier_supported(int N);
bool fourier_frames_ok(int N, int n, int frames);  // frames per workgroup 1 or 2, LDS fits
int fourier_threads(int N, int frames);
int fourier_lds_bytes(int N, int n, int frames);
hipError_t fourier_prepare(int N, int n, int frames);
hipError_t fourier_launch(int N, const FourierArgs &a, hipStream_t s, int frames);

}  // namespace fwr
