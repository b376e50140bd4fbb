// Launch interface of the multi-pass Fourier-domain Gerchberg path: the lenslet-averaging
// model of Eq. 4 on grids too large for one workgroup's LDS (N = 256).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace fwr {

struct FSArgs {
  const float *slopes;   // [B][2][n][n]
  float *out;            // [B][n+1][n+1], or [B][2][N][N] for the extended slopes
  float2 *spec;          // [B][N][N]: Z = TF(s_x + i s_y), rows in digit-reversed positions
  float2 *state;         // [B][N][N]: s_x + i s_y in real space where Eq. 5 or the output needs it
  float *rsum;           // [B][N]: row sums of s_x (Eq. 5)
  float *cpart;          // [B][N/16][N]: column sums of s_y over each block of 16 rows (Eq. 5)
  const float *alpha;    // [N][N] (column position, row position): loop coefficient of Z, / N^2
  const float2 *beta;    // loop coefficient of conj(Z(-l, -k)), / N^2
  const float2 *fin_a;   // final coefficients of Z and of conj(Z(-l, -k)), / N^2
  const float2 *fin_b;
  const float2 *tw256;   // W_256^e, e = 0..255
  const uint8_t *mask;   // [n][n]
  uint32_t *ctl;         // work counters of the persistent loop: [0] next item, [1] error, one count
                         // per frame on its own 256-byte line
  const uint32_t *loop_err = nullptr;  // set by the launcher after a persistent loop: its error word
  int wait_limit = 1 << 20;            // polls of a count before the persistent loop gives up
  int shape = 0;                       // 0: one launch per pass; 2: the loop as one persistent launch
  int B, n, o, n_iter, flags;  // flags: kFourierPeriodic, kFourierPeriodicEach (fourier.h)
};

bool fourier_mp_supported(int N);
size_t fourier_mp_workspace_bytes(int N, int max_batch);
size_t fourier_mp_ctl_words(int max_batch);
hipError_t fourier_mp_run(const FSArgs &a, bool extend, hipStream_t s);

}  // namespace fwr
