// Launch interface of the multi-pass (grid through HBM) Gerchberg path, N = 256.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace fwr {

enum : int { kMPPeriodic = 1, kMPPeriodicEach = 2 };

struct MPArgs {
  const float *slopes;   // [B][2][n][n]
  float *out;            // [B][n+1][n+1] or [B][2][N][N]
  // workspace, per frame pair: four N x N complex fields, the forcing rows and the sums
  float2 *phi, *spec, *sx, *sy;
  float2 *f0;            // [pairs][n+1][N], node (m, r + 16 q) of a row at 16 r + q
  float2 *sums;          // [pairs][2N]: C_n then R_m
  uint32_t *bad;         // [pairs][N/16]: per window row block, bit 0 (frame A) and bit 1 (frame B)
                         // set where an in-pupil measured slope is not finite
  const float *h_loop;   // [N][N], column position major, digit-reversed positions
  const float *h_final;
  const float2 *tw256;   // W_256^e, e = 0..255
  const uint8_t *mask;   // [n][n]
  const uint64_t *codes; // [N][16]: out-of-pupil bits of the 4 cells around each node, node (m, r + 16 q)
                         // in bits 4q..4q+3 of codes[16 m + r]
  uint32_t *ctl;         // work counters of the persistent loop kernel
  const uint32_t *loop_err = nullptr;  // set by the launcher after a persistent loop: its error word
  int B, n, o, n_iter, flags;
  int wait_limit = 1 << 20;  // polls of a count before the persistent loop gives up
  int col_shape = 0;     // launch shape: 0 = column pass with 16 threads per 256-point line, 1 = 64
                         // (quad sub-transforms), 2 = the loop as one persistent launch (16 threads)
};

bool multipass_supported(int N);
size_t multipass_workspace_bytes(int N, int n, int max_batch);
size_t multipass_ctl_words(int max_batch);
hipError_t multipass_run(const MPArgs &a, bool extend, hipStream_t s);
struct GenArgs;
hipError_t multipass_generate(const MPArgs &a, const GenArgs &g, hipStream_t s);

}  // namespace fwr
