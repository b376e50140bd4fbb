// Launch interface of the on-chip (LDS-resident) Gerchberg kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fwr {

enum : int { kFlagPeriodic = 1, kFlagPeriodicEach = 2, kFlagExtend = 4 };

struct OnchipArgs {
  const float *slopes;    // [B][2][n][n]
  float *out;             // [B][n+1][n+1], or [B][2][N][N] with kFlagExtend
  const float *h_loop;    // [4N][T]: loop filter for thread t's k-th column-phase output
  const float *h_final;   // [4N][T]: final (Wiener) filter, same layout
  const float2 *tw_lane;  // [T][4]: W_N^(j k)
  const uint32_t *codes;  // [(T+7)/8][4N]: 4 bits per node of thread t, nodes 8w..8w+7 in word w;
                          // bit 0: cell (m, n) outside the pupil, bit 1: cell (m-1, n-1),
                          // bit 2: cell (m, n-1), bit 3: cell (m-1, n)
  const float *start;     // optional [B][2][N][N]: out-of-pupil start slopes (NULL: zeros)
  float *resid;           // optional [B]: in-pupil misfit of the last iteration
  const uint8_t *mask;    // [n][n]: 1 = valid subaperture
  // optional device count: the batch is min(B, max(0, *count - count_off)) frames, read by the
  // kernel (workgroups past it exit at once); NULL = B frames
  const int32_t *count = nullptr;
  int count_off = 0;
  int B, n, o, n_iter, flags;
};

// `pairs`: frame pairs per workgroup (1, 2, 4, 8; see onchip_pairs_ok)
bool onchip_supported(int N);
bool onchip_pairs_ok(int N, int n, int pairs, bool periodic_each);  // instantiated and fits the LDS
int onchip_threads(int N, int pairs);                  // per workgroup
int onchip_lds_bytes(int N, int n, int pairs);         // per workgroup, static + dynamic
hipError_t onchip_prepare(int N, int n, int pairs);    // before the first launch with `pairs`
// `sched`: radix schedule of the in-lane DFTs (0 or 1) for the windowed kernel of 2x-padded
// plans (onchip_sched_ok); other launches take schedule 0
bool onchip_sched_ok(int N, int n);
hipError_t onchip_launch(int N, const OnchipArgs &a, hipStream_t s, int pairs, int sched);

}  // namespace fwr
