// Multi-pass Fourier-domain Gerchberg extension + reconstruction for the lenslet-averaging model
// of Eq. 4 at N = 256 (a 256 x 256 complex field is 512 KiB, over the LDS).
//
// One frame per complex field, Z = TF(s_x + i s_y), with step 2 of Algorithm 1 as
// Z' = alpha Z + beta conj(Z(-l, -k)) and the final reconstruction as A Z + B conj(Z(-l, -k))
// (see gerchberg_fourier.hip), split into grid-wide passes through a per-frame spectrum field:
//   rows : the inverse row FFTs of the spectrum, step 4 (the measurement inside the pupil) and
//          the forward row FFTs of the next iteration, 16 rows per block, in one pass (the model
//          has no real-space stencil, so no halo rows); or the same ending in the real-space
//          slopes with their Eq. 5 sums; or the start, the Eq. 5 fix, the outputs;
//   cols : forward column FFTs, the packed projector, inverse column FFTs.  Each block takes 16
//          column positions closed under k -> -k, so the mirrored frequency is in its LDS.  The
//          row FFTs leave frequency a + 16 b at position 16 a + b; the mirror of position
//          16 a + b is 16 (16 - a) + 15 - b (a > 0) or (16 - b) mod 16 (a = 0): position groups
//          a and 16 - a pair up, groups 0 and 8 are closed.  A block takes 8 contiguous
//          positions of group a and their 8 (contiguous) mirrors, or all of group 0 or 8.
// With launch shape 2 the loop's column passes and row steps run as one persistent launch
// (loop_kernel, below).
#include <algorithm>
#include <atomic>

#include "fft256.h"
#include "fourier.h"
#include "fourier_mp.h"

namespace fwr {
namespace fs {

using namespace mp;

constexpr int RB = NN / R;  // row blocks of 16 rows

enum : int {
  kInit = 0,        // measurement (zeros outside the pupil) -> forward rows -> spec
  kInitStore = 1,   // measurement -> state, Eq. 5 sums (no iteration)
  kStep = 2,        // spec -> inverse rows -> step 4 -> forward rows -> spec
  kStepStore = 3,   // spec -> inverse rows -> step 4 -> state, Eq. 5 sums
  kFixFwd = 4,      // state -> Eq. 5 (with `fix`) -> forward rows -> spec
  kFixExt = 5,      // state -> Eq. 5 (with `fix`) -> extended slopes [2][N][N]
  kOut = 6          // spec -> inverse rows -> (n+1) x (n+1) phase window (real part)
};

__device__ __forceinline__ size_t fld(int f) { return (size_t)f * NN * NN; }

constexpr int kCtl = 64;  // words between two per-frame counts of the persistent loop

// spectrum accesses shared between the workgroups of the persistent loop: agent-scope coherent
// (relaxed atomics), since the XCDs' L2 caches are not coherent with each other within a launch
template <bool COH>
__device__ __forceinline__ float2 ldc(const float2 *p) {
  if constexpr (COH) {
    const unsigned long long v = __hip_atomic_load(reinterpret_cast<unsigned long long *>(const_cast<float2 *>(p)),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_float2(__uint_as_float(uint32_t(v)), __uint_as_float(uint32_t(v >> 32)));
  } else {
    return *p;
  }
}
template <bool COH>
__device__ __forceinline__ void stc(float2 *p, float2 v) {
  if constexpr (COH) {
    const unsigned long long b = uint64_t(__float_as_uint(v.x)) | (uint64_t(__float_as_uint(v.y)) << 32);
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    *p = v;
  }
}
__device__ __forceinline__ float nan_f() { return __uint_as_float(0x7fc00000u); }

// measured s_x + i s_y of cell (m, c) of frame f, 0 outside the pupil
__device__ __forceinline__ float2 meas(const FSArgs &a, int f, int m, int c) {
  const unsigned i = unsigned(m - a.o), j = unsigned(c - a.o);
  const bool in = i < unsigned(a.n) && j < unsigned(a.n) && a.mask[i * a.n + j] != 0;
  const size_t plane = (size_t)a.n * a.n, idx = in ? (size_t)i * a.n + j : 0;
  const float *s = a.slopes + (size_t)f * 2 * plane;
  const float x = s[idx], y = s[plane + idx];  // (cell 0 when outside: a valid read)
  return in ? make_float2(x, y) : make_float2(0.f, 0.f);
}

__device__ __forceinline__ bool in_pupil(const FSArgs &a, int m, int c) {
  const unsigned i = unsigned(m - a.o), j = unsigned(c - a.o);
  return i < unsigned(a.n) && j < unsigned(a.n) && a.mask[i * a.n + j] != 0;
}

// One loop step on rows m0 .. m0 + 15 of frame f (the kStep mode of rows_kernel; the persistent
// loop runs it with COH): inverse row FFTs of the spectrum, step 4, forward row FFTs.  L: R padded
// lines; tw staged by the caller.
template <bool COH>
__device__ __forceinline__ void rows_step(const FSArgs &a, float2 *L, const float2 *tw, int t, int f, int m0) {
  const int rl = t >> 4, r = t & 15;
  constexpr int PASSES = R * NN / THREADS;  // one grid row per pass of the block
  float2 *S = a.spec + fld(f);
  {
    float2 v[PASSES];
#pragma unroll
    for (int c_ = 0; c_ < PASSES; ++c_) v[c_] = ldc<COH>(S + uint32_t((m0 + c_) * NN + t));
#pragma unroll
    for (int c_ = 0; c_ < PASSES; ++c_) L[c_ * LP + pad(t)] = v[c_];
  }
  __syncthreads();
  fft_stage_b<+1>(L + rl * LP, r);
  __syncthreads();
  fft_stage_a<+1>(L + rl * LP, r, tw);
  __syncthreads();
  // step 4: the measurement inside the pupil, the extrapolation outside
#pragma unroll
  for (int c_ = 0; c_ < PASSES; ++c_) {
    const int m = m0 + c_;
    if (in_pupil(a, m, t)) L[c_ * LP + pad(t)] = meas(a, f, m, t);
  }
  __syncthreads();
  fft_stage_a<-1>(L + rl * LP, r, tw);
  __syncthreads();
  fft_stage_b<-1>(L + rl * LP, r);
  __syncthreads();
#pragma unroll
  for (int c_ = 0; c_ < PASSES; ++c_) stc<COH>(S + uint32_t((m0 + c_) * NN + t), L[c_ * LP + pad(t)]);
}

// rows m0 .. m0 + 15 of frame blockIdx.y, row block blockIdx.x + b0
__global__ __launch_bounds__(THREADS) void rows_kernel(FSArgs a, int mode, int b0, int fix) {
  __shared__ float2 L[R * LP];
  __shared__ float2 tw[TW_RK];
  __shared__ float red[R * R];
  const int t = threadIdx.x, rl = t >> 4, r = t & 15;
  const int f = blockIdx.y, rb = blockIdx.x + b0, m0 = rb * R;
  stage_tw_rk(tw, a.tw256, t, THREADS);
  if (mode == kStep) {
    rows_step<false>(a, L, tw, t, f, m0);
    return;
  }
  constexpr int PASSES = R * NN / THREADS;  // one grid row per pass of the block
  if (mode == kInit && rb == 0 && t < kCtl) {  // the persistent loop's counts: the frame's, and with
    a.ctl[(size_t)kCtl * (f + 1) + t] = 0u;    // frame 0 the item counter and the error word
    if (f == 0) a.ctl[t] = 0u;
  }
  // a persistent loop that gave up: every frame's output is NaN
  const bool failed = a.loop_err != nullptr && *a.loop_err != 0u;
  if (mode == kInit || mode == kInitStore) {
#pragma unroll
    for (int c_ = 0; c_ < PASSES; ++c_) L[c_ * LP + pad(t)] = meas(a, f, m0 + c_, t);
  } else if (mode == kFixFwd || mode == kFixExt) {
    const float2 *S = a.state + fld(f);
    float2 v[PASSES];
#pragma unroll
    for (int c_ = 0; c_ < PASSES; ++c_) v[c_] = S[(size_t)(m0 + c_) * NN + t];
    if (fix) {
      // Eq. 5: s_x(m, N-1) -= R_m, s_y(N-1, c) -= C_c (C_c summed over the row blocks in order)
      if (t == NN - 1) {
#pragma unroll
        for (int c_ = 0; c_ < PASSES; ++c_) v[c_].x -= a.rsum[(size_t)f * NN + m0 + c_];
      }
      if (rb == RB - 1) {
        float cs = 0.f;
        for (int b = 0; b < RB; ++b) cs += a.cpart[((size_t)f * RB + b) * NN + t];
        v[PASSES - 1].y -= cs;
      }
    }
#pragma unroll
    for (int c_ = 0; c_ < PASSES; ++c_) L[c_ * LP + pad(t)] = v[c_];
  } else {
    const float2 *S = a.spec + fld(f);
#pragma unroll
    for (int c_ = 0; c_ < PASSES; ++c_) L[c_ * LP + pad(t)] = S[(size_t)(m0 + c_) * NN + t];
  }
  __syncthreads();
  if (mode == kStep || mode == kStepStore || mode == kOut) {
    fft_stage_b<+1>(L + rl * LP, r);
    __syncthreads();
    fft_stage_a<+1>(L + rl * LP, r, tw);
    __syncthreads();
  }
  if (mode == kOut) {
    const int n1 = a.n + 1;
    float *o = a.out + (size_t)f * n1 * n1;
#pragma unroll
    for (int c_ = 0; c_ < PASSES; ++c_) {
      const int m = m0 + c_;
      if (m >= a.o && m <= a.o + a.n && t >= a.o && t <= a.o + a.n)
        o[(size_t)(m - a.o) * n1 + (t - a.o)] = failed ? nan_f() : L[c_ * LP + pad(t)].x;
    }
    return;
  }
  if (mode == kStep || mode == kStepStore) {
    // step 4: the measurement inside the pupil, the extrapolation outside
#pragma unroll
    for (int c_ = 0; c_ < PASSES; ++c_) {
      const int m = m0 + c_;
      if (in_pupil(a, m, t)) L[c_ * LP + pad(t)] = meas(a, f, m, t);
    }
    __syncthreads();
  }
  if (mode == kFixExt) {
    const size_t gplane = (size_t)NN * NN;
    float *e = a.out + (size_t)f * 2 * gplane;
#pragma unroll
    for (int c_ = 0; c_ < PASSES; ++c_) {
      const float2 v = L[c_ * LP + pad(t)];
      e[(size_t)(m0 + c_) * NN + t] = failed ? nan_f() : v.x;
      e[gplane + (size_t)(m0 + c_) * NN + t] = failed ? nan_f() : v.y;
    }
    return;
  }
  if (mode == kInitStore || mode == kStepStore) {
    float2 *S = a.state + fld(f);
#pragma unroll
    for (int c_ = 0; c_ < PASSES; ++c_) S[(size_t)(m0 + c_) * NN + t] = L[c_ * LP + pad(t)];
    // Eq. 5 sums in a fixed order: R_m over the row (16 partials of 16), C partials over the block
    float part = 0.f;
#pragma unroll
    for (int q = 0; q < R; ++q) part += L[rl * LP + pad(r + R * q)].x;
    red[rl * R + r] = part;
    float cs = 0.f;
#pragma unroll
    for (int c_ = 0; c_ < PASSES; ++c_) cs += L[c_ * LP + pad(t)].y;
    a.cpart[((size_t)f * RB + rb) * NN + t] = cs;
    __syncthreads();
    if (r == 0) {
      float rs = 0.f;
      for (int q = 0; q < R; ++q) rs += red[rl * R + q];
      a.rsum[(size_t)f * NN + m0 + rl] = rs;
    }
    return;
  }
  // forward row FFTs -> spectrum
  fft_stage_a<-1>(L + rl * LP, r, tw);
  __syncthreads();
  fft_stage_b<-1>(L + rl * LP, r);
  __syncthreads();
  float2 *S = a.spec + fld(f);
#pragma unroll
  for (int c_ = 0; c_ < PASSES; ++c_) S[(size_t)(m0 + c_) * NN + t] = L[c_ * LP + pad(t)];
}

// column position held by line c of column block g, and the line holding its mirror
__device__ __forceinline__ int col_pos(int g, int c) {
  if (g == 0) return c;
  if (g == 1) return 8 * R + c;
  const int a = 1 + (g - 2) / 2, h = (g - 2) & 1;
  return c < 8 ? R * a + 8 * h + c : R * (R - a) + 8 * (1 - h) + (c - 8);
}
__device__ __forceinline__ int mirror_line(int g, int c) {
  if (g == 0) return (R - c) & (R - 1);
  return R - 1 - c;  // group 8: 128 + c <-> 128 + 15 - c; paired groups: line c <-> line 15 - c
}
// position of the mirrored frequency along a transformed line
__device__ __forceinline__ int mirror_pos(int p) {
  const int a = p >> 4, b = p & (R - 1);
  return a == 0 ? (R - b) & (R - 1) : R * (R - a) + (R - 1) - b;
}

// One column block g of frame f (the body of cols_kernel; the persistent loop runs it with COH):
// forward column FFTs, the packed projector, inverse column FFTs.  L: R padded lines; tw staged by
// the caller.
template <bool COH>
__device__ __forceinline__ void cols_block(const FSArgs &a, float2 *L, const float2 *tw, int t, int f, int g,
                                           int fin) {
  const int cl = t >> 4, r = t & 15;
  float2 *S = a.spec + fld(f);
  constexpr int NL = R * NN / THREADS;
  {
    const int c = t & (R - 1), row0 = t >> 4, p = col_pos(g, c);
    float2 v[NL];
#pragma unroll
    for (int c_ = 0; c_ < NL; ++c_) v[c_] = ldc<COH>(S + uint32_t((row0 + R * c_) * NN + p));
#pragma unroll
    for (int c_ = 0; c_ < NL; ++c_) L[c * LP + pad(row0 + R * c_)] = v[c_];
  }
  __syncthreads();
  fft_stage_a<-1>(L + cl * LP, r, tw);
  __syncthreads();
  fft_stage_b<-1>(L + cl * LP, r);
  __syncthreads();
  // Z' = alpha Z + beta conj(Zm) (loop) or A Z + B conj(Zm) (final), Zm = Z(-l, -k)
  const int pc = col_pos(g, cl), ml = mirror_line(g, cl);
  float2 out[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int q = r + R * j;
    const float2 z = L[cl * LP + pad(q)];
    const float2 zm = L[ml * LP + pad(mirror_pos(q))];
    const uint32_t ti = uint32_t(pc * NN + q);
    // (explicit fused multiply-adds: the same rounding whichever kernel inlines this)
    if (fin) {
      const float2 A = a.fin_a[ti], Bc = a.fin_b[ti];
      out[j] = make_float2(fmaf(Bc.y, zm.y, fmaf(Bc.x, zm.x, fmaf(-A.y, z.y, A.x * z.x))),
                           fmaf(-Bc.x, zm.y, fmaf(Bc.y, zm.x, fmaf(A.y, z.x, A.x * z.y))));
    } else {
      const float al = a.alpha[ti];
      const float2 be = a.beta[ti];
      out[j] = make_float2(fmaf(be.y, zm.y, fmaf(be.x, zm.x, al * z.x)), fmaf(-be.x, zm.y, fmaf(be.y, zm.x, al * z.y)));
    }
  }
  __syncthreads();  // every mirror read is done before the lines are overwritten
#pragma unroll
  for (int j = 0; j < R; ++j) L[cl * LP + pad(r + R * j)] = out[j];
  __syncthreads();
  fft_stage_b<+1>(L + cl * LP, r);
  __syncthreads();
  fft_stage_a<+1>(L + cl * LP, r, tw);
  __syncthreads();
  {
    const int c = t & (R - 1), row0 = t >> 4, p = col_pos(g, c);
#pragma unroll
    for (int c_ = 0; c_ < NL; ++c_)
      stc<COH>(S + uint32_t((row0 + R * c_) * NN + p), L[c * LP + pad(row0 + R * c_)]);
  }
}

__global__ __launch_bounds__(THREADS) void cols_kernel(FSArgs a, int fin) {
  __shared__ float2 L[R * LP];
  __shared__ float2 tw[TW_RK];
  const int t = threadIdx.x;
  stage_tw_rk(tw, a.tw256, t, THREADS);
  cols_block<false>(a, L, tw, t, blockIdx.y, blockIdx.x, fin);
}

// The loop's column passes and row steps, C_0, R_0, C_1, ..., R_{K-2}, C_{K-1} (K = n_iter), as
// one launch of resident workgroups that take items (step, frame, column block or row block) from
// a counter in order and wait, by polling a per-frame count, for the previous step of their own
// frame only (the Fried multi-pass loop's persistent launch, gerchberg_multipass.hip, with one frame
// per field).  Items wait only on earlier items, held by running workgroups: no deadlock at any
// residency.  A wait longer than a.wait_limit polls sets the error word; every workgroup stops and
// the outputs are written as NaN.  The counts are zeroed by the start pass (rows_kernel, kInit).
__global__ __launch_bounds__(THREADS) void loop_kernel(FSArgs a) {
  // the twiddles first, so that their reads fit the LDS instructions' immediate offsets
  __shared__ float2 lds[TW_RK + R * LP];
  __shared__ int s_item;
  float2 *const tw = lds, *const L = lds + TW_RK;
  const int t = threadIdx.x;
  stage_tw_rk(tw, a.tw256, t, THREADS);
  constexpr int per = 2 * R;  // items of one frame in one loop step (16 column blocks, 16 row blocks)
  const int step = a.B * per, nc = a.B * R;
  const int total = (a.n_iter - 1) * step + nc;
  uint32_t *next = a.ctl, *err = a.ctl + 1, *done = a.ctl + kCtl;
  int nxt = 0;
  if (t == 0) nxt = int(atomicAdd(next, 1u));
  for (;;) {
    if (t == 0) {
      int item = nxt;
      if (item < total) {
        nxt = int(atomicAdd(next, 1u));  // (the next item is taken while this one runs)
        const int k = item / step, rem = item % step;
        const int f = rem < nc ? rem / R : (rem - nc) / R;
        const uint32_t need = uint32_t(k * per + (rem < nc ? 0 : R));
        int spin = 0;
        while (__hip_atomic_load(done + kCtl * f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          if (((++spin & 63) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) ||
              spin > a.wait_limit) {
            __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            item = -1;
            break;
          }
          __builtin_amdgcn_s_sleep(8);
        }
      }
      s_item = item;
    }
    __syncthreads();
    const int item = s_item;
    if (item < 0 || item >= total) break;
    // (the thread index laundered per item, so that the bodies' address arithmetic is not hoisted
    // out of the item loop and held in registers across it; its range restated)
    int tl = t;
    asm volatile("" : "+v"(tl));
    __builtin_assume(tl >= 0 && tl < THREADS);
    const int k = item / step, rem = item % step;
    int f;
    if (rem < nc) {
      f = rem / R;
      cols_block<true>(a, L, tw, tl, f, rem % R, 0);
    } else {
      f = (rem - nc) / R;
      rows_step<true>(a, L, tw, tl, f, ((rem - nc) % R) * R);
    }
    (void)k;
    // every store of the item is complete (seen at agent scope) before the frame's count moves
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    if (t == 0) __hip_atomic_fetch_add(done + kCtl * f, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace fs

bool fourier_mp_supported(int N) { return N == mp::NN; }

size_t fourier_mp_workspace_bytes(int N, int max_batch) {
  if (N != mp::NN) return 0;
  const size_t B = (size_t)max_batch, NNs = (size_t)N * N;
  return B * (2 * NNs * sizeof(float2) + (size_t)N * sizeof(float) + (size_t)(N / 16) * N * sizeof(float)) +
         fourier_mp_ctl_words(max_batch) * sizeof(uint32_t);
}

size_t fourier_mp_ctl_words(int max_batch) { return (size_t)fs::kCtl * ((size_t)max_batch + 1); }

// resident workgroups of the persistent loop kernel on the current device (occupancy x CUs)
static int fs_loop_grid() {
  static std::atomic<int> grid[64] = {};  // (per device; concurrent first calls store the same value)
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (grid[dev].load() == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fs::loop_kernel, mp::THREADS, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    grid[dev].store((per_cu > 0 ? per_cu : 1) * cus);
  }
  return grid[dev].load();
}

hipError_t fourier_mp_run(const FSArgs &a0, bool extend, hipStream_t s) {
  using namespace fs;
  FSArgs a = a0;
  a.loop_err = nullptr;
  const dim3 grid(RB, a.B), blk(THREADS);
  const bool each = (a.flags & kFourierPeriodicEach) != 0;
  const int fix = ((a.flags & kFourierPeriodic) != 0 || (each && a.n_iter > 0)) ? 1 : 0;
  // launch shape 2: the loop's column passes and row steps in one persistent launch
  // (the item indices are 32-bit: calls with more items than that run one launch per pass)
  const long loop_items = (long)a.n_iter * a.B * 2 * R;
  const int lgrid = a.shape == 2 && !each && a.n_iter >= 2 && loop_items < (1L << 30) ? fs_loop_grid() : 0;
  if (a.n_iter == 0) {
    hipLaunchKernelGGL(rows_kernel, grid, blk, 0, s, a, int(kInitStore), 0, 0);
  } else if (lgrid > 0) {
    hipLaunchKernelGGL(rows_kernel, grid, blk, 0, s, a, int(kInit), 0, 0);
    // resident workgroups, at most half the items of one loop step (more only wait)
    const long cap = std::min<long>(lgrid, (long)a.B * R);
    hipLaunchKernelGGL(loop_kernel, dim3((unsigned)std::max<long>(cap, 1)), blk, 0, s, a);
    a.loop_err = a.ctl + 1;  // read by the output modes
    hipLaunchKernelGGL(rows_kernel, grid, blk, 0, s, a, int(kStepStore), 0, 0);
  } else {
    hipLaunchKernelGGL(rows_kernel, grid, blk, 0, s, a, int(kInit), 0, 0);
    for (int it = 0; it < a.n_iter; ++it) {
      const bool last = it == a.n_iter - 1;
      hipLaunchKernelGGL(cols_kernel, grid, blk, 0, s, a, 0);
      if (!last && !each) {
        hipLaunchKernelGGL(rows_kernel, grid, blk, 0, s, a, int(kStep), 0, 0);
        continue;
      }
      hipLaunchKernelGGL(rows_kernel, grid, blk, 0, s, a, int(kStepStore), 0, 0);
      if (!last) hipLaunchKernelGGL(rows_kernel, grid, blk, 0, s, a, int(kFixFwd), 0, 1);  // per-iteration Eq. 5
    }
  }
  if (extend) {
    hipLaunchKernelGGL(rows_kernel, grid, blk, 0, s, a, int(kFixExt), 0, fix);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(rows_kernel, grid, blk, 0, s, a, int(kFixFwd), 0, fix);
  hipLaunchKernelGGL(cols_kernel, grid, blk, 0, s, a, 1);
  // the output is the window rows o .. o + n
  const int w0 = a.o / mp::R, w1 = (a.o + a.n) / mp::R;
  hipLaunchKernelGGL(rows_kernel, dim3(w1 - w0 + 1, a.B), blk, 0, s, a, int(kOut), w0, 0);
  return hipGetLastError();
}

}  // namespace fwr
