// On-chip Gerchberg extension + Fourier reconstruction for padded grids N <= 128.
//
// Frames go in pairs.  Everything the loop iterates on is real, and every
// Fourier-domain operator in it is real and even, so the two frames of a pair
// ride in one complex field (frame A = real part, frame B = imaginary part)
// and share every FFT.  Per frame pair the loop state lives in registers and
// one N x N complex LDS tile; HBM is touched only to read the slopes and to
// write the result.  A workgroup takes PAIRS pairs (see Group below).
//
// Formulation (Fried model; exact rewrite of Algorithm 1 steps 1-4):
//   Step 2 of each iteration, phi~ = (G_x* S_x + G_y* S_y) / |G|^2 followed
//   by s~ = G phi~, is evaluated as
//     q   = G_x^T s_x + G_y^T s_y          (adjoint Fried stencil, real space)
//     phi = TF^-1 [ TF(q) / |G|^2 ]        (one real, even Fourier filter)
//     s'  = G phi                          (Fried stencil, real space)
//   and step 4 re-imposes the measurement inside the pupil.  With the cell
//   differences p = s_x + s_y (main diagonal) and r = s_x - s_y (anti-
//   diagonal), q (times 2) at a node is
//     q2 = F0 + sum over its 4 surrounding cells c outside the pupil of (phi - phi_c)
//   where phi_c is the diagonally opposite corner of cell c and F0 collects the
//   measured p, r of the in-pupil cells (constant over the iterations).
//   The final reconstruction (Eq. 2 with the Eq. 3 filter) is the same
//   Fourier step with 1 / (|G|^2 + gamma W_eta/W_phi).
//
// Thread layout: 4 lanes per grid line (see fft_lane.h), 4N threads per pair.
//   row phase    : thread (line = m, lane j) holds nodes (m, 4k + j), k < T
//   column phase : thread (line = c, lane j) holds rows 4k + j of LDS column c
// LDS tile: N rows x PITCH complex.  In the row phase a thread's k-th value
// sits at column T j + k of its row ("lane-blocked"), which makes the row
// reads of the inverse transform and the writes of the stencil hit the
// thread's own slots, so they need no barrier in between.
#include "fft_lane.h"
#include "lds_limit.h"
#include "onchip.h"

#include <cstdint>

// Minimum waves per SIMD the register allocation must allow for N <= 80 and one
// pair per workgroup (2: up to 256 VGPRs; 3: <= 168 VGPRs); larger groups raise it
// to what their waves need (Group::WAVES_PER_SIMD).
#ifndef FWR_ONCHIP_MIN_WAVES
#define FWR_ONCHIP_MIN_WAVES 2
#endif

// LDS row pitch = N + FWR_ONCHIP_PITCH_PAD complex elements
#ifndef FWR_ONCHIP_PITCH_PAD
#define FWR_ONCHIP_PITCH_PAD 1
#endif

namespace fwr {

template <int N>
struct Onchip {
  static constexpr int T = N / 4;
  static constexpr int THREADS = 4 * N;
  static constexpr int PITCH = N + FWR_ONCHIP_PITCH_PAD;  // complex elements per LDS row
  static constexpr int TILE = N * PITCH;  // complex elements
  // N <= 80: the per-node forcing F0 of the n+1 window rows lives in LDS (dynamic,
  // (n+1) * PITCH complex per pair), which leaves registers for two pairs per CU;
  // N = 128 keeps it in registers (one pair per CU: its tile alone is 132 KB).
  static constexpr bool F0_IN_LDS = N <= 80;
  static constexpr int WAVES_PER_SIMD = N <= 80 ? FWR_ONCHIP_MIN_WAVES : 2;
  // residual partials per frame pair: one set per wave (full waves) or per thread
  static constexpr int RED = THREADS % 64 == 0 ? 4 * (THREADS / 64) : 4 * THREADS;
};

// PAIRS frame pairs per workgroup (PAIRS x 4N threads).  The workgroup's barriers
// make every phase wait for its busiest SIMD; 4N threads make 5 waves at N = 80,
// i.e. 2 waves on one SIMD and 1 on the others, while 2 pairs make 10 waves
// (3, 3, 2, 2).  Registers must then allow ceil(waves / 4) waves per SIMD.
template <int N, int PAIRS>
struct Group {
  static constexpr int THREADS = PAIRS * Onchip<N>::THREADS;
  static constexpr int WAVES = (THREADS + 63) / 64;
  static constexpr int WAVES_PER_SIMD =
      (WAVES + 3) / 4 > Onchip<N>::WAVES_PER_SIMD ? (WAVES + 3) / 4 : Onchip<N>::WAVES_PER_SIMD;
  static constexpr int STATIC_LDS_BYTES = PAIRS * (Onchip<N>::TILE + 2 * N) * 8 + 2 * Onchip<N>::T * 4 * 8 +
                                          PAIRS * Onchip<N>::RED * 4;
  static int lds_bytes(int n) {
    return STATIC_LDS_BYTES + (Onchip<N>::F0_IN_LDS ? PAIRS * (n + 1) * Onchip<N>::PITCH * 8 : 0);
  }
};

// r + sum over the cells marked in c (bit b: the cell whose opposite corner is d_(b+1))
// of (ph - d), written as r + W ph - sum w_b d_b with W the number of marked cells
// (five FMAs per component)
__device__ __forceinline__ float2 outside_sum(float2 r, float2 ph, float2 d1, float2 d2, float2 d3, float2 d4,
                                             uint32_t c) {
  const float w1 = float(c & 1u), w2 = float((c >> 1) & 1u);
  const float w3 = float((c >> 2) & 1u), w4 = float((c >> 3) & 1u);
  const float W = float(__builtin_popcount(c & 15u));
  r.x = fmaf(W, ph.x, r.x);
  r.y = fmaf(W, ph.y, r.y);
  r.x = fmaf(-w1, d1.x, r.x);
  r.y = fmaf(-w1, d1.y, r.y);
  r.x = fmaf(-w2, d2.x, r.x);
  r.y = fmaf(-w2, d2.y, r.y);
  r.x = fmaf(-w3, d3.x, r.x);
  r.y = fmaf(-w3, d3.y, r.y);
  r.x = fmaf(-w4, d4.x, r.x);
  r.y = fmaf(-w4, d4.y, r.y);
  return r;
}

// c ? a : b on the bit patterns: exact, and both operands are always computed, so
// the compiler cannot sink the loads feeding one side into a branch
__device__ __forceinline__ float select_bits(bool c, float a, float b) {
  const uint32_t m = 0u - static_cast<uint32_t>(c);
  return __uint_as_float((__float_as_uint(a) & m) | (__float_as_uint(b) & ~m));
}

// A frame's non-finite input must not reach its partner through the shared complex field:
// measured and start slopes enter the field with non-finite values as zeros, and the frame
// is flagged so that its outputs are written as NaN.
__device__ __forceinline__ float nan_f() { return __uint_as_float(0x7fc00000u); }
// The test is integer arithmetic (1: not finite; an all-ones exponent carries into bit 31),
// and zero_if clears a non-finite value by masking its bits: no lane masks are held across
// the batched loads.
__device__ __forceinline__ uint32_t nonfinite_bit(float v) {
  return ((__float_as_uint(v) & 0x7f800000u) + 0x00800000u) >> 31;
}
__device__ __forceinline__ float zero_if(float v, uint32_t nf) { return __uint_as_float(__float_as_uint(v) & (nf - 1u)); }

// EACH: Eq. 5 after every iteration (flag kFlagPeriodicEach).
// WIN: the pruned loop of the 2x-padded window (n = N/2, o = N/4) with the window fixed at
// compile time, so that the zero lines and columns outside it fold away (launched only
// for such plans without start values or the extended-slope output).
// SCHED: radix schedule of the in-lane DFTs (see dft in fft_lane.h); schedule 1 is built for
// the WIN kernel of the sizes where the two schedules differ.
template <int N, bool EACH, int PAIRS, bool WIN = false, int SCHED = 0>
__global__ __launch_bounds__((Group<N, PAIRS>::THREADS))
__attribute__((amdgpu_waves_per_eu(Group<N, PAIRS>::WAVES_PER_SIMD)))
void gerchberg_onchip_kernel(OnchipArgs a) {
  using C = Onchip<N>;
  constexpr int T = C::T;
  constexpr int P = C::PITCH;
  __shared__ float2 buf_all[PAIRS * C::TILE];
  __shared__ float2 sums_all[PAIRS * 2 * N];  // Eq. 5: column sums C_n, then row sums R_m
  constexpr bool FULL_WAVES = C::THREADS % 64 == 0;
  __shared__ float red_all[PAIRS * C::RED];
  __shared__ float2 tw[T * 4];
  __shared__ float2 twi[T * 4];  // inverse twiddles with the lane signs of the signed quad DFT
  __shared__ uint32_t bad_all;   // non-finite input: bits 2 h (frame A) and 2 h + 1 (frame B) of pair h
  extern __shared__ float2 f0rows_all[];  // PAIRS x [(n+1)][PITCH], lane-blocked like the tile rows

  // this thread's frame pair within the workgroup and its LDS
  const int half = PAIRS == 1 ? 0 : int(threadIdx.x) / C::THREADS;
  const int t = int(threadIdx.x) - half * C::THREADS;
  float2 *const buf = buf_all + half * C::TILE;
  float2 *const sums = sums_all + half * 2 * N;
  float *const red = red_all + half * C::RED;
  float2 *const f0rows = f0rows_all + (C::F0_IN_LDS ? half * (a.n + 1) * P : 0);
  // row phase: the quad's grid row; column phase: LDS column t / 4 (the same number)
  const int col = t >> 2;
  const int line = col;
  const int j = t & 3;
  const QuadLane q(j);
  // frames of this launch: B, or the part of a device-side count the launch covers
  int nb = a.B;
  if (a.count != nullptr) {
    const int c = *a.count - a.count_off;
    nb = c < 0 ? 0 : (c < a.B ? c : a.B);
    if (2 * PAIRS * int(blockIdx.x) >= nb) return;  // the whole workgroup is past the batch
  }
  // a pair past the batch (last workgroup) computes on pair 0's input and writes nothing
  const bool active = 2 * (PAIRS * int(blockIdx.x) + half) < nb;
  const int fa = active ? 2 * (PAIRS * int(blockIdx.x) + half) : 0;
  const bool hasB = active && fa + 1 < nb;
  const int n = WIN ? N / 2 : a.n, o = WIN ? N / 4 : a.o;
  // with WIN: in-lane slots k whose node columns 4k + j (some lane j) meet the window
  // [o, o+n] (the support of q2), and the window plus one column either side (the
  // stencil's reach)
  constexpr auto kin_w = [](int k) { return !WIN || (4 * k + 3 >= N / 4 && 4 * k <= 3 * N / 4); };
  constexpr auto kin_r = [](int k) { return !WIN || (4 * k + 3 >= N / 4 - 1 && 4 * k <= 3 * N / 4 + 1); };
  // q2 is zero at the nodes of a window slot that lie outside the window (the lanes of the
  // two edge slots); their neighbour slots beyond the reach are not kept up to date
  auto clip_w = [&](float2 &v, int k) {
    if (WIN && (4 * k < N / 4 || 4 * k + 3 > 3 * N / 4)) {
      const int nn = 4 * k + j;
      const bool in = nn >= N / 4 && nn <= 3 * N / 4;
      v = make_float2(in ? v.x : 0.f, in ? v.y : 0.f);
    }
  };
  const int up = line == 0 ? N - 1 : line - 1;    // row m - 1
  const int dn = line == N - 1 ? 0 : line + 1;    // row m + 1

  if (threadIdx.x == 0) bad_all = 0;  // (the atomics come after the first barrier)
  uint32_t bad = 0;                   // this thread's non-finite bits (1: frame A, 2: frame B)
  for (int i = threadIdx.x; i < T * 4; i += Group<N, PAIRS>::THREADS) {
    const float2 w = a.tw_lane[i];
    const float sg = lane_sign(i & 3);
    tw[i] = w;
    twi[i] = make_float2(sg * w.x, -sg * w.y);
  }
  const float sj = lane_sign(j);

  // ---- per-node constants: out-of-pupil cell bits and the in-pupil forcing F0
  const int plane = n * n;
  const float *sa = a.slopes + (size_t)fa * 2 * plane;
  const float *sb = hasB ? sa + 2 * plane : nullptr;
  const float *sbb = hasB ? sb : sa;  // always-valid pointer for branch-free reads
  const float bflag = hasB ? 1.f : 0.f;
  const unsigned uplane = unsigned(plane);
  uint32_t codes[(T + 7) / 8];
#pragma unroll
  for (int w = 0; w < (T + 7) / 8; ++w) codes[w] = a.codes[w * C::THREADS + 4 * line + j];
  auto code_of = [&](int k) -> uint32_t { return (codes[k >> 3] >> (4 * (k & 7))) & 15u; };

  // F0 = -p(c1) + p(c2) + r(c3) - r(c4) over the in-pupil cells c1 = (m, n), c2 = (m-1, n-1),
  // c3 = (m, n-1), c4 = (m-1, n), with p = s_x + s_y, r = s_x - s_y.  The window's x and y
  // slopes are staged in the LDS tile with cells outside the pupil as zeros (whatever the
  // input holds there).  The staged planes also give the measured in-pupil row sums of s_x
  // and column sums of s_y: Eq. 5's R_m and C_n are these minus the same sums of the model
  // slopes.
  float2 f0[T];
#pragma unroll
  for (int k = 0; k < T; ++k) f0[k] = make_float2(0.f, 0.f);
  for (int i = t; i < 2 * N; i += C::THREADS) sums[i] = make_float2(0.f, 0.f);
  // four lanes per row (x plane) or column (y plane), then a quad reduction; cell (r, c) of
  // a plane at pv[r * pw + c]
  auto meas_sums = [&](const float2 *pv, int pw, bool rows) {
    for (int task = t; task < 4 * n; task += C::THREADS) {
      const int jj = task & 3, which = task >> 2;
      float2 acc = make_float2(0.f, 0.f);
      for (int i = jj; i < n; i += 4) acc = cadd(acc, rows ? pv[which * pw + i] : pv[i * pw + which]);
      acc.x += dpp_xor1(acc.x);
      acc.y += dpp_xor1(acc.y);
      acc.x += dpp_xor2(acc.x);
      acc.y += dpp_xor2(acc.y);
      if (jj == 0) sums[(rows ? N : 0) + o + which] = acc;
    }
  };
  // With the window fixed at compile time both planes are staged with a zero border (one row
  // above and below, 4 columns left and 5 right: every cell a window slot's node touches), so
  // that F0 is plain arithmetic on eight unconditional reads per node.
  constexpr bool PADF0 = WIN && (N + 4) * (N + 18) / 2 <= C::TILE;
  if constexpr (PADF0) {
    constexpr int NW = N / 2, PL = 4, PW = NW + 9, PH = NW + 2, PP = PH * PW;
    constexpr int CHP = (PP + C::THREADS - 1) / C::THREADS;
    {  // all loads first, then the LDS stores
      float va[2][CHP], vb[2][CHP];
#pragma unroll
      for (int c = 0; c < CHP; ++c) {
        const int i = t + c * C::THREADS;
        const int r = i / PW - 1, cc = i % PW - PL;
        const bool inside = i < PP && r >= 0 && r < NW && cc >= 0 && cc < NW;
        const int gi = inside ? r * NW + cc : 0;
        const bool v = inside && a.mask[gi] != 0;
#pragma unroll
        for (int pl = 0; pl < 2; ++pl) {
          const float xa = sa[pl * plane + gi], xb = sbb[pl * plane + gi];
          const uint32_t na = nonfinite_bit(xa), nb2 = hasB ? nonfinite_bit(xb) : 0u;
          bad |= v ? (na | (nb2 << 1)) : 0u;
          va[pl][c] = v ? zero_if(xa, na) : 0.f;
          vb[pl][c] = v && hasB ? zero_if(xb, nb2) : 0.f;
        }
      }
#pragma unroll
      for (int c = 0; c < CHP; ++c) {
        const int i = t + c * C::THREADS;
        if (i < PP) {
          buf[i] = make_float2(va[0][c], vb[0][c]);
          buf[PP + i] = make_float2(va[1][c], vb[1][c]);
        }
      }
    }
    __syncthreads();
    if (line >= o && line <= o + n) {
      const int b0 = (line - o + 1) * PW + PL - o, b1 = b0 - PW;  // cell (line - o, nn - o) = b0 + nn
#pragma unroll
      for (int k = 0; k < T; ++k) {
        if (!kin_w(k)) continue;
        const int nn = 4 * k + j;
        const float2 x1 = buf[b0 + nn], x2 = buf[b1 + nn - 1], x3 = buf[b0 + nn - 1], x4 = buf[b1 + nn];
        const float2 y1 = buf[PP + b0 + nn], y2 = buf[PP + b1 + nn - 1], y3 = buf[PP + b0 + nn - 1],
                     y4 = buf[PP + b1 + nn];
        // -(x1 + y1) + (x2 + y2) + (x3 - y3) - (x4 - y4)
        f0[k].x = ((x2.x - x1.x) + (x3.x - x4.x)) + ((y2.x - y1.x) + (y4.x - y3.x));
        f0[k].y = ((x2.y - x1.y) + (x3.y - x4.y)) + ((y2.y - y1.y) + (y4.y - y3.y));
        if ((k & 1) == 1) __builtin_amdgcn_sched_barrier(0);  // bound the reads in flight
      }
    }
    meas_sums(buf + PW + PL, PW, true);
    meas_sums(buf + PP + PW + PL, PW, false);
    __syncthreads();
  } else {
    // x plane, then y plane, at buf[r * n + c]
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = t; i < plane; i += C::THREADS) {
        const bool v = a.mask[i] != 0;
        const float va = sa[pass * plane + i];
        const float vb = sbb[pass * plane + i];
        const uint32_t na = nonfinite_bit(va), nb2 = hasB ? nonfinite_bit(vb) : 0u;
        bad |= v ? (na | (nb2 << 1)) : 0u;
        buf[i] = make_float2(v ? zero_if(va, na) : 0.f, v && hasB ? zero_if(vb, nb2) : 0.f);
      }
      __syncthreads();
      const float sgn3 = pass == 0 ? 1.f : -1.f;  // r = s_x - s_y
#pragma unroll
      for (int k = 0; k < T; ++k) {
        if (!kin_w(k)) continue;  // no pupil cell touches these nodes
        const uint32_t c = code_of(k);
        const int nn = 4 * k + j;
        const int nl = nn == 0 ? N - 1 : nn - 1;
        float2 f = f0[k];
        if (!(c & 1u)) { const float2 v = buf[(line - o) * n + (nn - o)]; f = csub(f, v); }
        if (!(c & 2u)) { const float2 v = buf[(up - o) * n + (nl - o)]; f = cadd(f, v); }
        if (!(c & 4u)) { const float2 v = buf[(line - o) * n + (nl - o)]; f.x = fmaf(sgn3, v.x, f.x); f.y = fmaf(sgn3, v.y, f.y); }
        if (!(c & 8u)) { const float2 v = buf[(up - o) * n + (nn - o)]; f.x = fmaf(-sgn3, v.x, f.x); f.y = fmaf(-sgn3, v.y, f.y); }
        f0[k] = f;
      }
      meas_sums(buf, n, pass == 0);
      __syncthreads();
    }
  }
  // measured sums kept in registers: this line's R_m and the C_n of column t / 4
  const float2 rmeas = sums[N + line], cmeas = sums[t >> 2];
  const bool in_rows = line >= o && line <= o + n;  // rows that can carry forcing
  if constexpr (C::F0_IN_LDS) {
    if (in_rows) {
#pragma unroll
      for (int k = 0; k < T; ++k) f0rows[(line - o) * P + T * j + k] = f0[k];
    }
  }
  const int f0row = (in_rows ? line - o : 0) * P + T * j;
  const float rowf = in_rows ? 1.f : 0.f;

  // Without start values, per-iteration Eq. 5 or the extended-slope output, the row
  // passes are pruned to the window.  q2 = G^T s where s differs from the model slopes
  // G phi only inside the pupil, and phi itself came from q2_prev through 1 / |G|^2, so
  // q2 = q2_prev (zero outside the window rows, by induction from F0) plus G^T of
  // in-pupil differences (window rows again); G^T vanishes on the singular set, so
  // nothing is lost there.  The forward row transforms run on the window rows o..o+n,
  // the inverse ones on those rows and one more on either side (the stencil's
  // neighbours); the other lines carry zeros.
  const bool prune = WIN || (!EACH && !(a.flags & kFlagExtend) && a.start == nullptr);
  const bool row_w = !prune || in_rows;
  const bool row_r1 = !prune || unsigned((line - (o - 1) + N) % N) < unsigned(n + 3);

  const bool want_resid = a.resid != nullptr && a.n_iter > 0;
  if (a.resid != nullptr && a.n_iter == 0 && t == 0 && active) {
    a.resid[fa] = 0.f;
    if (hasB) a.resid[fa + 1] = 0.f;
  }

  // neighbour column slots for n + 1 and n - 1 (lane-blocked layout)
  const int jp = (j + 1) & 3, jm = (j + 3) & 3;
  const int carry = j == 3 ? 1 : 0, borrow = j == 0 ? 1 : 0;

  // ---- Fourier step: x holds q2 (row layout) on entry, phi on exit.  Row lines with
  // `fwd` false must hold zeros (they are written as such); with `inv` false the line's
  // phi is not computed.
  // `mode` (a compile-time literal at each call) with WIN: 1 = the loop's transform of a
  // window-supported q2 whose result is needed on the window rows and one row either
  // side; 2 = the final one, whose input may also have the Eq. 5 rows 0 and N-1 and whose
  // result is needed on the window rows; 0 = no pruning of the column pass.
  // The signed transforms leave lane signs on the spectra: the row pass's on the LDS
  // columns it writes, the column pass's on its own values; the filter tables carry both.
  auto solve = [&](float2 *x, const float *h, bool fwd, bool inv, int mode) {
    if (fwd) line_fft_fwd_s<T, SCHED>(x, tw, j, q);
#pragma unroll
    for (int k = 0; k < T; ++k) buf[line * P + T * j + k] = x[k];
    __syncthreads();
    float2 y[T];
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const bool zero = (mode == 1 && !kin_w(k)) || (mode == 2 && !kin_w(k) && k != 0 && k != T - 1);
      y[k] = zero ? make_float2(0.f, 0.f) : buf[(4 * k + j) * P + col];
    }
    line_fft_fwd_s<T, SCHED>(y, tw, j, q);
    const float *ht = h + t * T;  // thread-contiguous: one address, immediate offsets
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const float hv = ht[k];
      y[k].x *= hv;
      y[k].y *= hv;
    }
    line_fft_inv_s<T, SCHED>(y, twi, j, sj, q);
#pragma unroll
    for (int k = 0; k < T; ++k) {
      if (mode == 1 ? kin_r(k) : kin_w(k)) buf[(4 * k + j) * P + col] = y[k];
    }
    __syncthreads();
    if (inv) {
#pragma unroll
      for (int k = 0; k < T; ++k) x[k] = buf[line * P + T * j + k];
      line_fft_inv_s<T, SCHED>(x, twi, j, sj, q);
    }
  };

  // Only k = T-1 (for n + 1) and k = 0 (for n - 1) can wrap; keeping the wrap
  // test out of the other (unrolled) indices leaves base + k addresses whose
  // offsets fold into the LDS instruction.
  const int base_p = T * jp + carry, base_m = T * jm - borrow;
  const int wrap_p = j == 3 ? 0 : T * jp + T - 1 + carry;  // slot for k = T-1
  const int wrap_m = j == 0 ? T * 3 + T - 1 : T * jm;     // slot for k = 0
  auto slot_p = [&](int k) { return k == T - 1 ? wrap_p : base_p + k; };
  auto slot_m = [&](int k) { return k == 0 ? wrap_m : base_m + k; };

  // ---- fast stencil: phi (x) -> q2 (x), measured slopes inside the pupil via F0
  auto stencil = [&](float2 *x) {
#pragma unroll
    for (int k = 0; k < T; ++k) {
      if (kin_r(k)) buf[line * P + T * j + k] = x[k];
    }
    // keep the per-node weights from being hoisted out of the iteration loop
    // as 4T live float registers: they are re-derived from 3 code words here
#pragma unroll
    for (int w = 0; w < (T + 7) / 8; ++w) asm volatile("" : "+v"(codes[w]));
    __syncthreads();
    if (row_w) {
#pragma unroll
      for (int k = 0; k < T; ++k) {
        if (!kin_w(k)) {
          x[k] = make_float2(0.f, 0.f);
          continue;
        }
        const int sp = slot_p(k), sm = slot_m(k);
        const float2 d1 = buf[dn * P + sp];  // (m+1, n+1)
        const float2 d2 = buf[up * P + sm];  // (m-1, n-1)
        const float2 d3 = buf[dn * P + sm];  // (m+1, n-1)
        const float2 d4 = buf[up * P + sp];  // (m-1, n+1)
        const uint32_t c = code_of(k);
        float2 r;
        if constexpr (C::F0_IN_LDS) {
          const float2 fv = f0rows[f0row + k];  // clamped address: always a valid read
          r = make_float2(fv.x * rowf, fv.y * rowf);
        } else {
          r = f0[k];
        }
        x[k] = outside_sum(r, x[k], d1, d2, d3, d4, c);
        clip_w(x[k], k);
        // bound the neighbour reads in flight (4 per node)
        if ((k & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    } else {
#pragma unroll
      for (int k = 0; k < T; ++k) x[k] = make_float2(0.f, 0.f);
    }
    __syncthreads();
  };

  // ---- final step: phi (x) -> q2 (x) with the measured slopes inside the pupil and,
  // with `fix`, Eq. 5 applied to the slopes first; with `write` the (optionally
  // periodised) slopes themselves are written out instead (returns true).
  //
  // Eq. 5 only rewrites s_x on column N-1 and s_y on row N-1: with
  // R_m = sum_n s_x(m, n) and C_n = sum_m s_y(m, n), s_x(m, N-1) drops by R_m and
  // s_y(N-1, n) by C_n.  Through the adjoint stencil this moves q2 only on the
  // border node lines:
  //   node (m, 0)   by -(R_m + R_{m-1}),   node (m, N-1) by +(R_m + R_{m-1}),
  //   node (0, n)   by -(C_n + C_{n-1}),   node (N-1, n) by +(C_n + C_{n-1}).
  // Outside the pupil the slopes are the model slopes of the periodic phase, whose
  // sums along a full row (x) or column (y) telescope to zero, so R_m and C_n are the
  // sums of the in-pupil misfits (measured - model) alone: the measured sums from the
  // set-up minus the model sums taken here.  When the step runs once (F0 is read for the
  // last time here) the negated in-pupil y model slopes take the place of F0 (the
  // thread's own LDS slots or registers); otherwise they are held in registers.  The
  // measured slopes themselves are read again only for the residual or the written
  // slopes.
  constexpr bool EY_IN_F0 = !EACH;
  auto final_step = [&](float2 *x, bool fix, bool write) -> bool {
#pragma unroll
    for (int k = 0; k < T; ++k) {
      if (kin_r(k)) buf[line * P + T * j + k] = x[k];
    }
    __syncthreads();
    const uint32_t fb = write || want_resid ? bad_all >> (2 * half) : 0u;  // non-finite frames of the pair
    const bool nan_a = (fb & 1u) != 0, nan_b = (fb & 2u) != 0;
    const unsigned wrow = unsigned(line >= o && line < o + n ? line - o : 0) * unsigned(n);
    const size_t gplane = (size_t)N * N;
    float *ea = a.out + (size_t)fa * 2 * gplane;  // extended slopes of frame A (write mode)
    float2 rowacc = make_float2(0.f, 0.f);  // minus the in-pupil model x slopes of the row
    // in-pupil misfit and measurement energy (a non-finite frame starts its energy at NaN, so
    // that the reduction makes its residual NaN)
    float ra = 0.f, rb = 0.f, na = nan_a ? nan_f() : 0.f, nb = nan_b ? nan_f() : 0.f;
    const bool need_meas = want_resid || write;
    float2 DY[EY_IN_F0 ? 1 : T];
    if (row_w) {  // (pruned: the other lines have no pupil cell and q2 = 0 there)
#pragma unroll
      for (int k = 0; k < T; ++k) {
        if (!kin_w(k)) {
          x[k] = make_float2(0.f, 0.f);
          continue;
        }
        const int nn = 4 * k + j;
        const uint32_t c4 = code_of(k);
        const bool meas = !(c4 & 1u);
        const unsigned widx = wrow + unsigned(nn >= o && nn < o + n ? nn - o : 0);
        const int sp = slot_p(k), sm = slot_m(k);
        const float2 ph = x[k];
        const float2 b = buf[line * P + sp];       // (m, n+1)
        const float2 c = buf[dn * P + T * j + k];  // (m+1, n)
        const float2 d1 = buf[dn * P + sp];        // (m+1, n+1)
        // cell (m, n): s_x = (b - a + d - c) / 2, s_y = (c - a + d - b) / 2
        const float2 gx = make_float2(0.5f * ((b.x - ph.x) + (d1.x - c.x)), 0.5f * ((b.y - ph.y) + (d1.y - c.y)));
        const float2 gy = make_float2(0.5f * ((c.x - ph.x) + (d1.x - b.x)), 0.5f * ((c.y - ph.y) + (d1.y - b.y)));
        // minus the in-pupil model slopes (exactly zero outside the pupil)
        const float2 mgx = make_float2(select_bits(meas, -gx.x, 0.f), select_bits(meas, -gx.y, 0.f));
        const float2 mgy = make_float2(select_bits(meas, -gy.x, 0.f), select_bits(meas, -gy.y, 0.f));
        rowacc = cadd(rowacc, mgx);
        if (need_meas) {
          // measured slopes, exactly zero outside the pupil (whatever the input holds there)
          const float mxa = select_bits(meas, sa[widx], 0.f), mya = select_bits(meas, sa[uplane + widx], 0.f);
          const float mxb = select_bits(meas, sbb[widx] * bflag, 0.f);
          const float myb = select_bits(meas, sbb[uplane + widx] * bflag, 0.f);
          if (want_resid) {
            const float2 ex = make_float2(select_bits(meas, mxa - gx.x, 0.f), select_bits(meas, mxb - gx.y, 0.f));
            const float2 ey = make_float2(select_bits(meas, mya - gy.x, 0.f), select_bits(meas, myb - gy.y, 0.f));
            ra = fmaf(ex.x, ex.x, fmaf(ey.x, ey.x, ra));
            rb = fmaf(ex.y, ex.y, fmaf(ey.y, ey.y, rb));
            na = fmaf(mxa, mxa, fmaf(mya, mya, na));
            nb = fmaf(mxb, mxb, fmaf(myb, myb, nb));
          }
          if (write && active) {
            const size_t idx = (size_t)line * N + nn;
            ea[idx] = nan_a ? nan_f() : select_bits(meas, mxa, gx.x);
            ea[gplane + idx] = nan_a ? nan_f() : select_bits(meas, mya, gy.x);
            if (hasB) {
              ea[2 * gplane + idx] = nan_b ? nan_f() : select_bits(meas, mxb, gx.y);
              ea[3 * gplane + idx] = nan_b ? nan_f() : select_bits(meas, myb, gy.y);
            }
          }
        }
        if (!write) {
          const float2 d2 = buf[up * P + sm];  // (m-1, n-1)
          const float2 d3 = buf[dn * P + sm];  // (m+1, n-1)
          const float2 d4 = buf[up * P + sp];  // (m-1, n+1)
          float2 r;
          if constexpr (C::F0_IN_LDS) {
            const float2 fv = f0rows[f0row + k];
            r = make_float2(fv.x * rowf, fv.y * rowf);
          } else {
            r = f0[k];
          }
          x[k] = outside_sum(r, ph, d1, d2, d3, d4, c4);
        clip_w(x[k], k);
        }
        if constexpr (EY_IN_F0 && C::F0_IN_LDS) {
          if (in_rows) f0rows[f0row + k] = mgy;  // after this thread's last read of the slot
        } else if constexpr (EY_IN_F0) {
          f0[k] = mgy;
        } else {
          DY[k] = mgy;
        }
        if ((k & 1) == 1) __builtin_amdgcn_sched_barrier(0);
      }
    } else {
#pragma unroll
      for (int k = 0; k < T; ++k) x[k] = make_float2(0.f, 0.f);
    }
    if (want_resid) {  // block reduction of the four sums (fixed order), then one write per frame
      constexpr int PARTS = FULL_WAVES ? C::THREADS / 64 : C::THREADS;
      if constexpr (FULL_WAVES) {
        for (int off = 32; off > 0; off >>= 1) {
          ra += __shfl_xor(ra, off);
          rb += __shfl_xor(rb, off);
          na += __shfl_xor(na, off);
          nb += __shfl_xor(nb, off);
        }
      }
      __syncthreads();
      if (!FULL_WAVES || (t & 63) == 0) {
        const int slot = FULL_WAVES ? (t >> 6) : t;
        red[4 * slot + 0] = ra;
        red[4 * slot + 1] = rb;
        red[4 * slot + 2] = na;
        red[4 * slot + 3] = nb;
      }
      __syncthreads();
      if (t == 0 && active) {
        float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
        for (int w = 0; w < PARTS; ++w) {
          s0 += red[4 * w];
          s1 += red[4 * w + 1];
          s2 += red[4 * w + 2];
          s3 += red[4 * w + 3];
        }
        // (a NaN energy passes the test: the residual of a non-finite frame is NaN)
        a.resid[fa] = !(s2 <= 0.f) ? sqrtf(s0 / s2) : 0.f;
        if (hasB) a.resid[fa + 1] = !(s3 <= 0.f) ? sqrtf(s1 / s3) : 0.f;
      }
    }
    if (fix) {
      // R_m: quad reduction of the per-lane partial row sums
      rowacc.x += dpp_xor1(rowacc.x);
      rowacc.y += dpp_xor1(rowacc.y);
      rowacc.x += dpp_xor2(rowacc.x);
      rowacc.y += dpp_xor2(rowacc.y);
      __syncthreads();  // every neighbour read of the tile and every misfit store is done
      if constexpr (!(EY_IN_F0 && C::F0_IN_LDS)) {
#pragma unroll
        for (int k = 0; k < T; ++k) buf[line * P + T * j + k] = EY_IN_F0 ? f0[k] : DY[k];
      }
      if (j == 0) sums[N + line] = cadd(rmeas, rowacc);
      __syncthreads();
      {  // C_n over the pupil rows: four lanes per column, fixed order (deterministic)
        const int nn = t >> 2, jj = t & 3;
        const int slot = T * (nn & 3) + (nn >> 2);
        float2 cs = make_float2(0.f, 0.f);
        for (int r = jj; r < n; r += 4)
          cs = cadd(cs, EY_IN_F0 && C::F0_IN_LDS ? f0rows[r * P + slot] : buf[(o + r) * P + slot]);
        cs.x += dpp_xor1(cs.x);
        cs.y += dpp_xor1(cs.y);
        cs.x += dpp_xor2(cs.x);
        cs.y += dpp_xor2(cs.y);
        if (jj == 0) sums[nn] = cadd(cmeas, cs);
      }
      __syncthreads();
      const float2 Rm = sums[N + line], Rm1 = sums[N + up];
      if (write) {
        // the thread re-reads the slopes it wrote above (same-thread order)
        if (active && j == 3) {  // s_x(m, N-1) -= R_m
          const size_t idx = (size_t)line * N + (N - 1);
          ea[idx] -= Rm.x;
          if (hasB) ea[2 * gplane + idx] -= Rm.y;
        }
        if (active && line == N - 1) {  // s_y(N-1, n) -= C_n
#pragma unroll
          for (int k = 0; k < T; ++k) {
            const size_t idx = (size_t)line * N + 4 * k + j;
            const float2 cn = sums[4 * k + j];
            ea[gplane + idx] -= cn.x;
            if (hasB) ea[3 * gplane + idx] -= cn.y;
          }
        }
      } else {
        const float2 rr = cadd(Rm, Rm1);
        if (j == 0) x[0] = csub(x[0], rr);          // node (m, 0)
        if (j == 3) x[T - 1] = cadd(x[T - 1], rr);  // node (m, N-1)
        if (line == 0 || line == N - 1) {
#pragma unroll
          for (int k = 0; k < T; ++k) {
            const int nn = 4 * k + j;
            const float2 cc = cadd(sums[nn], sums[nn == 0 ? N - 1 : nn - 1]);
            x[k] = line == 0 ? csub(x[k], cc) : cadd(x[k], cc);
          }
        }
      }
    }
    __syncthreads();
    return write;
  };

  const bool periodic = (a.flags & kFlagPeriodic) != 0;
  const bool extend = (a.flags & kFlagExtend) != 0;
  const bool need_final_step = periodic || extend || (EACH && a.n_iter > 0) || want_resid;
  const bool fix_final = periodic || (EACH && a.n_iter > 0);

  float2 x[T];
#pragma unroll
  for (int k = 0; k < T; ++k) x[k] = f0[k];  // q2 of the zero-padded start
  __syncthreads();                           // tables and forcing in LDS
  const bool has_start = !WIN && a.start != nullptr;  // (the WIN kernel is launched without start values)
  if (bad != 0 && !has_start) atomicOr(&bad_all, bad << (2 * half));
  if (has_start) {
    // q2 of the given start: add the adjoint stencil of the start slopes on the
    // out-of-pupil cells, -p(c1) + p(c2) + r(c3) - r(c4) (p = s_x + s_y, r = s_x - s_y),
    // staging p then r through the tile in the own-slot layout
    const size_t gplane = (size_t)N * N;
    const float *st = a.start + (size_t)fa * 2 * gplane;
    for (int pass = 0; pass < 2; ++pass) {
      const float sg = pass == 0 ? 1.f : -1.f;
#pragma unroll 4  // (staging only: a full unroll raises the register pressure of the whole kernel)
      for (int k = 0; k < T; ++k) {
        const size_t idx = (size_t)line * N + 4 * k + j;
        const float ax = st[idx], ay = st[gplane + idx];
        const float bx = hasB ? st[2 * gplane + idx] : 0.f, by = hasB ? st[3 * gplane + idx] : 0.f;
        // a non-finite start value makes p (or r) non-finite: that cell enters as zero
        const float pa = fmaf(sg, ay, ax), pb = fmaf(sg, by, bx);
        const uint32_t na = nonfinite_bit(pa), nb2 = nonfinite_bit(pb);
        bad |= na | (nb2 << 1);
        buf[line * P + T * j + k] = make_float2(zero_if(pa, na), zero_if(pb, nb2));
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < T; ++k) {
        const uint32_t c4 = code_of(k);
        const float2 own = buf[line * P + T * j + k];  // cell (m, n)
        const float2 ul = buf[up * P + slot_m(k)];     // cell (m-1, n-1)
        const float2 lf = buf[line * P + slot_m(k)];   // cell (m, n-1)
        const float2 upc = buf[up * P + T * j + k];    // cell (m-1, n)
        float2 r = x[k];
        if (pass == 0) {
          r.x += (c4 & 1u ? -own.x : 0.f) + (c4 & 2u ? ul.x : 0.f);
          r.y += (c4 & 1u ? -own.y : 0.f) + (c4 & 2u ? ul.y : 0.f);
        } else {
          r.x += (c4 & 4u ? lf.x : 0.f) - (c4 & 8u ? upc.x : 0.f);
          r.y += (c4 & 4u ? lf.y : 0.f) - (c4 & 8u ? upc.y : 0.f);
        }
        x[k] = r;
      }
      __syncthreads();
    }
    if (bad != 0) atomicOr(&bad_all, bad << (2 * half));
  }
  // (read after at least one more barrier: every solve and the final step begin with one)

  for (int it = 0; it < a.n_iter; ++it) {
    solve(x, a.h_loop, row_w, row_r1, WIN ? 1 : 0);
    if (it == a.n_iter - 1) break;
    if constexpr (EACH) final_step(x, true, false);
    else stencil(x);
  }
  if (need_final_step) {
    if (a.n_iter == 0) {
#pragma unroll
      for (int k = 0; k < T; ++k) x[k] = make_float2(0.f, 0.f);  // phi = 0
    }
    if (final_step(x, fix_final, extend)) return;
  } else if (a.n_iter > 0) {
    stencil(x);
  }
  // the output is the window rows; with Eq. 5 the border rows 0 and N-1 carry forcing
  solve(x, a.h_final, row_w || (fix_final && (line == 0 || line == N - 1)), row_w, WIN ? 2 : 0);

  // (n+1) x (n+1) node window
  if (active && line >= o && line <= o + n) {
    float *oa = a.out + (size_t)fa * (n + 1) * (n + 1);
    float *ob = oa + (size_t)(n + 1) * (n + 1);
    const uint32_t fb = bad_all >> (2 * half);
    const bool nan_a = (fb & 1u) != 0, nan_b = (fb & 2u) != 0;
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const int nn = 4 * k + j;
      if (nn >= o && nn <= o + n) {
        const size_t idx = (size_t)(line - o) * (n + 1) + (nn - o);
        oa[idx] = nan_a ? nan_f() : x[k].x;
        if (hasB) ob[idx] = nan_b ? nan_f() : x[k].y;
      }
    }
  }
}

// PAIRS > 1 is instantiated for the kernel without per-iteration Eq. 5, within 1024
// threads per workgroup
template <int N, int PAIRS>
constexpr bool pairs_instantiated() {
  return PAIRS == 1 || (Group<N, PAIRS>::THREADS <= 1024 && N <= 80);
}

// the compile-time window variant exists for every launch shape, so that the arithmetic
// of a frame pair does not depend on the number of pairs per workgroup
template <int PAIRS>
constexpr bool win_instantiated() {
  return true;
}

// the second radix schedule differs from the first for in-lane lengths above 5
template <int N>
constexpr bool sched_instantiated() {
  return Onchip<N>::T > 5;
}

template <int N, int PAIRS>
hipError_t launch_pairs(const OnchipArgs &a, hipStream_t s, int sched) {
  if constexpr (!pairs_instantiated<N, PAIRS>()) {
    return hipErrorInvalidValue;
  } else {
    const int groups = ((a.B + 1) / 2 + PAIRS - 1) / PAIRS;
    const size_t dyn = Onchip<N>::F0_IN_LDS ? size_t(PAIRS) * (a.n + 1) * Onchip<N>::PITCH * 8 : 0;
    const dim3 grid(groups), block(Group<N, PAIRS>::THREADS);
    if ((a.flags & kFlagPeriodicEach) != 0) {
      if constexpr (PAIRS == 1)
        hipLaunchKernelGGL((gerchberg_onchip_kernel<N, true, 1>), grid, block, dyn, s, a);
      else
        return hipErrorInvalidValue;
    } else {
      const bool win = a.n == N / 2 && a.o == N / 4 && a.start == nullptr && (a.flags & kFlagExtend) == 0;
      if constexpr (win_instantiated<PAIRS>()) {
        if (win) {
          if constexpr (sched_instantiated<N>()) {
            if (sched == 1) {
              hipLaunchKernelGGL((gerchberg_onchip_kernel<N, false, PAIRS, true, 1>), grid, block, dyn, s, a);
              return hipGetLastError();
            }
          }
          hipLaunchKernelGGL((gerchberg_onchip_kernel<N, false, PAIRS, true>), grid, block, dyn, s, a);
          return hipGetLastError();
        }
      }
      hipLaunchKernelGGL((gerchberg_onchip_kernel<N, false, PAIRS>), grid, block, dyn, s, a);
    }
    return hipGetLastError();
  }
}

template <int N>
hipError_t launch_onchip(const OnchipArgs &a, hipStream_t s, int pairs, int sched) {
  switch (pairs) {
    case 1: return launch_pairs<N, 1>(a, s, sched);
    case 2: return launch_pairs<N, 2>(a, s, sched);
    case 4: return launch_pairs<N, 4>(a, s, sched);
    case 8: return launch_pairs<N, 8>(a, s, sched);
    default: return hipErrorInvalidValue;
  }
}

template <int N, int PAIRS>
hipError_t prepare_pairs(int n) {
  if constexpr (!pairs_instantiated<N, PAIRS>()) {
    return hipSuccess;
  } else {
    // dynamic LDS above the default 64 KiB window must be requested explicitly
    const int dyn = Onchip<N>::F0_IN_LDS ? PAIRS * (n + 1) * Onchip<N>::PITCH * 8 : 0;
    const void *fns[4] = {reinterpret_cast<const void *>(&gerchberg_onchip_kernel<N, false, PAIRS>),
                          PAIRS == 1 ? reinterpret_cast<const void *>(&gerchberg_onchip_kernel<N, true, 1>)
                                     : nullptr,
                          nullptr, nullptr};
    if constexpr (win_instantiated<PAIRS>())
      fns[2] = reinterpret_cast<const void *>(&gerchberg_onchip_kernel<N, false, PAIRS, true>);
    if constexpr (sched_instantiated<N>())
      fns[3] = reinterpret_cast<const void *>(&gerchberg_onchip_kernel<N, false, PAIRS, true, 1>);
    hipError_t e = hipSuccess;
    for (int i = 0; i < 4 && e == hipSuccess; ++i)
      if (fns[i]) e = raise_dynamic_lds(fns[i], dyn);
    return e;
  }
}

template <int N>
hipError_t prepare_onchip(int n, int pairs) {
  switch (pairs) {
    case 1: return prepare_pairs<N, 1>(n);
    case 2: return prepare_pairs<N, 2>(n);
    case 4: return prepare_pairs<N, 4>(n);
    case 8: return prepare_pairs<N, 8>(n);
    default: return hipErrorInvalidValue;
  }
}

template <int N>
bool pairs_ok(int n, int pairs, bool each) {
  bool inst = false;
  switch (pairs) {
    case 1: inst = true; break;
    case 2: inst = pairs_instantiated<N, 2>(); break;
    case 4: inst = pairs_instantiated<N, 4>(); break;
    case 8: inst = pairs_instantiated<N, 8>(); break;
    default: return false;
  }
  if (!inst || (each && pairs != 1)) return false;
  int bytes = 0;
  switch (pairs) {
    case 1: bytes = Group<N, 1>::lds_bytes(n); break;
    case 2: bytes = Group<N, 2>::lds_bytes(n); break;
    case 4: bytes = Group<N, 4>::lds_bytes(n); break;
    case 8: bytes = Group<N, 8>::lds_bytes(n); break;
  }
  return bytes <= 160 * 1024;
}

#define FWR_ONCHIP_SIZES(X) X(8) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(80) X(128)

// The grid sizes are spread over several translation units so that they compile in
// parallel: this file is compiled once per unit with FWR_ONCHIP_UNIT = 0 ... 4.  Unit 0
// holds the size dispatch and the small sizes; units 1 ... 4 hold the explicit
// instantiations of the large ones (FWR_ONCHIP_UNIT undefined: everything in one unit).
#ifndef FWR_ONCHIP_UNIT
#define FWR_ONCHIP_UNIT -1
#endif
#define FWR_ONCHIP_INST(NN)                                                                  \
  template hipError_t launch_onchip<NN>(const OnchipArgs &, hipStream_t, int, int);        \
  template hipError_t prepare_onchip<NN>(int, int);
#define FWR_ONCHIP_EXTERN(NN)                                                                \
  extern template hipError_t launch_onchip<NN>(const OnchipArgs &, hipStream_t, int, int); \
  extern template hipError_t prepare_onchip<NN>(int, int);
#if FWR_ONCHIP_UNIT < 0 || FWR_ONCHIP_UNIT == 1
FWR_ONCHIP_INST(80)
#else
FWR_ONCHIP_EXTERN(80)
#endif
#if FWR_ONCHIP_UNIT < 0 || FWR_ONCHIP_UNIT == 2
FWR_ONCHIP_INST(128)
#else
FWR_ONCHIP_EXTERN(128)
#endif
#if FWR_ONCHIP_UNIT < 0 || FWR_ONCHIP_UNIT == 3
FWR_ONCHIP_INST(64)
#else
FWR_ONCHIP_EXTERN(64)
#endif
#if FWR_ONCHIP_UNIT < 0 || FWR_ONCHIP_UNIT == 4
FWR_ONCHIP_INST(48)
FWR_ONCHIP_INST(40)
#else
FWR_ONCHIP_EXTERN(48)
FWR_ONCHIP_EXTERN(40)
#endif

#if FWR_ONCHIP_UNIT <= 0

bool onchip_supported(int N) {
  switch (N) {
#define FWR_CASE(NN) case NN: return true;
    FWR_ONCHIP_SIZES(FWR_CASE)
#undef FWR_CASE
    default: return false;
  }
}

int onchip_threads(int N, int pairs) { return 4 * N * pairs; }
int onchip_lds_bytes(int N, int n, int pairs) {
  switch (N) {
#define FWR_CASE(NN)                                   \
  case NN:                                             \
    switch (pairs) {                                   \
      case 1: return Group<NN, 1>::lds_bytes(n);       \
      case 2: return Group<NN, 2>::lds_bytes(n);       \
      case 4: return Group<NN, 4>::lds_bytes(n);       \
      case 8: return Group<NN, 8>::lds_bytes(n);       \
      default: return 0;                               \
    }
    FWR_ONCHIP_SIZES(FWR_CASE)
#undef FWR_CASE
    default: return 0;
  }
}

bool onchip_pairs_ok(int N, int n, int pairs, bool each) {
  switch (N) {
#define FWR_CASE(NN) case NN: return pairs_ok<NN>(n, pairs, each);
    FWR_ONCHIP_SIZES(FWR_CASE)
#undef FWR_CASE
    default: return false;
  }
}

hipError_t onchip_prepare(int N, int n, int pairs) {
  switch (N) {
#define FWR_CASE(NN) case NN: return prepare_onchip<NN>(n, pairs);
    FWR_ONCHIP_SIZES(FWR_CASE)
#undef FWR_CASE
    default: return hipErrorInvalidValue;
  }
}

bool onchip_sched_ok(int N, int n) {
  if (2 * n != N || N % 4 != 0) return false;
  switch (N) {
#define FWR_CASE(NN) case NN: return sched_instantiated<NN>();
    FWR_ONCHIP_SIZES(FWR_CASE)
#undef FWR_CASE
    default: return false;
  }
}

hipError_t onchip_launch(int N, const OnchipArgs &a, hipStream_t s, int pairs, int sched) {
  switch (N) {
#define FWR_CASE(NN) case NN: return launch_onchip<NN>(a, s, pairs, sched);
    FWR_ONCHIP_SIZES(FWR_CASE)
#undef FWR_CASE
    default: return hipErrorInvalidValue;
  }
}

#endif  // FWR_ONCHIP_UNIT <= 0

}  // namespace fwr
