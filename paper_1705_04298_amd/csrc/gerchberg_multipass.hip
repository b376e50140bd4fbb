// Multi-pass Gerchberg extension + Fourier reconstruction for grids too large
// for one workgroup's LDS (N = 256: 512 KiB per frame pair).
//
// Same formulation as the on-chip kernel (two frames per complex field; the
// loop step is q = G^T s, phi = TF^-1[TF(q) / |G|^2], s' = G phi; see
// gerchberg_onchip.hip), split into grid-wide phases that exchange whole
// fields through HBM (the 64 MiB working set of 64 frame pairs, two complex
// fields each, stays in the MALL):
//   row_fwd     : stencil (or F0 at the start) on 16-row blocks + forward row FFTs  -> SPEC
//   col         : forward column FFTs, filter, inverse column FFTs on 16-column tiles
//   row_inv     : inverse row FFTs -> PHI
//   row_inv_fwd : between two solves of the pruned loop, row_inv and the next row_fwd in
//                 one pass (phi stays in LDS)  -> second spectrum field, read by col
// and, once per call, the explicit final step (cell slopes, Eq. 5 sums and
// fix, scatter to q) and the output kernels.  With launch shape 2 the loop's col
// and row_inv_fwd steps run as one persistent launch (loop_kernel, below) whose
// workgroups hand the spectra to one another.
//
// Without per-iteration Eq. 5 the loop is pruned to the window, as in the on-chip
// kernel: q2 vanishes outside the n+1 window rows (it is G^T of slopes that differ from
// the model slopes of phi only inside the pupil, and phi came from the previous q2), so
// row_fwd runs on the blocks of the window rows (zeros elsewhere in them), col reads only
// the window rows and writes back only the rows the next pass needs, and row_inv runs on
// the blocks of the window rows and one row either side.  The last solve before an
// explicit final step writes all rows (phi is exact everywhere; only its rows were
// skipped).
//
// FFT of a 256-point line: 16 threads, 16 x 16 decomposition through LDS.
// Stage A: thread r takes points 16a + r, DFT-16 over a, twiddle W_256^(r k1);
// stage B: thread k1 takes the 16 contiguous results, DFT-16.  Position
// 16 k1 + k2 then holds frequency k1 + 16 k2 (digit-reversed); the filter
// table is laid out in that order and the inverse undoes it.  Lines are
// padded by one element every 16, plus one (273 per line), to spread LDS banks.
#include <algorithm>
#include <atomic>

#include "fft256.h"
#include "multipass.h"

namespace fwr {

namespace mp {

__device__ __forceinline__ size_t field(int pair) { return (size_t)pair * NN * NN; }

constexpr int kCtlStride = 64;  // words between two work counts of the persistent loop (ctl)

// The forcing rows F0 hold each thread's 16 nodes (m, r + 16 q), q = 0..15, contiguously at
// [row][16 r + q], so that a thread loads them as eight 16-byte words; the node codes are packed
// per thread as well: codes[16 m + r] holds the 4-bit code of node (m, r + 16 q) in bits 4q..4q+3.
__device__ __forceinline__ void load_forcing(const float2 *row, int r, float2 (&f)[R]) {
  const float4 *p = reinterpret_cast<const float4 *>(row + R * r);
#pragma unroll
  for (int h = 0; h < R / 2; ++h) {
    const float4 v = p[h];
    f[2 * h] = make_float2(v.x, v.y);
    f[2 * h + 1] = make_float2(v.z, v.w);
  }
}
__device__ __forceinline__ uint32_t node_code(uint64_t w, int q) { return uint32_t(w >> (4 * q)) & 15u; }

__device__ __forceinline__ void load_tw(float2 *tw, const float2 *g, int t) {
  stage_tw_rk(tw, g, t, THREADS);  // (256-thread workgroups)
}

// in-pupil test of cell (cm, cn) (indices mod N)
__device__ __forceinline__ bool in_pupil(const uint8_t *mask, int n, int o, int cm, int cn) {
  cm &= NN - 1;
  cn &= NN - 1;
  const unsigned i = unsigned(cm - o), j = unsigned(cn - o);
  return i < unsigned(n) && j < unsigned(n) && mask[i * n + j] != 0;
}

// A frame's non-finite input must not reach its partner through the shared complex field:
// every measured slope enters the field through clean() (non-finite values as zeros), and
// the frame is flagged so that its output is written as NaN.
__device__ __forceinline__ bool finite(float v) { return (__float_as_uint(v) & 0x7f800000u) != 0x7f800000u; }
__device__ __forceinline__ float clean(float v) { return finite(v) ? v : 0.f; }
__device__ __forceinline__ float nan_f() { return __uint_as_float(0x7fc00000u); }

// Loads and stores of the spectrum fields that workgroups of the persistent loop kernel hand to
// one another within the launch (COH): relaxed atomics at agent scope, i.e. accesses coherent
// across the XCDs' L2 caches (the L2s of a multi-XCD device are not coherent with each other
// within a kernel; plain accesses may hit a stale line).  The other kernels use plain accesses.
template <bool COH>
__device__ __forceinline__ float2 ld2(const float2 *p) {
  if constexpr (COH) {
    const unsigned long long v = __hip_atomic_load(reinterpret_cast<unsigned long long *>(const_cast<float2 *>(p)),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_float2(__uint_as_float(uint32_t(v)), __uint_as_float(uint32_t(v >> 32)));
  } else {
    return *p;
  }
}
template <bool COH>
__device__ __forceinline__ void st2(float2 *p, float2 v) {
  if constexpr (COH) {
    const unsigned long long b = uint64_t(__float_as_uint(v.x)) | (uint64_t(__float_as_uint(v.y)) << 32);
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    *p = v;
  }
}

// measured (s_x, s_y) of cell (cm, cn) for frames A (real) and B (imag), cleaned; returns
// the frames' non-finite bits (1: A, 2: B)
__device__ __forceinline__ uint32_t measured(const MPArgs &a, int pair, int cm, int cn, float2 &sx, float2 &sy) {
  const int n = a.n, plane = n * n;
  const int idx = (cm - a.o) * n + (cn - a.o);
  const float *sa = a.slopes + (size_t)(2 * pair) * 2 * plane;
  const bool hasB = 2 * pair + 1 < a.B;
  const float ax = sa[idx], ay = sa[plane + idx];
  const float bx = hasB ? sa[2 * plane + idx] : 0.f, by = hasB ? sa[3 * plane + idx] : 0.f;
  sx = make_float2(clean(ax), clean(bx));
  sy = make_float2(clean(ay), clean(by));
  return (finite(ax) && finite(ay) ? 0u : 1u) | (finite(bx) && finite(by) ? 0u : 2u);
}

// non-finite bits of the pair, from the window row blocks' words (all N/16 words are loaded
// at once; those past the window's blocks are not written by this plan and are ignored)
__device__ __forceinline__ uint32_t pair_bad(const MPArgs &a, int pair) {
  const int nb = (a.o + a.n) / R - a.o / R + 1;
  const uint32_t *w = a.bad + (size_t)pair * (NN / R);
  uint32_t bad = a.loop_err != nullptr && *a.loop_err != 0 ? 3u : 0u;  // (the loop gave up: every frame)
#pragma unroll
  for (int b = 0; b < NN / R; ++b) {
    const uint32_t v = w[b];
    bad |= b < nb ? v : 0u;
  }
  return bad;
}

// ---------------------------------------------------------------- row phase
// mode 0: q2 = F0 (start of the loop; also stores F0 rows of the window)
// mode 1: q2 = F0 + sum over out-of-pupil cells of (phi - phi_diagonal)
// mode 2: mode 1 plus Eq. 5 on the border node columns of the window rows:
//         node (m, 0) by -(R_m + R_{m-1}), node (m, N-1) by +(R_m + R_{m-1})
// mode 3: Eq. 5 on the border node rows: node (0, n) by -(C_n + C_{n-1}), node (N-1, n) by
//         +(C_n + C_{n-1}); row blocks 0 and N/16 - 1, only rows 0 and N-1 are written.  A
//         mode-2 launch runs it on its last two blocks (after the nw window blocks; nw is also
//         the number of column-sum partials).
// R_m = sums[N + m] and the column-sum partials come from eq5_kernel.
// blocks start at row block b0
__global__ __launch_bounds__(THREADS) void row_fwd_kernel(MPArgs a, int mode_arg, int b0, int nw) {
  // phi rows m0-1 .. m0+16; once the stencil has read them, the same LDS holds the 16
  // padded lines of the row transforms (R * LP <= (R + 2) * NN), so four blocks fit a CU
  __shared__ float2 ph[(R + 2) * NN];
  static_assert(R * LP <= (R + 2) * NN, "line buffer must fit in the phi rows");
  float2 *const L = ph;
  __shared__ float2 tw[TW_RK];
  __shared__ uint32_t badw;  // mode 0: the block's non-finite bits
  const int t = threadIdx.x, rl = t >> 4, r = t & 15;
  const int mode = mode_arg == 2 && int(blockIdx.x) >= nw ? 3 : mode_arg;  // uniform per block
  if (t == 0) badw = 0;
  const int pair = blockIdx.y, m0 = mode == 3 ? (int(blockIdx.x) == nw ? 0 : NN - R) : (blockIdx.x + b0) * R;
  const int m = m0 + rl;
  load_tw(tw, a.tw256, t);
  if (mode == 1 || mode == 2) {
    const float2 *P = a.phi + field(pair);
#pragma unroll
    for (int c_ = 0; c_ < (R + 2) * NN / THREADS; ++c_) {  // (constant trip count: unrolled, loads batched)
      const int i = t + c_ * THREADS;
      const int row = (m0 - 1 + i / NN) & (NN - 1);
      ph[i] = P[(size_t)row * NN + (i % NN)];
    }
  }
  const bool win_row = m >= a.o && m <= a.o + a.n;
  float2 *F0 = a.f0 + (size_t)pair * (a.n + 1) * NN;
  // the forcing and the node codes of this thread's nodes, loaded with the phi rows (from
  // a valid row on the lines outside the window, whose result is replaced by zero)
  float2 f0v[R];
  uint64_t cw = 0;
  if (mode == 1 || mode == 2) {
    load_forcing(F0 + (size_t)(win_row ? m - a.o : 0) * NN, r, f0v);
    cw = a.codes[m * R + r];
  }
  __syncthreads();
  float2 fq[R];
  uint32_t bad = 0;  // mode 0: every in-pupil cell is cell (m, nn) of one window-row node
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int nn = r + R * q;
    float2 f = make_float2(0.f, 0.f);
    if (mode == 0) {
      if (win_row) {
        const int nl = (nn - 1) & (NN - 1), up = (m - 1) & (NN - 1);
        float2 sx, sy;
        if (in_pupil(a.mask, a.n, a.o, m, nn)) { bad |= measured(a, pair, m, nn, sx, sy); f = csub(f, cadd(sx, sy)); }
        if (in_pupil(a.mask, a.n, a.o, up, nl)) { measured(a, pair, up, nl, sx, sy); f = cadd(f, cadd(sx, sy)); }
        if (in_pupil(a.mask, a.n, a.o, m, nl)) { measured(a, pair, m, nl, sx, sy); f = cadd(f, csub(sx, sy)); }
        if (in_pupil(a.mask, a.n, a.o, up, nn)) { measured(a, pair, up, nn, sx, sy); f = csub(f, csub(sx, sy)); }
      }
    } else if (mode != 3) {
      f = f0v[q];
      const uint32_t c = node_code(cw, q);
      const float2 p0 = ph[(rl + 1) * NN + nn];
      const int np = (nn + 1) & (NN - 1), nm = (nn - 1) & (NN - 1);
      const float2 d1 = ph[(rl + 2) * NN + np], d2 = ph[rl * NN + nm];
      const float2 d3 = ph[(rl + 2) * NN + nm], d4 = ph[rl * NN + np];
      if (c & 1) f = cadd(f, csub(p0, d1));
      if (c & 2) f = cadd(f, csub(p0, d2));
      if (c & 4) f = cadd(f, csub(p0, d3));
      if (c & 8) f = cadd(f, csub(p0, d4));
      if (!win_row) f = make_float2(0.f, 0.f);  // (q2 = 0 on the other rows)
      if (mode == 2 && win_row && (nn == 0 || nn == NN - 1)) {
        const float2 *Rs = a.sums + (size_t)pair * 2 * NN + NN;
        const float2 r0 = m <= a.o + a.n - 1 ? Rs[m] : make_float2(0.f, 0.f);
        const float2 r1 = m - 1 >= a.o ? Rs[m - 1] : make_float2(0.f, 0.f);
        const float2 rr = cadd(r0, r1);
        f = nn == 0 ? csub(f, rr) : cadd(f, rr);
      }
    }
    fq[q] = f;
  }
  if (mode == 0 && win_row) {  // the forcing rows, each thread's 16 nodes as eight 16-byte words
    float4 *F4 = reinterpret_cast<float4 *>(F0 + (size_t)(m - a.o) * NN + R * r);
#pragma unroll
    for (int h = 0; h < R / 2; ++h) F4[h] = make_float4(fq[2 * h].x, fq[2 * h].y, fq[2 * h + 1].x, fq[2 * h + 1].y);
  }
  if (mode == 3) {  // (q2 = 0 on the block's other rows)
    // C_n for n = t from the b0 <= N/16 partials (fixed order, loads issued together), staged in
    // the phi-row LDS that this mode does not use
    const float2 *part = a.sx + field(pair);  // column-sum partials [nw][N]
    float2 pv[NN / R];
#pragma unroll
    for (int b = 0; b < NN / R; ++b) pv[b] = part[(b < nw ? b : 0) * NN + t];
    float2 cn = make_float2(0.f, 0.f);
#pragma unroll
    for (int b = 0; b < NN / R; ++b)
      if (b < nw) cn = cadd(cn, pv[b]);
    ph[t] = cn;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int nn = r + R * q, nl = (nn - 1) & (NN - 1);
      const float2 cc = cadd(ph[nn], ph[nl]);
      fq[q] = m == 0 ? make_float2(-cc.x, -cc.y) : (m == NN - 1 ? cc : make_float2(0.f, 0.f));
    }
  }
  if (bad != 0) atomicOr(&badw, bad);
  __syncthreads();  // every stencil read of the phi rows is done
#pragma unroll
  for (int q = 0; q < R; ++q) L[rl * LP + pad(r + R * q)] = fq[q];
  __syncthreads();
  fft_stage_a<-1>(L + rl * LP, r, tw);
  __syncthreads();
  fft_stage_b<-1>(L + rl * LP, r);
  __syncthreads();
  if (mode == 0 && t == 0) a.bad[(size_t)pair * (NN / R) + blockIdx.x] = badw;  // (b0 = the first window block)
  // the start pass also zeroes the persistent loop's counters: the pair's count, and with pair 0
  // the item counter and the error word
  if (mode == 0 && blockIdx.x == 0 && t < kCtlStride) {
    a.ctl[(size_t)kCtlStride * (pair + 1) + t] = 0u;
    if (pair == 0) a.ctl[t] = 0u;
  }
  float2 *S = a.spec + field(pair);
#pragma unroll
  for (int c_ = 0; c_ < R * NN / THREADS; ++c_) {  // (constant trip count: unrolled, loads batched)
    const int i = t + c_ * THREADS;
    const int row = i / NN, p = i % NN;
    // rows 0 and N-1 belong to the border blocks of a mode-2 launch (never window rows)
    const bool border_row = m0 + row == 0 || m0 + row == NN - 1;
    if (mode == 3 ? border_row : !(mode_arg == 2 && border_row)) S[(size_t)(m0 + row) * NN + p] = L[row * LP + pad(p)];
  }
}

// Eq. 5 sums from the in-pupil misfits (measured - model slopes of phi), on the window's row
// blocks: R_m (fixed-order row sums) to sums[N + m] for every row of the block, and the
// block's partial column sums of the y misfits to the column-sum partials [block][N] (kept in
// the s_x field, unused on this path).  Outside the pupil the slopes are the model slopes of
// the periodic phase, whose full-row (x) and full-column (y) sums vanish, so R_m and C_n are
// these misfit sums alone.
// (the block's y misfits reuse the LDS of its phi rows once every thread has read them: 36 KB of
// LDS instead of 68 KB, four blocks per CU instead of two)
__global__ __launch_bounds__(THREADS) void eq5_kernel(MPArgs a, int b0) {
  __shared__ float2 ph[(R + 1) * NN];
  __shared__ float2 part[THREADS];
  const int t = threadIdx.x, rl = t >> 4, r = t & 15;
  const int pair = blockIdx.y, m0 = (blockIdx.x + b0) * R, m = m0 + rl;
  const float2 *P = a.phi + field(pair);
#pragma unroll
  for (int c_ = 0; c_ < (R + 1) * NN / THREADS; ++c_) {  // (constant trip count: unrolled, loads batched)
    const int i = t + c_ * THREADS;
    const int row = (m0 + i / NN) & (NN - 1);
    ph[i] = P[(size_t)row * NN + (i % NN)];
  }
  const int n = a.n, o = a.o, plane = n * n;
  const float *sa = a.slopes + (size_t)(2 * pair) * 2 * plane;
  const bool hasB = 2 * pair + 1 < a.B;
  const float *sb = hasB ? sa + 2 * plane : sa;
  float2 mx[R], my[R];
  bool inp[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int nn = r + R * q;
    const bool inw = unsigned(m - o) < unsigned(n) && unsigned(nn - o) < unsigned(n);
    const int idx = inw ? (m - o) * n + (nn - o) : 0;
    inp[q] = inw && a.mask[idx] != 0;
    mx[q] = make_float2(sa[idx], hasB ? sb[idx] : 0.f);
    my[q] = make_float2(sa[plane + idx], hasB ? sb[plane + idx] : 0.f);
  }
  __syncthreads();
  float2 acc = make_float2(0.f, 0.f);
  float2 ey[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int nn = r + R * q, np = (nn + 1) & (NN - 1);
    const float2 a0 = ph[rl * NN + nn], b = ph[rl * NN + np];
    const float2 c = ph[(rl + 1) * NN + nn], d = ph[(rl + 1) * NN + np];
    const float2 gx = make_float2(0.5f * ((b.x - a0.x) + (d.x - c.x)), 0.5f * ((b.y - a0.y) + (d.y - c.y)));
    const float2 gy = make_float2(0.5f * ((c.x - a0.x) + (d.x - b.x)), 0.5f * ((c.y - a0.y) + (d.y - b.y)));
    // (cleaned here, after the barrier, so that the loads above stay in flight across it)
    const float2 mxc = make_float2(clean(mx[q].x), clean(mx[q].y)), myc = make_float2(clean(my[q].x), clean(my[q].y));
    const float2 ex = inp[q] ? csub(mxc, gx) : make_float2(0.f, 0.f);
    ey[q] = inp[q] ? csub(myc, gy) : make_float2(0.f, 0.f);
    acc = cadd(acc, ex);
  }
  __syncthreads();  // every read of the phi rows is done: their LDS takes the y misfits
#pragma unroll
  for (int q = 0; q < R; ++q) ph[rl * NN + r + R * q] = ey[q];
  part[t] = acc;
  __syncthreads();
  if (r == 0) {  // fixed-order row sum
    float2 s2 = make_float2(0.f, 0.f);
    for (int i = 0; i < R; ++i) s2 = cadd(s2, part[rl * R + i]);
    a.sums[(size_t)pair * 2 * NN + NN + m] = s2;
  }
  float2 cs = make_float2(0.f, 0.f);  // column t over the block's rows, fixed order
#pragma unroll
  for (int i = 0; i < R; ++i) cs = cadd(cs, ph[i * NN + t]);
  (a.sx + field(pair))[(size_t)blockIdx.x * NN + t] = cs;
}

// ---------------------------------------------------------------- column phase
// rows outside [rlo, rhi] (and, with `border`, other than 0 and N-1) are read as zeros;
// only rows in [wlo, whi] are written back
// (reads the spectrum from `in`, writes it to a.spec; the two may be the same field)
// TPL threads per 256-point line (the launch shape the autotuner picks): 16 (radix-16 DFTs in
// registers, four workgroups per CU) or 64 (one wave per line, quad sub-transforms: four times
// the waves for the same lines, for small batches)
// One 16-column tile (the body of col_kernel; the persistent loop kernel runs it with COH and
// with threads past the tile's R * TPL idle).  L: R padded lines; tw, tw16 staged by the caller.
template <int TPL, bool COH>
__device__ __forceinline__ void col_tile(const MPArgs &a, float2 *L, const float2 *tw, const float2 *tw16, int t,
                                         int pair, int c0, const float2 *in, const float *h, int rlo, int rhi,
                                         int wlo, int whi, int border) {
  constexpr int CT = R * TPL;
  const bool act = t < CT;
  const int cl = t / TPL, u = t % TPL;
  const QuadLane q(u & 3);
  const float2 *Sin = in + field(pair);
  float2 *S = a.spec + field(pair);
  // rows outside [rlo, rhi] load row rlo (a cache hit) and are replaced by zeros: every
  // load is issued first and kept unconditional, so that they are not serialised behind
  // divergent branches
  constexpr int NL = R * NN / CT;
  float2 v[NL];
  if (act) {
#pragma unroll
    for (int c_ = 0; c_ < NL; ++c_) {
      const int row = (t + c_ * CT) / R, cc = (t + c_ * CT) % R;
      const bool in = (row >= rlo && row <= rhi) || (border && (row == 0 || row == NN - 1));
      v[c_] = ld2<COH>(Sin + uint32_t((in ? row : rlo) * NN + c0 + cc));  // (unsigned: no sign extension)
    }
#pragma unroll
    for (int c_ = 0; c_ < NL; ++c_) asm volatile("" : "+v"(v[c_].x), "+v"(v[c_].y));
#pragma unroll
    for (int c_ = 0; c_ < NL; ++c_) {
      const int row = (t + c_ * CT) / R, cc = (t + c_ * CT) % R;
      const bool in = (row >= rlo && row <= rhi) || (border && (row == 0 || row == NN - 1));
      L[cc * LP + pad(row)] = in ? v[c_] : make_float2(0.f, 0.f);
    }
  }
  __syncthreads();
  if constexpr (TPL == 16) {
    if (act) fft_stage_a<-1>(L + cl * LP, u, tw);
    __syncthreads();
    if (act) fft_stage_b<-1>(L + cl * LP, u);
  } else {
    fft_quad_stage_a<-1>(L + cl * LP, u, tw, tw16, q);
    __syncthreads();
    fft_quad_stage_b<-1>(L + cl * LP, u, tw16, q);
  }
  __syncthreads();
  if (act) {
    const float *hc = h + uint32_t((c0 + cl) * NN);
#pragma unroll
    for (int i = 0; i < NN / TPL; ++i) {
      const int p = u + TPL * i;
      const float2 w = L[cl * LP + pad(p)];
      const float hv = hc[p];
      L[cl * LP + pad(p)] = make_float2(w.x * hv, w.y * hv);
    }
  }
  __syncthreads();
  if constexpr (TPL == 16) {
    if (act) fft_stage_b<+1>(L + cl * LP, u);
    __syncthreads();
    if (act) fft_stage_a<+1>(L + cl * LP, u, tw);
  } else {
    fft_quad_stage_b<+1>(L + cl * LP, u, tw16, q);
    __syncthreads();
    fft_quad_stage_a<+1>(L + cl * LP, u, tw, tw16, q);
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int c_ = 0; c_ < R * NN / CT; ++c_) {  // (constant trip count: unrolled, loads batched)
      const int i = t + c_ * CT;
      const int row = i / R, cc = i % R;
      if (row >= wlo && row <= whi) st2<COH>(S + uint32_t(row * NN + c0 + cc), L[cc * LP + pad(row)]);
    }
  }
}

template <int TPL>
__global__ __launch_bounds__(R * TPL) void col_kernel(MPArgs a, const float2 *in, const float *h, int rlo, int rhi,
                                                      int wlo, int whi, int border) {
  static_assert(TPL == 16 || TPL == 64, "16 or 64 threads per line");
  __shared__ float2 L[R * LP];
  __shared__ float2 tw[TW_RK];  // TPL = 16: tw_rk_entry; TPL = 64: the lane-ordered stage-A twiddles
  __shared__ float2 tw16[16];
  const int t = threadIdx.x;
  if (TPL == 16)
    stage_tw_rk(tw, a.tw256, t, R * TPL);
  else if (t < NN)
    tw[t] = twq_entry(a.tw256, t);
  if (TPL == 64 && t < 16) tw16[t] = tw16_entry(a.tw256, t);
  col_tile<TPL, false>(a, L, tw, tw16, t, blockIdx.y, blockIdx.x * R, in, h, rlo, rhi, wlo, whi, border);
}

// ---------------------------------------------------------------- inverse rows
// Inverse row FFTs of 16 spectrum rows m0 .. m0+15 of a pair (the body of row_inv_kernel; the
// persistent loop runs it with COH for the loop's last solve, its threads past the first 256
// idle): phi rows, or with to_out the (n+1) x (n+1) node window of phi as the pair's two phase
// frames (NaN for a flagged frame).
template <bool COH>
__device__ __forceinline__ void row_inv_block(const MPArgs &a, float2 *L, const float2 *tw, int t, int pair, int m0,
                                              bool to_out) {
  const int rl = t >> 4, r = t & 15;
  const bool act = t < THREADS;
  const float2 *S = a.spec + field(pair);
  constexpr int NL = R * NN / THREADS;
  if (act) {
    float2 v[NL];
#pragma unroll
    for (int c_ = 0; c_ < NL; ++c_) {  // (constant trip count: unrolled, loads batched)
      const int i = t + c_ * THREADS;
      v[c_] = ld2<COH>(S + uint32_t((m0 + i / NN) * NN + i % NN));
    }
#pragma unroll
    for (int c_ = 0; c_ < NL; ++c_) {
      const int i = t + c_ * THREADS;
      L[(i / NN) * LP + pad(i % NN)] = v[c_];
    }
  }
  __syncthreads();
  if (act) fft_stage_b<+1>(L + rl * LP, r);
  __syncthreads();
  if (act) fft_stage_a<+1>(L + rl * LP, r, tw);
  __syncthreads();
  if (!act) return;
  if (!to_out) {
    float2 *Ph = a.phi + field(pair);
#pragma unroll
    for (int c_ = 0; c_ < NL; ++c_) {
      const int i = t + c_ * THREADS;
      const int row = i / NN, p = i % NN;
      Ph[(size_t)(m0 + row) * NN + p] = L[row * LP + pad(p)];
    }
    return;
  }
  const int n1 = a.n + 1;
  float *oa = a.out + (size_t)(2 * pair) * n1 * n1;
  const bool hasB = 2 * pair + 1 < a.B;
  const uint32_t bad = pair_bad(a, pair);
#pragma unroll
  for (int c_ = 0; c_ < NL; ++c_) {
    const int i = t + c_ * THREADS;
    const int m = m0 + i / NN, p = i % NN;
    if (m < a.o || m > a.o + a.n || p < a.o || p > a.o + a.n) continue;
    const float2 w = L[(i / NN) * LP + pad(p)];
    const size_t idx = (size_t)(m - a.o) * n1 + (p - a.o);
    oa[idx] = bad & 1u ? nan_f() : w.x;
    if (hasB) oa[(size_t)n1 * n1 + idx] = bad & 2u ? nan_f() : w.y;
  }
}

__global__ __launch_bounds__(THREADS) void row_inv_kernel(MPArgs a, int b0, int to_out) {
  __shared__ float2 L[R * LP];
  __shared__ float2 tw[TW_RK];
  const int t = threadIdx.x;
  load_tw(tw, a.tw256, t);
  row_inv_block<false>(a, L, tw, t, blockIdx.y, (blockIdx.x + b0) * R, to_out != 0);
}

// ---------------------------------------------------------------- inverse rows + next forward rows
constexpr int FT = (R + 2) * 16;  // 18 lines of 16 threads
// One window block (the body of row_inv_fwd_kernel; the persistent loop kernel runs it with COH).
// L: R + 2 padded lines; tw staged by the caller.
template <bool COH>
__device__ __forceinline__ void row_inv_fwd_block(const MPArgs &a, float2 *L, const float2 *tw, int t, int pair,
                                                  int m0, float2 *out) {
  const int rl = t >> 4, r = t & 15;
  const bool own = rl < R;  // the threads of lines 16 and 17 transform but own no output row
  const int m = m0 + (own ? rl : 0);
  const float2 *S = a.spec + field(pair);
  constexpr int NL = (R + 2) * NN / FT;
  float2 v[NL];  // (every load issued before the first LDS store)
#pragma unroll
  for (int c_ = 0; c_ < NL; ++c_) {  // (constant trip count: unrolled, loads batched)
    const int i = t + c_ * FT;
    const int row = i / NN, p = i % NN;
    v[c_] = ld2<COH>(S + uint32_t(((m0 - 1 + row) & (NN - 1)) * NN + p));
  }
  const bool win_row = own && m >= a.o && m <= a.o + a.n;
  const float2 *F0 = a.f0 + (size_t)pair * (a.n + 1) * NN;
  float2 f0v[R];
  load_forcing(F0 + (size_t)(win_row ? m - a.o : 0) * NN, r, f0v);
  const uint64_t cw = a.codes[m * R + r];
#pragma unroll
  for (int c_ = 0; c_ < NL; ++c_) {
    const int i = t + c_ * FT;
    L[(i / NN) * LP + pad(i % NN)] = v[c_];
  }
  __syncthreads();
  fft_stage_b<+1>(L + rl * LP, r);
  __syncthreads();
  fft_stage_a<+1>(L + rl * LP, r, tw);
  __syncthreads();
  // line j now holds phi row m0 - 1 + j; the stencil of row m reads lines rl .. rl + 2
  const int sl = own ? rl : 0;
  float2 fq[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int nn = r + R * q;
    float2 f = f0v[q];
    const uint32_t c = node_code(cw, q);
    const int np = (nn + 1) & (NN - 1), nm = (nn - 1) & (NN - 1);
    const float2 p0 = L[(sl + 1) * LP + pad(nn)];
    const float2 d1 = L[(sl + 2) * LP + pad(np)], d2 = L[sl * LP + pad(nm)];
    const float2 d3 = L[(sl + 2) * LP + pad(nm)], d4 = L[sl * LP + pad(np)];
    if (c & 1) f = cadd(f, csub(p0, d1));
    if (c & 2) f = cadd(f, csub(p0, d2));
    if (c & 4) f = cadd(f, csub(p0, d3));
    if (c & 8) f = cadd(f, csub(p0, d4));
    if (!win_row) f = make_float2(0.f, 0.f);  // (q2 = 0 on the other rows)
    fq[q] = f;
  }
  __syncthreads();  // every stencil read of the phi rows is done
#pragma unroll
  for (int q = 0; q < R; ++q) L[rl * LP + pad(r + R * q)] = fq[q];
  __syncthreads();
  fft_stage_a<-1>(L + rl * LP, r, tw);  // (lines 16 and 17 are transformed too and dropped)
  __syncthreads();
  fft_stage_b<-1>(L + rl * LP, r);
  __syncthreads();
  if (t < NN) {
    float2 *D = out + field(pair);
#pragma unroll
    for (int row = 0; row < R; ++row) st2<COH>(D + uint32_t((m0 + row) * NN + t), L[row * LP + pad(t)]);
  }
}

// One loop step between two column passes when phi is needed only by the next stencil: a
// window block takes the spectrum rows m0-1 .. m0+16, runs their inverse row FFTs (phi rows,
// kept in LDS), then the stencil (as row_fwd mode 1) and the forward row FFTs of its 16 rows.
// The blocks' halo rows overlap, so the result goes to `out`, not back to a.spec.
__global__ __launch_bounds__(FT) void row_inv_fwd_kernel(MPArgs a, float2 *out, int b0) {
  __shared__ float2 L[(R + 2) * LP];
  __shared__ float2 tw[TW_RK];
  const int t = threadIdx.x;
  stage_tw_rk(tw, a.tw256, t, FT);
  row_inv_fwd_block<false>(a, L, tw, t, blockIdx.y, (blockIdx.x + b0) * R, out);
}

// ---------------------------------------------------------------- persistent loop
// The pruned loop's column passes and fused row steps, C_0, RF_0, C_1, ..., RF_{K-2}, C_{K-1},
// then the last solve's inverse row FFTs (K = n_iter), as one launch of resident workgroups that
// take work items in that order from a counter: item = (step, pair, 16-column tile or row
// block).  An item waits until every item of its pair in the previous step is done (a per-pair
// count), so pairs move through the steps independently and one pair's loads overlap another's
// transforms, without a grid-wide barrier between the steps.  Items are taken in order and wait
// only on earlier items, taken by workgroups that are running, so the launch cannot deadlock
// whatever the number of resident workgroups.  A wait longer than a.wait_limit polls (~1 us each;
// default 2^20) sets the error word; every workgroup then stops, and the frames are written as
// NaN (pair_bad).  The counters are zeroed by the start pass (row_fwd_kernel, mode 0).
struct LoopArgs {
  uint32_t *ctl;          // [0] next item, [1] error, [64 (pair + 1)] items of the pair done (one
                          // 256-byte line per count: the waiting workgroups poll them)
  int pairs, nr, wb0;     // frame pairs; window row blocks per pair and the first one
  int wlo, whi;           // rows the column passes read (the window rows)
  int rlo, rhi;           // rows they write back (the stencil's reach)
  int last_wlo, last_whi; // rows the last column pass writes back
  int ri_b0, nri;         // row blocks of the last solve's inverse row FFTs (phi)
};

// item -> (column tile, fused row block or last-solve row block; step k, pair, tile / block index)
struct LoopItem {
  int kind;  // 0 column tile, 1 fused row step block, 2 the last solve's inverse row block
  int k, pair, sub;
};
// phase-major: the items of step k (every pair's column tiles, then every pair's row blocks) before
// those of step k + 1 (an order that lags the row blocks half a step behind the column tiles, so
// that every wait has the same slack, was measured slower: 0.753 against 0.727 ms per 128 frames)
__device__ __forceinline__ LoopItem loop_item(int item, const LoopArgs &l, int n_iter) {
  const int per = R + l.nr;
  const int ri0 = (n_iter - 1) * l.pairs * per + l.pairs * R;  // (the last solve's items follow)
  LoopItem it;
  if (item >= ri0) {
    it.kind = 2;
    it.k = n_iter - 1;
    it.pair = (item - ri0) / l.nri;
    it.sub = (item - ri0) % l.nri;
    return it;
  }
  const int k = item / (l.pairs * per), rem = item % (l.pairs * per);
  const int nc = l.pairs * R;
  it.kind = rem < nc ? 0 : 1;
  it.k = k;
  it.pair = rem < nc ? rem / R : (rem - nc) / l.nr;
  it.sub = rem < nc ? rem % R : (rem - nc) % l.nr;
  return it;
}

// (4 waves per SIMD: 3 workgroups per CU, as the LDS allows; letting the compiler use more registers
// instead, without spills, left one workgroup per CU by the occupancy query: 1.11 ms per 128 frames)
__global__ __launch_bounds__(FT, 4) void loop_kernel(MPArgs a, LoopArgs l) {
  // one array, the twiddles first: their reads (base 17 r, offsets k) then fit the immediate offset
  // fields of the LDS instructions, with no address register per offset
  __shared__ float2 lds[TW_RK + (R + 2) * LP];
  float2 *const tw = lds, *const L = lds + TW_RK;
  __shared__ int s_item;
  const int t = threadIdx.x;
  stage_tw_rk(tw, a.tw256, t, FT);
  const int per = R + l.nr;  // items of one pair in one loop step (column tiles + row blocks)
  const int total = (a.n_iter - 1) * l.pairs * per + l.pairs * (R + l.nri);
  uint32_t *next = l.ctl, *err = l.ctl + 1, *done = l.ctl + kCtlStride;
  int nxt = 0;
  if (t == 0) nxt = int(atomicAdd(next, 1u));
  for (;;) {
    if (t == 0) {
      int item = nxt;
      if (item < total) {
        nxt = int(atomicAdd(next, 1u));  // (the next item is taken while this one runs)
        const LoopItem w = loop_item(item, l, a.n_iter);
        const int pair = w.pair;
        const uint32_t need = uint32_t(w.k * per + (w.kind == 0 ? 0 : R));
        int spin = 0;
        while (__hip_atomic_load(done + kCtlStride * pair, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          if (((++spin & 63) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) ||
              spin > a.wait_limit) {
            __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            item = -1;
            break;
          }
          __builtin_amdgcn_s_sleep(8);  // (polls spaced out: they share the memory path with the items)
        }
      }
      s_item = item;
    }
    __syncthreads();
    const int item = s_item;
    if (item < 0 || item >= total) break;
    // (the thread index laundered per item, so that the bodies' address arithmetic is not hoisted
    // out of the item loop and held in registers across it)
    int tl = t;
    asm volatile("" : "+v"(tl));
    __builtin_assume(tl >= 0 && tl < FT);  // (its range, which the laundering hides)
    const LoopItem w = loop_item(item, l, a.n_iter);
    const int pair = w.pair;
    if (w.kind == 0) {
      const bool last = w.k == a.n_iter - 1;
      col_tile<16, true>(a, L, tw, nullptr, tl, pair, w.sub * R, w.k == 0 ? a.spec : a.sy, a.h_loop, l.wlo,
                         l.whi, last ? l.last_wlo : l.rlo, last ? l.last_whi : l.rhi, 0);
    } else if (w.kind == 1) {
      row_inv_fwd_block<true>(a, L, tw, tl, pair, (l.wb0 + w.sub) * R, a.sy);
    } else {
      row_inv_block<true>(a, L, tw, tl, pair, (l.ri_b0 + w.sub) * R, false);
    }
    // every store of the item is complete (seen at agent scope) before the pair's count moves
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    if (t == 0) __hip_atomic_fetch_add(done + kCtlStride * pair, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------- final step
// cell slopes: measured inside the pupil (bit for bit), G phi outside; row sums R_m
__global__ __launch_bounds__(THREADS) void slopes_kernel(MPArgs a, int phi_zero) {
  __shared__ float2 ph[(R + 1) * NN];
  __shared__ float2 part[THREADS];
  const int t = threadIdx.x, rl = t >> 4, r = t & 15;
  const int pair = blockIdx.y, m0 = blockIdx.x * R, m = m0 + rl;
  const float2 *P = a.phi + field(pair);
#pragma unroll
  for (int c_ = 0; c_ < (R + 1) * NN / THREADS; ++c_) {  // (constant trip count: unrolled, loads batched)
    const int i = t + c_ * THREADS;
    const int row = (m0 + i / NN) & (NN - 1);
    ph[i] = phi_zero ? make_float2(0.f, 0.f) : P[(size_t)row * NN + (i % NN)];
  }
  // the measured slopes and the mask of this thread's cells, loaded with the phi rows and
  // unconditionally (cells outside the window read cell 0 and are not used)
  const int n = a.n, o = a.o, plane = n * n;
  const float *sa = a.slopes + (size_t)(2 * pair) * 2 * plane;
  const bool hasB = 2 * pair + 1 < a.B;
  const float *sb = hasB ? sa + 2 * plane : sa;
  float2 mx[R], my[R];
  bool inp[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int nn = r + R * q;
    const bool inw = unsigned(m - o) < unsigned(n) && unsigned(nn - o) < unsigned(n);
    const int idx = inw ? (m - o) * n + (nn - o) : 0;
    inp[q] = inw && a.mask[idx] != 0;
    mx[q] = make_float2(sa[idx], sb[idx]);
    my[q] = make_float2(sa[plane + idx], sb[plane + idx]);
  }
  __syncthreads();
  float2 *SX = a.sx + field(pair), *SY = a.sy + field(pair);
  float2 acc = make_float2(0.f, 0.f);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int nn = r + R * q, np = (nn + 1) & (NN - 1);
    const float2 a0 = ph[rl * NN + nn], b = ph[rl * NN + np];
    const float2 c = ph[(rl + 1) * NN + nn], d = ph[(rl + 1) * NN + np];
    float2 sx = make_float2(0.5f * ((b.x - a0.x) + (d.x - c.x)), 0.5f * ((b.y - a0.y) + (d.y - c.y)));
    float2 sy = make_float2(0.5f * ((c.x - a0.x) + (d.x - b.x)), 0.5f * ((c.y - a0.y) + (d.y - b.y)));
    if (inp[q]) {  // measured inside the pupil (bit for bit; cleaned), G phi outside
      sx = make_float2(clean(mx[q].x), hasB ? clean(mx[q].y) : 0.f);
      sy = make_float2(clean(my[q].x), hasB ? clean(my[q].y) : 0.f);
    }
    SX[(size_t)m * NN + nn] = sx;
    SY[(size_t)m * NN + nn] = sy;
    acc = cadd(acc, sx);
  }
  part[t] = acc;
  __syncthreads();
  if (r == 0) {  // fixed-order row sum
    float2 s = make_float2(0.f, 0.f);
    for (int i = 0; i < R; ++i) s = cadd(s, part[rl * R + i]);
    a.sums[(size_t)pair * 2 * NN + NN + m] = s;
  }
}

// column sums C_n (fixed order), then Eq. 5 on column N-1 of s_x and row N-1 of s_y
__global__ __launch_bounds__(THREADS) void periodic_kernel(MPArgs a) {
  const int pair = blockIdx.x, t = threadIdx.x;
  float2 *SX = a.sx + field(pair), *SY = a.sy + field(pair);
  float2 *sums = a.sums + (size_t)pair * 2 * NN;
  float2 cs = make_float2(0.f, 0.f);
#pragma unroll 32
  for (int m = 0; m < NN; ++m) cs = cadd(cs, SY[(size_t)m * NN + t]);
  __syncthreads();  // all column reads done before row N-1 changes
  SY[(size_t)(NN - 1) * NN + t] = csub(SY[(size_t)(NN - 1) * NN + t], cs);
  SX[(size_t)t * NN + NN - 1] = csub(SX[(size_t)t * NN + NN - 1], sums[NN + t]);
}

// extended slopes out: frame A from the real parts, frame B from the imaginary parts
__global__ __launch_bounds__(THREADS) void ext_out_kernel(MPArgs a) {
  const int pair = blockIdx.y, m = blockIdx.x, t = threadIdx.x;
  const float2 *SX = a.sx + field(pair), *SY = a.sy + field(pair);
  const size_t plane = (size_t)NN * NN;
  float *oa = a.out + (size_t)(2 * pair) * 2 * plane;
  const bool hasB = 2 * pair + 1 < a.B;
  const size_t idx = (size_t)m * NN + t;
  const float2 x = SX[idx], y = SY[idx];
  const uint32_t bad = pair_bad(a, pair);
  oa[idx] = bad & 1u ? nan_f() : x.x;
  oa[plane + idx] = bad & 1u ? nan_f() : y.x;
  if (hasB) {
    oa[2 * plane + idx] = bad & 2u ? nan_f() : x.y;
    oa[3 * plane + idx] = bad & 2u ? nan_f() : y.y;
  }
}

// q2 = -p(m,n) + p(m-1,n-1) + r(m,n-1) - r(m-1,n), p = s_x + s_y, r = s_x - s_y; row FFT
__global__ __launch_bounds__(THREADS) void scatter_kernel(MPArgs a) {
  __shared__ float2 L[R * LP];
  __shared__ float2 tw[TW_RK];
  const int t = threadIdx.x, rl = t >> 4, r = t & 15;
  const int pair = blockIdx.y, m0 = blockIdx.x * R, m = m0 + rl, up = (m - 1) & (NN - 1);
  load_tw(tw, a.tw256, t);
  const float2 *SX = a.sx + field(pair), *SY = a.sy + field(pair);
  for (int q = 0; q < R; ++q) {
    const int nn = r + R * q, nm = (nn - 1) & (NN - 1);
    const float2 p_mn = cadd(SX[(size_t)m * NN + nn], SY[(size_t)m * NN + nn]);
    const float2 p_ul = cadd(SX[(size_t)up * NN + nm], SY[(size_t)up * NN + nm]);
    const float2 r_ml = csub(SX[(size_t)m * NN + nm], SY[(size_t)m * NN + nm]);
    const float2 r_un = csub(SX[(size_t)up * NN + nn], SY[(size_t)up * NN + nn]);
    L[rl * LP + pad(nn)] = cadd(csub(p_ul, p_mn), csub(r_ml, r_un));
  }
  __syncthreads();
  fft_stage_a<-1>(L + rl * LP, r, tw);
  __syncthreads();
  fft_stage_b<-1>(L + rl * LP, r);
  __syncthreads();
  float2 *S = a.spec + field(pair);
#pragma unroll
  for (int c_ = 0; c_ < R * NN / THREADS; ++c_) {  // (constant trip count: unrolled, loads batched)
    const int i = t + c_ * THREADS;
    const int row = i / NN, p = i % NN;
    S[(size_t)(m0 + row) * NN + p] = L[row * LP + pad(p)];
  }
}

}  // namespace mp

size_t multipass_workspace_bytes(int N, int n, int max_batch) {
  if (N != mp::NN) return 0;
  const size_t pairs = (size_t)(max_batch + 1) / 2;
  const size_t f = (size_t)N * N * sizeof(float2);
  return pairs * (4 * f + (size_t)(n + 1) * N * sizeof(float2) + 2 * (size_t)N * sizeof(float2) +
                 (size_t)(N / mp::R) * sizeof(uint32_t)) +
         multipass_ctl_words(max_batch) * sizeof(uint32_t);
}

size_t multipass_ctl_words(int max_batch) { return mp::kCtlStride * ((size_t)(max_batch + 1) / 2 + 1); }

// resident workgroups of the persistent loop kernel on the current device (occupancy x CUs)
static int loop_grid() {
  static std::atomic<int> grid[64] = {};  // (per device; concurrent first calls store the same value)
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (grid[dev].load() == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mp::loop_kernel, mp::FT, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    grid[dev].store((per_cu > 0 ? per_cu : 1) * cus);
  }
  return grid[dev].load();
}

bool multipass_supported(int N) { return N == mp::NN; }

hipError_t multipass_run(const MPArgs &a0, bool extend, hipStream_t s) {
  using namespace mp;
  MPArgs a = a0;
  const int pairs = (a.B + 1) / 2;
  const dim3 rows(NN / R, pairs), blk(THREADS);
  const bool periodic = (a.flags & kMPPeriodic) != 0;
  const bool each = (a.flags & kMPPeriodicEach) != 0;
  const bool explicit_final = periodic || extend || (each && a.n_iter > 0);
  const bool fix_final = periodic || (each && a.n_iter > 0);
  // Eq. 5 after the loop from the in-pupil misfits, without full slope fields.  Its border-row
  // blocks write node rows 0 and N-1, which must not be window rows: with o = 1 row N-1 = o + n
  // is one, so that case takes the explicit path.
  const bool eq5_sums = periodic && !extend && !each && a.n_iter > 0 && a.o >= 2;
  // window rows [o, o+n] and the stencil's reach [o-1, o+n+1]; their row blocks
  // (with o = 1 the reach wraps around: every row)
  const int wlo = a.o, whi = a.o + a.n;
  const int rlo = a.o >= 2 ? a.o - 1 : 0, rhi = a.o >= 2 ? a.o + a.n + 1 : NN - 1;
  const int wb0 = wlo / R, wb1 = whi / R, rb0 = rlo / R, rb1 = rhi / R;
  const dim3 wrows(wb1 - wb0 + 1, pairs), rrows(rb1 - rb0 + 1, pairs);
  auto col = [&](const float2 *in, const float *h, int rlo_, int rhi_, int wlo_, int whi_, int border) {
    if (a.col_shape == 1)
      hipLaunchKernelGGL(col_kernel<64>, rows, dim3(R * 64), 0, s, a, in, h, rlo_, rhi_, wlo_, whi_, border);
    else
      hipLaunchKernelGGL(col_kernel<16>, rows, dim3(R * 16), 0, s, a, in, h, rlo_, rhi_, wlo_, whi_, border);
  };
  auto explicit_q = [&](bool phi_zero, bool fix) {
    hipLaunchKernelGGL(slopes_kernel, rows, blk, 0, s, a, phi_zero ? 1 : 0);
    if (fix) hipLaunchKernelGGL(periodic_kernel, dim3(pairs), blk, 0, s, a);
  };
  // start: q2 = F0 (also fills the F0 rows), forward row FFTs of the window rows
  hipLaunchKernelGGL(row_fwd_kernel, wrows, blk, 0, s, a, 0, wb0, 0);
  // Between two solves of the pruned loop phi only feeds the next stencil: the inverse and
  // the next forward row pass run as one kernel, writing the spectrum to the s_y field (unused
  // until after the loop), which the next column pass reads back into the spectrum field.
  float2 *const spec2 = a.sy;
  const float2 *col_in = a.spec;
  // launch shape 2: the loop's column passes and fused row steps in one persistent launch
  // (the item indices are 32-bit: calls with more items than that run one launch per pass)
  const long loop_items = (long)a.n_iter * pairs * (R + (wb1 - wb0 + 1) + NN / R);
  const int lgrid = a.col_shape == 2 && !each && a.n_iter >= 2 && loop_items < (1L << 30) ? loop_grid() : 0;
  if (lgrid > 0) {
    const bool full_last = explicit_final && !eq5_sums;  // (as full_out of the last iteration below)
    LoopArgs l{};
    l.ctl = a.ctl;
    l.pairs = pairs;
    l.nr = wb1 - wb0 + 1;
    l.wb0 = wb0;
    l.wlo = wlo;
    l.whi = whi;
    l.rlo = rlo;
    l.rhi = rhi;
    l.last_wlo = full_last ? 0 : rlo;
    l.last_whi = full_last ? NN - 1 : rhi;
    l.ri_b0 = full_last ? 0 : rb0;  // the loop's last solve: inverse row FFTs of these row blocks
    l.nri = full_last ? NN / R : rb1 - rb0 + 1;
    // resident workgroups, at most half the items of one loop step (more only wait: measured)
    const long cap = std::min<long>(lgrid, (long)pairs * (R + l.nr) / 2);
    hipLaunchKernelGGL(loop_kernel, dim3((unsigned)std::max<long>(cap, 1)), dim3(FT), 0, s, a, l);
    a.loop_err = a.ctl + 1;  // read by the output kernels (pair_bad)
  }
  for (int it = 0; it < (lgrid > 0 ? 0 : a.n_iter); ++it) {
    const bool last = it == a.n_iter - 1;
    // q2 is window-supported here unless per-iteration Eq. 5 made it explicit
    const bool win_in = !each || it == 0;
    const bool full_out = each || (last && explicit_final && !eq5_sums);  // phi needed on every row
    col(col_in, a.h_loop, win_in ? wlo : 0, win_in ? whi : NN - 1,
                       full_out ? 0 : rlo, full_out ? NN - 1 : rhi, 0);
    col_in = a.spec;
    if (!last && !each) {
      hipLaunchKernelGGL(row_inv_fwd_kernel, wrows, dim3(FT), 0, s, a, spec2, wb0);
      col_in = spec2;
      continue;
    }
    if (full_out)
      hipLaunchKernelGGL(row_inv_kernel, rows, blk, 0, s, a, 0, 0);
    else
      hipLaunchKernelGGL(row_inv_kernel, rrows, blk, 0, s, a, rb0, 0);
    if (last) break;
    explicit_q(false, true);  // per-iteration Eq. 5
    hipLaunchKernelGGL(scatter_kernel, rows, blk, 0, s, a);
  }
  bool win_final = true;  // q2 of the final solve window-supported (plus rows 0 and N-1 with Eq. 5)
  bool border = false;
  if (eq5_sums) {
    hipLaunchKernelGGL(eq5_kernel, wrows, blk, 0, s, a, wb0);
    // the window blocks (mode 2) and the two border-row blocks (mode 3) in one launch
    hipLaunchKernelGGL(row_fwd_kernel, dim3(wb1 - wb0 + 3, pairs), blk, 0, s, a, 2, wb0, wb1 - wb0 + 1);
    border = true;
  } else if (explicit_final) {
    explicit_q(a.n_iter == 0, fix_final);
    if (extend) {
      hipLaunchKernelGGL(ext_out_kernel, dim3(NN, pairs), blk, 0, s, a);
      return hipGetLastError();
    }
    hipLaunchKernelGGL(scatter_kernel, rows, blk, 0, s, a);
    win_final = false;
  } else if (a.n_iter > 0) {
    hipLaunchKernelGGL(row_fwd_kernel, wrows, blk, 0, s, a, 1, wb0, 0);
  }
  // the output is the window rows
  col(a.spec, a.h_final, win_final ? wlo : 0, win_final ? whi : NN - 1, wlo,
                     whi, border ? 1 : 0);
  hipLaunchKernelGGL(row_inv_kernel, wrows, blk, 0, s, a, wb0, 1);  // (phi's window rows straight to the output)
  return hipGetLastError();
}

}  // namespace fwr

// ---------------------------------------------------------------- device frames, N = 256
#include "gen.h"

namespace fwr {
namespace mp {

__device__ __forceinline__ uint64_t philox_pair(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                uint32_t k1, uint32_t *out4) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = uint64_t(0xD2511F53u) * c0;
    const uint64_t p1 = uint64_t(0xCD9E8D57u) * c2;
    const uint32_t n0 = uint32_t(p1 >> 32) ^ c1 ^ k0, n1 = uint32_t(p1);
    const uint32_t n2 = uint32_t(p0 >> 32) ^ c3 ^ k1, n3 = uint32_t(p0);
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out4[0] = c0;
  out4[1] = c1;
  out4[2] = c2;
  out4[3] = c3;
  return 0;
}

__device__ __forceinline__ float2 bm(uint32_t a, uint32_t b) {
  const float u1 = (float(a >> 8) + 1.0f) * (1.0f / 16777216.0f);
  const float u2 = float(b >> 8) * (1.0f / 16777216.0f);
  const float r = sqrtf(-2.0f * logf(u1));
  float s, c;
  sincospif(2.0f * u2, &s, &c);
  return make_float2(r * c, r * s);
}

// spectrum in digit-reversed positions (row position q, column position c)
__global__ __launch_bounds__(THREADS) void gen_spectrum_kernel(MPArgs a, GenArgs g) {
  const int pair = blockIdx.y;
  const uint64_t gp = g.first_pair + pair + (g.d_counter ? *g.d_counter / 2 : 0);
  float2 *S = a.spec + field(pair);
  const float dk = 1.0f / (float(NN) * g.d);
  for (int i = threadIdx.x; i < R * NN; i += THREADS) {
    const int q = blockIdx.x * R + i / NN, c = i % NN;
    const int l = (q >> 4) + 16 * (q & 15), k = (c >> 4) + 16 * (c & 15);
    float amp = 0.f;
    if (l != 0 || k != 0) {
      const int ks = k < NN / 2 ? k : k - NN, ls = l < NN / 2 ? l : l - NN;
      const float kap2 = (float(ks) * ks + float(ls) * ls) * dk * dk;
      const float psd = g.vk_const * powf(g.r0, -5.0f / 3.0f) * powf(kap2 + 1.0f / (g.L0 * g.L0), -11.0f / 6.0f);
      amp = sqrtf(psd) * dk;
    }
    uint32_t r4[4];
    philox_pair(uint32_t(gp), uint32_t(gp >> 32), uint32_t(l * NN + k), 0u, g.seed_lo, g.seed_hi, r4);
    const float2 z = bm(r4[0], r4[1]);
    S[(size_t)q * NN + c] = make_float2(z.x * amp, z.y * amp);
  }
}

// inverse column transforms only (for the generator)
__global__ __launch_bounds__(THREADS) void col_inv_kernel(MPArgs a) {
  __shared__ float2 L[R * LP];
  __shared__ float2 tw[TW_RK];
  const int t = threadIdx.x, cl = t >> 4, r = t & 15;
  const int pair = blockIdx.y, c0 = blockIdx.x * R;
  load_tw(tw, a.tw256, t);
  float2 *S = a.spec + field(pair);
#pragma unroll
  for (int c_ = 0; c_ < R * NN / THREADS; ++c_) {  // (constant trip count: unrolled, loads batched)
    const int i = t + c_ * THREADS;
    const int row = i / R, cc = i % R;
    L[cc * LP + pad(row)] = S[(size_t)row * NN + c0 + cc];
  }
  __syncthreads();
  fft_stage_b<+1>(L + cl * LP, r);
  __syncthreads();
  fft_stage_a<+1>(L + cl * LP, r, tw);
  __syncthreads();
#pragma unroll
  for (int c_ = 0; c_ < R * NN / THREADS; ++c_) {  // (constant trip count: unrolled, loads batched)
    const int i = t + c_ * THREADS;
    const int row = i / R, cc = i % R;
    S[(size_t)row * NN + c0 + cc] = L[cc * LP + pad(row)];
  }
}

// slopes (+ noise, valid subapertures) and node phase from the screen pair in PHI
__global__ __launch_bounds__(THREADS) void gen_slopes_kernel(MPArgs a, GenArgs g) {
  const int pair = blockIdx.y;
  const uint64_t gp = g.first_pair + pair + (g.d_counter ? *g.d_counter / 2 : 0);
  const float2 *P = a.phi + field(pair);
  const int n = g.n, o = g.o, plane = n * n;
  const bool hasB = 2 * pair + 1 < g.B;
  float *sa = g.slopes + (size_t)(2 * pair) * 2 * plane;
  for (int idx = blockIdx.x * THREADS + threadIdx.x; idx < plane; idx += gridDim.x * THREADS) {
    const int i = idx / n, jj = idx - i * n, m = o + i, c = o + jj;
    const float2 p00 = P[(size_t)m * NN + c], p01 = P[(size_t)m * NN + c + 1];
    const float2 p10 = P[(size_t)(m + 1) * NN + c], p11 = P[(size_t)(m + 1) * NN + c + 1];
    const float2 sx = make_float2(0.5f * ((p01.x - p00.x) + (p11.x - p10.x)), 0.5f * ((p01.y - p00.y) + (p11.y - p10.y)));
    const float2 sy = make_float2(0.5f * ((p10.x - p00.x) + (p11.x - p01.x)), 0.5f * ((p10.y - p00.y) + (p11.y - p01.y)));
    uint32_t r4[4];
    philox_pair(uint32_t(gp), uint32_t(gp >> 32), uint32_t(idx), 1u, g.seed_lo, g.seed_hi, r4);
    const float2 na = bm(r4[0], r4[1]), nb = bm(r4[2], r4[3]);
    const float valid = g.mask[idx] ? 1.f : 0.f;
    sa[idx] = valid * (sx.x + g.sigma * na.x);
    sa[plane + idx] = valid * (sy.x + g.sigma * na.y);
    if (hasB) {
      sa[2 * plane + idx] = valid * (sx.y + g.sigma * nb.x);
      sa[3 * plane + idx] = valid * (sy.y + g.sigma * nb.y);
    }
  }
  if (g.phase) {
    const int n1 = n + 1;
    float *pa = g.phase + (size_t)(2 * pair) * n1 * n1;
    for (int idx = blockIdx.x * THREADS + threadIdx.x; idx < n1 * n1; idx += gridDim.x * THREADS) {
      const int i = idx / n1, jj = idx - i * n1;
      const float2 v = P[(size_t)(o + i) * NN + o + jj];
      pa[idx] = v.x;
      if (hasB) pa[(size_t)n1 * n1 + idx] = v.y;
    }
  }
}

__global__ void mp_counter_add_kernel(uint64_t *c, uint64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c += v;
}

}  // namespace mp

hipError_t multipass_generate(const MPArgs &a, const GenArgs &g, hipStream_t s) {
  using namespace mp;
  const int pairs = (g.B + 1) / 2;
  const dim3 rows(NN / R, pairs), blk(THREADS);
  hipLaunchKernelGGL(gen_spectrum_kernel, rows, blk, 0, s, a, g);
  hipLaunchKernelGGL(col_inv_kernel, rows, blk, 0, s, a);
  hipLaunchKernelGGL(row_inv_kernel, rows, blk, 0, s, a, 0, 0);
  hipLaunchKernelGGL(gen_slopes_kernel, dim3(16, pairs), blk, 0, s, a, g);
  if (g.d_counter) hipLaunchKernelGGL(mp_counter_add_kernel, dim3(1), dim3(64), 0, s, g.d_counter, uint64_t(2 * pairs));
  return hipGetLastError();
}

}  // namespace fwr
