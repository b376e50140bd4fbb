// Fourier-domain Gerchberg extension + reconstruction for slope models without a compact
// real-space stencil (the lenslet-averaging model of Eq. 4), padded grids N <= 128.
//
// One frame per complex field: Z = TF(s_x + i s_y).  With X = TF(s_x), Y = TF(s_y) and
// Z~ = conj(Z(-l, -k)), X = (Z + Z~) / 2 and Y = (Z - Z~) / (2i), so step 2 of Algorithm 1
// (LSQ phase, then the model slopes: X' = a X + c Y, Y' = conj(c) X + b Y with
// a = |G_x|^2 / |G|^2, b = |G_y|^2 / |G|^2, c = G_x conj(G_y) / |G|^2) becomes
//     Z' = alpha Z + beta Z~,   alpha = (a + b) / 2 + Im c (real),  beta = (a - b) / 2 + i Re c,
// and the final reconstruction (Eq. 2 with the Eq. 3 filter) is
//     Phi = A Z + B Z~,   A = (R_x - i R_y) / 2,  B = (R_x + i R_y) / 2.
// The plan tabulates alpha, beta, A, B per thread and slot (1/N^2 of the unnormalised inverse
// folded in).  Z~ comes through LDS: after the forward column transforms every thread writes
// its column of the spectrum in natural frequency order and reads the mirrored column.
//
// Layout and line transforms as in the on-chip Fried kernel (4 lanes per grid line, LDS tile
// N x (N+1) complex per frame); the state between iterations is s_x + i s_y in registers
// (row layout).  The measured slopes of the window rows stay in LDS for N <= 80; at N = 128 the
// tile alone takes 132 KB, and step 4 reads them from global memory (L2-resident) instead.
#include "fft_lane.h"
#include "fourier.h"
#include "lds_limit.h"

#include <cstdint>

namespace fwr {
namespace fourier {

template <int N>
struct Shape {
  static constexpr int T = N / 4;
  static constexpr int THREADS = 4 * N;
  static constexpr int P = N + 1;
  static constexpr int TILE = N * P;
  static constexpr bool MEAS_IN_LDS = N <= 80;  // measured window rows kept in LDS
};

// FR frames per workgroup (see the on-chip kernel: N = 80 makes 5 waves per frame)
template <int N, int FR>
struct FGroup {
  static constexpr int THREADS = FR * Shape<N>::THREADS;
  static constexpr int WAVES = (THREADS + 63) / 64;
  static constexpr int WAVES_PER_SIMD = (WAVES + 3) / 4 > 2 ? (WAVES + 3) / 4 : 2;
  static constexpr int STATIC_LDS_BYTES = FR * (Shape<N>::TILE + 2 * N) * 8 + Shape<N>::T * 4 * 8;
  static int dyn_bytes(int n) { return Shape<N>::MEAS_IN_LDS ? FR * n * Shape<N>::P * 8 : 0; }
  static int lds_bytes(int n) { return STATIC_LDS_BYTES + dyn_bytes(n); }
};

__device__ __forceinline__ float select_bits(bool c, float a, float b) {
  const uint32_t m = 0u - static_cast<uint32_t>(c);
  return __uint_as_float((__float_as_uint(a) & m) | (__float_as_uint(b) & ~m));
}

template <int N, int FR>
__global__ __launch_bounds__((FGroup<N, FR>::THREADS))
__attribute__((amdgpu_waves_per_eu(FGroup<N, FR>::WAVES_PER_SIMD)))
void fourier_kernel(FourierArgs a) {
  constexpr int T = Shape<N>::T, P = Shape<N>::P, TILE = Shape<N>::TILE, TH = Shape<N>::THREADS;
  __shared__ float2 buf_all[FR * TILE];
  __shared__ float2 sums_all[FR * N];
  __shared__ float2 tw[T * 4];
  extern __shared__ float2 meas_all[];  // FR x [n][P]: measured s_x + i s_y of the window rows

  const int half = FR == 1 ? 0 : int(threadIdx.x) / TH;
  const int t = int(threadIdx.x) - half * TH;
  float2 *const buf = buf_all + half * TILE;
  float2 *const sums = sums_all + half * N;
  float2 *const meas = meas_all + (Shape<N>::MEAS_IN_LDS ? half * a.n * P : 0);
  const int line = t >> 2, j = t & 3;
  const QuadLane q(j);
  const bool active = FR * int(blockIdx.x) + half < a.B;  // frames past the batch write nothing
  const int f = active ? FR * int(blockIdx.x) + half : 0;
  const int n = a.n, o = a.o, plane = n * n;

  for (int i = threadIdx.x; i < T * 4; i += FGroup<N, FR>::THREADS) tw[i] = a.tw_lane[i];

  // measured slopes of the window rows, lane-blocked: grid column c -> slot T (c % 4) + c / 4
  const float *sf = a.slopes + (size_t)f * 2 * plane;
  // all loads of a chunk are issued before its LDS stores (cells outside the window read
  // cell 0 and are replaced by zeros): one memory latency per chunk, not per element
  constexpr int CH = (N / 2 * N + TH - 1) / TH;
  for (int i0 = t; Shape<N>::MEAS_IN_LDS && i0 < n * N; i0 += CH * TH) {
    float vx[CH], vy[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = i0 + u * TH, r = i / N, c = i - r * N;
      const bool in = i < n * N && c >= o && c < o + n;
      const int g = in ? r * n + c - o : 0;
      vx[u] = sf[g];
      vy[u] = sf[plane + g];
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = i0 + u * TH, r = i / N, c = i - r * N;
      const bool in = i < n * N && c >= o && c < o + n;
      if (i < n * N) meas[r * P + T * (c & 3) + (c >> 2)] = in ? make_float2(vx[u], vy[u]) : make_float2(0.f, 0.f);
    }
  }
  __syncthreads();
  const uint32_t pup = a.inpupil[t];
  const bool in_rows = line >= o && line < o + n;
  const int mrow = (in_rows ? line - o : 0) * P + T * j;
  // measured s_x + i s_y of cell (line, 4k + j) (any value outside the window; only in-pupil
  // cells are used): from LDS, or from global memory where the LDS cannot hold the rows
  auto meas_at = [&](int k) -> float2 {
    if constexpr (Shape<N>::MEAS_IN_LDS) {
      return meas[mrow + k];
    } else {
      const int c = 4 * k + j - o;
      const int g = in_rows && c >= 0 && c < n ? (line - o) * n + c : 0;
      return make_float2(sf[g], sf[plane + g]);
    }
  };

  float2 x[T];  // s_x + i s_y of cells (line, 4k + j): the measurement, zeros or the start outside
  const float *stf = a.start ? a.start + (size_t)f * 2 * N * N + (size_t)line * N + j : nullptr;
#pragma unroll
  for (int k = 0; k < T; ++k) {
    const bool in = in_rows && ((pup >> k) & 1u);
    const float2 v = meas_at(k);
    const float ox = stf ? stf[4 * k] : 0.f, oy = stf ? stf[N * N + 4 * k] : 0.f;
    x[k] = make_float2(select_bits(in, v.x, ox), select_bits(in, v.y, oy));
  }

  // column-phase frequencies: LDS column c holds x-frequency kf(c); slot k of lane j holds
  // y-frequency l = k + T beta(j); the mirrored x-frequency sits in column cm
  const int beta_of[4] = {0, 2, 1, 3};
  const int kf = (line % T) + T * beta_of[line / T];
  const int kfm = kf == 0 ? 0 : N - kf;
  const int cm = T * beta_of[kfm / T] + kfm % T;
  const int lbase = T * beta_of[j];

  // one Fourier step: x (row layout, real space) -> x; `fin` selects the final filter
  auto solve = [&](bool fin) {
    line_fft_fwd<T>(x, tw, j, q);
#pragma unroll
    for (int k = 0; k < T; ++k) buf[line * P + T * j + k] = x[k];
    __syncthreads();
    float2 y[T];
#pragma unroll
    for (int k = 0; k < T; ++k) y[k] = buf[(4 * k + j) * P + line];
    line_fft_fwd<T>(y, tw, j, q);
    __syncthreads();  // column reads done before the spectrum exchange reuses the tile
#pragma unroll
    for (int k = 0; k < T; ++k) buf[line * P + lbase + k] = y[k];  // [column position][l]
    __syncthreads();
    const size_t tb = (size_t)t * T;
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const int l = lbase + k, lm = l == 0 ? 0 : N - l;
      const float2 zm = buf[cm * P + lm];
      const float2 z = y[k];
      if (fin) {
        const float2 A = a.fin_a[tb + k], Bc = a.fin_b[tb + k];
        // A z + B conj(zm)
        y[k] = make_float2(A.x * z.x - A.y * z.y + Bc.x * zm.x + Bc.y * zm.y,
                           A.x * z.y + A.y * z.x + Bc.y * zm.x - Bc.x * zm.y);
      } else {
        const float al = a.alpha[tb + k];
        const float2 be = a.beta[tb + k];
        // alpha z + beta conj(zm)
        y[k] = make_float2(al * z.x + be.x * zm.x + be.y * zm.y, al * z.y + be.y * zm.x - be.x * zm.y);
      }
    }
    __syncthreads();  // mirror reads done before the tile is rewritten
    line_fft_inv<T>(y, tw, j, q);
#pragma unroll
    for (int k = 0; k < T; ++k) buf[(4 * k + j) * P + line] = y[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < T; ++k) x[k] = buf[line * P + T * j + k];
    line_fft_inv<T>(x, tw, j, q);
  };

  // Eq. 5: s_x(m, N-1) -= R_m (row sum of s_x), s_y(N-1, n) -= C_n (column sum of s_y)
  auto eq5 = [&]() {
    float rs = 0.f;
#pragma unroll
    for (int k = 0; k < T; ++k) rs += x[k].x;
    rs += dpp_xor1(rs);
    rs += dpp_xor2(rs);
#pragma unroll
    for (int k = 0; k < T; ++k) buf[line * P + T * j + k] = x[k];  // own slots: no hazard
    __syncthreads();
    if (t < N) {  // fixed-order column sums
      const int slot = T * (t & 3) + (t >> 2);
      float cs = 0.f;
      for (int m = 0; m < N; ++m) cs += buf[m * P + slot].y;
      sums[t] = make_float2(0.f, cs);
    }
    __syncthreads();
    if (j == 3) x[T - 1].x -= rs;
    if (line == N - 1) {
#pragma unroll
      for (int k = 0; k < T; ++k) x[k].y -= sums[4 * k + j].y;
    }
    __syncthreads();  // the column sums are read before the next use of the buffers
  };
  // in-pupil misfit of the last iteration, before step 4: ||P (s' - s0)|| / ||P s0||
  auto residual = [&]() {
    float num = 0.f, den = 0.f;
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const bool in = in_rows && ((pup >> k) & 1u);
      const float2 v = meas_at(k);
      const float dx = x[k].x - v.x, dy = x[k].y - v.y;
      num += in ? dx * dx + dy * dy : 0.f;
      den += in ? v.x * v.x + v.y * v.y : 0.f;
    }
    num += dpp_xor1(num);
    num += dpp_xor2(num);
    den += dpp_xor1(den);
    den += dpp_xor2(den);
    if (j == 0) sums[line] = make_float2(num, den);
    __syncthreads();
    if (t < 64) {  // fixed-order sum over the lines: lane-wise, then a butterfly over the wave
      float nt = 0.f, dt = 0.f;
      for (int m = t; m < N; m += 64) {
        nt += sums[m].x;
        dt += sums[m].y;
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        nt += __shfl_xor(nt, off);
        dt += __shfl_xor(dt, off);
      }
      if (t == 0 && active) a.resid[f] = !(dt <= 0.f) ? sqrtf(nt / dt) : 0.f;  // (NaN stays NaN)
    }
    __syncthreads();  // the line sums are read before the buffer is used again
  };
  // step 4: the measurement inside the pupil, the extrapolation outside
  auto replace = [&]() {
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const bool in = in_rows && ((pup >> k) & 1u);
      const float2 v = meas_at(k);
      x[k] = make_float2(select_bits(in, v.x, x[k].x), select_bits(in, v.y, x[k].y));
    }
  };
  if (a.resid != nullptr && a.n_iter == 0 && t == 0 && active) a.resid[f] = 0.f;
  for (int it = 0; it < a.n_iter; ++it) {
    solve(false);
    if (a.resid != nullptr && it == a.n_iter - 1) {
      residual();
      // (keeps the residual's reads of the measurement apart from step 4's: shared, they cost
      // the loop 69 spilled VGPRs)
      asm volatile("" ::: "memory");
    }
    replace();
    if (a.flags & kFourierPeriodicEach) eq5();
  }

  if (a.flags & kFourierPeriodic) eq5();

  if (a.flags & kFourierExtend) {
    if (active) {
      const size_t gplane = (size_t)N * N;
      float *ea = a.out + (size_t)f * 2 * gplane;
#pragma unroll
      for (int k = 0; k < T; ++k) {
        const size_t idx = (size_t)line * N + 4 * k + j;
        ea[idx] = x[k].x;
        ea[gplane + idx] = x[k].y;
      }
    }
    return;
  }

  solve(true);
  if (active && line >= o && line <= o + n) {
    float *oa = a.out + (size_t)f * (n + 1) * (n + 1);
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const int nn = 4 * k + j;
      if (nn >= o && nn <= o + n) oa[(size_t)(line - o) * (n + 1) + (nn - o)] = x[k].x;
    }
  }
}

}  // namespace fourier

#define FWR_FOURIER_SIZES(X) X(8) X(16) X(24) X(32) X(40) X(48) X(64) X(80) X(128)

namespace {

template <int N, int FR>
int lds_of(int n) {
  return fourier::FGroup<N, FR>::lds_bytes(n);
}

// two frames per workgroup only where both tiles fit the LDS (not at N = 128)
template <int N>
constexpr bool two_frames_instantiated() {
  return 8 * N <= 1024 && fourier::FGroup<N, 2>::STATIC_LDS_BYTES <= 160 * 1024;
}

template <int N>
bool frames_ok_n(int n, int frames) {
  if (frames == 1) return lds_of<N, 1>(n) <= 160 * 1024;
  if constexpr (two_frames_instantiated<N>()) {
    if (frames == 2) return lds_of<N, 2>(n) <= 160 * 1024;
  }
  return false;
}

template <int N>
hipError_t prepare_n(int n, int frames) {
  if constexpr (two_frames_instantiated<N>()) {
    if (frames == 2)
      return raise_dynamic_lds(reinterpret_cast<const void *>(&fourier::fourier_kernel<N, 2>),
                               fourier::FGroup<N, 2>::dyn_bytes(n));
  }
  if (frames != 1) return hipErrorInvalidValue;
  return raise_dynamic_lds(reinterpret_cast<const void *>(&fourier::fourier_kernel<N, 1>),
                           fourier::FGroup<N, 1>::dyn_bytes(n));
}

template <int N>
hipError_t launch_n(const FourierArgs &a, hipStream_t s, int frames) {
  const int groups = (a.B + frames - 1) / frames;
  if constexpr (two_frames_instantiated<N>()) {
    if (frames == 2) {
      hipLaunchKernelGGL((fourier::fourier_kernel<N, 2>), dim3(groups), dim3(fourier::FGroup<N, 2>::THREADS),
                         size_t(fourier::FGroup<N, 2>::dyn_bytes(a.n)), s, a);
      return hipGetLastError();
    }
  }
  if (frames != 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((fourier::fourier_kernel<N, 1>), dim3(groups), dim3(fourier::FGroup<N, 1>::THREADS),
                     size_t(fourier::FGroup<N, 1>::dyn_bytes(a.n)), s, a);
  return hipGetLastError();
}

}  // namespace

bool fourier_supported(int N) {
  switch (N) {
#define FWR_CASE(NN) case NN: return true;
    FWR_FOURIER_SIZES(FWR_CASE)
#undef FWR_CASE
    default: return false;
  }
}

bool fourier_frames_ok(int N, int n, int frames) {
  switch (N) {
#define FWR_CASE(NN) case NN: return frames_ok_n<NN>(n, frames);
    FWR_FOURIER_SIZES(FWR_CASE)
#undef FWR_CASE
    default: return false;
  }
}

int fourier_threads(int N, int frames) { return 4 * N * frames; }

int fourier_lds_bytes(int N, int n, int frames) {
  switch (N) {
#define FWR_CASE(NN) case NN: return frames == 1 ? lds_of<NN, 1>(n) : frames_ok_n<NN>(n, frames) ? lds_of<NN, 2>(n) : 0;
    FWR_FOURIER_SIZES(FWR_CASE)
#undef FWR_CASE
    default: return 0;
  }
}

hipError_t fourier_prepare(int N, int n, int frames) {
  switch (N) {
#define FWR_CASE(NN) case NN: return prepare_n<NN>(n, frames);
    FWR_FOURIER_SIZES(FWR_CASE)
#undef FWR_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t fourier_launch(int N, const FourierArgs &a, hipStream_t s, int frames) {
  switch (N) {
#define FWR_CASE(NN) case NN: return launch_n<NN>(a, s, frames);
    FWR_FOURIER_SIZES(FWR_CASE)
#undef FWR_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fwr
