// Device-side synthetic frames: von Karman phase screens on the padded N x N
// grid (periodic, pitch d), Fried slopes on the (n+1) x (n+1) node window of the
// lenslet array, white slope noise, valid subapertures only.
//
// One workgroup makes two frames: complex white Gaussian noise shaped by
// sqrt(Phi_vK(kappa)) dkappa is inverse-transformed once; the real and the
// imaginary parts are two independent screens.  Random numbers come from the
// counter-based Philox4x32-10 generator (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC 2011) keyed by the seed, with the
// counter (frame pair, position, stream), then Box-Muller.  Frames therefore
// depend only on (seed, frame index), not on the batch they are made in.
//
// The FFT reuses the on-chip line transforms (4 lanes per line, see
// fft_lane.h); the spectrum is generated directly in the transform's
// digit-reversed position order.
#include "fft_lane.h"
#include "gen.h"

#include <cstdint>

namespace fwr {
namespace gen {

// ------------------------------------------------------------------ Philox4x32-10
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = uint64_t(0xD2511F53u) * c.x;
    const uint64_t p1 = uint64_t(0xCD9E8D57u) * c.z;
    const uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0);
    const uint32_t hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// two standard normals from two uint32 (Box-Muller on (0, 1] uniforms)
__device__ __forceinline__ float2 box_muller(uint32_t a, uint32_t b) {
  const float u1 = (float(a >> 8) + 1.0f) * (1.0f / 16777216.0f);  // (0, 1]
  const float u2 = float(b >> 8) * (1.0f / 16777216.0f);           // [0, 1)
  const float r = sqrtf(-2.0f * logf(u1));
  float s, c;
  sincospif(2.0f * u2, &s, &c);
  return make_float2(r * c, r * s);
}

__device__ __forceinline__ float vk_amp(int l, int k, int N, const GenArgs &a) {
  // sqrt(Phi_vK(kappa)) dkappa with kappa = (k', l') / (N d), signed indices; 0 at the piston
  if (l == 0 && k == 0) return 0.f;
  const int ks = k < (N + 1) / 2 ? k : k - N, ls = l < (N + 1) / 2 ? l : l - N;
  const float dk = 1.0f / (float(N) * a.d);
  const float kap2 = (float(ks) * ks + float(ls) * ls) * dk * dk;
  const float psd = a.vk_const * powf(a.r0, -5.0f / 3.0f) * powf(kap2 + 1.0f / (a.L0 * a.L0), -11.0f / 6.0f);
  return sqrtf(psd) * dk;
}

template <int N>
__global__ __launch_bounds__(4 * N) void gen_onchip_kernel(GenArgs a) {
  constexpr int T = N / 4, THREADS = 4 * N, P = N + 1;
  __shared__ float2 buf[N * P];
  __shared__ float2 tw[T * 4];
  const int t = threadIdx.x, line = t >> 2, j = t & 3;
  const QuadLane q(j);
  const uint64_t pair = a.first_pair + blockIdx.x + (a.d_counter ? *a.d_counter / 2 : 0);
  const int fa = 2 * blockIdx.x;
  const bool hasB = fa + 1 < a.B;
  for (int i = t; i < T * 4; i += THREADS) {
    const int k2 = i >> 2, jj = i & 3;
    // W_N^(jj k2) from the constexpr-free device sincospi (twiddles of a generator need not be exact)
    float s, c;
    sincospif(-2.0f * float(jj * k2) / float(N), &s, &c);
    tw[i] = make_float2(c, s);
  }
  __syncthreads();
  const int beta[4] = {0, 2, 1, 3};
  // column-phase layout: thread (column position c = line, lane j) holds the column-frequency
  // positions l = k + T beta(j); column position c holds row frequency (c % T) + T beta(c / T)
  const int kf = (line % T) + T * beta[line / T];
  float2 y[T];
#pragma unroll
  for (int k = 0; k < T; ++k) {
    const int lf = k + T * beta[j];
    const U4 r = philox4x32_10(U4{uint32_t(pair), uint32_t(pair >> 32), uint32_t(lf * N + kf), 0u}, a.seed_lo,
                               a.seed_hi);
    const float2 g = box_muller(r.x, r.y);
    const float amp = vk_amp(lf, kf, N, a);
    y[k] = make_float2(g.x * amp, g.y * amp);
  }
  // inverse column transforms, transpose, inverse row transforms (unnormalised = plain sum)
  line_fft_inv<T>(y, tw, j, q);
#pragma unroll
  for (int k = 0; k < T; ++k) buf[(4 * k + j) * P + line] = y[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < T; ++k) y[k] = buf[line * P + T * j + k];
  line_fft_inv<T>(y, tw, j, q);
  __syncthreads();
  // phase in natural layout
#pragma unroll
  for (int k = 0; k < T; ++k) buf[line * P + 4 * k + j] = y[k];
  __syncthreads();
  // slopes on the lenslet window (grid cells [o, o+n)), phase on its nodes
  const int n = a.n, o = a.o, plane = n * n;
  float *sa = a.slopes + (size_t)fa * 2 * plane;
  for (int idx = t; idx < plane; idx += THREADS) {
    const int i = idx / n, jj = idx - i * n;
    const int m = o + i, c = o + jj;
    const float2 p00 = buf[m * P + c], p01 = buf[m * P + c + 1];
    const float2 p10 = buf[(m + 1) * P + c], p11 = buf[(m + 1) * P + c + 1];
    const float2 sx = make_float2(0.5f * ((p01.x - p00.x) + (p11.x - p10.x)), 0.5f * ((p01.y - p00.y) + (p11.y - p10.y)));
    const float2 sy = make_float2(0.5f * ((p10.x - p00.x) + (p11.x - p01.x)), 0.5f * ((p10.y - p00.y) + (p11.y - p01.y)));
    const U4 r = philox4x32_10(U4{uint32_t(pair), uint32_t(pair >> 32), uint32_t(idx), 1u}, a.seed_lo, a.seed_hi);
    const float2 na = box_muller(r.x, r.y), nb = box_muller(r.z, r.w);
    const float valid = a.mask[idx] ? 1.f : 0.f;
    sa[idx] = valid * (sx.x + a.sigma * na.x);
    sa[plane + idx] = valid * (sy.x + a.sigma * na.y);
    if (hasB) {
      sa[2 * plane + idx] = valid * (sx.y + a.sigma * nb.x);
      sa[3 * plane + idx] = valid * (sy.y + a.sigma * nb.y);
    }
  }
  if (a.phase) {
    const int n1 = n + 1;
    float *pa = a.phase + (size_t)fa * n1 * n1;
    for (int idx = t; idx < n1 * n1; idx += THREADS) {
      const int i = idx / n1, jj = idx - i * n1;
      const float2 v = buf[(o + i) * P + o + jj];
      pa[idx] = v.x;
      if (hasB) pa[(size_t)n1 * n1 + idx] = v.y;
    }
  }
}

__global__ void counter_add_kernel(uint64_t *c, uint64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c += v;
}

// Fried slopes of node phases (Sec. 2; the model the reconstruction inverts), one frame per
// blockIdx.y, cells in grid-stride order: s_x = (phi(m, n+1) - phi(m, n) + phi(m+1, n+1) -
// phi(m+1, n)) / 2, s_y with rows and columns exchanged; plus the noise; zero outside the pupil.
__global__ __launch_bounds__(256) void fried_slopes_kernel(const float *phase, const float *noise,
                                                           const uint8_t *mask, float *slopes, int n) {
  const int f = blockIdx.y, n1 = n + 1, plane = n * n;
  const float *p = phase + (size_t)f * n1 * n1;
  float *sa = slopes + (size_t)f * 2 * plane;
  const float *na = noise ? noise + (size_t)f * 2 * plane : nullptr;
  for (int idx = blockIdx.x * 256 + threadIdx.x; idx < plane; idx += gridDim.x * 256) {
    const int i = idx / n, c = idx - i * n;
    const float a = p[i * n1 + c], b = p[i * n1 + c + 1], cc = p[(i + 1) * n1 + c], e = p[(i + 1) * n1 + c + 1];
    float sx = 0.5f * ((b - a) + (e - cc)), sy = 0.5f * ((cc - a) + (e - b));
    if (na) {
      sx += na[idx];
      sy += na[plane + idx];
    }
    const bool v = mask[idx] != 0;
    sa[idx] = v ? sx : 0.f;
    sa[plane + idx] = v ? sy : 0.f;
  }
}

}  // namespace gen

hipError_t fried_slopes_launch(const float *phase, const float *noise, const uint8_t *mask, float *slopes, int B,
                               int n, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  const int blocks = (n * n + 255) / 256;
  hipLaunchKernelGGL(gen::fried_slopes_kernel, dim3(blocks < 64 ? blocks : 64, B), dim3(256), 0, s, phase, noise,
                     mask, slopes, n);
  return hipGetLastError();
}

#define FWR_GEN_SIZES(X) X(8) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(80) X(128)

bool gen_supported(int N) {
  switch (N) {
#define FWR_CASE(NN) case NN: return true;
    FWR_GEN_SIZES(FWR_CASE)
#undef FWR_CASE
    default: return false;
  }
}

hipError_t gen_launch(int N, const GenArgs &a, hipStream_t s) {
  const int groups = (a.B + 1) / 2;
  switch (N) {
#define FWR_CASE(NN) \
  case NN: hipLaunchKernelGGL(gen::gen_onchip_kernel<NN>, dim3(groups), dim3(4 * NN), 0, s, a); break;
    FWR_GEN_SIZES(FWR_CASE)
#undef FWR_CASE
    default: return hipErrorInvalidValue;
  }
  if (a.d_counter) hipLaunchKernelGGL(gen::counter_add_kernel, dim3(1), dim3(64), 0, s, a.d_counter, uint64_t(2 * groups));
  return hipGetLastError();
}

}  // namespace fwr
