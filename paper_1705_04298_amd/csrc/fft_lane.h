// In-register mixed-radix DFTs and the cross-lane radix-4 stage used by the
// on-chip Gerchberg kernel (gfx950, wave64).
//
// A line of N = 4 * T complex points is held by a quad of lanes: lane j owns
// the points with index = j (mod 4), T of them, in registers.  A forward DFT
// of the line is (decimation in time over the lane digit):
//   1. an in-register DFT of length T over each lane's points,
//   2. multiplication by the twiddle W_N^(j k) (k = in-register frequency),
//   3. a 4-point DFT across the quad, done as two radix-2 stages on DPP
//      quad permutations (no LDS traffic).
// Afterwards lane j holds frequencies k + T * beta(j), beta = (0, 2, 1, 3).
// The inverse runs the same steps in reverse order with conjugate factors
// and no 1/N scaling (the caller folds normalisation into its filter).
//
// Twiddle constants of the in-register stages are compile-time values from a
// constexpr double-precision Taylor evaluation rounded to float.
#pragma once

#include <hip/hip_runtime.h>

#include <numeric>
#include <type_traits>
#include <utility>

namespace fwr {

// ------------------------------------------------------------------ constexpr trig
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int i = 1; i < 40; ++i) {
    term *= -x * x / double((2 * i - 1) * (2 * i));
    sum += term;
  }
  return sum;
}
constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int i = 1; i < 40; ++i) {
    term *= -x * x / double((2 * i) * (2 * i + 1));
    sum += term;
  }
  return sum;
}
// cos / sin of 2 pi e / L, argument reduced to [-pi, pi]
constexpr double cos2pi(long e, long L) {
  e %= L;
  if (e < 0) e += L;
  double x = 2.0 * kPi * double(e) / double(L);
  if (x > kPi) x -= 2.0 * kPi;
  return taylor_cos(x);
}
constexpr double sin2pi(long e, long L) {
  e %= L;
  if (e < 0) e += L;
  double x = 2.0 * kPi * double(e) / double(L);
  if (x > kPi) x -= 2.0 * kPi;
  return taylor_sin(x);
}

// ------------------------------------------------------------------ helpers
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i (DIR = -1) or +i (DIR = +1)
template <int DIR>
__device__ __forceinline__ float2 mul_i(float2 a) {
  if constexpr (DIR < 0) return make_float2(a.y, -a.x);
  else return make_float2(-a.y, a.x);
}
__device__ __forceinline__ float2 cmul(float2 a, float2 w) {
  return make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}
__device__ __forceinline__ float2 cmul_conj(float2 a, float2 w) {  // a * conj(w)
  return make_float2(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y);
}

// multiply by W_L^(DIR * E) = exp(DIR * 2 pi i E / L), E compile-time
template <int L, int DIR, int E>
__device__ __forceinline__ float2 twiddle(float2 a) {
  constexpr int e = ((E % L) + L) % L;
  if constexpr (e == 0) {
    return a;
  } else if constexpr (2 * e == L) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (4 * e == L) {
    return mul_i<DIR>(a);
  } else if constexpr (4 * e == 3 * L) {
    return mul_i<-DIR>(a);
  } else if constexpr (8 * e == L || 8 * e == 3 * L || 8 * e == 5 * L || 8 * e == 7 * L) {
    constexpr float r = 0.70710678118654752440f;
    constexpr float c = float(cos2pi(e, L)) > 0 ? r : -r;
    constexpr float s = float(DIR * sin2pi(e, L)) > 0 ? r : -r;
    // (a.x + i a.y)(c + i s) with |c| = |s| = r
    const float px = a.x * c, py = a.y * c;
    if constexpr ((c > 0) == (s > 0)) return make_float2(px - py, px + py);
    else return make_float2(px + py, py - px);
  } else {
    constexpr float c = float(cos2pi(e, L));
    constexpr float s = float(DIR * sin2pi(e, L));
    return make_float2(fmaf(a.x, c, -a.y * s), fmaf(a.x, s, a.y * c));
  }
}

// ------------------------------------------------------------------ butterflies
template <int DIR>
__device__ __forceinline__ void bfly2(float2 *x) {
  const float2 a = x[0], b = x[1];
  x[0] = cadd(a, b);
  x[1] = csub(a, b);
}

template <int DIR>
__device__ __forceinline__ void bfly3(float2 *x) {
  constexpr float h = 0.86602540378443864676f;  // sin(2 pi / 3)
  const float2 t = cadd(x[1], x[2]);
  const float2 dd = csub(x[1], x[2]);
  const float2 a = x[0];
  x[0] = cadd(a, t);
  const float2 m = make_float2(fmaf(-0.5f, t.x, a.x), fmaf(-0.5f, t.y, a.y));
  const float2 s = make_float2(h * dd.x, h * dd.y);
  // X1 = m + DIR * i * s, X2 = m - DIR * i * s
  x[1] = cadd(m, mul_i<DIR>(s));
  x[2] = csub(m, mul_i<DIR>(s));
}

template <int DIR>
__device__ __forceinline__ void bfly4(float2 *x) {
  const float2 a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
  const float2 c = cadd(x[1], x[3]), d = mul_i<DIR>(csub(x[1], x[3]));
  x[0] = cadd(a, c);
  x[2] = csub(a, c);
  x[1] = cadd(b, d);
  x[3] = csub(b, d);
}

template <int DIR>
__device__ __forceinline__ void bfly5(float2 *x) {
  constexpr float c1 = float(cos2pi(1, 5)), c2 = float(cos2pi(2, 5));
  constexpr float s1 = float(sin2pi(1, 5)), s2 = float(sin2pi(2, 5));
  const float2 x0 = x[0];
  const float2 t1 = cadd(x[1], x[4]), t2 = cadd(x[2], x[3]);
  const float2 t3 = csub(x[1], x[4]), t4 = csub(x[2], x[3]);
  x[0] = cadd(x0, cadd(t1, t2));
  const float2 a1 = make_float2(fmaf(c2, t2.x, fmaf(c1, t1.x, x0.x)), fmaf(c2, t2.y, fmaf(c1, t1.y, x0.y)));
  const float2 a2 = make_float2(fmaf(c1, t2.x, fmaf(c2, t1.x, x0.x)), fmaf(c1, t2.y, fmaf(c2, t1.y, x0.y)));
  const float2 b1 = make_float2(fmaf(s2, t4.x, s1 * t3.x), fmaf(s2, t4.y, s1 * t3.y));
  const float2 b2 = make_float2(fmaf(-s1, t4.x, s2 * t3.x), fmaf(-s1, t4.y, s2 * t3.y));
  // forward: X1 = a1 - i b1, X4 = a1 + i b1, X2 = a2 - i b2, X3 = a2 + i b2
  x[1] = cadd(a1, mul_i<DIR>(b1));
  x[4] = csub(a1, mul_i<DIR>(b1));
  x[2] = cadd(a2, mul_i<DIR>(b2));
  x[3] = csub(a2, mul_i<DIR>(b2));
}

// inverse of a modulo m (a, m coprime; m = 1 gives 0)
constexpr int modinv(int a, int m) {
  for (int x = 0; x < m; ++x)
    if ((a * x) % m == 1 % m) return x;
  return 0;
}

template <int L>
constexpr int first_radix() {
  if constexpr (L % 4 == 0) return 4;
  else if constexpr (L % 2 == 0) return 2;
  else if constexpr (L % 3 == 0) return 3;
  else return 5;
}

// radix taken first by the alternative schedule: the largest of 5, 3, 2 that divides L
template <int L>
constexpr int last_radix() {
  if constexpr (L % 5 == 0) return 5;
  else if constexpr (L % 3 == 0) return 3;
  else return 2;
}

// Natural-order in-place DFT of length L on x[0..L-1]:
//   X[k] = sum_n x[n] exp(DIR * 2 pi i n k / L), no scaling.
// Radix schedule SCHED 0: radix 4 (else 2, 3, 5) first, prime-factor (Good-Thomas, no
// twiddles) when the two factors are coprime; SCHED 1: Cooley-Tukey with twiddles at every
// level, radix 5 (else 3, else 2) first.  Both are exact DFTs; they round differently.
template <int L, int DIR, int SCHED = 0>
__device__ __forceinline__ void dft(float2 *x) {
  if constexpr (L == 1) {
  } else if constexpr (L == 2) {
    bfly2<DIR>(x);
  } else if constexpr (L == 3) {
    bfly3<DIR>(x);
  } else if constexpr (L == 4) {
    bfly4<DIR>(x);
  } else if constexpr (L == 5) {
    bfly5<DIR>(x);
  } else if constexpr (SCHED == 0 && std::gcd(first_radix<L>(), L / first_radix<L>()) == 1) {
    // coprime factors L = R M: prime-factor (Good-Thomas) algorithm, no twiddles.
    // Input n = (M n1 + R n2) mod L, output k = (M M' k1 + R R' k2) mod L with
    // M M' = 1 (mod R), R R' = 1 (mod M); then W_L^(n k) = W_R^(n1 k1) W_M^(n2 k2).
    constexpr int R = first_radix<L>();
    constexpr int M = L / R;
    constexpr int Mi = modinv(M % R, R), Ri = modinv(R % M, M);
    float2 s[R][M];
    static_for<0, R>([&](auto r) {
      static_for<0, M>([&](auto i) { s[r][i] = x[(M * decltype(r)::value + R * decltype(i)::value) % L]; });
      dft<M, DIR>(s[r]);
    });
    static_for<0, M>([&](auto k2) {
      float2 t[R];
      static_for<0, R>([&](auto r) { t[r] = s[r][k2]; });
      dft<R, DIR>(t);
      static_for<0, R>([&](auto k1) {
        x[(M * Mi * decltype(k1)::value + R * Ri * decltype(k2)::value) % L] = t[k1];
      });
    });
  } else {
    static_assert(L % 2 == 0 || L % 3 == 0 || L % 5 == 0, "radix 2/3/5 lengths only");
    constexpr int R = SCHED == 0 ? first_radix<L>() : last_radix<L>();
    constexpr int M = L / R;
    float2 s[R][M];
    static_for<0, R>([&](auto r) {
      static_for<0, M>([&](auto i) { s[r][i] = x[R * i + r]; });
      dft<M, DIR, SCHED>(s[r]);
    });
    static_for<1, R>([&](auto r) {
      static_for<1, M>([&](auto k) { s[r][k] = twiddle<L, DIR, decltype(r)::value * decltype(k)::value>(s[r][k]); });
    });
    static_for<0, M>([&](auto k) {
      float2 t[R];
      static_for<0, R>([&](auto r) { t[r] = s[r][k]; });
      dft<R, DIR, SCHED>(t);
      static_for<0, R>([&](auto q) { x[k + M * q] = t[q]; });
    });
  }
}

// ------------------------------------------------------------------ cross-lane radix-4
// DPP quad permutations: xor 1 = quad_perm(1,0,3,2), xor 2 = quad_perm(2,3,0,1).
__device__ __forceinline__ float dpp_xor1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_xor2(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
}

// Per-lane constants of the quad stage.
struct QuadLane {
  float sg1;   // +1 on lanes 0,1 ; -1 on lanes 2,3   (xor-2 stage)
  float sg0;   // +1 on lanes 0,2 ; -1 on lanes 1,3   (xor-1 stage)
  bool is3;
  __device__ explicit QuadLane(int j) : sg1((j & 2) ? -1.f : 1.f), sg0((j & 1) ? -1.f : 1.f), is3(j == 3) {}
};

// forward 4-point DFT across the quad; lane j ends with output index beta(j)
__device__ __forceinline__ float2 quad_dft_fwd(float2 v, const QuadLane &q) {
  float2 p = make_float2(dpp_xor2(v.x), dpp_xor2(v.y));
  v = make_float2(fmaf(q.sg1, v.x, p.x), fmaf(q.sg1, v.y, p.y));
  if (q.is3) v = make_float2(v.y, -v.x);  // * (-i)
  p = make_float2(dpp_xor1(v.x), dpp_xor1(v.y));
  return make_float2(fmaf(q.sg0, v.x, p.x), fmaf(q.sg0, v.y, p.y));
}
// inverse (unnormalised: returns 4x the lane's input-side value)
__device__ __forceinline__ float2 quad_dft_inv(float2 v, const QuadLane &q) {
  float2 p = make_float2(dpp_xor1(v.x), dpp_xor1(v.y));
  v = make_float2(fmaf(q.sg0, v.x, p.x), fmaf(q.sg0, v.y, p.y));
  if (q.is3) v = make_float2(-v.y, v.x);  // * (+i)
  p = make_float2(dpp_xor2(v.x), dpp_xor2(v.y));
  return make_float2(fmaf(q.sg1, v.x, p.x), fmaf(q.sg1, v.y, p.y));
}

// Signed quad DFTs: each radix-2 stage is one v_fmac_f32 per component with the partner
// lane's value as its DPP source, v += c * v(partner), c = the lane's stage sign (+-1).
// Since c^2 = 1 this is c times the standard stage output, so lane j ends with its
// standard result times S_j = (+1, -1, -1, +1)[j] (the product of its two stage signs;
// the lane-3 rotation between the stages is linear and carries the sign through).  The
// caller folds S_j into its next per-element operation.  The DPP source register must
// not have been written by a VALU instruction in the two preceding slots: the s_nop
// gives that distance, and the second instruction reads a register the first does not
// write.  A quad's four lanes are always active together.
__device__ __forceinline__ void stage_xor1(float2 &v, float c) {
  asm("s_nop 1\n\t"
      "v_fmac_f32_dpp %0, %0, %2 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %1, %1, %2 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf bound_ctrl:1"
      : "+v"(v.x), "+v"(v.y)
      : "v"(c));
}
__device__ __forceinline__ void stage_xor2(float2 &v, float c) {
  asm("s_nop 1\n\t"
      "v_fmac_f32_dpp %0, %0, %2 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %1, %1, %2 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1"
      : "+v"(v.x), "+v"(v.y)
      : "v"(c));
}
__device__ __forceinline__ float lane_sign(int j) { return (j == 1 || j == 2) ? -1.f : 1.f; }

__device__ __forceinline__ float2 quad_dft_fwd_s(float2 v, const QuadLane &q) {
  stage_xor2(v, q.sg1);
  if (q.is3) v = make_float2(v.y, -v.x);  // * (-i)
  stage_xor1(v, q.sg0);
  return v;
}
__device__ __forceinline__ float2 quad_dft_inv_s(float2 v, const QuadLane &q) {
  stage_xor1(v, q.sg0);
  if (q.is3) v = make_float2(-v.y, v.x);  // * (+i)
  stage_xor2(v, q.sg1);
  return v;
}

// Full line transforms.  tw[4 k + j] = W_N^(j k) = exp(-2 pi i j k / N), in LDS
// (the 16 quads of a wave read the same four entries: broadcast, no conflicts).
template <int T>
__device__ __forceinline__ void line_fft_fwd(float2 *x, const float2 *tw, int j, const QuadLane &q) {
  dft<T, -1>(x);
#pragma unroll
  for (int k = 1; k < T; ++k) x[k] = cmul(x[k], tw[4 * k + j]);
#pragma unroll
  for (int k = 0; k < T; ++k) x[k] = quad_dft_fwd(x[k], q);
}
template <int T>
__device__ __forceinline__ void line_fft_inv(float2 *x, const float2 *tw, int j, const QuadLane &q) {
#pragma unroll
  for (int k = 0; k < T; ++k) x[k] = quad_dft_inv(x[k], q);
#pragma unroll
  for (int k = 1; k < T; ++k) x[k] = cmul_conj(x[k], tw[4 * k + j]);
  dft<T, +1>(x);
}

// Signed line transforms (see quad_dft_fwd_s): the forward one returns lane j's values
// times S_j; the inverse one takes unsigned input and `twi[4 k + j]` = S_j conj(tw[4 k + j])
// (with `sj` = S_j for k = 0), so that its output is unsigned.
template <int T, int SCHED = 0>
__device__ __forceinline__ void line_fft_fwd_s(float2 *x, const float2 *tw, int j, const QuadLane &q) {
  dft<T, -1, SCHED>(x);
#pragma unroll
  for (int k = 1; k < T; ++k) x[k] = cmul(x[k], tw[4 * k + j]);
#pragma unroll
  for (int k = 0; k < T; ++k) x[k] = quad_dft_fwd_s(x[k], q);
}
template <int T, int SCHED = 0>
__device__ __forceinline__ void line_fft_inv_s(float2 *x, const float2 *twi, int j, float sj, const QuadLane &q) {
#pragma unroll
  for (int k = 0; k < T; ++k) x[k] = quad_dft_inv_s(x[k], q);
  x[0] = make_float2(sj * x[0].x, sj * x[0].y);
#pragma unroll
  for (int k = 1; k < T; ++k) x[k] = cmul(x[k], twi[4 * k + j]);
  dft<T, +1, SCHED>(x);
}

}  // namespace fwr
