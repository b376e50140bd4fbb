// C ABI of libfwr: plan construction (double-precision tables, rounded to
// float once), argument validation and asynchronous launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/fwr.h"
#include <complex>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "fourier.h"
#include "fourier_mp.h"
#include "gen.h"
#include "hudgin.h"
#include "learned.h"
#include "multipass.h"
#include "onchip.h"


namespace {

constexpr uint32_t kMagic = 0x46575231u;  // "FWR1"
constexpr double kPi = 3.14159265358979323846264338327950288;

// Von Karman PSD prefactor [24/5 Gamma(6/5)]^(5/6) Gamma(11/6)^2 / (2 pi^(11/3)).
double vk_constant() {
  return std::pow(24.0 / 5.0 * std::tgamma(6.0 / 5.0), 5.0 / 6.0) * std::pow(std::tgamma(11.0 / 6.0), 2.0) /
         (2.0 * std::pow(kPi, 11.0 / 3.0));
}

}  // namespace

struct fwr_plan_s {
  uint32_t magic = 0;
  int device = 0;
  int n = 0, N = 0, o = 0, n_iter = 0, flags = 0, max_batch = 0;
  hipStream_t stream = nullptr;
  void *d_mem = nullptr;
  const float *h_loop = nullptr;
  const float *h_final = nullptr;
  const float2 *tw_lane = nullptr;
  const uint32_t *codes = nullptr;
  int pairs = 1;  // frame pairs per workgroup of the on-chip kernel
  int sched = 0;  // radix schedule of its in-lane DFTs (windowed kernel of 2x-padded plans)
  // Fourier-domain path (slope models without a compact stencil)
  bool fourier = false;
  fwr::FourierArgs fa{};
  bool fourier_mp = false;  // the Fourier-domain path through HBM (N = 256)
  fwr::FSArgs fs{};
  int frames = 1;  // frames per workgroup of the Fourier-domain kernel
  // multi-pass path (N = 256)
  bool multipass = false;
  fwr::MPArgs mp{};
  const uint8_t *dmask = nullptr;  // [n][n] valid subapertures on the device (generator)
  const int32_t *hudgin_src = nullptr;  // [2][N][N] source cells of the Hudgin extension (on-chip plans)
  double d = 0.0;                  // lenslet pitch [m]
  // gather buffers when the plan serves as the fallback of fwr_reconstruct_learned (first use)
  void *fb_mem = nullptr;
  int32_t *fb_idx = nullptr, *fb_count = nullptr;
  float *fb_slopes = nullptr, *fb_phase = nullptr;
};

namespace {

bool valid(fwr_plan_t p) { return p != nullptr && p->magic == kMagic; }

// frame pairs per workgroup that the on-chip kernel is built for
constexpr int kPairsOptions[] = {1, 2, 4, 8};

// Autotuned choices, per device and problem shape (process-wide).
struct TuneKey {
  int device, N, n, n_iter;
  bool each;
  int model;
  bool operator<(const TuneKey &o) const {
    return std::tie(device, N, n, n_iter, each, model) < std::tie(o.device, o.N, o.n, o.n_iter, o.each, o.model);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tuned;

// stored value: launch unit (frame pairs, or frames for the Fourier-domain kernel) + 16 x schedule
void remember_pairs(int device, int N, int n, int n_iter, bool each, int pairs, int model = FWR_MODEL_FRIED,
                    int sched = 0) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tuned[TuneKey{device, N, n, n_iter, each, model}] = pairs + 16 * sched;
}

int tuned_value(int device, int N, int n, int n_iter, bool each, int model) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tuned.find(TuneKey{device, N, n, n_iter, each, model});
  return it == g_tuned.end() ? 0 : it->second;
}

// The tuned choice when there is one.  Otherwise: two pairs when one pair's waves
// number 4k + 1 (k >= 1), where a lone workgroup leaves one SIMD with twice the waves
// of the others and every phase waits for it (N = 80: 5 waves; two pairs make
// 3, 3, 2, 2); one pair elsewhere, where larger groups measured slower (they lower the
// register budget per wave).
int tuned_pairs(int device, int N, int n, int n_iter, bool each) {
  if (const int v = tuned_value(device, N, n, n_iter, each, FWR_MODEL_FRIED)) return v % 16;
  const int waves = (fwr::onchip_threads(N, 1) + 63) / 64;
  if (waves > 4 && waves % 4 == 1 && fwr::onchip_pairs_ok(N, n, 2, each)) return 2;
  return 1;
}

// Squared Fried transfer function |G_x|^2 + |G_y|^2 = 4 (u^2 + v^2),
// u = sin(pi k/N) cos(pi l/N), v = sin(pi l/N) cos(pi k/N).
double fried_g2(int l, int k, int N) {
  const double sk = std::sin(kPi * k / N), ck = std::cos(kPi * k / N);
  const double sl = std::sin(kPi * l / N), cl = std::cos(kPi * l / N);
  const double u = sk * cl, v = sl * ck;
  return 4.0 * (u * u + v * v);
}

bool singular(int l, int k, int N) {
  return (l == 0 && k == 0) || (N % 2 == 0 && l == N / 2 && k == N / 2);
}

// gamma * W_eta / W_phi at DFT index (l, k): sigma^2 d^2 / Phi_vK(kappa), kappa = (k', l') / (N d)
double regulariser(const fwr_params &p, int l, int k) {
  const int N = p.n_grid;
  if (p.alpha_map) return p.alpha_map[(size_t)l * N + k];
  if (p.gamma == 0.0) return 0.0;
  const int ks = k < (N + 1) / 2 ? k : k - N;
  const int ls = l < (N + 1) / 2 ? l : l - N;
  const double kap2 = (double(ks) * ks + double(ls) * ls) / (double(N) * N * p.d * p.d);
  const double phi = vk_constant() * std::pow(p.r0, -5.0 / 3.0) * std::pow(kap2 + 1.0 / (p.L0 * p.L0), -11.0 / 6.0);
  return p.gamma * p.noise_var * p.d * p.d / phi;
}

// 1 / (2 |G|^2 N^2) (loop) and 1 / (2 (|G|^2 + gamma W_eta/W_phi) N^2) (final), 0 on the singular set
void filter_values(const fwr_params &p, int l, int k, double &hl, double &hf) {
  const int N = p.n_grid;
  const double norm = 1.0 / (2.0 * double(N) * double(N));
  hl = hf = 0.0;
  if (singular(l, k, N)) return;
  const double g2 = fried_g2(l, k, N);
  hl = norm / g2;
  const double den = g2 + regulariser(p, l, k);
  hf = den > 0.0 ? norm / den : 0.0;
}

// Hudgin extension (Sec. 3.2): the source cell of every grid cell, x slopes from the nearest
// in-pupil cell of the column, y slopes from the nearest of the row (upper / left on a tie),
// -1 where the line has none; [2][N][N]
std::vector<int32_t> hudgin_sources(const fwr_params &p) {
  const int n = p.n_sub, N = p.n_grid, o = (N - n) / 2;
  auto in_pupil = [&](int cm, int cn) {
    const int i = cm - o, jj = cn - o;
    return i >= 0 && i < n && jj >= 0 && jj < n && p.mask[(size_t)i * n + jj] != 0;
  };
  std::vector<int32_t> hsrc(2 * (size_t)N * N, -1);
  for (int m = 0; m < N; ++m)
    for (int c = 0; c < N; ++c) {
      int best = -1, bd = N + 1;
      for (int r = 0; r < N; ++r)
        if (in_pupil(r, c) && std::abs(r - m) < bd) {
          bd = std::abs(r - m);
          best = (r - o) * n + (c - o);
        }
      hsrc[(size_t)m * N + c] = best;
      best = -1;
      bd = N + 1;
      for (int q = 0; q < N; ++q)
        if (in_pupil(m, q) && std::abs(q - c) < bd) {
          bd = std::abs(q - c);
          best = (m - o) * n + (q - o);
        }
      hsrc[(size_t)N * N + (size_t)m * N + c] = best;
    }
  return hsrc;
}

fwr_status plan_multipass(const fwr_params &p, fwr_plan_t *out);
fwr_status plan_fourier(const fwr_params &p, fwr_plan_t *out);

}  // namespace

extern "C" {

const char *fwr_status_string(int32_t s) {
  switch (s) {
    case FWR_OK: return "ok";
    case FWR_E_INVAL: return "invalid argument";
    case FWR_E_UNSUPPORTED: return "unsupported configuration";
    case FWR_E_NOMEM: return "device allocation failed";
    case FWR_E_DEVICE: return "HIP runtime error";
    case FWR_E_STATE: return "invalid plan handle";
    default: return "unknown status";
  }
}

fwr_status fwr_plan(const fwr_params *params, fwr_plan_t *out) {
  if (out == nullptr) return FWR_E_INVAL;
  *out = nullptr;
  if (params == nullptr) return FWR_E_INVAL;
  const fwr_params &p = *params;
  const int n = p.n_sub, N = p.n_grid;
  if (n < 1 || N <= n || (N - n) % 2 != 0 || p.mask == nullptr) return FWR_E_INVAL;
  if (p.n_iter < 0 || p.n_iter > 10000 || p.max_batch < 1) return FWR_E_INVAL;
  if (N > 256) return FWR_E_UNSUPPORTED;
  if (p.alpha_map != nullptr) {
    // W_eta / W_phi of real processes: finite, >= 0 and even, alpha(-l, -k) = alpha(l, k); the
    // kernels' Fourier operators must be real and even (two frames share a complex field)
    for (int l = 0; l < N; ++l)
      for (int k = 0; k < N; ++k) {
        const double a = p.alpha_map[(size_t)l * N + k];
        if (!(a >= 0.0) || !std::isfinite(a) || a != p.alpha_map[(size_t)((N - l) % N) * N + (N - k) % N])
          return FWR_E_INVAL;
      }
  }
  // pixel-size correction of the lenslet-averaging model: 0 <= d_px < d (sinc model only)
  if (!(p.d_px >= 0.0) || !std::isfinite(p.d_px)) return FWR_E_INVAL;
  if (p.d_px > 0.0) {
    if (p.model != FWR_MODEL_SINC) return FWR_E_UNSUPPORTED;
    if (!(p.d > 0.0) || !(p.d_px < p.d)) return FWR_E_INVAL;
  }
  // the physical parameters of Eq. 3 feed the final filter of both slope models
  if (p.alpha_map == nullptr && p.gamma != 0.0) {
    if (!(p.gamma > 0.0) || !(p.noise_var >= 0.0) || !(p.r0 > 0.0) || !(p.L0 > 0.0) || !(p.d > 0.0))
      return FWR_E_INVAL;
  }
  if (p.model == FWR_MODEL_SINC) return plan_fourier(p, out);
  if (p.model != FWR_MODEL_FRIED) return FWR_E_UNSUPPORTED;
  if (fwr::multipass_supported(N)) return plan_multipass(p, out);
  if (!fwr::onchip_supported(N)) return FWR_E_UNSUPPORTED;

  const int T = N / 4, threads = fwr::onchip_threads(N, 1);
  static const int beta[4] = {0, 2, 1, 3};

  // host tables; the filters carry the lane signs the kernel's signed quad transforms
  // leave on the spectrum: S_(c / T) of the row pass that wrote LDS column c and S_jj of
  // the column pass, S = (+1, -1, -1, +1)
  static const double lane_s[4] = {1.0, -1.0, -1.0, 1.0};
  std::vector<float> h_loop((size_t)T * threads), h_final((size_t)T * threads);
  for (int c = 0; c < N; ++c) {
    const int kf = (c % T) + T * beta[c / T];  // row frequency held in LDS column c
    for (int jj = 0; jj < 4; ++jj) {
      const int tt = 4 * c + jj;
      const double sg = lane_s[c / T] * lane_s[jj];
      for (int k2 = 0; k2 < T; ++k2) {
        const int lf = k2 + T * beta[jj];      // column frequency of this output
        double hl, hf;
        filter_values(p, lf, kf, hl, hf);
        h_loop[(size_t)tt * T + k2] = float(sg * hl);
        h_final[(size_t)tt * T + k2] = float(sg * hf);
      }
    }
  }
  std::vector<float2> tw((size_t)T * 4);
  for (int k2 = 0; k2 < T; ++k2)
    for (int jj = 0; jj < 4; ++jj) {
      const double ang = -2.0 * kPi * double(jj) * double(k2) / double(N);
      tw[(size_t)k2 * 4 + jj] = make_float2(float(std::cos(ang)), float(std::sin(ang)));
    }
  // per-thread node codes: 4 bits per node (m, 4k + j) of thread t = 4m + j; a set bit marks an
  // adjacent cell outside the pupil: bit 0 (m, n), bit 1 (m-1, n-1), bit 2 (m, n-1), bit 3 (m-1, n)
  const int o = (N - n) / 2;
  auto in_pupil = [&](int cm, int cn) {
    cm = (cm + N) % N;
    cn = (cn + N) % N;
    const int i = cm - o, jj = cn - o;
    return i >= 0 && i < n && jj >= 0 && jj < n && p.mask[(size_t)i * n + jj] != 0;
  };
  const int words = (T + 7) / 8;
  std::vector<uint32_t> codes((size_t)words * threads, 0u);
  for (int m = 0; m < N; ++m)
    for (int jj = 0; jj < 4; ++jj)
      for (int k = 0; k < T; ++k) {
        const int nn = 4 * k + jj;
        const uint32_t c = (in_pupil(m, nn) ? 0u : 1u) | (in_pupil(m - 1, nn - 1) ? 0u : 2u) |
                           (in_pupil(m, nn - 1) ? 0u : 4u) | (in_pupil(m - 1, nn) ? 0u : 8u);
        codes[(size_t)(k / 8) * threads + 4 * m + jj] |= c << (4 * (k % 8));
      }

  const bool each = p.periodic_each_iter != 0;
  if (!fwr::onchip_pairs_ok(N, n, 1, each)) return FWR_E_UNSUPPORTED;
  auto *plan = new (std::nothrow) fwr_plan_s();
  if (plan == nullptr) return FWR_E_NOMEM;
  bool prepared = hipGetDevice(&plan->device) == hipSuccess;
  for (int pairs : kPairsOptions)
    if (prepared && fwr::onchip_pairs_ok(N, n, pairs, each))
      prepared = fwr::onchip_prepare(N, n, pairs) == hipSuccess;
  if (!prepared) {
    delete plan;
    return FWR_E_DEVICE;
  }
  plan->pairs = tuned_pairs(plan->device, N, n, p.n_iter, each);
  plan->sched = tuned_value(plan->device, N, n, p.n_iter, each, FWR_MODEL_FRIED) / 16;
  const size_t b_h = h_loop.size() * sizeof(float);
  const size_t b_tw = tw.size() * sizeof(float2);
  const size_t off_hf = b_h, off_tw = 2 * b_h, off_codes = 2 * b_h + b_tw;
  const size_t off_dmask = off_codes + codes.size() * sizeof(uint32_t);
  const std::vector<int32_t> hsrc = hudgin_sources(p);
  const size_t off_hudgin = (off_dmask + (size_t)n * n + 15) & ~size_t(15);
  const size_t total = off_hudgin + hsrc.size() * sizeof(int32_t);
  std::vector<uint8_t> dmask((size_t)n * n);
  for (size_t i = 0; i < dmask.size(); ++i) dmask[i] = p.mask[i] ? 1 : 0;
  char *mem = nullptr;
  if (hipMalloc(reinterpret_cast<void **>(&mem), total) != hipSuccess) {
    delete plan;
    return FWR_E_NOMEM;
  }
  hipError_t e = hipMemcpy(mem, h_loop.data(), b_h, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_hf, h_final.data(), b_h, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_tw, tw.data(), b_tw, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(mem + off_codes, codes.data(), codes.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_dmask, dmask.data(), dmask.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_hudgin, hsrc.data(), hsrc.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = fwr::hudgin_prepare(N);
  if (e != hipSuccess) {
    (void)hipFree(mem);
    delete plan;
    return FWR_E_DEVICE;
  }
  plan->magic = kMagic;
  plan->n = n;
  plan->N = N;
  plan->o = o;
  plan->n_iter = p.n_iter;
  plan->flags = (p.periodic ? fwr::kFlagPeriodic : 0) | (p.periodic_each_iter ? fwr::kFlagPeriodicEach : 0);
  plan->max_batch = p.max_batch;
  plan->stream = static_cast<hipStream_t>(p.stream);
  plan->d_mem = mem;
  plan->h_loop = reinterpret_cast<const float *>(mem);
  plan->h_final = reinterpret_cast<const float *>(mem + off_hf);
  plan->tw_lane = reinterpret_cast<const float2 *>(mem + off_tw);
  plan->codes = reinterpret_cast<const uint32_t *>(mem + off_codes);
  plan->dmask = reinterpret_cast<const uint8_t *>(mem + off_dmask);
  plan->hudgin_src = reinterpret_cast<const int32_t *>(mem + off_hudgin);
  plan->d = p.d;
  *out = plan;
  return FWR_OK;
}

// Argument checks of one extension / reconstruction call (no device work).
static fwr_status check_args(fwr_plan_t plan, const float *in, const float *out, int32_t B, bool extend,
                             const float *start, const float *resid) {
  if (!valid(plan)) return FWR_E_STATE;
  if (B < 0 || B > plan->max_batch) return FWR_E_INVAL;
  if (B == 0) return FWR_OK;
  if (in == nullptr || out == nullptr) return FWR_E_INVAL;
  if ((start != nullptr || resid != nullptr) && (plan->multipass || plan->fourier_mp)) return FWR_E_UNSUPPORTED;
  // with no iteration the start is the extension itself: Eq. 2/3 of (measurement inside, start
  // outside); the extended-slope output, Eq. 5 and the residual need iterations
  if (start != nullptr && plan->n_iter == 0 && (extend || resid != nullptr || (plan->flags & fwr::kFlagPeriodic)))
    return FWR_E_INVAL;
  return FWR_OK;
}

// `count` (device int32, on-chip plans only): the launch covers B frames of which the first
// min(B, *count - count_off) are processed (see OnchipArgs).
static fwr_status run(fwr_plan_t plan, const float *in, float *out, int32_t B, bool extend,
                      const float *start = nullptr, float *resid = nullptr, hipStream_t stream = nullptr,
                      bool use_stream = false, const int32_t *count = nullptr, int count_off = 0,
                      bool beside_others = false) {
  if (const fwr_status c = check_args(plan, in, out, B, extend, start, resid); c != FWR_OK) return c;
  if (B == 0) return FWR_OK;
  const hipStream_t st = use_stream ? stream : plan->stream;
  if (count != nullptr && (plan->fourier || plan->multipass)) return FWR_E_UNSUPPORTED;
  if (plan->fourier_mp) {
    fwr::FSArgs a = plan->fs;
    a.slopes = in;
    a.out = out;
    a.B = B;
    a.flags = ((plan->flags & fwr::kFlagPeriodic) ? fwr::kFourierPeriodic : 0) |
              ((plan->flags & fwr::kFlagPeriodicEach) ? fwr::kFourierPeriodicEach : 0);
    a.shape = beside_others ? 0 : plan->sched;  // (as on the Fried multi-pass path below)
    return fwr::fourier_mp_run(a, extend, st) == hipSuccess ? FWR_OK : FWR_E_DEVICE;
  }
  if (plan->fourier) {
    fwr::FourierArgs a = plan->fa;
    a.slopes = in;
    a.out = out;
    a.start = start;
    a.resid = resid;
    a.B = B;
    a.flags = ((plan->flags & fwr::kFlagPeriodic) ? fwr::kFourierPeriodic : 0) |
              ((plan->flags & fwr::kFlagPeriodicEach) ? fwr::kFourierPeriodicEach : 0) |
              (extend ? fwr::kFourierExtend : 0);
    return fwr::fourier_launch(plan->N, a, st, plan->frames) == hipSuccess ? FWR_OK : FWR_E_DEVICE;
  }
  if (plan->multipass) {
    fwr::MPArgs a = plan->mp;
    a.slopes = in;
    a.out = out;
    a.B = B;
    // beside other items of a grouped call the loop runs one launch per pass: the persistent
    // loop's resident workgroups wait in place and hold CUs that the concurrent items need
    // (measured on the mixed step: 1.050 ms per step against 1.089 ms)
    a.col_shape = beside_others && plan->sched == 2 ? 0 : plan->sched;
    return fwr::multipass_run(a, extend, st) == hipSuccess ? FWR_OK : FWR_E_DEVICE;
  }
  fwr::OnchipArgs a;
  a.slopes = in;
  a.out = out;
  a.h_loop = plan->h_loop;
  a.h_final = plan->h_final;
  a.tw_lane = plan->tw_lane;
  a.codes = plan->codes;
  a.mask = plan->dmask;
  a.B = B;
  a.n = plan->n;
  a.o = plan->o;
  a.n_iter = plan->n_iter;
  a.flags = plan->flags | (extend ? fwr::kFlagExtend : 0);
  a.start = start;
  a.resid = resid;
  a.count = count;
  a.count_off = count_off;
  return fwr::onchip_launch(plan->N, a, st, plan->pairs, plan->sched) == hipSuccess ? FWR_OK : FWR_E_DEVICE;
}

fwr_status fwr_extend(fwr_plan_t plan, const float *d_slopes, float *d_ext, int32_t B) {
  return run(plan, d_slopes, d_ext, B, true);
}

fwr_status fwr_reconstruct(fwr_plan_t plan, const float *d_slopes, float *d_phase, int32_t B) {
  return run(plan, d_slopes, d_phase, B, false);
}

fwr_status fwr_extend_start(fwr_plan_t plan, const float *d_slopes, const float *d_start, float *d_ext,
                            float *d_resid, int32_t B) {
  return run(plan, d_slopes, d_ext, B, true, d_start, d_resid);
}

fwr_status fwr_reconstruct_start(fwr_plan_t plan, const float *d_slopes, const float *d_start, float *d_phase,
                                 float *d_resid, int32_t B) {
  return run(plan, d_slopes, d_phase, B, false, d_start, d_resid);
}

fwr_status fwr_reconstruct_group(const fwr_work *work, int32_t n_work, void *stream) {
  static std::mutex mu;
  static std::vector<hipStream_t> pool;
  static std::vector<hipEvent_t> evs;
  if (n_work < 0 || (n_work > 0 && work == nullptr)) return FWR_E_INVAL;
  // every item is checked before anything is enqueued
  for (int i = 0; i < n_work; ++i) {
    const fwr_work &w = work[i];
    if (!valid(w.plan)) return FWR_E_STATE;
    for (int k = 0; k < i; ++k)
      if (work[k].plan == w.plan) return FWR_E_INVAL;  // a plan's workspace serves one item
    if (const fwr_status c = check_args(w.plan, w.d_slopes, w.d_phase, w.B, false, w.d_start, w.d_resid);
        c != FWR_OK)
      return c;
  }
  if (n_work == 0) return FWR_OK;
  std::lock_guard<std::mutex> lock(mu);
  const hipStream_t main = static_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(main, &cap) != hipSuccess) return FWR_E_DEVICE;
  // One item runs on the caller's stream, the others on library streams forked from it.  HIP gives
  // a process a few hardware queues (4 by default) and binds each stream to one of them; streams
  // that share a queue run one after the other.  n - 1 library streams beside
  // the caller's leave n = 4 items on four queues where the process holds no other streams; where
  // it does, the queue least likely to be shared is the caller's (often the first stream bound),
  // so the caller's stream takes the item with the longest chain of launches (the first multi-pass
  // plan, else the first item), enqueued after the others so their single launches start first.
  // The streams and events are made outside any capture (at least 8 on the first call).
  const int need = n_work - 1;
  const int want = need > 8 ? need : 8;
  if ((int)pool.size() < need && cap != hipStreamCaptureStatusNone) return FWR_E_UNSUPPORTED;
  while ((int)pool.size() < want) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return FWR_E_DEVICE;
    pool.push_back(s);
  }
  while ((int)evs.size() < want + 1) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return FWR_E_DEVICE;
    evs.push_back(e);
  }
  int lead = 0;
  for (int i = 0; i < n_work; ++i)
    if (work[i].plan->multipass || work[i].plan->fourier_mp) {
      lead = i;
      break;
    }
  hipEvent_t fork = evs[want];
  if (need > 0 && hipEventRecord(fork, main) != hipSuccess) return FWR_E_DEVICE;
  fwr_status status = FWR_OK;
  int forked = 0;
  bool fork_ok = true;
  for (int i = 0; i < n_work; ++i) {
    if (i == lead) continue;
    const hipStream_t st = pool[forked];
    if (hipStreamWaitEvent(st, fork, 0) != hipSuccess) {
      status = FWR_E_DEVICE;
      fork_ok = false;
      break;
    }
    ++forked;
    const fwr_work &w = work[i];
    const fwr_status r =
        run(w.plan, w.d_slopes, w.d_phase, w.B, false, w.d_start, w.d_resid, st, true, nullptr, 0, n_work > 1);
    if (r != FWR_OK && status == FWR_OK) status = r;
  }
  if (fork_ok) {
    const fwr_work &w = work[lead];
    const fwr_status r =
        run(w.plan, w.d_slopes, w.d_phase, w.B, false, w.d_start, w.d_resid, main, true, nullptr, 0, n_work > 1);
    if (r != FWR_OK && status == FWR_OK) status = r;
  }
  // every forked branch joins back into the caller's stream, also after a failed launch
  for (int i = 0; i < forked; ++i)
    if (hipEventRecord(evs[i], pool[i]) != hipSuccess || hipStreamWaitEvent(main, evs[i], 0) != hipSuccess)
      status = FWR_E_DEVICE;
  return status;
}

fwr_status fwr_generate(fwr_plan_t plan, uint64_t seed, uint64_t first_frame, uint64_t *d_counter, float r0,
                        float L0, float noise_sigma, float *d_slopes, float *d_phase, int32_t B) {
  if (!valid(plan)) return FWR_E_STATE;
  if (plan->fourier) return FWR_E_UNSUPPORTED;  // the generator samples Fried slopes
  if (B < 0 || B > plan->max_batch || (first_frame & 1u)) return FWR_E_INVAL;
  if (B == 0) return FWR_OK;
  if (d_slopes == nullptr || !(r0 > 0.f) || !(L0 > 0.f) || !(noise_sigma >= 0.f) || !(plan->d > 0.0))
    return FWR_E_INVAL;
  fwr::GenArgs g{};
  g.slopes = d_slopes;
  g.phase = d_phase;
  g.mask = plan->dmask;
  g.d_counter = d_counter;
  g.first_pair = first_frame / 2;
  g.seed_lo = uint32_t(seed);
  g.seed_hi = uint32_t(seed >> 32);
  g.r0 = r0;
  g.L0 = L0;
  g.d = float(plan->d);
  g.sigma = noise_sigma;
  g.vk_const = float(vk_constant());
  g.B = B;
  g.n = plan->n;
  g.o = plan->o;
  hipError_t e;
  if (plan->multipass) {
    fwr::MPArgs a = plan->mp;
    a.B = B;
    e = fwr::multipass_generate(a, g, plan->stream);
  } else {
    e = fwr::gen_launch(plan->N, g, plan->stream);
  }
  return e == hipSuccess ? FWR_OK : FWR_E_DEVICE;
}

fwr_status fwr_fried_slopes(fwr_plan_t plan, const float *d_phase, const float *d_noise, float *d_slopes,
                            int32_t B) {
  if (!valid(plan)) return FWR_E_STATE;
  if (plan->fourier || plan->fourier_mp || plan->dmask == nullptr) return FWR_E_UNSUPPORTED;
  if (B < 0 || B > plan->max_batch) return FWR_E_INVAL;
  if (B == 0) return FWR_OK;
  if (d_phase == nullptr || d_slopes == nullptr) return FWR_E_INVAL;
  return fwr::fried_slopes_launch(d_phase, d_noise, plan->dmask, d_slopes, B, plan->n, plan->stream) == hipSuccess
             ? FWR_OK
             : FWR_E_DEVICE;
}

fwr_status fwr_hudgin_extend(fwr_plan_t plan, const float *d_slopes, float *d_ext, int32_t B) {
  if (!valid(plan)) return FWR_E_STATE;
  if (plan->hudgin_src == nullptr) return FWR_E_UNSUPPORTED;
  if (B < 0 || B > plan->max_batch) return FWR_E_INVAL;
  if (B == 0) return FWR_OK;
  if (d_slopes == nullptr || d_ext == nullptr) return FWR_E_INVAL;
  fwr::HudginArgs a{};
  a.slopes = d_slopes;
  a.out = d_ext;
  a.src_x = plan->hudgin_src;
  a.src_y = plan->hudgin_src + (size_t)plan->N * plan->N;
  a.B = B;
  a.n = plan->n;
  a.N = plan->N;
  return fwr::hudgin_launch(a, plan->stream) == hipSuccess ? FWR_OK : FWR_E_DEVICE;
}

}  // extern "C"

// Argument checks shared by the two learned calls (B = 0 passes; nothing is enqueued).
static fwr_status check_learned(fwr_plan_t plan, fwr_plan_t fallback, fwr_cnn_t cnn, const float *d_slopes,
                                const float *d_start, const float *d_phase, const float *d_resid, float threshold,
                                int32_t B) {
  if (!valid(plan) || !valid(fallback)) return FWR_E_STATE;
  int cn = 0, cN = 0, cmax = 0;
  hipStream_t cs = nullptr;
  if (!fwr::cnn_info(cnn, &cn, &cN, &cmax, &cs)) return FWR_E_STATE;
  if (cn != plan->n || cN != plan->N || fallback->n != plan->n || fallback->N != plan->N) return FWR_E_INVAL;
  if (cs != plan->stream || fallback->stream != plan->stream) return FWR_E_INVAL;
  if (B < 0 || B > plan->max_batch || B > fallback->max_batch || B > cmax) return FWR_E_INVAL;
  if (B == 0) return FWR_OK;
  if (d_slopes == nullptr || d_start == nullptr || d_phase == nullptr || d_resid == nullptr ||
      std::isnan(threshold))
    return FWR_E_INVAL;
  if (plan->multipass || plan->fourier) return FWR_E_UNSUPPORTED;
  if (plan->n_iter < 1) return FWR_E_INVAL;  // the residual is that of the last iteration
  return FWR_OK;
}

extern "C" {

fwr_status fwr_reconstruct_learned(fwr_plan_t plan, fwr_plan_t fallback, fwr_cnn_t cnn, const float *d_slopes,
                                   float *d_start, float *d_phase, float *d_resid, float threshold, int32_t B,
                                   int32_t *h_count) {
  if (h_count != nullptr) *h_count = 0;
  if (const fwr_status c = check_learned(plan, fallback, cnn, d_slopes, d_start, d_phase, d_resid, threshold, B);
      c != FWR_OK || B == 0)
    return c;
  const int n = plan->n;
  const size_t per_s = (size_t)2 * n * n, per_p = (size_t)(n + 1) * (n + 1);
  if (fallback->fb_mem == nullptr) {
    const size_t mb = (size_t)fallback->max_batch;
    const size_t idx_bytes = ((mb + 1) * sizeof(int32_t) + 255) / 256 * 256;
    void *mem = nullptr;
    if (hipMalloc(&mem, idx_bytes + mb * (per_s + per_p) * sizeof(float)) != hipSuccess) return FWR_E_NOMEM;
    fallback->fb_mem = mem;
    fallback->fb_idx = static_cast<int32_t *>(mem);
    fallback->fb_count = fallback->fb_idx + mb;
    fallback->fb_slopes = reinterpret_cast<float *>(static_cast<char *>(mem) + idx_bytes);
    fallback->fb_phase = fallback->fb_slopes + mb * per_s;
  }
  const hipStream_t st = plan->stream;
  fwr_status r = fwr_cnn_forward(cnn, d_slopes, d_start, B);
  if (r != FWR_OK) return r;
  r = run(plan, d_slopes, d_phase, B, false, d_start, d_resid);
  if (r != FWR_OK) return r;
  if (fwr::fallback_select(d_resid, threshold, B, fallback->fb_idx, fallback->fb_count, st) != hipSuccess)
    return FWR_E_DEVICE;
  int32_t count = 0;
  if (hipMemcpyAsync(&count, fallback->fb_count, sizeof(count), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return FWR_E_DEVICE;
  if (count < 0 || count > B) return FWR_E_DEVICE;
  if (count > 0) {
    if (fwr::fallback_gather(d_slopes, fallback->fb_idx, fallback->fb_slopes, count, int(per_s), st) != hipSuccess)
      return FWR_E_DEVICE;
    r = run(fallback, fallback->fb_slopes, fallback->fb_phase, count, false);
    if (r != FWR_OK) return r;
    if (fwr::fallback_scatter(fallback->fb_phase, fallback->fb_idx, d_phase, count, int(per_p), st) != hipSuccess)
      return FWR_E_DEVICE;
  }
  if (h_count != nullptr) *h_count = count;
  return FWR_OK;
}

fwr_status fwr_reconstruct_learned_noalloc(fwr_plan_t plan, fwr_plan_t fallback, fwr_cnn_t cnn,
                                           const float *d_slopes, float *d_start, float *d_phase, float *d_resid,
                                           float threshold, int32_t B, int32_t *d_count) {
  if (const fwr_status c = check_learned(plan, fallback, cnn, d_slopes, d_start, d_phase, d_resid, threshold, B);
      c != FWR_OK)
    return c;
  if (B > FWR_NOALLOC_MAX_FRAMES) return FWR_E_INVAL;
  if (fallback->fourier) return FWR_E_UNSUPPORTED;  // the chunked fallback needs the on-chip Fried kernel
  const hipStream_t st = plan->stream;
  void *base = nullptr;
  if (fwr::fallback_scratch(&base) != hipSuccess) return FWR_E_DEVICE;
  int32_t *idx = static_cast<int32_t *>(base);
  int32_t *cnt = reinterpret_cast<int32_t *>(static_cast<char *>(base) + fwr::kNoallocCountOffset);
  if (B == 0) {  // the select kernel of an empty batch writes the count 0 (a kernel, not a memset node)
    if (d_count != nullptr && fwr::fallback_select(nullptr, threshold, 0, idx, d_count, st) != hipSuccess)
      return FWR_E_DEVICE;
    return FWR_OK;
  }
  const int n = plan->n;
  const size_t per_s = (size_t)2 * n * n, per_p = (size_t)(n + 1) * (n + 1);
  // chunk capacity: an even number of frames, so that the frames of the gathered list pair up
  // (two frames per complex field) exactly as in the one-batch fallback
  const size_t room = FWR_NOALLOC_SCRATCH_BYTES - fwr::kNoallocChunkOffset;
  const int cap = int(2 * (room / (2 * (per_s + per_p) * sizeof(float))));
  if (cap < 2) return FWR_E_UNSUPPORTED;
  float *chunk_s = reinterpret_cast<float *>(static_cast<char *>(base) + fwr::kNoallocChunkOffset);
  float *chunk_p = chunk_s + (size_t)cap * per_s;
  fwr_status r = fwr_cnn_forward(cnn, d_slopes, d_start, B);
  if (r != FWR_OK) return r;
  r = run(plan, d_slopes, d_phase, B, false, d_start, d_resid);
  if (r != FWR_OK) return r;
  if (fwr::fallback_select(d_resid, threshold, B, idx, cnt, st) != hipSuccess) return FWR_E_DEVICE;
  for (int off = 0; off < B; off += cap) {
    const int cb = B - off < cap ? B - off : cap;
    if (fwr::fallback_gather_counted(d_slopes, idx, cnt, off, chunk_s, cb, int(per_s), st) != hipSuccess)
      return FWR_E_DEVICE;
    r = run(fallback, chunk_s, chunk_p, cb, false, nullptr, nullptr, st, true, cnt, off);
    if (r != FWR_OK) return r;
    if (fwr::fallback_scatter_counted(chunk_p, idx, cnt, off, d_phase, cb, int(per_p), st) != hipSuccess)
      return FWR_E_DEVICE;
  }
  if (d_count != nullptr &&
      hipMemcpyAsync(d_count, cnt, sizeof(int32_t), hipMemcpyDeviceToDevice, st) != hipSuccess)
    return FWR_E_DEVICE;
  return FWR_OK;
}

fwr_status fwr_set_stream(fwr_plan_t plan, void *stream) {
  if (!valid(plan)) return FWR_E_STATE;
  plan->stream = static_cast<hipStream_t>(stream);
  return FWR_OK;
}

fwr_status fwr_plan_launch_info(fwr_plan_t plan, int32_t *threads, int32_t *frames_per_group,
                                int32_t *lds_bytes) {
  if (!valid(plan)) return FWR_E_STATE;
  if (plan->multipass || plan->fourier_mp) {  // (the column pass's workgroup; the persistent loop's)
    if (threads) *threads = plan->multipass && plan->sched == 1 ? 1024 : (plan->multipass && plan->sched == 2 ? 288 : 256);
    if (frames_per_group) *frames_per_group = plan->multipass ? 2 : 1;
    if (lds_bytes) *lds_bytes = 0;
    return FWR_OK;
  }
  if (plan->fourier) {
    if (threads) *threads = fwr::fourier_threads(plan->N, plan->frames);
    if (frames_per_group) *frames_per_group = plan->frames;
    if (lds_bytes) *lds_bytes = fwr::fourier_lds_bytes(plan->N, plan->n, plan->frames);
    return FWR_OK;
  }
  if (threads) *threads = fwr::onchip_threads(plan->N, plan->pairs);
  if (frames_per_group) *frames_per_group = 2 * plan->pairs;
  if (lds_bytes) *lds_bytes = fwr::onchip_lds_bytes(plan->N, plan->n, plan->pairs);
  return FWR_OK;
}

fwr_status fwr_plan_set_group(fwr_plan_t plan, int32_t frames_per_group) {
  if (!valid(plan)) return FWR_E_STATE;
  if (plan->multipass) return frames_per_group == 2 ? FWR_OK : FWR_E_UNSUPPORTED;
  if (plan->fourier_mp) return frames_per_group == 1 ? FWR_OK : FWR_E_UNSUPPORTED;
  if (plan->fourier) {
    if (frames_per_group < 1) return FWR_E_INVAL;
    if (!fwr::fourier_frames_ok(plan->N, plan->n, frames_per_group)) return FWR_E_UNSUPPORTED;
    plan->frames = frames_per_group;
    return FWR_OK;
  }
  if (frames_per_group < 2 || frames_per_group % 2 != 0) return FWR_E_INVAL;
  const bool each = (plan->flags & fwr::kFlagPeriodicEach) != 0;
  if (!fwr::onchip_pairs_ok(plan->N, plan->n, frames_per_group / 2, each)) return FWR_E_UNSUPPORTED;
  plan->pairs = frames_per_group / 2;
  return FWR_OK;
}

fwr_status fwr_plan_set_schedule(fwr_plan_t plan, int32_t schedule) {
  if (!valid(plan)) return FWR_E_STATE;
  if (schedule < 0 || schedule > 2) return FWR_E_INVAL;
  if (schedule == 2 && !plan->multipass && !plan->fourier_mp) return FWR_E_UNSUPPORTED;
  if (schedule == 1 && !plan->multipass &&
      (plan->fourier || plan->fourier_mp || (plan->flags & fwr::kFlagPeriodicEach) != 0 ||
       !fwr::onchip_sched_ok(plan->N, plan->n)))
    return FWR_E_UNSUPPORTED;
  plan->sched = schedule;
  return FWR_OK;
}

fwr_status fwr_plan_set_wait_limit(fwr_plan_t plan, int32_t polls) {
  if (!valid(plan)) return FWR_E_STATE;
  if (!plan->multipass && !plan->fourier_mp) return FWR_E_UNSUPPORTED;
  if (polls < 1 || polls > (1 << 24)) return FWR_E_INVAL;
  if (plan->multipass) plan->mp.wait_limit = polls;
  else plan->fs.wait_limit = polls;
  return FWR_OK;
}

fwr_status fwr_plan_get_schedule(fwr_plan_t plan, int32_t *schedule) {
  if (!valid(plan)) return FWR_E_STATE;
  if (schedule == nullptr) return FWR_E_INVAL;
  *schedule = plan->sched;
  return FWR_OK;
}

fwr_status fwr_plan_autotune(fwr_plan_t plan, int32_t B, int32_t *frames_per_group) {
  if (!valid(plan)) return FWR_E_STATE;
  if (B < 1 || B > plan->max_batch) return FWR_E_INVAL;
  const bool each = (plan->flags & fwr::kFlagPeriodicEach) != 0;
  const int n = plan->n, N = plan->N;
  // candidate launch shapes: frame pairs per workgroup (on-chip) or frames (Fourier-domain);
  // the multi-pass paths have one (a frame pair, or a frame, per field) and their loop shapes
  const bool mp = plan->multipass || plan->fourier_mp;
  int *unit = plan->fourier ? &plan->frames : &plan->pairs;
  auto shape_ok = [&](int u) {
    if (mp) return u == 1;
    return plan->fourier ? fwr::fourier_frames_ok(N, n, u) : fwr::onchip_pairs_ok(N, n, u, each);
  };
  // the kernels' work does not depend on the slope values: time them on zeros
  float *d_in = nullptr, *d_out = nullptr;
  const size_t in_bytes = (size_t)B * 2 * n * n * sizeof(float);
  const size_t out_bytes = (size_t)B * (n + 1) * (n + 1) * sizeof(float);
  if (hipMalloc(reinterpret_cast<void **>(&d_in), in_bytes) != hipSuccess) return FWR_E_NOMEM;
  if (hipMalloc(reinterpret_cast<void **>(&d_out), out_bytes) != hipSuccess) {
    (void)hipFree(d_in);
    return FWR_E_NOMEM;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
            hipMemsetAsync(d_in, 0, in_bytes, plan->stream) == hipSuccess;
  const int before = *unit, sched_before = plan->sched;
  // radix schedules: both where the windowed on-chip kernel has two, else the first; the
  // multi-pass path's launch shapes (column passes of 16 or 64 threads per line, or the loop as
  // one persistent launch)
  const int n_sched = mp ? 3 : (!plan->fourier && !each && fwr::onchip_sched_ok(N, n) ? 2 : 1);
  // (the lenslet-averaging multi-pass path has shapes 0 and 2: one launch per pass or persistent)
  int best = before, best_sched = sched_before;
  float best_ms = 0.f;
  for (int pairs : kPairsOptions) {
    for (int sc = 0; sc < n_sched; ++sc) {
      if (!ok) break;
      if (!shape_ok(pairs) || (plan->fourier_mp && sc == 1)) continue;
      *unit = pairs;
      plan->sched = sc;
      float ms = 0.f;
      ok = run(plan, d_in, d_out, B, false) == FWR_OK && hipEventRecord(e0, plan->stream) == hipSuccess;
      for (int r = 0; r < 3 && ok; ++r) ok = run(plan, d_in, d_out, B, false) == FWR_OK;
      ok = ok && hipEventRecord(e1, plan->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
           hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
      // a later candidate (larger group, second schedule) must win by more than timing noise
      if (ok && (best_ms == 0.f || ms < 0.97f * best_ms)) {
        best = pairs;
        best_sched = sc;
        best_ms = ms;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(d_in);
  (void)hipFree(d_out);
  *unit = ok ? best : before;
  plan->sched = ok ? best_sched : sched_before;
  if (!ok) return FWR_E_DEVICE;
  remember_pairs(plan->device, N, n, plan->n_iter, each, best, plan->fourier ? FWR_MODEL_SINC : FWR_MODEL_FRIED,
                 plan->sched);
  if (frames_per_group) *frames_per_group = plan->fourier ? best : 2 * best;
  return FWR_OK;
}

fwr_status fwr_destroy(fwr_plan_t plan) {
  if (!valid(plan)) return FWR_E_STATE;
  (void)hipStreamSynchronize(plan->stream);
  (void)hipFree(plan->d_mem);
  (void)hipFree(plan->fb_mem);
  plan->magic = 0;
  delete plan;
  return FWR_OK;
}

}  // extern "C"

namespace {

fwr_status plan_multipass(const fwr_params &p, fwr_plan_t *out) {
  const int n = p.n_sub, N = p.n_grid, o = (N - n) / 2;
  // filter tables: [column position c][row position q], position -> frequency (pos / 16) + 16 (pos % 16)
  auto freq = [](int pos) { return (pos >> 4) + 16 * (pos & 15); };
  std::vector<float> hl((size_t)N * N), hf((size_t)N * N);
  for (int c = 0; c < N; ++c)
    for (int q = 0; q < N; ++q) {
      double a, b;
      filter_values(p, freq(q), freq(c), a, b);
      hl[(size_t)c * N + q] = float(a);
      hf[(size_t)c * N + q] = float(b);
    }
  std::vector<float2> tw(N);
  for (int e = 0; e < N; ++e) {
    const double ang = -2.0 * kPi * double(e) / double(N);
    tw[e] = make_float2(float(std::cos(ang)), float(std::sin(ang)));
  }
  std::vector<uint8_t> mask((size_t)n * n);
  for (size_t i = 0; i < mask.size(); ++i) mask[i] = p.mask[i] ? 1 : 0;
  auto in_pupil = [&](int cm, int cn) {
    cm = (cm + N) % N;
    cn = (cn + N) % N;
    const int i = cm - o, jj = cn - o;
    return i >= 0 && i < n && jj >= 0 && jj < n && mask[(size_t)i * n + jj] != 0;
  };
  // node codes packed per thread of the row passes: node (m, r + 16 q) in bits 4q..4q+3 of word 16 m + r
  std::vector<uint64_t> codes((size_t)N * 16, 0u);
  for (int m = 0; m < N; ++m)
    for (int nn = 0; nn < N; ++nn) {
      const uint64_t c = uint64_t((in_pupil(m, nn) ? 0 : 1) | (in_pupil(m - 1, nn - 1) ? 0 : 2) |
                                  (in_pupil(m, nn - 1) ? 0 : 4) | (in_pupil(m - 1, nn) ? 0 : 8));
      codes[(size_t)m * 16 + nn % 16] |= c << (4 * (nn / 16));
    }

  auto *plan = new (std::nothrow) fwr_plan_s();
  if (plan == nullptr) return FWR_E_NOMEM;
  if (hipGetDevice(&plan->device) != hipSuccess) {
    delete plan;
    return FWR_E_DEVICE;
  }
  const size_t b_h = hl.size() * sizeof(float), b_tw = tw.size() * sizeof(float2);
  const size_t off_hf = b_h, off_tw = 2 * b_h, off_codes = off_tw + b_tw;
  const size_t b_codes = codes.size() * sizeof(uint64_t), off_mask = off_codes + b_codes;
  const size_t off_ws = (off_mask + mask.size() + 255) & ~size_t(255);
  const size_t ws = fwr::multipass_workspace_bytes(N, n, p.max_batch);
  char *mem = nullptr;
  if (hipMalloc(reinterpret_cast<void **>(&mem), off_ws + ws) != hipSuccess) {
    delete plan;
    return FWR_E_NOMEM;
  }
  hipError_t e = hipMemcpy(mem, hl.data(), b_h, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_hf, hf.data(), b_h, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_tw, tw.data(), b_tw, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_mask, mask.data(), mask.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_codes, codes.data(), b_codes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(mem);
    delete plan;
    return FWR_E_DEVICE;
  }
  const size_t pairs = (size_t)(p.max_batch + 1) / 2;
  const size_t fbytes = (size_t)N * N * sizeof(float2);
  char *w = mem + off_ws;
  fwr::MPArgs &a = plan->mp;
  a.phi = reinterpret_cast<float2 *>(w);
  a.spec = reinterpret_cast<float2 *>(w + pairs * fbytes);
  a.sx = reinterpret_cast<float2 *>(w + 2 * pairs * fbytes);
  a.sy = reinterpret_cast<float2 *>(w + 3 * pairs * fbytes);
  a.f0 = reinterpret_cast<float2 *>(w + 4 * pairs * fbytes);
  a.sums = reinterpret_cast<float2 *>(w + 4 * pairs * fbytes + pairs * (size_t)(n + 1) * N * sizeof(float2));
  a.bad = reinterpret_cast<uint32_t *>(a.sums + pairs * 2 * (size_t)N);
  a.ctl = a.bad + pairs * (size_t)(N / 16);
  a.h_loop = reinterpret_cast<const float *>(mem);
  a.h_final = reinterpret_cast<const float *>(mem + off_hf);
  a.tw256 = reinterpret_cast<const float2 *>(mem + off_tw);
  a.mask = reinterpret_cast<const uint8_t *>(mem + off_mask);
  a.codes = reinterpret_cast<const uint64_t *>(mem + off_codes);
  a.n = n;
  a.o = o;
  a.n_iter = p.n_iter;
  a.flags = (p.periodic ? fwr::kMPPeriodic : 0) | (p.periodic_each_iter ? fwr::kMPPeriodicEach : 0);
  plan->magic = kMagic;
  plan->n = n;
  plan->N = N;
  plan->o = o;
  plan->n_iter = p.n_iter;
  plan->max_batch = p.max_batch;
  plan->stream = static_cast<hipStream_t>(p.stream);
  plan->d_mem = mem;
  plan->multipass = true;
  plan->dmask = a.mask;
  plan->d = p.d;
  // the column-pass shape autotuned earlier in the process for this shape, else 16 threads per line
  plan->sched = tuned_value(plan->device, N, n, p.n_iter, p.periodic_each_iter != 0, FWR_MODEL_FRIED) / 16;
  *out = plan;
  return FWR_OK;
}

}  // namespace

namespace {

// Lenslet-averaging (sinc) model of Eq. 4 at DFT index (l, k): the Hermitian part of
// exp(i pi (k' + l') / N) 2i sin(pi k' (1 - delta) / N) sinc(l' / N) (x) and its transpose (y),
// signed k', l'; zero on the Nyquist row and column of an even grid.  delta = d_px / d: the edge
// averages lie (1 - delta) d apart (the pixel-size correction remarked after Eq. 4).
void sinc_g(int l, int k, int N, double delta, std::complex<double> &gx, std::complex<double> &gy) {
  gx = gy = 0.0;
  if (N % 2 == 0 && (l == N / 2 || k == N / 2)) return;
  const double ks = k < (N + 1) / 2 ? k : k - N, ls = l < (N + 1) / 2 ? l : l - N;
  auto sinc = [](double u) { return u == 0.0 ? 1.0 : std::sin(kPi * u) / (kPi * u); };
  const std::complex<double> shift = std::polar(1.0, kPi * (ks + ls) / N);
  const std::complex<double> two_i(0.0, 2.0);
  gx = shift * two_i * std::sin(kPi * ks * (1.0 - delta) / N) * sinc(ls / N);
  gy = shift * two_i * std::sin(kPi * ls * (1.0 - delta) / N) * sinc(ks / N);
}

bool sinc_singular(int l, int k, int N) {
  return (l == 0 && k == 0) || (N % 2 == 0 && (l == N / 2 || k == N / 2));
}

// Packed-projector coefficients of the sinc model at DFT index (l, k), 1 / N^2 of the
// unnormalised inverse transforms folded in: the loop's Z' = alpha Z + beta conj(Z(-l, -k))
// (alpha = (a + b) / 2 + Im c, beta = (a - b) / 2 + i Re c with a = |G_x|^2 / |G|^2,
// b = |G_y|^2 / |G|^2, c = G_x conj(G_y) / |G|^2), and the final A Z + B conj(Z(-l, -k))
// (A, B = (R_x -/+ i R_y) / 2, R = G* / (|G|^2 + gamma W_eta / W_phi), Eq. 3).
void sinc_coeffs(const fwr_params &p, int l, int k, float &alpha, float2 &beta, float2 &fin_a, float2 &fin_b) {
  const int N = p.n_grid;
  const double inv = 1.0 / (double(N) * double(N));
  std::complex<double> gx, gy;
  sinc_g(l, k, N, p.d_px / p.d, gx, gy);
  const double g2 = std::norm(gx) + std::norm(gy);
  double al = 0.0;
  std::complex<double> be = 0.0, fa = 0.0, fb = 0.0;
  if (!sinc_singular(l, k, N)) {
    const double a = std::norm(gx) / g2, b = std::norm(gy) / g2;
    const std::complex<double> cc = gx * std::conj(gy) / g2;
    al = 0.5 * (a + b) + cc.imag();
    be = std::complex<double>(0.5 * (a - b), cc.real());
  }
  const double den = g2 + regulariser(p, l, k);
  if (den > 0.0 && !(p.gamma == 0.0 && p.alpha_map == nullptr && sinc_singular(l, k, N))) {
    const std::complex<double> rx = std::conj(gx) / den, ry = std::conj(gy) / den;
    const std::complex<double> I(0.0, 1.0);
    fa = 0.5 * (rx - I * ry);
    fb = 0.5 * (rx + I * ry);
  }
  alpha = float(al * inv);
  beta = make_float2(float(be.real() * inv), float(be.imag() * inv));
  fin_a = make_float2(float(fa.real() * inv), float(fa.imag() * inv));
  fin_b = make_float2(float(fb.real() * inv), float(fb.imag() * inv));
}

// Multi-pass plan of the sinc model (N = 256): coefficient tables [column position][row
// position] in the digit-reversed order the 256-point line transforms leave, and the workspace
fwr_status plan_fourier_mp(const fwr_params &p, fwr_plan_t *out) {
  const int n = p.n_sub, N = p.n_grid, o = (N - n) / 2;
  auto freq = [](int pos) { return (pos >> 4) + 16 * (pos & 15); };
  const size_t NNs = (size_t)N * N;
  std::vector<float> alpha(NNs);
  std::vector<float2> betat(NNs), fin_a(NNs), fin_b(NNs);
  for (int c = 0; c < N; ++c)
    for (int q = 0; q < N; ++q) {
      const size_t i = (size_t)c * N + q;
      sinc_coeffs(p, freq(q), freq(c), alpha[i], betat[i], fin_a[i], fin_b[i]);
    }
  std::vector<float2> tw(N);
  for (int e = 0; e < N; ++e) {
    const double ang = -2.0 * kPi * double(e) / double(N);
    tw[e] = make_float2(float(std::cos(ang)), float(std::sin(ang)));
  }
  std::vector<uint8_t> mask((size_t)n * n);
  for (size_t i = 0; i < mask.size(); ++i) mask[i] = p.mask[i] ? 1 : 0;
  auto *plan = new (std::nothrow) fwr_plan_s();
  if (plan == nullptr) return FWR_E_NOMEM;
  if (hipGetDevice(&plan->device) != hipSuccess) {
    delete plan;
    return FWR_E_DEVICE;
  }
  const size_t b_a = NNs * sizeof(float), b_c = NNs * sizeof(float2), b_tw = tw.size() * sizeof(float2);
  const size_t off_b = b_a, off_fa = off_b + b_c, off_fb = off_fa + b_c, off_tw = off_fb + b_c;
  const size_t off_mask = off_tw + b_tw, off_ws = (off_mask + mask.size() + 255) & ~size_t(255);
  const size_t ws = fwr::fourier_mp_workspace_bytes(N, p.max_batch);
  char *mem = nullptr;
  if (hipMalloc(reinterpret_cast<void **>(&mem), off_ws + ws) != hipSuccess) {
    delete plan;
    return FWR_E_NOMEM;
  }
  hipError_t e = hipMemcpy(mem, alpha.data(), b_a, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_b, betat.data(), b_c, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_fa, fin_a.data(), b_c, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_fb, fin_b.data(), b_c, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_tw, tw.data(), b_tw, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_mask, mask.data(), mask.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(mem);
    delete plan;
    return FWR_E_DEVICE;
  }
  const size_t B = (size_t)p.max_batch;
  char *w = mem + off_ws;
  fwr::FSArgs &a = plan->fs;
  a.spec = reinterpret_cast<float2 *>(w);
  a.state = reinterpret_cast<float2 *>(w + B * NNs * sizeof(float2));
  a.rsum = reinterpret_cast<float *>(w + 2 * B * NNs * sizeof(float2));
  a.cpart = a.rsum + B * N;
  a.ctl = reinterpret_cast<uint32_t *>(a.cpart + B * (size_t)(N / 16) * N);
  a.alpha = reinterpret_cast<const float *>(mem);
  a.beta = reinterpret_cast<const float2 *>(mem + off_b);
  a.fin_a = reinterpret_cast<const float2 *>(mem + off_fa);
  a.fin_b = reinterpret_cast<const float2 *>(mem + off_fb);
  a.tw256 = reinterpret_cast<const float2 *>(mem + off_tw);
  a.mask = reinterpret_cast<const uint8_t *>(mem + off_mask);
  a.n = n;
  a.o = o;
  a.n_iter = p.n_iter;
  plan->magic = kMagic;
  plan->n = n;
  plan->N = N;
  plan->o = o;
  plan->n_iter = p.n_iter;
  plan->flags = (p.periodic ? fwr::kFlagPeriodic : 0) | (p.periodic_each_iter ? fwr::kFlagPeriodicEach : 0);
  plan->max_batch = p.max_batch;
  plan->stream = static_cast<hipStream_t>(p.stream);
  plan->d_mem = mem;
  plan->fourier = true;
  plan->fourier_mp = true;
  plan->dmask = a.mask;
  plan->d = p.d;
  // the loop's launch shape autotuned earlier in the process for this shape, else one launch per pass
  plan->sched = tuned_value(plan->device, N, n, p.n_iter, p.periodic_each_iter != 0, FWR_MODEL_SINC) / 16;
  *out = plan;
  return FWR_OK;
}

fwr_status plan_fourier(const fwr_params &p, fwr_plan_t *out) {
  const int n = p.n_sub, N = p.n_grid, o = (N - n) / 2;
  if (fwr::fourier_mp_supported(N)) return plan_fourier_mp(p, out);
  if (!fwr::fourier_supported(N)) return FWR_E_UNSUPPORTED;
  if (!fwr::fourier_frames_ok(N, n, 1)) return FWR_E_UNSUPPORTED;
  const int T = N / 4, threads = fwr::fourier_threads(N, 1);
  static const int beta[4] = {0, 2, 1, 3};
  std::vector<float> alpha((size_t)T * threads);
  std::vector<float2> betat((size_t)T * threads), fin_a((size_t)T * threads), fin_b((size_t)T * threads);
  for (int c = 0; c < N; ++c) {
    const int kf = (c % T) + T * beta[c / T];  // x-frequency held in LDS column c
    for (int jj = 0; jj < 4; ++jj) {
      const size_t base = (size_t)(4 * c + jj) * T;
      for (int k2 = 0; k2 < T; ++k2) {
        const int l = k2 + T * beta[jj];      // y-frequency of this slot
        sinc_coeffs(p, l, kf, alpha[base + k2], betat[base + k2], fin_a[base + k2], fin_b[base + k2]);
      }
    }
  }
  std::vector<float2> tw((size_t)T * 4);
  for (int k2 = 0; k2 < T; ++k2)
    for (int jj = 0; jj < 4; ++jj) {
      const double ang = -2.0 * kPi * double(jj) * double(k2) / double(N);
      tw[(size_t)k2 * 4 + jj] = make_float2(float(std::cos(ang)), float(std::sin(ang)));
    }
  // in-pupil bits: bit k of thread t = 4m + j marks cell (m, 4k + j)
  std::vector<uint32_t> pup(threads, 0u);
  for (int m = 0; m < N; ++m)
    for (int jj = 0; jj < 4; ++jj)
      for (int k = 0; k < T; ++k) {
        const int i = m - o, c = 4 * k + jj - o;
        if (i >= 0 && i < n && c >= 0 && c < n && p.mask[(size_t)i * n + c]) pup[4 * m + jj] |= 1u << k;
      }
  auto *plan = new (std::nothrow) fwr_plan_s();
  if (plan == nullptr) return FWR_E_NOMEM;
  bool prepared = hipGetDevice(&plan->device) == hipSuccess;
  for (int frames = 1; frames <= 2 && prepared; ++frames)
    if (fwr::fourier_frames_ok(N, n, frames)) prepared = fwr::fourier_prepare(N, n, frames) == hipSuccess;
  if (!prepared) {
    delete plan;
    return FWR_E_DEVICE;
  }
  const size_t b_a = alpha.size() * sizeof(float), b_c = betat.size() * sizeof(float2);
  const size_t b_tw = tw.size() * sizeof(float2), b_p = pup.size() * sizeof(uint32_t);
  const std::vector<int32_t> hsrc = hudgin_sources(p);
  const size_t b_h = hsrc.size() * sizeof(int32_t);
  const size_t off_b = b_a, off_fa = off_b + b_c, off_fb = off_fa + b_c, off_tw = off_fb + b_c,
               off_p = off_tw + b_tw, off_h = (off_p + b_p + 15) & ~size_t(15), total = off_h + b_h;
  char *mem = nullptr;
  if (hipMalloc(reinterpret_cast<void **>(&mem), total) != hipSuccess) {
    delete plan;
    return FWR_E_NOMEM;
  }
  hipError_t e = hipMemcpy(mem, alpha.data(), b_a, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_b, betat.data(), b_c, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_fa, fin_a.data(), b_c, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_fb, fin_b.data(), b_c, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_tw, tw.data(), b_tw, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_p, pup.data(), b_p, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + off_h, hsrc.data(), b_h, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = fwr::hudgin_prepare(N);
  if (e != hipSuccess) {
    (void)hipFree(mem);
    delete plan;
    return FWR_E_DEVICE;
  }
  fwr::FourierArgs &a = plan->fa;
  a.alpha = reinterpret_cast<const float *>(mem);
  a.beta = reinterpret_cast<const float2 *>(mem + off_b);
  a.fin_a = reinterpret_cast<const float2 *>(mem + off_fa);
  a.fin_b = reinterpret_cast<const float2 *>(mem + off_fb);
  a.tw_lane = reinterpret_cast<const float2 *>(mem + off_tw);
  a.inpupil = reinterpret_cast<const uint32_t *>(mem + off_p);
  plan->hudgin_src = reinterpret_cast<const int32_t *>(mem + off_h);
  a.n = n;
  a.o = o;
  a.n_iter = p.n_iter;
  plan->magic = kMagic;
  plan->n = n;
  plan->N = N;
  plan->o = o;
  plan->n_iter = p.n_iter;
  plan->flags = (p.periodic ? fwr::kFlagPeriodic : 0) | (p.periodic_each_iter ? fwr::kFlagPeriodicEach : 0);
  plan->max_batch = p.max_batch;
  plan->stream = static_cast<hipStream_t>(p.stream);
  plan->d_mem = mem;
  plan->fourier = true;
  plan->d = p.d;
  // tuned earlier in the process, else two frames when one frame's waves number 4k + 1
  const int tuned = tuned_value(plan->device, N, n, p.n_iter, false, FWR_MODEL_SINC);
  const int waves = (fwr::fourier_threads(N, 1) + 63) / 64;
  plan->frames = tuned ? tuned : (waves > 4 && waves % 4 == 1 && fwr::fourier_frames_ok(N, n, 2)) ? 2 : 1;
  *out = plan;
  return FWR_OK;
}

}  // namespace

