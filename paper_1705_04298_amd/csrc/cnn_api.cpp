// C ABI of the learned initial extension (CNN): create, parameters in/out,
// forward, backward (loss + gradients), Adam step.  All compute is in cnn.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/fwr.h"
#include "cnn.h"
#include "learned.h"

using namespace fwr::cnn_launch;

namespace {

constexpr uint32_t kCnnMagic = 0x464E4E31u;  // "FNN1"

size_t master_w(int l) { return (size_t)kCoutS[l] * 9 * kCinS[l]; }
size_t master_total() {
  size_t n = 0;
  for (int l = 0; l < kLayers; ++l) n += master_w(l) + kCoutS[l];
  return n;
}
size_t oracle_total() {
  size_t n = 0;
  for (int l = 0; l < kLayers; ++l) n += (size_t)kCout[l] * kCin[l] * 9 + kCout[l];
  return n;
}

}  // namespace

struct fwr_cnn_s {
  uint32_t magic = 0;
  int n = 0, N = 0, max_batch = 0, training = 0;
  float scale = 1.f;
  double outside = 0.0;  // out-of-pupil grid cells (loss normalisation)
  hipStream_t stream = nullptr;
  void *mem = nullptr;
  uint8_t *mask = nullptr;
  float *w = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;  // master layout, per layer w then bias
  size_t woff[kLayers] = {}, boff[kLayers] = {};
  uint16_t *wt[kLayers] = {}, *wtb[kLayers] = {};
  uint16_t *feat = nullptr, *act[kLayers - 1] = {}, *dz[2] = {}, *dz7 = nullptr;
  float *loss = nullptr;
  long step = 0;
};

namespace {

bool valid(fwr_cnn_t c) { return c != nullptr && c->magic == kCnnMagic; }

}  // namespace

bool fwr::cnn_info(fwr_cnn_t c, int *n_sub, int *n_grid, int *max_batch, hipStream_t *stream) {
  if (!valid(c)) return false;
  *n_sub = c->n;
  *n_grid = c->N;
  *max_batch = c->max_batch;
  *stream = c->stream;
  return true;
}

namespace {

fwr_status repack(fwr_cnn_t c) {
  for (int l = 0; l < kLayers; ++l) {
    if (pack(c->w + c->woff[l], c->wt[l], c->wtb[l], kCinS[l], kCoutS[l], kpad_of(kCinS[l]), kpad_of(kCoutS[l]),
             c->stream) != hipSuccess)
      return FWR_E_DEVICE;
  }
  return FWR_OK;
}

}  // namespace

extern "C" {

fwr_status fwr_cnn_create(int32_t n_sub, int32_t n_grid, const uint8_t *mask, int32_t max_batch, float input_scale,
                          int32_t training, void *stream, fwr_cnn_t *out) {
  if (out == nullptr) return FWR_E_INVAL;
  *out = nullptr;
  if (mask == nullptr || n_sub < 1 || n_grid <= n_sub || (n_grid - n_sub) % 2 || max_batch < 1 ||
      !(input_scale > 0.f))
    return FWR_E_INVAL;
  if ((n_grid * n_grid) % 64 != 0 || n_grid < 16) return FWR_E_UNSUPPORTED;
  if (conv_prepare(n_grid) != hipSuccess) return FWR_E_UNSUPPORTED;
  auto *c = new (std::nothrow) fwr_cnn_s();
  if (c == nullptr) return FWR_E_NOMEM;
  c->n = n_sub;
  c->N = n_grid;
  c->max_batch = max_batch;
  c->training = training ? 1 : 0;
  c->scale = input_scale;
  c->stream = static_cast<hipStream_t>(stream);
  const size_t pix = (size_t)max_batch * n_grid * n_grid;
  const size_t P = master_total();
  // layout: params (4 x P floats) | loss | bf16 weights | mask | features | activations | gradients
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) & ~size_t(255);
    return o;
  };
  const size_t o_params = take(4 * P * sizeof(float));
  const size_t o_loss = take(sizeof(float));
  size_t o_wt[kLayers], o_wtb[kLayers];
  for (int l = 0; l < kLayers; ++l) {
    o_wt[l] = take((size_t)kCoutS[l] * kpad_of(kCinS[l]) * 2);
    o_wtb[l] = take((size_t)kCinS[l] * kpad_of(kCoutS[l]) * 2);
  }
  const size_t o_mask = take((size_t)n_sub * n_sub);
  const size_t o_feat = take(pix * 8 * 2);
  const int nact = c->training ? kLayers - 1 : 2;
  size_t o_act[kLayers - 1] = {};
  for (int l = 0; l < nact; ++l) o_act[l] = take(pix * 32 * 2);
  size_t o_dz[2] = {}, o_dz7 = 0;
  if (c->training) {
    o_dz[0] = take(pix * 32 * 2);
    o_dz[1] = take(pix * 32 * 2);
    o_dz7 = take(pix * 16 * 2);
  }
  char *mem = nullptr;
  if (hipMalloc(reinterpret_cast<void **>(&mem), off) != hipSuccess) {
    delete c;
    return FWR_E_NOMEM;
  }
  c->mem = mem;
  c->w = reinterpret_cast<float *>(mem + o_params);
  c->g = c->w + P;
  c->m1 = c->g + P;
  c->m2 = c->m1 + P;
  size_t po = 0;
  for (int l = 0; l < kLayers; ++l) {
    c->woff[l] = po;
    po += master_w(l);
    c->boff[l] = po;
    po += kCoutS[l];
  }
  c->loss = reinterpret_cast<float *>(mem + o_loss);
  for (int l = 0; l < kLayers; ++l) {
    c->wt[l] = reinterpret_cast<uint16_t *>(mem + o_wt[l]);
    c->wtb[l] = reinterpret_cast<uint16_t *>(mem + o_wtb[l]);
  }
  c->mask = reinterpret_cast<uint8_t *>(mem + o_mask);
  c->feat = reinterpret_cast<uint16_t *>(mem + o_feat);
  for (int l = 0; l < nact; ++l) c->act[l] = reinterpret_cast<uint16_t *>(mem + o_act[l]);
  if (c->training) {
    c->dz[0] = reinterpret_cast<uint16_t *>(mem + o_dz[0]);
    c->dz[1] = reinterpret_cast<uint16_t *>(mem + o_dz[1]);
    c->dz7 = reinterpret_cast<uint16_t *>(mem + o_dz7);
  }
  std::vector<uint8_t> m((size_t)n_sub * n_sub);
  size_t inside = 0;
  for (size_t i = 0; i < m.size(); ++i) {
    m[i] = mask[i] ? 1 : 0;
    inside += m[i];
  }
  c->outside = double(n_grid) * n_grid - double(inside);
  hipError_t e = hipMemcpy(c->mask, m.data(), m.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(c->w, 0, 4 * P * sizeof(float));
  if (e != hipSuccess) {
    (void)hipFree(mem);
    delete c;
    return FWR_E_DEVICE;
  }
  c->magic = kCnnMagic;
  *out = c;
  return FWR_OK;
}

fwr_status fwr_cnn_set_params(fwr_cnn_t c, const float *h_params, int32_t count) {
  if (!valid(c)) return FWR_E_STATE;
  if (h_params == nullptr || count != (int32_t)oracle_total()) return FWR_E_INVAL;
  std::vector<float> master(master_total(), 0.f);
  size_t src = 0;
  for (int l = 0; l < kLayers; ++l) {
    const int O = kCout[l], C = kCin[l], CS = kCinS[l];
    for (int o = 0; o < O; ++o)
      for (int ci = 0; ci < C; ++ci)
        for (int t = 0; t < 9; ++t) master[c->woff[l] + ((size_t)o * 9 + t) * CS + ci] = h_params[src + ((size_t)o * C + ci) * 9 + t];
    src += (size_t)O * C * 9;
    for (int o = 0; o < O; ++o) master[c->boff[l] + o] = h_params[src + o];
    src += O;
  }
  const size_t P = master_total();
  hipError_t e = hipMemcpyAsync(c->w, master.data(), P * sizeof(float), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->m1, 0, 2 * P * sizeof(float), c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return FWR_E_DEVICE;
  c->step = 0;
  return repack(c);
}

static fwr_status read_master(fwr_cnn_t c, const float *dev, float *h_out, int32_t count) {
  if (!valid(c)) return FWR_E_STATE;
  if (h_out == nullptr || count != (int32_t)oracle_total()) return FWR_E_INVAL;
  std::vector<float> master(master_total());
  if (hipMemcpyAsync(master.data(), dev, master.size() * sizeof(float), hipMemcpyDeviceToHost, c->stream) !=
          hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return FWR_E_DEVICE;
  size_t dst = 0;
  for (int l = 0; l < kLayers; ++l) {
    const int O = kCout[l], C = kCin[l], CS = kCinS[l];
    for (int o = 0; o < O; ++o)
      for (int ci = 0; ci < C; ++ci)
        for (int t = 0; t < 9; ++t) h_out[dst + ((size_t)o * C + ci) * 9 + t] = master[c->woff[l] + ((size_t)o * 9 + t) * CS + ci];
    dst += (size_t)O * C * 9;
    for (int o = 0; o < O; ++o) h_out[dst + o] = master[c->boff[l] + o];
    dst += O;
  }
  return FWR_OK;
}

fwr_status fwr_cnn_get_params(fwr_cnn_t c, float *h_params, int32_t count) {
  if (!valid(c)) return FWR_E_STATE;
  return read_master(c, c->w, h_params, count);
}

fwr_status fwr_cnn_get_grads(fwr_cnn_t c, float *h_grads, int32_t count) {
  if (!valid(c)) return FWR_E_STATE;
  return read_master(c, c->g, h_grads, count);
}

fwr_status fwr_cnn_forward(fwr_cnn_t c, const float *d_slopes, float *d_pred, int32_t B) {
  if (!valid(c)) return FWR_E_STATE;
  if (B < 0 || B > c->max_batch) return FWR_E_INVAL;
  if (B == 0) return FWR_OK;
  if (d_slopes == nullptr || d_pred == nullptr) return FWR_E_INVAL;
  const int N = c->N;
  if (features(d_slopes, c->mask, c->feat, B, c->n, N, c->scale, c->stream) != hipSuccess) return FWR_E_DEVICE;
  const uint16_t *in = c->feat;
  for (int l = 0; l < kLayers; ++l) {
    void *o = (l == kLayers - 1) ? static_cast<void *>(d_pred) : static_cast<void *>(c->act[c->training ? l : (l & 1)]);
    if (conv(l, in, c->wt[l], c->w + c->boff[l], o, B, N, 1.f / c->scale, c->stream) != hipSuccess)
      return FWR_E_DEVICE;
    in = static_cast<const uint16_t *>(o);
  }
  return FWR_OK;
}

}  // extern "C"

namespace {

// Parameter gradients from c->dz7 (the last layer's output gradient) back through the network.
fwr_status backprop(fwr_cnn_t c, int32_t B) {
  const int N = c->N;
  const size_t P = master_total();
  hipStream_t s = c->stream;
  if (hipMemsetAsync(c->g, 0, P * sizeof(float), s) != hipSuccess) return FWR_E_DEVICE;
  const uint16_t *dz = c->dz7;
  for (int l = kLayers - 1; l >= 0; --l) {
    const uint16_t *xin = l == 0 ? c->feat : c->act[l - 1];
    if (wgrad(l, xin, dz, c->g + c->woff[l], c->g + c->boff[l], B, N, s) != hipSuccess) return FWR_E_DEVICE;
    if (l > 0) {
      uint16_t *dx = c->dz[l & 1];
      if (conv_bwd_data(l, dz, c->wtb[l], c->act[l - 1], dx, B, N, s) != hipSuccess) return FWR_E_DEVICE;
      dz = dx;
    }
  }
  return FWR_OK;
}

fwr_status read_loss(fwr_cnn_t c, float *h_loss) {
  if (h_loss) {
    if (hipMemcpyAsync(h_loss, c->loss, sizeof(float), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      return FWR_E_DEVICE;
  }
  return FWR_OK;
}

}  // namespace

extern "C" {

fwr_status fwr_cnn_backward(fwr_cnn_t c, const float *d_pred, const float *d_target, int32_t B, float *h_loss) {
  if (!valid(c)) return FWR_E_STATE;
  if (!c->training) return FWR_E_UNSUPPORTED;
  if (B < 1 || B > c->max_batch || d_pred == nullptr || d_target == nullptr) return FWR_E_INVAL;
  const float inv_count = float(1.0 / (double(B) * 2.0 * c->outside));
  hipStream_t s = c->stream;
  if (hipMemsetAsync(c->loss, 0, sizeof(float), s) != hipSuccess) return FWR_E_DEVICE;
  if (loss_grad(d_pred, d_target, c->mask, c->dz7, c->loss, B, c->n, c->N, c->scale, inv_count, s) != hipSuccess)
    return FWR_E_DEVICE;
  if (const fwr_status r = backprop(c, B); r != FWR_OK) return r;
  return read_loss(c, h_loss);
}

fwr_status fwr_cnn_loss_grad(fwr_cnn_t c, const float *d_pred, const float *d_target, float *d_grad, int32_t B,
                             float *h_loss) {
  if (!valid(c)) return FWR_E_STATE;
  if (B < 1 || B > c->max_batch || d_pred == nullptr || d_target == nullptr || d_grad == nullptr)
    return FWR_E_INVAL;
  const float inv_count = float(1.0 / (double(B) * 2.0 * c->outside));
  if (hipMemsetAsync(c->loss, 0, sizeof(float), c->stream) != hipSuccess) return FWR_E_DEVICE;
  if (loss_grad_map(d_pred, d_target, c->mask, d_grad, c->loss, B, c->n, c->N, c->scale, inv_count, c->stream) !=
      hipSuccess)
    return FWR_E_DEVICE;
  return read_loss(c, h_loss);
}

fwr_status fwr_cnn_backward_grad(fwr_cnn_t c, const float *d_grad, int32_t B) {
  if (!valid(c)) return FWR_E_STATE;
  if (!c->training) return FWR_E_UNSUPPORTED;
  if (B < 1 || B > c->max_batch || d_grad == nullptr) return FWR_E_INVAL;
  if (grad_in(d_grad, c->dz7, B, c->N, 1.f / c->scale, c->stream) != hipSuccess) return FWR_E_DEVICE;
  return backprop(c, B);
}

fwr_status fwr_cnn_adam_step(fwr_cnn_t c, float lr) {
  if (!valid(c)) return FWR_E_STATE;
  if (!c->training || !(lr > 0.f)) return FWR_E_INVAL;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  c->step += 1;
  // bias corrections from the same (FP32) betas the moment updates use
  const float c1 = float(1.0 - std::pow(double(b1), double(c->step)));
  const float c2 = float(1.0 - std::pow(double(b2), double(c->step)));
  if (adam(c->w, c->g, c->m1, c->m2, (int)master_total(), lr, b1, b2, eps, c1, c2, c->stream) != hipSuccess)
    return FWR_E_DEVICE;
  return repack(c);
}

fwr_status fwr_cnn_set_stream(fwr_cnn_t c, void *stream) {
  if (!valid(c)) return FWR_E_STATE;
  c->stream = static_cast<hipStream_t>(stream);
  return FWR_OK;
}

fwr_status fwr_cnn_destroy(fwr_cnn_t c) {
  if (!valid(c)) return FWR_E_STATE;
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(c->mem);
  c->magic = 0;
  delete c;
  return FWR_OK;
}

}  // extern "C"
