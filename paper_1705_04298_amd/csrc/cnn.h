// Launchers of the CNN kernels (learned initial extension).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fwr {
namespace cnn_launch {

// Layer geometry: 7 layers, stored channel counts (padded) in / out.
constexpr int kLayers = 7;
constexpr int kCin[kLayers] = {3, 32, 32, 32, 32, 32, 32};
constexpr int kCout[kLayers] = {32, 32, 32, 32, 32, 32, 2};
constexpr int kCinS[kLayers] = {8, 32, 32, 32, 32, 32, 32};
constexpr int kCoutS[kLayers] = {32, 32, 32, 32, 32, 32, 16};
constexpr int kpad_of(int cin_s) { return ((9 * cin_s + 31) / 32) * 32; }

hipError_t conv_prepare(int N);  // once per grid size, before the first conv / conv_bwd_data
hipError_t conv(int layer, const uint16_t *x, const uint16_t *wt, const float *bias, void *out, int B, int N,
                float out_scale, hipStream_t s);
hipError_t conv_bwd_data(int layer, const uint16_t *dz, const uint16_t *wtb, const uint16_t *act_prev, uint16_t *dx,
                         int B, int N, hipStream_t s);
hipError_t wgrad(int layer, const uint16_t *x, const uint16_t *dz, float *dw, float *db, int B, int N, hipStream_t s);
hipError_t features(const float *slopes, const uint8_t *mask, uint16_t *feat, int B, int n, int N, float scale,
                    hipStream_t s);
hipError_t loss_grad(const float *pred, const float *target, const uint8_t *mask, uint16_t *dz7, float *loss, int B,
                     int n, int N, float scale, float inv_count, hipStream_t s);
// the same loss with dloss/dpred (slope units) as a float map [B][2][N][N] (zero inside the pupil)
hipError_t loss_grad_map(const float *pred, const float *target, const uint8_t *mask, float *grad, float *loss, int B,
                         int n, int N, float scale, float inv_count, hipStream_t s);
// dz7 from dloss/dpred (slope units)
hipError_t grad_in(const float *grad, uint16_t *dz7, int B, int N, float inv_scale, hipStream_t s);
hipError_t adam(float *w, const float *g, float *m1, float *m2, int count, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t s);
hipError_t pack(const float *w, uint16_t *wt, uint16_t *wtb, int cin_s, int cout_s, int kpad_f, int kpad_b,
                hipStream_t s);

}  // namespace cnn_launch
}  // namespace fwr
