// Layout of the learned cost model's parameters and its device launchers.
#pragma once

#include <cstdint>

namespace qk {

constexpr int kMlpF = 20;   // features (same order as segment_features)
constexpr int kMlpH = 64;   // hidden units per layer
// flat FP32 parameter vector: W1 [F][H], b1 [H], W2 [H][H], b2 [H], W3 [H], b3
constexpr int kOW1 = 0;
constexpr int kOb1 = kOW1 + kMlpF * kMlpH;
constexpr int kOW2 = kOb1 + kMlpH;
constexpr int kOb2 = kOW2 + kMlpH * kMlpH;
constexpr int kOW3 = kOb2 + kMlpH;
constexpr int kOb3 = kOW3 + kMlpH;
constexpr int kMlpParams = kOb3 + 1;
// per-row backward cache: h1 [H], h2 [H], dz2 [H], dz1 [H], dy
constexpr int kMlpCache = 4 * kMlpH + 1;

// idx (optional) selects rows of X / T for batch position b; Y and cache are
// indexed by batch position.  T == nullptr or cache == nullptr: forward only.
int mlp_launch_rows(const float* params, const float* X, const int* idx, const float* T, int64_t B, float inv_b,
                    float* Y, float* cache, void* stream);
int mlp_launch_grads(const float* X, const int* idx, const float* cache, int64_t B, float* grads, void* stream);
int mlp_launch_adam(float* params, const float* grads, float* m, float* v, float lr, float b1, float b2, float eps,
                    int step, void* stream);
int mlp_launch_loss(const float* Y, const float* T, const int* idx, int64_t B, float* out, void* stream);

}  // namespace qk
