// Learned cost model: a 2-hidden-layer ReLU MLP (F = 20 inputs, H = 64), FP32,
// trained on the device by these kernels.
//
//   z1 = x W1 + b1, h1 = relu(z1), z2 = h1 W2 + b2, h2 = relu(z2), y = h2 W3 + b3
//   loss = (1/B) sum_b (y_b - t_b)^2
//
// k_mlp_rows   -- one thread per row: forward pass, and (with targets) the
//                 per-row backward quantities h1, h2, dz2, dz1, dy.
// k_mlp_grads  -- one thread per parameter: sums the per-row contributions in
//                 row order (deterministic, no atomics).
// k_mlp_adam   -- one thread per parameter: Adam with bias correction.
// k_mlp_loss   -- one workgroup: the batch loss.
#include <hip/hip_runtime.h>

#include "mlp.hpp"

namespace qk {

namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_mlp_rows(const float* __restrict__ params, const float* __restrict__ X,
                                                       const int* __restrict__ idx, const float* __restrict__ T,
                                                       int64_t B, float inv_b, float* __restrict__ Y,
                                                       float* __restrict__ cache)
{
    __shared__ float P[kMlpParams];
    for (int p = threadIdx.x; p < kMlpParams; p += kThreads) P[p] = params[p];
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (b >= B) return;
    const int64_t row = idx ? idx[b] : b;
    float x[kMlpF];
#pragma unroll
    for (int i = 0; i < kMlpF; ++i) x[i] = X[row * kMlpF + i];
    float h1[kMlpH], h2[kMlpH];
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) {
        float z = P[kOb1 + j];
#pragma unroll
        for (int i = 0; i < kMlpF; ++i) z = fmaf(x[i], P[kOW1 + i * kMlpH + j], z);
        h1[j] = z > 0.f ? z : 0.f;
    }
    float y = P[kOb3];
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) {
        float z = P[kOb2 + j];
#pragma unroll 16
        for (int i = 0; i < kMlpH; ++i) z = fmaf(h1[i], P[kOW2 + i * kMlpH + j], z);
        h2[j] = z > 0.f ? z : 0.f;
        y = fmaf(h2[j], P[kOW3 + j], y);
    }
    Y[b] = y;
    if (!T || !cache) return;
    const float dy = 2.f * (y - T[row]) * inv_b;
    float* c = cache + b * kMlpCache;
    float dz2[kMlpH];
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) {
        dz2[j] = h2[j] > 0.f ? dy * P[kOW3 + j] : 0.f;
        c[j] = h1[j];
        c[kMlpH + j] = h2[j];
        c[2 * kMlpH + j] = dz2[j];
    }
#pragma unroll
    for (int i = 0; i < kMlpH; ++i) {
        float s = 0.f;
        if (h1[i] > 0.f) {
#pragma unroll 16
            for (int j = 0; j < kMlpH; ++j) s = fmaf(dz2[j], P[kOW2 + i * kMlpH + j], s);
        }
        c[3 * kMlpH + i] = s;
    }
    c[4 * kMlpH] = dy;
}

__global__ __launch_bounds__(kThreads) void k_mlp_grads(const float* __restrict__ X, const int* __restrict__ idx,
                                                        const float* __restrict__ cache, int64_t B,
                                                        float* __restrict__ grads)
{
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= kMlpParams) return;
    float s = 0.f;
    if (p < kOb1) {                       // W1[i][j] += x_i dz1_j
        const int i = p / kMlpH, j = p % kMlpH;
        for (int64_t b = 0; b < B; ++b) {
            const int64_t row = idx ? idx[b] : b;
            s = fmaf(X[row * kMlpF + i], cache[b * kMlpCache + 3 * kMlpH + j], s);
        }
    } else if (p < kOW2) {                // b1[j] += dz1_j
        const int j = p - kOb1;
        for (int64_t b = 0; b < B; ++b) s += cache[b * kMlpCache + 3 * kMlpH + j];
    } else if (p < kOb2) {                // W2[i][j] += h1_i dz2_j
        const int q = p - kOW2, i = q / kMlpH, j = q % kMlpH;
        for (int64_t b = 0; b < B; ++b)
            s = fmaf(cache[b * kMlpCache + i], cache[b * kMlpCache + 2 * kMlpH + j], s);
    } else if (p < kOW3) {                // b2[j] += dz2_j
        const int j = p - kOb2;
        for (int64_t b = 0; b < B; ++b) s += cache[b * kMlpCache + 2 * kMlpH + j];
    } else if (p < kOb3) {                // W3[j] += h2_j dy
        const int j = p - kOW3;
        for (int64_t b = 0; b < B; ++b)
            s = fmaf(cache[b * kMlpCache + kMlpH + j], cache[b * kMlpCache + 4 * kMlpH], s);
    } else {                              // b3 += dy
        for (int64_t b = 0; b < B; ++b) s += cache[b * kMlpCache + 4 * kMlpH];
    }
    grads[p] = s;
}

__global__ __launch_bounds__(kThreads) void k_mlp_adam(float* __restrict__ params, const float* __restrict__ grads,
                                                       float* __restrict__ m, float* __restrict__ v, int np,
                                                       float lr, float b1, float b2, float eps, float bc1, float bc2)
{
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= np) return;
    const float g = grads[p];
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    params[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

__global__ __launch_bounds__(kThreads) void k_mlp_loss(const float* __restrict__ Y, const float* __restrict__ T,
                                                       const int* __restrict__ idx, int64_t B, float* out)
{
    __shared__ double red[kThreads];
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < B; b += kThreads) {
        const int64_t row = idx ? idx[b] : b;
        const double r = (double)Y[b] - (double)T[row];
        s += r * r;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (float)(red[0] / (double)(B > 0 ? B : 1));
}

}  // namespace

int mlp_launch_rows(const float* params, const float* X, const int* idx, const float* T, int64_t B, float inv_b,
                    float* Y, float* cache, void* stream)
{
    if (B <= 0) return 0;
    const uint32_t grid = (uint32_t)((B + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_mlp_rows, dim3(grid), dim3(kThreads), 0, (hipStream_t)stream, params, X, idx, T, B, inv_b,
                       Y, cache);
    return (int)hipGetLastError();
}

int mlp_launch_grads(const float* X, const int* idx, const float* cache, int64_t B, float* grads, void* stream)
{
    const uint32_t grid = (kMlpParams + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_mlp_grads, dim3(grid), dim3(kThreads), 0, (hipStream_t)stream, X, idx, cache, B, grads);
    return (int)hipGetLastError();
}

int mlp_launch_adam(float* params, const float* grads, float* m, float* v, float lr, float b1, float b2, float eps,
                    int step, void* stream)
{
    const float bc1 = 1.f - powf(b1, (float)step), bc2 = 1.f - powf(b2, (float)step);
    const uint32_t grid = (kMlpParams + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_mlp_adam, dim3(grid), dim3(kThreads), 0, (hipStream_t)stream, params, grads, m, v,
                       kMlpParams, lr, b1, b2, eps, bc1, bc2);
    return (int)hipGetLastError();
}

int mlp_launch_loss(const float* Y, const float* T, const int* idx, int64_t B, float* out, void* stream)
{
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(kThreads), 0, (hipStream_t)stream, Y, T, idx, B, out);
    return (int)hipGetLastError();
}

}  // namespace qk
