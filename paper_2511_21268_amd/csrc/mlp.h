// Small MLP (8 -> 64 -> 64 -> 4, tanh hidden layers) that maps the features of
// one AMG level to the coefficients of its degree-4 polynomial smoother.
// Weights are held in BF16 on the device (used by forward and backward) with an
// FP32 master copy updated by Adam; all accumulation is FP32.  Every reduction
// over samples is a fixed-order loop, so training is deterministic.
//
// Parameter vector (MLP_NPARAM entries):
//   W1[64][8] b1[64] W2[64][64] b2[64] W3[4][64] b3[4]
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amgk {

constexpr int MLP_IN = 8, MLP_H = 64, MLP_OUT = 4;
constexpr int MLP_W1 = 0, MLP_B1 = MLP_W1 + MLP_H * MLP_IN, MLP_W2 = MLP_B1 + MLP_H,
              MLP_B2 = MLP_W2 + MLP_H * MLP_H, MLP_W3 = MLP_B2 + MLP_H, MLP_B3 = MLP_W3 + MLP_OUT * MLP_H,
              MLP_NPARAM = MLP_B3 + MLP_OUT;
constexpr int MLP_ACT = 2 * MLP_H;                    // stored activations per sample (h1, h2)
constexpr int MLP_DEL = MLP_OUT + 2 * MLP_H;          // stored deltas per sample (dy, dh2, dh1)

__device__ inline float bf16_to_f32(uint16_t b) { return __uint_as_float(((unsigned)b) << 16); }

// round to nearest even; NaN stays NaN
__device__ inline uint16_t f32_to_bf16(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// One thread per sample: Y = W3 tanh(W2 tanh(W1 x + b1) + b2) + b3.
__global__ __launch_bounds__(64) void k_mlp_fwd(const uint16_t *__restrict__ w, const float *__restrict__ X, int B,
                                                float *__restrict__ Y, float *__restrict__ act)
{
    int s = blockIdx.x * 64 + threadIdx.x;
    if (s >= B) return;
    float x[MLP_IN], h1[MLP_H], h2[MLP_H];
    for (int j = 0; j < MLP_IN; j++) x[j] = X[s * MLP_IN + j];
    for (int i = 0; i < MLP_H; i++) {
        float a = bf16_to_f32(w[MLP_B1 + i]);
        for (int j = 0; j < MLP_IN; j++) a = fmaf(bf16_to_f32(w[MLP_W1 + i * MLP_IN + j]), x[j], a);
        h1[i] = tanhf(a);
    }
    for (int i = 0; i < MLP_H; i++) {
        float a = bf16_to_f32(w[MLP_B2 + i]);
        for (int j = 0; j < MLP_H; j++) a = fmaf(bf16_to_f32(w[MLP_W2 + i * MLP_H + j]), h1[j], a);
        h2[i] = tanhf(a);
    }
    for (int i = 0; i < MLP_OUT; i++) {
        float a = bf16_to_f32(w[MLP_B3 + i]);
        for (int j = 0; j < MLP_H; j++) a = fmaf(bf16_to_f32(w[MLP_W3 + i * MLP_H + j]), h2[j], a);
        Y[s * MLP_OUT + i] = a;
    }
    if (act) {
        for (int i = 0; i < MLP_H; i++) { act[s * MLP_ACT + i] = h1[i]; act[s * MLP_ACT + MLP_H + i] = h2[i]; }
    }
}

// Per-sample back-propagation of the loss L = mean over samples and outputs of
// (Y - T)^2: dy = 2 (y - t) / (4 B), dh2 = W3^T dy * (1 - h2^2),
// dh1 = W2^T dh2 * (1 - h1^2).
__global__ __launch_bounds__(64) void k_mlp_delta(const uint16_t *__restrict__ w, const float *__restrict__ act,
                                                  const float *__restrict__ Y, const float *__restrict__ T, int B,
                                                  float *__restrict__ del)
{
    int s = blockIdx.x * 64 + threadIdx.x;
    if (s >= B) return;
    const float *h1 = act + s * MLP_ACT, *h2 = h1 + MLP_H;
    float dy[MLP_OUT], dh2[MLP_H];
    const float scale = 2.0f / (float)(MLP_OUT * B);
    for (int i = 0; i < MLP_OUT; i++) dy[i] = scale * (Y[s * MLP_OUT + i] - T[s * MLP_OUT + i]);
    for (int j = 0; j < MLP_H; j++) {
        float a = 0.0f;
        for (int i = 0; i < MLP_OUT; i++) a = fmaf(bf16_to_f32(w[MLP_W3 + i * MLP_H + j]), dy[i], a);
        dh2[j] = a * (1.0f - h2[j] * h2[j]);
    }
    float *d = del + s * MLP_DEL;
    for (int i = 0; i < MLP_OUT; i++) d[i] = dy[i];
    for (int j = 0; j < MLP_H; j++) d[MLP_OUT + j] = dh2[j];
    for (int j = 0; j < MLP_H; j++) {
        float a = 0.0f;
        for (int i = 0; i < MLP_H; i++) a = fmaf(bf16_to_f32(w[MLP_W2 + i * MLP_H + j]), dh2[i], a);
        d[MLP_OUT + MLP_H + j] = a * (1.0f - h1[j] * h1[j]);
    }
}

// Gradient of every parameter: one thread per parameter, samples summed in
// index order.  Thread 0 also writes the loss.
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ X, const float *__restrict__ act,
                                                  const float *__restrict__ del, const float *__restrict__ Y,
                                                  const float *__restrict__ T, int B, float *__restrict__ grad,
                                                  float *__restrict__ loss)
{
    int p = blockIdx.x * 256 + threadIdx.x;
    if (p == 0 && loss) {
        float l = 0.0f;
        for (int s = 0; s < B; s++)
            for (int i = 0; i < MLP_OUT; i++) {
                float e = Y[s * MLP_OUT + i] - T[s * MLP_OUT + i];
                l = fmaf(e, e, l);
            }
        *loss = l / (float)(MLP_OUT * B);
    }
    if (p >= MLP_NPARAM) return;
    float g = 0.0f;
    if (p < MLP_B1) {                       // W1[i][j] : dh1[i] x[j]
        int i = (p - MLP_W1) / MLP_IN, j = (p - MLP_W1) % MLP_IN;
        for (int s = 0; s < B; s++) g = fmaf(del[s * MLP_DEL + MLP_OUT + MLP_H + i], X[s * MLP_IN + j], g);
    } else if (p < MLP_W2) {                // b1[i]
        int i = p - MLP_B1;
        for (int s = 0; s < B; s++) g += del[s * MLP_DEL + MLP_OUT + MLP_H + i];
    } else if (p < MLP_B2) {                // W2[i][j] : dh2[i] h1[j]
        int i = (p - MLP_W2) / MLP_H, j = (p - MLP_W2) % MLP_H;
        for (int s = 0; s < B; s++) g = fmaf(del[s * MLP_DEL + MLP_OUT + i], act[s * MLP_ACT + j], g);
    } else if (p < MLP_W3) {                // b2[i]
        int i = p - MLP_B2;
        for (int s = 0; s < B; s++) g += del[s * MLP_DEL + MLP_OUT + i];
    } else if (p < MLP_B3) {                // W3[i][j] : dy[i] h2[j]
        int i = (p - MLP_W3) / MLP_H, j = (p - MLP_W3) % MLP_H;
        for (int s = 0; s < B; s++) g = fmaf(del[s * MLP_DEL + i], act[s * MLP_ACT + MLP_H + j], g);
    } else {                                // b3[i]
        int i = p - MLP_B3;
        for (int s = 0; s < B; s++) g += del[s * MLP_DEL + i];
    }
    grad[p] = g;
}

// Adam on the FP32 master weights, then the BF16 copy (round to nearest even).
__global__ void k_mlp_adam(float *__restrict__ master, uint16_t *__restrict__ w, const float *__restrict__ grad,
                           float *__restrict__ m, float *__restrict__ v, int step, float lr, float b1, float b2,
                           float eps)
{
    int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    if (step > 0) {
        float g = grad[p];
        float mp = b1 * m[p] + (1.0f - b1) * g;
        float vp = b2 * v[p] + (1.0f - b2) * g * g;
        m[p] = mp;
        v[p] = vp;
        float mh = mp / (1.0f - powf(b1, (float)step));
        float vh = vp / (1.0f - powf(b2, (float)step));
        master[p] = master[p] - lr * mh / (sqrtf(vh) + eps);
    }
    w[p] = f32_to_bf16(master[p]);
}

}  // namespace amgk
