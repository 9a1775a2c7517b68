// Small multilayer perceptrons on bfloat16 matrix cores: host-side launch
// interface of mlp_kernels.hip (library internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace navsim {

// C[m, n] = sum_k A(m, k) B(n, k), bfloat16 operands, float accumulation.
// A(m, k) = A[m lda + k] when a_kmajor, else A[k lda + m]; B likewise.
// Epilogue: + bias[n] (optional) + bias_rows[row_idx[m] ldbr + n] (optional),
// activation (0 none, 1 leaky ReLU with `slope`, 2 tanh), then stored as float to Cf
// and/or as bfloat16 (round to nearest even) to Cb.
struct GemmArgs {
    int M = 0, N = 0, K = 0;
    const uint16_t *A = nullptr;
    int64_t lda = 0;
    bool a_kmajor = true;
    const uint16_t *B = nullptr;
    int64_t ldb = 0;
    bool b_kmajor = true;
    const float *bias = nullptr;
    const float *bias_rows = nullptr;
    const int32_t *row_idx = nullptr;
    int64_t ldbr = 0;
    int act = 0;
    float slope = 0.0f;
    float *Cf = nullptr;
    int64_t ldcf = 0;
    uint16_t *Cb = nullptr;
    int64_t ldcb = 0;
    // optional: rows = min(M, *m_dev * m_mul), read on the device (the grid
    // still covers M rows; workgroups past the rows return at once)
    const int32_t *m_dev = nullptr;
    int m_mul = 1;
};

hipError_t launch_gemm(const GemmArgs &g, hipStream_t s);

// dZ = dH * act'(H) for leaky ReLU (H is the layer's bfloat16 output, whose
// sign is that of its input); writes float dZf and bfloat16 dZb, [M, N] rows
// of stride ld.  act 0: dZ = dH.
hipError_t launch_act_backward(int M, int N, const float *dH, const uint16_t *H, int act,
                               float slope, float *dZf, uint16_t *dZb, hipStream_t s);

// out[n] = sum over m of X[m, n] (float, [M, N] rows), in a fixed order:
// chunks of 32 rows in order, then the chunk sums in order.  `partial`
// holds ceil(M / 32) * N floats.
hipError_t launch_col_sum(int M, int N, const float *X, float *partial, float *out,
                          hipStream_t s);

// Weighted squared error of outputs Y [M, D] to targets T [M, D]: row loss
// L[m] = sum_d w[d] (Y - T)^2 and dY = 2 w (Y - T) / M (float and bfloat16).
hipError_t launch_sq_loss(int M, int D, const float *Y, const float *T, const float *w,
                          float *L, float *dYf, uint16_t *dYb, hipStream_t s);

// AdamW (decoupled weight decay): for i < n,
//   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
//   p = p (1 - lr wd) - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
// decay applied where decay_mask[i] != 0; pb = bfloat16(p).
hipError_t launch_adamw(int64_t n, float *p, uint16_t *pb, const float *g, float *m, float *v,
                        const uint8_t *decay_mask, float lr, float b1, float b2, float eps,
                        float wd, int64_t t, hipStream_t s);

// Actor input rows [N][m + 4] in bfloat16: 1 / (obs - beta) for the m pooled
// ranges (reciprocal transform, beta device scalar), the 4 other features as
// they are.
hipError_t launch_actor_input(int N, int m, const float *obs, const float *beta, uint16_t *x,
                              hipStream_t s);

// Gaussian exploration noise on actions [N][2], clipped to [-1, 1]; the step
// index is *step_ctr (device {lo, hi}) + step_off.
hipError_t launch_actor_noise(int N, float *act, float std, const uint32_t *step_ctr, int step_off,
                              uint32_t key0, uint32_t key1, hipStream_t s);

// The whole actor in one launch (inputs, every layer, tanh, noise): weights
// as a padded bf16 image, layer l [npad[l]][kpad[l]] at w_off[l], zeros in
// the padding; npad[l] <= kpad[l + 1]; kpad and kmax multiples of 32, npad of
// 16, kmax >= every kpad.
constexpr int kActorMaxLayers = 5;
struct ActorArgs {
    int N = 0, m = 0, layers = 0, kmax = 0;
    int wmax = 0;  // actor_fused_wmax: bf16 elements of the largest padded weight block
    int kpad[kActorMaxLayers] = {}, npad[kActorMaxLayers] = {};
    int64_t w_off[kActorMaxLayers] = {}, b_off[kActorMaxLayers] = {};
    const uint16_t *w = nullptr;
    const float *b = nullptr;  // biases, padded with zeros to npad
    const float *beta = nullptr;
    const float *obs = nullptr;
    float *act = nullptr;
    float slope = 0.01f, std = 0.0f;
    const uint32_t *step_ctr = nullptr;
    int step_off = 0;
    uint32_t key0 = 0, key1 = 0;
};
hipError_t launch_actor_fused(const ActorArgs &a, hipStream_t s);
// LDS bytes of that launch: two [16][kmax + 8] bf16 activation buffers, the
// largest layer's padded weights and 16 action pairs (it is used only when
// this is <= 64 KiB).
size_t actor_fused_lds_bytes(int layers, const int *kpad, const int *npad, int kmax);
int actor_fused_wmax(int layers, const int *kpad, const int *npad);

// Float to bfloat16 (round to nearest even), n elements.
hipError_t launch_to_bf16(int64_t n, const float *x, uint16_t *y, hipStream_t s);

}  // namespace navsim
