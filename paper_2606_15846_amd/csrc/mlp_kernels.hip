// Kernels of the small bfloat16 perceptrons (the learned reset proposal's
// network): a tiled GEMM on the gfx950 matrix cores with a fused
// bias/activation epilogue, the activation backward, column sums, the squared
// error loss and AdamW.  Accumulation is always float.
#include <math.h>

#include <algorithm>

#include "mlp_internal.hpp"
#include "philox.hpp"

namespace navsim {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 64, kBN = 64, kBK = 32;
constexpr int kLdsK = kBK + 8;  // padded row (80 bytes) of a staged tile
constexpr int kGemmThreads = 256;
constexpr int kColChunk = 32;  // rows per partial column sum

__device__ __forceinline__ uint16_t to_bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;  // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);                    // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16_bits(uint16_t b) {
    return __uint_as_float((uint32_t)b << 16);
}

// Stage rows [r0, r0 + 64) x k [k0, k0 + 32) of a matrix whose element (r, k)
// is X[r ld + k] (kmajor) or X[k ld + r], as T[r][k] in LDS; zeros outside
// [0, R) x [0, K).
template <bool KMAJOR>
__device__ __forceinline__ void stage_tile(uint16_t (*T)[kLdsK], const uint16_t *X, int64_t ld,
                                           int R, int K, int r0, int k0, bool vec_ok, int tid) {
    if (KMAJOR) {
        const int r = tid >> 2, kk = (tid & 3) * 8;
        const int gr = r0 + r, gk = k0 + kk;
        uint16_t v[8];
        if (vec_ok && gr < R && gk + 8 <= K) {
            const uint4 q = *reinterpret_cast<const uint4 *>(X + (int64_t)gr * ld + gk);
            *reinterpret_cast<uint4 *>(&T[r][kk]) = q;
            return;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
            v[j] = (gr < R && gk + j < K) ? X[(int64_t)gr * ld + gk + j] : (uint16_t)0;
#pragma unroll
        for (int j = 0; j < 8; ++j) T[r][kk + j] = v[j];
    } else {
        const int kr = tid >> 3, rr = (tid & 7) * 8;
        const int gk = k0 + kr, gr = r0 + rr;
        uint16_t v[8];
        if (vec_ok && gk < K && gr + 8 <= R) {
            const uint4 q = *reinterpret_cast<const uint4 *>(X + (int64_t)gk * ld + gr);
            const uint16_t *w = reinterpret_cast<const uint16_t *>(&q);
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = w[j];
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                v[j] = (gk < K && gr + j < R) ? X[(int64_t)gk * ld + gr + j] : (uint16_t)0;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) T[rr + j][kr] = v[j];
    }
}

// One workgroup computes a 64 x 64 block of C; each of its four wavefronts a
// 32 x 32 quarter as 2 x 2 tiles of the 16 x 16 x 32 bfloat16 MFMA.
// Fragment layout of v_mfma_f32_16x16x32_bf16: lane l supplies row l % 16 of
// A and column l % 16 of B, k = 8 (l / 16) .. 8 (l / 16) + 7; it receives
// C[4 (l / 16) + r][l % 16], r = 0..3.
template <bool AK, bool BK>
__global__ __launch_bounds__(kGemmThreads) void gemm_kernel(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kBM][kLdsK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kBN][kLdsK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    int M = g.M;
    if (g.m_dev) {
        // rows known only on the device: the grid covers g.M, the rest exits
        const int64_t md = (int64_t)*g.m_dev * g.m_mul;
        M = md < (int64_t)M ? (int)(md > 0 ? md : 0) : M;
        if (m0 >= M) return;
    }
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const bool a_vec = (g.lda % 8 == 0) && (((uintptr_t)g.A & 15) == 0);
    const bool b_vec = (g.ldb % 8 == 0) && (((uintptr_t)g.B & 15) == 0);
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    for (int k0 = 0; k0 < g.K; k0 += kBK) {
        stage_tile<AK>(As, g.A, g.lda, M, g.K, m0, k0, a_vec, tid);
        stage_tile<BK>(Bs, g.B, g.ldb, g.N, g.K, n0, k0, b_vec, tid);
        __syncthreads();
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            a[i] = *reinterpret_cast<const bf16x8 *>(&As[wm + 16 * i + fr][fk]);
            b[i] = *reinterpret_cast<const bf16x8 *>(&Bs[wn + 16 * i + fr][fk]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn + 16 * j + fr;
            if (n >= g.N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + (lane >> 4) * 4 + r;
                if (m >= M) continue;
                float v = acc[i][j][r];
                if (g.bias) v += g.bias[n];
                if (g.bias_rows) v += g.bias_rows[(int64_t)g.row_idx[m] * g.ldbr + n];
                if (g.act == 1 && !(v > 0.0f)) v *= g.slope;
                if (g.act == 2) v = tanhf(v);
                if (g.Cf) g.Cf[(int64_t)m * g.ldcf + n] = v;
                if (g.Cb) g.Cb[(int64_t)m * g.ldcb + n] = to_bf16_bits(v);
            }
        }
}

__global__ void act_backward_kernel(int64_t n, int N, const float *dH, const uint16_t *H, int act,
                                    float slope, float *dZf, uint16_t *dZb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float d = dH[i];
    if (act == 1 && !(from_bf16_bits(H[i]) > 0.0f)) d *= slope;
    if (dZf) dZf[i] = d;
    if (dZb) dZb[i] = to_bf16_bits(d);
}

__global__ void col_sum_chunks_kernel(int M, int N, const float *X, float *partial) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (n >= N) return;
    const int m1 = min(M, (c + 1) * kColChunk);
    float s = 0.0f;
    for (int m = c * kColChunk; m < m1; ++m) s += X[(int64_t)m * N + n];
    partial[(int64_t)c * N + n] = s;
}

__global__ void col_sum_final_kernel(int chunks, int N, const float *partial, float *out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.0f;
    for (int c = 0; c < chunks; ++c) s += partial[(int64_t)c * N + n];
    out[n] = s;
}

__global__ void sq_loss_kernel(int M, int D, const float *Y, const float *T, const float *w,
                               float *L, float *dYf, uint16_t *dYb) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    float l = 0.0f;
    for (int d = 0; d < D; ++d) {
        const float e = Y[(int64_t)m * D + d] - T[(int64_t)m * D + d];
        l += w[d] * (e * e);
        const float gd = (2.0f * w[d] * e) / (float)M;
        if (dYf) dYf[(int64_t)m * D + d] = gd;
        if (dYb) dYb[(int64_t)m * D + d] = to_bf16_bits(gd);
    }
    if (L) L[m] = l;
}

__global__ void adamw_kernel(int64_t n, float *p, uint16_t *pb, const float *g, float *m, float *v,
                             const uint8_t *decay_mask, float lr, float b1, float b2, float eps,
                             float wd, float bc1, float bc2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    float pi = p[i];
    if (!decay_mask || decay_mask[i]) pi = pi * (1.0f - lr * wd);
    pi = pi - lr * ((mi / bc1) / (sqrtf(vi / bc2) + eps));
    p[i] = pi;
    if (pb) pb[i] = to_bf16_bits(pi);
}

__global__ void to_bf16_kernel(int64_t n, const float *x, uint16_t *y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = to_bf16_bits(x[i]);
}

// Actor input: x[e][j] = bf16(1 / (obs[e][j] - beta)) for the m pooled
// ranges (the reciprocal transform), bf16(obs[e][j]) for the 4 goal and
// velocity features.
__global__ void actor_input_kernel(int N, int m, const float *obs, const float *beta,
                                   uint16_t *x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int row = m + 4;
    if (i >= (int64_t)N * row) return;
    const int j = (int)(i % row);
    const float v = obs[i];
    x[i] = to_bf16_bits(j < m ? 1.0f / (v - *beta) : v);
}

// Exploration noise: a = clip(a + std n, -1, 1) with n standard normal from
// Box-Muller on Philox(e, n mod 2^32, n div 2^32, 11) words 0 and 1 at step
// n = *step_ctr + step_off (double precision, rounded to float).
__global__ void actor_noise_kernel(int N, float *act, float std, const uint32_t *step_ctr,
                                   int step_off, uint32_t key0, uint32_t key1) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N) return;
    const uint64_t n = (((uint64_t)step_ctr[1] << 32) | (uint64_t)step_ctr[0]) + (uint64_t)step_off;
    uint32_t c[4] = {(uint32_t)e, (uint32_t)n, (uint32_t)(n >> 32), 11u};
    philox4x32_10(c, key0, key1);
    const double u1 = ((double)c[0] + 0.5) / 4294967296.0, u2 = ((double)c[1] + 0.5) / 4294967296.0;
    const double r = sqrt(-2.0 * log(u1)), t = 2.0 * 3.14159265358979323846 * u2;
    const float n0 = (float)(r * cos(t)), n1 = (float)(r * sin(t));
    float a0 = act[2 * e] + std * n0, a1 = act[2 * e + 1] + std * n1;
    act[2 * e] = fminf(1.0f, fmaxf(-1.0f, a0));
    act[2 * e + 1] = fminf(1.0f, fmaxf(-1.0f, a1));
}

// Whole actor in one launch: a workgroup of 4 wavefronts takes 16 observation
// rows, builds their bf16 inputs in LDS (reciprocal range transform), then
// runs every layer as 16 x 16 x 32 bf16 MFMA tiles, wavefront w taking the
// layer's 16-column blocks w, w + 4, ..., with the weights staged in LDS by
// the workgroup from a padded bf16 image (k-contiguous rows, K padded to 32,
// N to 16, zeros outside), and writes bias + activation to the next layer's
// input rows.  The last layer applies tanh; then one lane per row draws the
// row's exploration noise pair (one Box-Muller transform), adds, clips and
// stores both action components.  Same tiles, k order and rounding points as
// the layer-by-layer GEMM path.
// Threads of the one-launch actor: 8 wavefronts, one 16-column block of a
// layer (<= 128 wide) each, so that a wavefront's serial chain per layer is
// one block's products and epilogue.
constexpr int kActorThreads = 512;
constexpr int kActorWaves = kActorThreads / 64;
constexpr int kActorBlocks = 8 / kActorWaves;  // column blocks per wavefront
constexpr int kActorPasses = 2048 / kActorThreads;  // 16 rows x 128 columns per pass set

__global__ __launch_bounds__(kActorThreads) void actor_fused_kernel(ActorArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint16_t act_lds[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row0 = blockIdx.x * 16;
    const int ld = a.kmax + 8;  // LDS row pitch (bf16): 16 B past a bank cycle
    uint16_t *cur_in = act_lds;        // this layer's input rows [16][ld]
    uint16_t *nxt_in = act_lds + 16 * ld;  // the next layer's
    uint16_t *wl = act_lds + 32 * ld;  // this layer's weights
    float *s_act = reinterpret_cast<float *>(wl + a.wmax);  // [16][2] actions before noise
    const int row = a.m + 4;
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    // A layer's weights and biases go to registers one layer ahead: layer
    // l + 1's loads are in flight while layer l runs on the matrix cores.
    // Weights: np kp / 8 <= 128 * 128 / 8 = 2048 vectors, kActorPasses per
    // thread; rows of kp bf16 stored with pitch kp + 8 (conflict-free fragment
    // reads); thread t copies 16-byte column t % 16 of rows t / 16 + (T / 16) i.
    const int wc = threadIdx.x & 15, wr0 = threadIdx.x >> 4;
    constexpr int kRowStep = kActorThreads / 16;
    uint4 t8[kActorPasses];
    float bias[kActorBlocks];
    auto load_layer = [&](int l) {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.w + a.w_off[l]);
        const int rv = a.kpad[l] / 8, np = a.npad[l];
#pragma unroll
        for (int t = 0; t < kActorPasses; ++t) {
            const int rw = wr0 + kRowStep * t;
            t8[t] = (wc < rv && rw < np) ? src[rw * rv + wc] : make_uint4(0u, 0u, 0u, 0u);
        }
        // this lane's biases, for its wavefront's column blocks (np <= 128)
#pragma unroll
        for (int t = 0; t < kActorBlocks; ++t) {
            const int n0 = 16 * (wave + kActorWaves * t);
            bias[t] = n0 < np ? a.b[a.b_off[l] + n0 + fr] : 0.0f;
        }
    };
    load_layer(0);
    // inputs: 16 rows x kpad[0] (<= 128) columns, kActorPasses per thread, loads first
    {
        const int kp0 = a.kpad[0];
        const float beta = *a.beta;
        float v[kActorPasses];
        // every load in bounds (clamped row and column, N >= 1) and issued
        // back to back; out-of-range entries are then replaced by 0
#pragma unroll
        for (int t = 0; t < kActorPasses; ++t) {
            const int q = threadIdx.x + kActorThreads * t, r = q >> 7, j = q & 127, e = row0 + r;
            v[t] = a.obs[(int64_t)min(e, a.N - 1) * row + min(j, row - 1)];
        }
#pragma unroll
        for (int t = 0; t < kActorPasses; ++t) {
            const int q = threadIdx.x + kActorThreads * t, r = q >> 7, j = q & 127, e = row0 + r;
            if (!(e < a.N && j < row)) v[t] = 0.0f;
        }
#pragma unroll
        for (int t = 0; t < kActorPasses; ++t) {
            const int q = threadIdx.x + kActorThreads * t, r = q >> 7, j = q & 127;
            if (j < kp0)
                cur_in[r * ld + j] =
                    to_bf16_bits(j < a.m && row0 + r < a.N ? 1.0f / (v[t] - beta) : v[t]);
        }
    }
    for (int l = 0; l < a.layers; ++l) {
        const int kp = a.kpad[l], np = a.npad[l];
        {
            uint4 *dst = reinterpret_cast<uint4 *>(wl);
            const int rv = kp / 8;
#pragma unroll
            for (int t = 0; t < kActorPasses; ++t) {
                const int rw = wr0 + kRowStep * t;
                if (wc < rv && rw < np) dst[rw * (rv + 1) + wc] = t8[t];
            }
        }
        float bias_l[kActorBlocks];
#pragma unroll
        for (int t = 0; t < kActorBlocks; ++t) bias_l[t] = bias[t];
        __syncthreads();  // inputs and weights in LDS
        if (l + 1 < a.layers) load_layer(l + 1);
        const uint16_t *W = wl;
        const bool last = l + 1 == a.layers;
        // Every fragment is read before the first product, from positions
        // clamped into this layer's K and N (always in bounds), so the reads
        // share one LDS round trip; products past K are then skipped.
        const int nkb = kp / 32;  // 1..4
        bf16x8 av[4];             // the rows' input fragments, shared by every column block
        bf16x8 bv[kActorBlocks][4];  // this wavefront's column blocks
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
            av[kb] = *reinterpret_cast<const bf16x8 *>(&cur_in[fr * ld + 32 * min(kb, nkb - 1) + fk]);
#pragma unroll
        for (int t = 0; t < kActorBlocks; ++t) {
            const int n0 = min(16 * (wave + kActorWaves * t), np - 16);
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
                bv[t][kb] = *reinterpret_cast<const bf16x8 *>(W + (n0 + fr) * (kp + 8) +
                                                              32 * min(kb, nkb - 1) + fk);
        }
#pragma unroll
        for (int t = 0; t < kActorBlocks; ++t) {
            const int n0 = 16 * (wave + kActorWaves * t);
            if (n0 >= np) break;
            f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
                if (kb < nkb) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[kb], bv[t][kb], acc, 0, 0, 0);
            const int n = n0 + fr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rr = (lane >> 4) * 4 + r;
                float v = acc[r] + bias_l[t];
                if (!last) {
                    if (!(v > 0.0f)) v *= a.slope;
                    nxt_in[rr * ld + n] = to_bf16_bits(v);
                } else if (n < 2) {
                    s_act[rr * 2 + n] = tanhf(v);
                }
            }
        }
        if (!last) {
            // zero the padding columns [np, kpad[l + 1]) of the next input
            const int kn = a.kpad[l + 1], wpad = kn - np;
            for (int q = threadIdx.x; q < 16 * wpad; q += kActorThreads) {
                const int r = q / wpad;
                nxt_in[r * ld + np + (q - r * wpad)] = 0;
            }
            uint16_t *t = cur_in;
            cur_in = nxt_in;
            nxt_in = t;
        }
        __syncthreads();  // next layer's inputs written, this layer's weights no longer read
    }
    // noise, clip and store: one lane per row
    if (threadIdx.x < 16) {
        const int e = row0 + threadIdx.x;
        if (e < a.N) {
            float v0 = s_act[threadIdx.x * 2], v1 = s_act[threadIdx.x * 2 + 1];
            if (a.std > 0.0f) {
                const uint64_t st =
                    (((uint64_t)a.step_ctr[1] << 32) | (uint64_t)a.step_ctr[0]) + (uint64_t)a.step_off;
                uint32_t c[4] = {(uint32_t)e, (uint32_t)st, (uint32_t)(st >> 32), 11u};
                philox4x32_10(c, a.key0, a.key1);
                const double u1 = ((double)c[0] + 0.5) / 4294967296.0;
                const double u2 = ((double)c[1] + 0.5) / 4294967296.0;
                const double rad = sqrt(-2.0 * log(u1));
                const double t = 2.0 * 3.14159265358979323846 * u2;
                v0 = fminf(1.0f, fmaxf(-1.0f, v0 + a.std * (float)(rad * cos(t))));
                v1 = fminf(1.0f, fmaxf(-1.0f, v1 + a.std * (float)(rad * sin(t))));
            }
            a.act[(int64_t)e * 2] = v0;
            a.act[(int64_t)e * 2 + 1] = v1;
        }
    }
}

unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

size_t actor_fused_lds_bytes(int layers, const int *kpad, const int *npad, int kmax) {
    return ((size_t)32 * (kmax + 8) + (size_t)actor_fused_wmax(layers, kpad, npad)) *
               sizeof(uint16_t) +
           16 * 2 * sizeof(float);
}

int actor_fused_wmax(int layers, const int *kpad, const int *npad) {
    int wmax = 0;
    for (int l = 0; l < layers; ++l) wmax = std::max(wmax, (kpad[l] + 8) * npad[l]);
    return (wmax + 7) & ~7;  // keeps the action floats after it 16-byte aligned
}

hipError_t launch_actor_fused(const ActorArgs &a, hipStream_t s) {
    if (a.N <= 0) return hipSuccess;
    const size_t lds = actor_fused_lds_bytes(a.layers, a.kpad, a.npad, a.kmax);
    hipLaunchKernelGGL(actor_fused_kernel, dim3((unsigned)((a.N + 15) / 16)), dim3(kActorThreads), lds,
                       s, a);
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs &g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    const dim3 grid((unsigned)((g.N + kBN - 1) / kBN), (unsigned)((g.M + kBM - 1) / kBM));
    if (g.a_kmajor && g.b_kmajor)
        hipLaunchKernelGGL((gemm_kernel<true, true>), grid, dim3(kGemmThreads), 0, s, g);
    else if (g.a_kmajor)
        hipLaunchKernelGGL((gemm_kernel<true, false>), grid, dim3(kGemmThreads), 0, s, g);
    else if (g.b_kmajor)
        hipLaunchKernelGGL((gemm_kernel<false, true>), grid, dim3(kGemmThreads), 0, s, g);
    else
        hipLaunchKernelGGL((gemm_kernel<false, false>), grid, dim3(kGemmThreads), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_act_backward(int M, int N, const float *dH, const uint16_t *H, int act,
                               float slope, float *dZf, uint16_t *dZb, hipStream_t s) {
    const int64_t n = (int64_t)M * N;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(act_backward_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, N, dH, H,
                       act, slope, dZf, dZb);
    return hipGetLastError();
}

hipError_t launch_col_sum(int M, int N, const float *X, float *partial, float *out,
                          hipStream_t s) {
    if (N == 0) return hipSuccess;
    const int chunks = (M + kColChunk - 1) / kColChunk;
    if (chunks > 0)
        hipLaunchKernelGGL(col_sum_chunks_kernel, dim3(blocks_for(N, 256), (unsigned)chunks),
                           dim3(256), 0, s, M, N, X, partial);
    hipLaunchKernelGGL(col_sum_final_kernel, dim3(blocks_for(N, 256)), dim3(256), 0, s, chunks, N,
                       partial, out);
    return hipGetLastError();
}

hipError_t launch_sq_loss(int M, int D, const float *Y, const float *T, const float *w,
                          float *L, float *dYf, uint16_t *dYb, hipStream_t s) {
    if (M == 0) return hipSuccess;
    hipLaunchKernelGGL(sq_loss_kernel, dim3(blocks_for(M, 256)), dim3(256), 0, s, M, D, Y, T, w,
                       L, dYf, dYb);
    return hipGetLastError();
}

hipError_t launch_adamw(int64_t n, float *p, uint16_t *pb, const float *g, float *m, float *v,
                        const uint8_t *decay_mask, float lr, float b1, float b2, float eps,
                        float wd, int64_t t, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const float bc1 = (float)(1.0 - pow((double)b1, (double)t));
    const float bc2 = (float)(1.0 - pow((double)b2, (double)t));
    hipLaunchKernelGGL(adamw_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, p, pb, g, m, v,
                       decay_mask, lr, b1, b2, eps, wd, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_actor_input(int N, int m, const float *obs, const float *beta, uint16_t *x,
                              hipStream_t s) {
    const int64_t n = (int64_t)N * (m + 4);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(actor_input_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, N, m, obs,
                       beta, x);
    return hipGetLastError();
}

hipError_t launch_actor_noise(int N, float *act, float std, const uint32_t *step_ctr, int step_off,
                              uint32_t key0, uint32_t key1, hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(actor_noise_kernel, dim3(blocks_for(N, 256)), dim3(256), 0, s, N, act, std,
                       step_ctr, step_off, key0, key1);
    return hipGetLastError();
}

hipError_t launch_to_bf16(int64_t n, const float *x, uint16_t *y, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, x, y);
    return hipGetLastError();
}

}  // namespace navsim
