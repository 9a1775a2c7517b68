// Host side of the policy in the loop (C ABI in include/navsim_policy.h): the
// actor's parameters, its forward pass as matrix-core GEMMs with fused
// epilogues, and rollouts that alternate actor and step launches, optionally
// captured once into a HIP graph.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "mlp_internal.hpp"
#include "navsim_host.hpp"
#include "navsim_policy.h"

using namespace navsim;

struct navsim_policy_s {
    navsim_t h = nullptr;
    int device = 0, N = 0, m = 0, L = 0;
    float slope = 0.01f;
    std::vector<int32_t> dims;
    std::vector<int64_t> w_off, b_off;
    int64_t beta_off = 0, nparams = 0;
    float *p = nullptr;
    uint16_t *pb = nullptr;
    uint16_t *x = nullptr, *hid[2] = {nullptr, nullptr};
    uint32_t *step_ctr = nullptr;
    // one-launch actor: padded bf16 weights and padded biases
    bool fused = false;
    ActorArgs fa{};
    uint16_t *wpad = nullptr;
    float *bpad = nullptr;
    // captured rollout
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    StepParams graph_params{};
    const float *graph_obs0 = nullptr;
    float graph_std = 0.0f;
    int graph_steps = 0, graph_kernel = -1, graph_tile_envs = 0;
};

namespace {

void drop_policy_graph(navsim_policy_s *q) {
    if (q->graph) (void)hipGraphExecDestroy(q->graph);
    q->graph = nullptr;
    q->graph_steps = 0;
}

// act = actor(obs) (+ noise at step index *step_ctr + step_off).
navsim_status actor_forward(navsim_policy_s *q, const float *obs, float *act, float std,
                            int step_off, hipStream_t s) {
    if (q->fused) {
        ActorArgs a = q->fa;
        a.obs = obs;
        a.act = act;
        a.std = std;
        a.step_off = step_off;
        NS_HIP(launch_actor_fused(a, s));
        return NAVSIM_OK;
    }
    NS_HIP(launch_actor_input(q->N, q->m, obs, q->p + q->beta_off, q->x, s));
    const uint16_t *in = q->x;
    for (int l = 0; l < q->L; ++l) {
        GemmArgs g;
        g.M = q->N;
        g.N = q->dims[l + 1];
        g.K = q->dims[l];
        g.A = in;
        g.lda = q->dims[l];
        g.B = q->pb + q->w_off[l];
        g.ldb = q->dims[l];
        g.bias = q->p + q->b_off[l];
        if (l + 1 < q->L) {
            g.act = 1;
            g.slope = q->slope;
            g.Cb = q->hid[l & 1];
            g.ldcb = g.N;
            in = q->hid[l & 1];
        } else {
            g.act = 2;
            g.Cf = act;
            g.ldcf = 2;
        }
        NS_HIP(launch_gemm(g, s));
    }
    if (std > 0.0f)
        NS_HIP(launch_actor_noise(q->N, act, std, q->step_ctr, step_off,
                                  (uint32_t)(q->h->cfg.seed & 0xffffffffu),
                                  (uint32_t)(q->h->cfg.seed >> 32), s));
    return NAVSIM_OK;
}

navsim_status policy_steps(navsim_t h, navsim_policy_s *q, const StepParams &p0, int steps,
                           const float *obs0, float std, int kernel, hipStream_t s) {
    const int64_t N = h->cfg.num_envs;
    const int row = h->cfg.num_sectors + 4;
    for (int i = 0; i < steps; ++i) {
        StepParams p = p0;
        p.act_out = nullptr;
        p.act = p0.act_out + (int64_t)i * N * 2;
        p.obs += (int64_t)i * N * row;
        p.reward += (int64_t)i * N;
        p.term += (int64_t)i * N;
        p.trunc += (int64_t)i * N;
        if (p.final_obs) p.final_obs += (int64_t)i * N * row;
        const float *in = i == 0 ? obs0 : p0.obs + (int64_t)(i - 1) * N * row;
        navsim_status st = actor_forward(q, in, p0.act_out + (int64_t)i * N * 2, std, i, s);
        if (st != NAVSIM_OK) return st;
        const hipError_t e =
            kernel == NAVSIM_KERNEL_PLAIN ? launch_plain(p, s) : launch_fused(p, h->tile_envs, s);
        if (e != hipSuccess) return fail(NAVSIM_E_HIP, "kernel launch: %s", hipGetErrorString(e));
    }
    return NAVSIM_OK;
}

}  // namespace

extern "C" {

navsim_status navsim_policy_create(navsim_t h, int32_t hidden, int32_t hidden_layers,
                                   float leaky_slope, navsim_policy_t *out) {
    if (!out) return fail(NAVSIM_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!h) return fail(NAVSIM_E_BAD_HANDLE, "handle is NULL");
    if (hidden < 1 || hidden > 1024 || hidden_layers < 1 || hidden_layers > 4 ||
        !finite_pos(leaky_slope))
        return fail(NAVSIM_E_INVALID_ARG,
                    "need hidden in 1..1024, hidden_layers in 1..4, leaky_slope > 0");
    DeviceGuard dg(h->device);
    if (dg.err != hipSuccess) return fail(NAVSIM_E_HIP, "hipSetDevice: %s", hipGetErrorString(dg.err));
    navsim_policy_s *q = new (std::nothrow) navsim_policy_s();
    if (!q) return fail(NAVSIM_E_OOM, "host allocation failed");
    q->h = h;
    q->device = h->device;
    q->N = h->cfg.num_envs;
    q->m = h->cfg.num_sectors;
    q->slope = leaky_slope;
    q->L = hidden_layers + 1;
    q->dims.push_back(q->m + 4);
    for (int l = 0; l < hidden_layers; ++l) q->dims.push_back(hidden);
    q->dims.push_back(2);
    int64_t off = 0;
    for (int l = 0; l < q->L; ++l) {
        q->w_off.push_back(off);
        off = (off + (int64_t)q->dims[l + 1] * q->dims[l] + 7) & ~(int64_t)7;
        q->b_off.push_back(off);
        off = (off + q->dims[l + 1] + 7) & ~(int64_t)7;
    }
    q->beta_off = off;
    q->nparams = off + 8;
    // the one-launch actor when every layer fits 128 inputs
    int kmax = 0;
    q->fused = q->L <= kActorMaxLayers;
    int64_t wo = 0, bo = 0;
    for (int l = 0; l < q->L && q->fused; ++l) {
        q->fa.kpad[l] = (q->dims[l] + 31) & ~31;
        q->fa.npad[l] = (q->dims[l + 1] + 15) & ~15;
        q->fa.w_off[l] = wo;
        q->fa.b_off[l] = bo;
        wo += (int64_t)q->fa.kpad[l] * q->fa.npad[l];
        bo += q->fa.npad[l];
        kmax = std::max(kmax, q->fa.kpad[l]);
        q->fused = q->fa.kpad[l] <= 128;
    }
    q->fused = q->fused && actor_fused_lds_bytes(q->L, q->fa.kpad, q->fa.npad, kmax) <= 65536;
    const size_t N = (size_t)q->N;
    bool ok = hipMalloc((void **)&q->p, (size_t)q->nparams * 4) == hipSuccess &&
              hipMalloc((void **)&q->pb, (size_t)q->nparams * 2) == hipSuccess &&
              hipMalloc((void **)&q->x, N * (q->m + 4) * 2) == hipSuccess &&
              hipMalloc((void **)&q->hid[0], N * hidden * 2) == hipSuccess &&
              hipMalloc((void **)&q->hid[1], N * hidden * 2) == hipSuccess &&
              hipMalloc((void **)&q->step_ctr, 8) == hipSuccess;
    ok = ok && hipMemset(q->p, 0, (size_t)q->nparams * 4) == hipSuccess &&
         hipMemset(q->pb, 0, (size_t)q->nparams * 2) == hipSuccess &&
         hipMemset(q->step_ctr, 0, 8) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    if (ok && q->fused) {
        ok = hipMalloc((void **)&q->wpad, (size_t)wo * 2) == hipSuccess &&
             hipMalloc((void **)&q->bpad, (size_t)bo * 4) == hipSuccess &&
             hipMemset(q->wpad, 0, (size_t)wo * 2) == hipSuccess &&
             hipMemset(q->bpad, 0, (size_t)bo * 4) == hipSuccess &&
             hipDeviceSynchronize() == hipSuccess;
        ActorArgs &a = q->fa;
        a.N = q->N;
        a.m = q->m;
        a.layers = q->L;
        a.kmax = kmax;
        a.wmax = actor_fused_wmax(q->L, a.kpad, a.npad);
        a.w = q->wpad;
        a.b = q->bpad;
        a.beta = q->p + q->beta_off;
        a.slope = q->slope;
        a.step_ctr = q->step_ctr;
        a.key0 = (uint32_t)(h->cfg.seed & 0xffffffffu);
        a.key1 = (uint32_t)(h->cfg.seed >> 32);
    }
    if (!ok) {
        (void)navsim_policy_destroy(q);
        return fail(NAVSIM_E_OOM, "allocating the actor failed");
    }
    *out = q;
    return NAVSIM_OK;
}

navsim_status navsim_policy_layout(navsim_policy_t q, int32_t *num_layers, int32_t *dims,
                                   int64_t *offsets, int64_t *count) {
    if (!q) return fail(NAVSIM_E_BAD_HANDLE, "policy is NULL");
    if (num_layers) *num_layers = q->L;
    if (count) *count = q->nparams;
    if (dims)
        for (int l = 0; l <= q->L; ++l) dims[l] = q->dims[l];
    if (offsets) {
        for (int l = 0; l < q->L; ++l) {
            offsets[2 * l] = q->w_off[l];
            offsets[2 * l + 1] = q->b_off[l];
        }
        offsets[2 * q->L] = q->beta_off;
    }
    return NAVSIM_OK;
}

navsim_status navsim_policy_set_params(navsim_policy_t q, const float *host, int64_t count) {
    if (!q) return fail(NAVSIM_E_BAD_HANDLE, "policy is NULL");
    if (!host || count != q->nparams)
        return fail(NAVSIM_E_INVALID_ARG, "host buffer of %lld floats required",
                    (long long)q->nparams);
    DeviceGuard dg(q->device);
    NS_HIP(hipDeviceSynchronize());
    NS_HIP(hipMemcpy(q->p, host, (size_t)count * 4, hipMemcpyHostToDevice));
    NS_HIP(launch_to_bf16(count, q->p, q->pb, nullptr));
    if (q->fused) {
        // padded images for the one-launch actor (same bf16 rounding as the
        // layer-by-layer path: nearest even)
        std::vector<uint16_t> w((size_t)q->fa.w_off[q->L - 1] +
                                    (size_t)q->fa.npad[q->L - 1] * q->fa.kpad[q->L - 1],
                                0);
        std::vector<float> b((size_t)q->fa.b_off[q->L - 1] + q->fa.npad[q->L - 1], 0.0f);
        for (int l = 0; l < q->L; ++l) {
            for (int o = 0; o < q->dims[l + 1]; ++o) {
                for (int i = 0; i < q->dims[l]; ++i) {
                    uint32_t u;
                    const float f = host[q->w_off[l] + (int64_t)o * q->dims[l] + i];
                    memcpy(&u, &f, 4);
                    uint16_t bits;
                    if ((u & 0x7fffffffu) > 0x7f800000u)
                        bits = 0x7fc0u;
                    else
                        bits = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
                    w[q->fa.w_off[l] + (int64_t)o * q->fa.kpad[l] + i] = bits;
                }
                b[q->fa.b_off[l] + o] = host[q->b_off[l] + o];
            }
        }
        NS_HIP(hipMemcpy(q->wpad, w.data(), w.size() * 2, hipMemcpyHostToDevice));
        NS_HIP(hipMemcpy(q->bpad, b.data(), b.size() * 4, hipMemcpyHostToDevice));
    }
    NS_HIP(hipDeviceSynchronize());
    return NAVSIM_OK;
}

navsim_status navsim_policy_act(navsim_policy_t q, const float *obs, float *act, float noise_std,
                                uint64_t step, void *stream) {
    if (!q) return fail(NAVSIM_E_BAD_HANDLE, "policy is NULL");
    if (!obs || !act) return fail(NAVSIM_E_INVALID_ARG, "obs and act are required");
    if (!(noise_std >= 0.0f) || !isfinite(noise_std))
        return fail(NAVSIM_E_INVALID_ARG, "noise_std must be finite and >= 0");
    DeviceGuard dg(q->device);
    const hipStream_t s = (hipStream_t)stream;
    NS_HIP(launch_set_step(q->step_ctr, step, s));
    return actor_forward(q, obs, act, noise_std, 0, s);
}

navsim_status navsim_policy_rollout(navsim_t h, navsim_policy_t q, int32_t steps,
                                    uint64_t first_step, const float *obs0, float noise_std,
                                    float *act, float *obs, float *reward, uint8_t *terminated,
                                    uint8_t *truncated, float *final_obs, int32_t kernel,
                                    int32_t flags, void *stream) {
    if (!h) return fail(NAVSIM_E_BAD_HANDLE, "handle is NULL");
    if (!q || q->h != h) return fail(NAVSIM_E_BAD_HANDLE, "policy is NULL or of another handle");
    if (!h->loaded) return fail(NAVSIM_E_STATE, "navsim_load_maps has not been called");
    if (!h->initialized) return fail(NAVSIM_E_STATE, "navsim_reset (mask NULL) must come first");
    if (steps < 1 || steps > 4096) return fail(NAVSIM_E_INVALID_ARG, "steps must be in 1..4096");
    if (!obs0 || !act || !obs || !reward || !terminated || !truncated)
        return fail(NAVSIM_E_INVALID_ARG,
                    "obs0, act, obs, reward, terminated, truncated are required");
    if (kernel != NAVSIM_KERNEL_FUSED && kernel != NAVSIM_KERNEL_PLAIN)
        return fail(NAVSIM_E_INVALID_ARG, "unknown kernel %d", kernel);
    if (flags & ~NAVSIM_ROLLOUT_GRAPH) return fail(NAVSIM_E_INVALID_ARG, "unknown flags 0x%x", flags);
    if (h->hook.run)
        return fail(NAVSIM_E_UNSUPPORTED,
                    "rollouts use the in-kernel sampler: detach the reset proposer first");
    if (!(noise_std >= 0.0f) || !isfinite(noise_std))
        return fail(NAVSIM_E_INVALID_ARG, "noise_std must be finite and >= 0");
    DeviceGuard dg(h->device);
    if (dg.err != hipSuccess) return fail(NAVSIM_E_HIP, "hipSetDevice: %s", hipGetErrorString(dg.err));
    StepParams p = make_step_params(h);
    p.mode = 0;
    p.act_out = act;  // the actions buffer; each step reads its row
    p.obs = obs;
    p.reward = reward;
    p.term = terminated;
    p.trunc = truncated;
    p.final_obs = final_obs;
    const hipStream_t s = (hipStream_t)stream;
    NS_HIP(launch_set_step(q->step_ctr, first_step, s));
    if (!(flags & NAVSIM_ROLLOUT_GRAPH)) return policy_steps(h, q, p, steps, obs0, noise_std, kernel, s);
    // every launch parameter (buffers, maps, settings) is part of the key
    const bool same = q->graph && q->graph_steps == steps && q->graph_kernel == kernel &&
                      q->graph_tile_envs == h->tile_envs && q->graph_obs0 == obs0 &&
                      q->graph_std == noise_std &&
                      memcmp(&q->graph_params, &p, sizeof p) == 0;
    if (!same) {
        drop_policy_graph(q);
        if (!q->capture_stream)
            NS_HIP(hipStreamCreateWithFlags(&q->capture_stream, hipStreamNonBlocking));
        NS_HIP(hipStreamBeginCapture(q->capture_stream, hipStreamCaptureModeThreadLocal));
        const navsim_status st =
            policy_steps(h, q, p, steps, obs0, noise_std, kernel, q->capture_stream);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(q->capture_stream, &graph);
        if (st != NAVSIM_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess)
            return fail(NAVSIM_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        hipGraphExec_t exec = nullptr;
        const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e2 != hipSuccess)
            return fail(NAVSIM_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
        q->graph = exec;
        q->graph_params = p;
        q->graph_steps = steps;
        q->graph_kernel = kernel;
        q->graph_tile_envs = h->tile_envs;
        q->graph_obs0 = obs0;
        q->graph_std = noise_std;
    }
    NS_HIP(hipGraphLaunch(q->graph, s));
    return NAVSIM_OK;
}

navsim_status navsim_policy_destroy(navsim_policy_t q) {
    if (!q) return fail(NAVSIM_E_BAD_HANDLE, "policy is NULL");
    {
        DeviceGuard dg(q->device);
        (void)hipDeviceSynchronize();
        drop_policy_graph(q);
        void *ptrs[] = {q->p, q->pb, q->x, q->hid[0], q->hid[1], q->step_ctr, q->wpad, q->bpad};
        for (void *v : ptrs)
            if (v) (void)hipFree(v);
        if (q->capture_stream) (void)hipStreamDestroy(q->capture_stream);
    }
    delete q;
    return NAVSIM_OK;
}

}  // extern "C"
