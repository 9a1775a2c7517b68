// Host side of the learned reset proposal (C ABI in
// include/navsim_reset_proposal.h): C-free bitsets, pooled map inputs,
// difficulty-bin tables, the network's parameters and optimiser state, and
// the sequences of kernel launches for labelling, training and proposing.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <random>
#include <vector>

#include "mlp_internal.hpp"
#include "navsim_host.hpp"
#include "navsim_reset_proposal.h"
#include "reach_internal.hpp"
#include "rp_scratch.hpp"

using namespace navsim;

namespace {

// Device buffer that grows on demand.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t n) {
        if (n <= bytes) return hipSuccess;
        if (p) {
            // earlier launches may still use the old buffer
            const hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return e;
            (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
        const hipError_t e = hipMalloc(&p, n);
        if (e == hipSuccess) bytes = n;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T *as() const {
        return (T *)p;
    }
};

// Bin of a hop count: the same double-precision comparisons the header
// states (d = h s against d_lo + k w and d_lo + (k + 1) w).
int bin_of(double s, int h, double lo, double hi, int nb) {
    if (h < 0) return -1;
    const double d = (double)h * s;
    const double w = (hi - lo) / (double)nb;
    for (int k = 0; k < nb; ++k)
        if (d >= lo + (double)k * w && d < lo + (double)(k + 1) * w) return k;
    return -1;
}

}  // namespace

struct navsim_rp_s {
    navsim_t h = nullptr;
    int device = 0;
    navsim_rp_config cfg{};
    int num_maps = 0, d0 = 0, L = 0, max_hops = 0;
    std::vector<int32_t> dims;
    std::vector<int64_t> w_off, b_off;
    int64_t nparams = 0;
    float s_common = 0.0f;
    ReachParams rp{};
    // tables
    ReachDesc *maps = nullptr;
    uint32_t *bits = nullptr;
    int32_t *free_cells = nullptr;
    int8_t *hop_bin = nullptr;
    int32_t *bin_hi = nullptr;
    float *pool = nullptr;         // [maps][1024]
    uint16_t *pool_rows = nullptr; // [maps nb][1024 + nb]
    // parameters and optimiser
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    uint16_t *pb = nullptr;
    uint8_t *decay = nullptr;
    float *wloss = nullptr;        // loss weights [5]
    int64_t adam_t = 0;
    uint32_t train_step = 0;
    void *scratch = nullptr;       // fixed per-device workspace (navsim_rp_propose_noalloc)
    uint64_t param_version = 0;    // bumped whenever the parameters change
    // learned resets inside the step (navsim_rp_attach): one device block
    struct Attach {
        bool on = false;
        int props = 0, tries = 0, cap = 0;
        void *block = nullptr;
        int32_t *bin = nullptr, *src = nullptr, *hops = nullptr;  // [N]
        uint8_t *defer = nullptr;                                 // [N]
        float *pose = nullptr;                                    // [N][5]
        uint32_t *r_env = nullptr, *r_ep = nullptr;               // [cap]
        int32_t *r_map = nullptr, *r_bin = nullptr, *n_dev = nullptr;
        unsigned long long *stats = nullptr;                      // [8]
        float *ct = nullptr, *y = nullptr;
        uint16_t *z = nullptr, *hc0 = nullptr, *hc1 = nullptr;
        int32_t *ridx = nullptr;
        int32_t *pend = nullptr, *best = nullptr;  // [cap] requests left to the tail launch
        int4 *tail = nullptr;                      // [cap][tail_rounds] round slots
        int tail_rounds = 0;                       // rounds after the head rounds
        uint64_t ct_version = ~0ull;
    } at;
    // workspaces
    DevBuf ctable, colsum, x, hid[4], y, dyf, dyb, dh, dzf, dzb, lrows, zc, ridx, yc, hc[2],
        bmap, bbin, target, chosen, zp, rp_idx, yp;
};

namespace {

template <typename T>
navsim_status upload_vec(T **dst, const std::vector<T> &src) {
    const size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
    if (hipMalloc((void **)dst, bytes) != hipSuccess)
        return fail(NAVSIM_E_OOM, "hipMalloc of %zu bytes failed", bytes);
    if (!src.empty())
        NS_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return NAVSIM_OK;
}

void free_rp(navsim_rp_s *r) {
    void *ptrs[] = {r->maps, r->bits, r->free_cells, r->hop_bin, r->bin_hi, r->pool,
                    r->pool_rows, r->p, r->g, r->m, r->v, r->pb, r->decay, r->wloss};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    DevBuf *bufs[] = {&r->ctable, &r->colsum, &r->x, &r->hid[0], &r->hid[1], &r->hid[2],
                      &r->hid[3], &r->y, &r->dyf, &r->dyb, &r->dh, &r->dzf, &r->dzb, &r->lrows,
                      &r->zc, &r->ridx, &r->yc, &r->hc[0], &r->hc[1], &r->bmap, &r->bbin,
                      &r->target, &r->chosen, &r->zp, &r->rp_idx, &r->yp};
    for (DevBuf *b : bufs) b->release();
}

#define RP_HIP(call)                                                                 \
    do {                                                                             \
        hipError_t _e = (call);                                                      \
        if (_e != hipSuccess) return fail(NAVSIM_E_HIP, "%s: %s", #call, hipGetErrorString(_e)); \
    } while (0)
#define RP_BUF(buf, bytes)                                                                    \
    do {                                                                                      \
        if ((buf).ensure(bytes) != hipSuccess) return fail(NAVSIM_E_OOM, "workspace of %zu bytes", (size_t)(bytes)); \
    } while (0)

int hidden_width(const navsim_rp_s *r) { return r->cfg.hidden; }

// Bytes of the constant first-layer table (one row per (map, bin)).
size_t ctable_bytes(const navsim_rp_s *r) {
    return (size_t)r->num_maps * r->cfg.num_bins * hidden_width(r) * sizeof(float);
}

// Writes ct[(map, bin)] = W1[:, :1024 + nb] [pool | one-hot] + b1 (float,
// ctable_bytes(r) bytes).
navsim_status refresh_ctable(navsim_rp_s *r, float *ct, hipStream_t s) {
    const int rows = r->num_maps * r->cfg.num_bins, Hd = hidden_width(r);
    GemmArgs g;
    g.M = rows;
    g.N = Hd;
    g.K = kPoolCells + r->cfg.num_bins;
    g.A = r->pool_rows;
    g.lda = kPoolCells + r->cfg.num_bins;
    g.B = r->pb + r->w_off[0];
    g.ldb = r->d0;
    g.bias = r->p + r->b_off[0];
    g.Cf = ct;
    g.ldcf = Hd;
    RP_HIP(launch_gemm(g, s));
    return NAVSIM_OK;
}

// Network outputs for noise rows (constant part of layer 1 from the table
// ct): Z [R][nz] bf16, row_idx [R] -> Y [R][5] float; hidden activations in
// hc0, hc1 (bf16, R x hidden each).
navsim_status forward_noise(navsim_rp_s *r, int R, const uint16_t *Z, const int32_t *row_idx,
                            float *Y, const float *ct, uint16_t *hc0, uint16_t *hc1,
                            hipStream_t s, const int32_t *m_dev = nullptr, int m_mul = 1) {
    const int Hd = hidden_width(r);
    uint16_t *hc[2] = {hc0, hc1};
    const float slope = r->cfg.leaky_slope;
    GemmArgs g;
    g.M = R;
    g.N = Hd;
    g.K = r->cfg.noise_dim;
    g.A = Z;
    g.lda = r->cfg.noise_dim;
    g.B = r->pb + r->w_off[0] + kPoolCells + r->cfg.num_bins;
    g.ldb = r->d0;
    g.bias_rows = ct;
    g.row_idx = row_idx;
    g.ldbr = Hd;
    g.act = 1;
    g.slope = slope;
    g.Cb = hc[0];
    g.ldcb = Hd;
    g.m_dev = m_dev;
    g.m_mul = m_mul;
    RP_HIP(launch_gemm(g, s));
    int cur = 0;
    for (int l = 1; l < r->L; ++l) {
        GemmArgs q;
        q.M = R;
        q.N = r->dims[l + 1];
        q.K = r->dims[l];
        q.A = hc[cur];
        q.lda = r->dims[l];
        q.B = r->pb + r->w_off[l];
        q.ldb = r->dims[l];
        q.bias = r->p + r->b_off[l];
        q.m_dev = m_dev;
        q.m_mul = m_mul;
        if (l + 1 < r->L) {
            q.act = 1;
            q.slope = slope;
            q.Cb = hc[1 - cur];
            q.ldcb = q.N;
        } else {
            q.Cf = Y;
            q.ldcf = q.N;
        }
        RP_HIP(launch_gemm(q, s));
        cur = 1 - cur;
    }
    return NAVSIM_OK;
}

// Forward on explicit inputs X [n][d0], keeping every layer's bf16 output in
// r->hid[] (for the backward pass) and the float outputs in Y [n][5].
navsim_status forward_full(navsim_rp_s *r, int n, const uint16_t *X, float *Y, hipStream_t s) {
    const uint16_t *in = X;
    for (int l = 0; l < r->L; ++l) {
        GemmArgs g;
        g.M = n;
        g.N = r->dims[l + 1];
        g.K = r->dims[l];
        g.A = in;
        g.lda = r->dims[l];
        g.B = r->pb + r->w_off[l];
        g.ldb = r->dims[l];
        g.bias = r->p + r->b_off[l];
        if (l + 1 < r->L) {
            RP_BUF(r->hid[l], (size_t)n * g.N * 2);
            g.act = 1;
            g.slope = r->cfg.leaky_slope;
            g.Cb = r->hid[l].as<uint16_t>();
            g.ldcb = g.N;
            in = r->hid[l].as<uint16_t>();
        } else {
            g.Cf = Y;
            g.ldcf = g.N;
        }
        RP_HIP(launch_gemm(g, s));
    }
    return NAVSIM_OK;
}

// Loss rows and gradient of the mean weighted squared error into r->g.
// Layer gradients alternate between two (float, bf16) buffer pairs.
navsim_status backward_full(navsim_rp_s *r, int n, const uint16_t *X, const float *Y,
                            const float *T, float *loss_rows, hipStream_t s) {
    const int out = r->dims[r->L];
    const int Hmax = *std::max_element(r->dims.begin() + 1, r->dims.end());
    RP_BUF(r->dyf, (size_t)n * Hmax * 4);
    RP_BUF(r->dyb, (size_t)n * Hmax * 2);
    RP_BUF(r->dzf, (size_t)n * Hmax * 4);
    RP_BUF(r->dzb, (size_t)n * Hmax * 2);
    RP_BUF(r->dh, (size_t)n * Hmax * 4);
    RP_BUF(r->colsum, (size_t)((n + 31) / 32 + 1) * Hmax * 4);
    float *zf[2] = {r->dyf.as<float>(), r->dzf.as<float>()};
    uint16_t *zb[2] = {r->dyb.as<uint16_t>(), r->dzb.as<uint16_t>()};
    RP_HIP(launch_sq_loss(n, out, Y, T, r->wloss, loss_rows, zf[0], zb[0], s));
    int cur = 0;
    for (int l = r->L - 1; l >= 0; --l) {
        const int no = r->dims[l + 1], ni = r->dims[l];
        const uint16_t *Hin = l == 0 ? X : r->hid[l - 1].as<uint16_t>();
        GemmArgs gw;  // dW = dz^T Hin
        gw.M = no;
        gw.N = ni;
        gw.K = n;
        gw.A = zb[cur];
        gw.lda = no;
        gw.a_kmajor = false;
        gw.B = Hin;
        gw.ldb = ni;
        gw.b_kmajor = false;
        gw.Cf = r->g + r->w_off[l];
        gw.ldcf = ni;
        RP_HIP(launch_gemm(gw, s));
        RP_HIP(launch_col_sum(n, no, zf[cur], r->colsum.as<float>(), r->g + r->b_off[l], s));
        if (l == 0) break;
        GemmArgs gx;  // dH = dz W
        gx.M = n;
        gx.N = ni;
        gx.K = no;
        gx.A = zb[cur];
        gx.lda = no;
        gx.B = r->pb + r->w_off[l];
        gx.ldb = ni;
        gx.b_kmajor = false;
        gx.Cf = r->dh.as<float>();
        gx.ldcf = ni;
        RP_HIP(launch_gemm(gx, s));
        RP_HIP(launch_act_backward(n, ni, r->dh.as<float>(), r->hid[l - 1].as<uint16_t>(), 1,
                                   r->cfg.leaky_slope, zf[1 - cur], zb[1 - cur], s));
        cur = 1 - cur;
    }
    return NAVSIM_OK;
}

navsim_status adamw_step(navsim_rp_s *r, const float *grad, float lr, float wd, hipStream_t s) {
    r->adam_t += 1;
    r->param_version += 1;
    RP_HIP(launch_adamw(r->nparams, r->p, r->pb, grad, r->m, r->v, r->decay, lr, 0.9f, 0.999f,
                        1e-8f, wd, r->adam_t, s));
    return NAVSIM_OK;
}

// Arguments shared by the two proposal entry points.
navsim_status check_propose(const navsim_rp_s *r, int32_t n, const int32_t *map,
                            const int32_t *bin, const uint32_t *env, const uint32_t *episode,
                            int32_t proposals, int32_t max_tries, const float *pose,
                            const int32_t *hops, const int32_t *source, const int32_t *checks) {
    if (!r) return fail(NAVSIM_E_BAD_HANDLE, "proposer is NULL");
    if (n < 0 || proposals < 0 || proposals > 4096 || max_tries < 0)
        return fail(NAVSIM_E_INVALID_ARG, "n >= 0, proposals in 0..4096, max_tries >= 0");
    if ((int64_t)n * proposals > (1 << 24))
        return fail(NAVSIM_E_INVALID_ARG, "n * proposals must be <= 2^24");
    if (n > 0 && (!map || !bin || !env || !episode || !pose || !hops || !source || !checks))
        return fail(NAVSIM_E_INVALID_ARG, "all arrays are required");
    return NAVSIM_OK;
}

// Device buffers of one proposal call: the constant first-layer table, noise
// inputs, their table rows, network outputs and two hidden activations.
struct ProposeWork {
    float *ct = nullptr;
    uint16_t *z = nullptr;
    int32_t *row_idx = nullptr;
    float *y = nullptr;
    uint16_t *hc0 = nullptr, *hc1 = nullptr;
};

constexpr size_t align_up(size_t b) { return (b + 255) & ~(size_t)255; }

// Fixed-workspace bytes of a call with n requests x `proposals` draws (0
// when proposals is 0: the rejection sampler alone uses no workspace).
size_t noalloc_bytes(const navsim_rp_s *r, int32_t n, int32_t proposals) {
    if (proposals <= 0 || n <= 0) return 0;
    const size_t R = (size_t)n * (size_t)proposals, Hd = (size_t)hidden_width(r);
    return align_up(ctable_bytes(r)) + align_up(R * r->cfg.noise_dim * 2) + align_up(R * 4) +
           align_up(R * 5 * 4) + 2 * align_up(R * Hd * 2);
}

// Noise draws, network outputs, then the exact checks and the rejection
// sampler behind them (w holds the buffers when proposals > 0).
navsim_status propose_run(navsim_rp_s *r, int32_t n, const int32_t *map, const int32_t *bin,
                          const uint32_t *env, const uint32_t *episode, int32_t proposals,
                          int32_t max_tries, float *pose, int32_t *hops, int32_t *source,
                          int32_t *checks, float *y_out, const ProposeWork &w, hipStream_t s) {
    const float *y = nullptr;
    if (proposals > 0) {
        const int64_t R = (int64_t)n * proposals;
        navsim_status st = refresh_ctable(r, w.ct, s);
        if (st != NAVSIM_OK) return st;
        NoiseArgs na;
        na.n = n;
        na.per = proposals;
        na.nz = r->cfg.noise_dim;
        na.nbins = r->cfg.num_bins;
        na.num_maps = r->num_maps;
        na.c0 = env;
        na.c1 = episode;
        na.c1_const = 0u;
        na.stream = 8u;
        na.map = map;
        na.bin = bin;
        na.z = w.z;
        na.row_idx = w.row_idx;
        RP_HIP(launch_noise(na, r->rp.key0, r->rp.key1, s));
        if ((st = forward_noise(r, (int)R, na.z, na.row_idx, w.y, w.ct, w.hc0, w.hc1, s)) !=
            NAVSIM_OK)
            return st;
        y = w.y;
        if (y_out) RP_HIP(hipMemcpyAsync(y_out, y, (size_t)R * 5 * 4, hipMemcpyDeviceToDevice, s));
    }
    ProposeArgs pa;
    pa.n = n;
    pa.props = proposals;
    pa.tries = max_tries;
    pa.map = map;
    pa.bin = bin;
    pa.env = env;
    pa.episode = episode;
    pa.y = y;
    pa.pose = pose;
    pa.hops = hops;
    pa.source = source;
    pa.checks = checks;
    RP_HIP(launch_propose(r->rp, pa, s));
    return NAVSIM_OK;
}

// The in-step proposal pass (navsim_s::ResetHook::run): requests of the envs
// that deferred their reset, noise draws and network outputs for them, then
// the exact checks with the rejection sampler behind them; pairs go to the
// envs' rows of the pose table.
navsim_status rp_hook_run(void *ctx, hipStream_t s) {
    navsim_rp_s *r = (navsim_rp_s *)ctx;
    navsim_rp_s::Attach &A = r->at;
    navsim_t h = r->h;
    CompactArgs ca;
    ca.N = h->cfg.num_envs;
    ca.cap = A.cap;
    ca.defer = A.defer;
    ca.bin = A.bin;
    ca.env_map = h->env_map;
    ca.ep = h->st.ep;
    ca.env = A.r_env;
    ca.episode = A.r_ep;
    ca.map = A.r_map;
    ca.rbin = A.r_bin;
    ca.src = A.src;
    ca.n_out = A.n_dev;
    ca.stats = A.stats;
    ca.n_pend = A.n_dev + 1;  // the pending count shares the counters' block
    RP_HIP(launch_compact(ca, s));
    const float *y = nullptr;
    if (A.props > 0) {
        navsim_status st = NAVSIM_OK;
        if (A.ct_version != r->param_version) {
            if ((st = refresh_ctable(r, A.ct, s)) != NAVSIM_OK) return st;
            A.ct_version = r->param_version;
        }
        NoiseArgs na;
        na.n = A.cap;
        na.per = A.props;
        na.nz = r->cfg.noise_dim;
        na.nbins = r->cfg.num_bins;
        na.num_maps = r->num_maps;
        na.c0 = A.r_env;
        na.c1 = A.r_ep;
        na.c1_const = 0u;
        na.stream = 8u;
        na.map = A.r_map;
        na.bin = A.r_bin;
        na.z = A.z;
        na.row_idx = A.ridx;
        na.n_dev = A.n_dev;
        RP_HIP(launch_noise(na, r->rp.key0, r->rp.key1, s));
        if ((st = forward_noise(r, A.cap * A.props, A.z, A.ridx, A.y, A.ct, A.hc0, A.hc1, s,
                                A.n_dev, A.props)) != NAVSIM_OK)
            return st;
        y = A.y;
    }
    ProposeArgs pa;
    pa.n = A.cap;
    pa.props = A.props;
    pa.tries = A.tries;
    pa.map = A.r_map;
    pa.bin = A.r_bin;
    pa.env = A.r_env;
    pa.episode = A.r_ep;
    pa.y = y;
    pa.pose = A.pose;
    pa.hops = A.hops;
    pa.source = A.src;
    pa.checks = nullptr;
    pa.n_dev = A.n_dev;
    pa.slot = (const int32_t *)A.r_env;
    pa.stats = A.stats + 2;
    // the few requests with no valid candidate in their head rounds set the
    // launch's time when their rounds run one after another: their remaining
    // rounds go to one tail launch, one workgroup per round
    const int tail_rounds =
        std::max(0, (int)(((int64_t)A.props + A.tries + propose_width(A.cap) - 1) /
                          propose_width(A.cap)) - kProposeHeadRounds);
    if (tail_rounds > 0) {
        pa.head_rounds = kProposeHeadRounds;
        pa.pend = A.pend;
        pa.n_pend = A.n_dev + 1;
        pa.best = A.best;
        pa.tail = A.tail;
    }
    RP_HIP(launch_propose(r->rp, pa, s));
    if (tail_rounds > 0) RP_HIP(launch_propose_tail(r->rp, pa, tail_rounds, s));
    return NAVSIM_OK;
}

void detach_rp(navsim_rp_s *r) {
    navsim_t h = r->h;
    if (h && h->hook.ctx == r) h->hook = navsim_s::ResetHook{};
    if (r->at.block) {
        (void)hipDeviceSynchronize();  // steps in flight may still use the block
        (void)hipFree(r->at.block);
    }
    r->at = navsim_rp_s::Attach{};
}

}  // namespace

extern "C" {

navsim_status navsim_rp_create(navsim_t h, const navsim_rp_config *cfg, navsim_rp_t *out) {
    if (!out) return fail(NAVSIM_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!h) return fail(NAVSIM_E_BAD_HANDLE, "handle is NULL");
    if (!cfg) return fail(NAVSIM_E_INVALID_ARG, "cfg is NULL");
    if (!h->loaded) return fail(NAVSIM_E_STATE, "navsim_load_maps has not been called");
    const navsim_rp_config &c = *cfg;
    if (c.num_bins < 1 || c.num_bins > kReachMaxBins)
        return fail(NAVSIM_E_INVALID_ARG, "num_bins must be in 1..%d", kReachMaxBins);
    if (!(c.d_lo_m >= 0.0f) || !(c.d_hi_m > c.d_lo_m) || !isfinite(c.d_hi_m))
        return fail(NAVSIM_E_INVALID_ARG, "need 0 <= d_lo_m < d_hi_m");
    if (c.noise_dim < 1 || c.noise_dim > 64)
        return fail(NAVSIM_E_INVALID_ARG, "noise_dim must be in 1..64");
    if (c.hidden < 16 || c.hidden > 1024 || c.hidden % 16 != 0)
        return fail(NAVSIM_E_INVALID_ARG, "hidden must be a multiple of 16 in 16..1024");
    if (c.hidden_layers < 1 || c.hidden_layers > 4)
        return fail(NAVSIM_E_INVALID_ARG, "hidden_layers must be in 1..4");
    if (!finite_pos(c.leaky_slope)) return fail(NAVSIM_E_INVALID_ARG, "leaky_slope must be > 0");
    const int M = h->num_maps;
    for (int k = 0; k < M; ++k) {
        const int W = h->host_w[k], H = h->host_h[k];
        if (W < 32 || H < 32 || (int64_t)H * ((W + 31) / 32) > kReachMaxWords)
            return fail(NAVSIM_E_UNSUPPORTED,
                        "map %d is %dx%d: proposals need W, H >= 32 and H ceil(W/32) <= %d", k, W,
                        H, kReachMaxWords);
    }
    DeviceGuard dg(h->device);
    if (dg.err != hipSuccess) return fail(NAVSIM_E_HIP, "hipSetDevice: %s", hipGetErrorString(dg.err));
    navsim_rp_s *r = new (std::nothrow) navsim_rp_s();
    if (!r) return fail(NAVSIM_E_OOM, "host allocation failed");
    r->h = h;
    r->device = h->device;
    r->cfg = c;
    r->num_maps = M;
    // bitsets, free lists, pooled occupancy
    std::vector<ReachDesc> descs(M);
    std::vector<uint32_t> bits;
    std::vector<int32_t> freel;
    std::vector<float> pool((size_t)M * kPoolCells, 0.0f);
    for (int k = 0; k < M; ++k) {
        const int W = h->host_w[k], H = h->host_h[k];
        ReachDesc &d = descs[k];
        d.W = W;
        d.H = H;
        d.wpr = (W + 31) / 32;
        d.words = d.wpr * H;
        d.bit_off = (int64_t)bits.size();
        d.free_off = (int64_t)freel.size();
        d.free_cnt = h->host_free_cnt[k];
        d.s = h->host_res[k];
        bits.resize(bits.size() + d.words, 0u);
        const int32_t *fl = h->host_free.data() + h->host_free_off[k];
        for (int q = 0; q < d.free_cnt; ++q) {
            const int cell = fl[q], i = cell % W, j = cell / W;
            bits[d.bit_off + (int64_t)j * d.wpr + (i >> 5)] |= 1u << (i & 31);
            freel.push_back(cell);
        }
        const uint8_t *occ = h->host_occ.data() + h->host_occ_off[k];
        for (int q = 0; q < 32; ++q)
            for (int p = 0; p < 32; ++p) {
                float v = 0.0f;
                for (int j = q * H / 32; j < (q + 1) * H / 32 && v == 0.0f; ++j)
                    for (int i = p * W / 32; i < (p + 1) * W / 32; ++i)
                        if (occ[(int64_t)j * W + i]) {
                            v = 1.0f;
                            break;
                        }
                pool[(size_t)k * kPoolCells + q * 32 + p] = v;
            }
    }
    // hop-count bins: the search depth is the largest hop count in any bin,
    // over the smallest cell size among the maps
    double smin = 1e30;
    for (int k = 0; k < M; ++k) smin = std::min(smin, (double)h->host_res[k]);
    bool same_res = true;
    for (int k = 1; k < M; ++k) same_res = same_res && h->host_res[k] == h->host_res[0];
    if (!same_res) {
        delete r;
        return fail(NAVSIM_E_UNSUPPORTED, "proposals need one cell size for all maps");
    }
    const double lo = (double)c.d_lo_m, hi = (double)c.d_hi_m;
    int maxh = (int)(hi / smin) + 2;
    while (maxh > 0 && bin_of(smin, maxh, lo, hi, c.num_bins) < 0) --maxh;
    if (maxh <= 0 || maxh > 65535) {
        delete r;
        return fail(NAVSIM_E_INVALID_ARG, "the bins cover no hop count in 1..65535");
    }
    std::vector<int8_t> hop_bin(maxh + 1);
    std::vector<int32_t> bin_hi(c.num_bins, -1);
    for (int q = 0; q <= maxh; ++q) {
        hop_bin[q] = (int8_t)bin_of(smin, q, lo, hi, c.num_bins);
        if (hop_bin[q] >= 0) bin_hi[hop_bin[q]] = q;
    }
    r->max_hops = maxh;
    // network layout
    r->d0 = kPoolCells + c.num_bins + c.noise_dim;
    r->L = c.hidden_layers + 1;
    r->dims.push_back(r->d0);
    for (int l = 0; l < c.hidden_layers; ++l) r->dims.push_back(c.hidden);
    r->dims.push_back(5);
    int64_t off = 0;
    for (int l = 0; l < r->L; ++l) {
        r->w_off.push_back(off);
        off += (int64_t)r->dims[l + 1] * r->dims[l];
        off = (off + 7) & ~(int64_t)7;
        r->b_off.push_back(off);
        off += r->dims[l + 1];
        off = (off + 7) & ~(int64_t)7;
    }
    r->nparams = off;
    std::vector<float> params((size_t)off, 0.0f);
    std::vector<uint8_t> decay((size_t)off, 0);
    std::mt19937_64 gen(c.seed);
    for (int l = 0; l < r->L; ++l) {
        const double bound = 1.0 / sqrt((double)r->dims[l]);
        std::uniform_real_distribution<double> U(-bound, bound);
        const int64_t n = (int64_t)r->dims[l + 1] * r->dims[l];
        for (int64_t q = 0; q < n; ++q) {
            params[r->w_off[l] + q] = (float)U(gen);
            decay[r->w_off[l] + q] = 1;
        }
    }
    const float wl[5] = {1.0f, 1.0f, 0.0f, 1.0f, 1.0f};
    navsim_status st = NAVSIM_OK;
    auto fail_out = [&](navsim_status e) {
        free_rp(r);
        delete r;
        return e;
    };
    if ((st = upload_vec(&r->maps, descs)) != NAVSIM_OK) return fail_out(st);
    if ((st = upload_vec(&r->bits, bits)) != NAVSIM_OK) return fail_out(st);
    if ((st = upload_vec(&r->free_cells, freel)) != NAVSIM_OK) return fail_out(st);
    if ((st = upload_vec(&r->hop_bin, hop_bin)) != NAVSIM_OK) return fail_out(st);
    if ((st = upload_vec(&r->bin_hi, bin_hi)) != NAVSIM_OK) return fail_out(st);
    if ((st = upload_vec(&r->pool, pool)) != NAVSIM_OK) return fail_out(st);
    if ((st = upload_vec(&r->p, params)) != NAVSIM_OK) return fail_out(st);
    if ((st = upload_vec(&r->decay, decay)) != NAVSIM_OK) return fail_out(st);
    if ((st = upload_vec(&r->wloss, std::vector<float>(wl, wl + 5))) != NAVSIM_OK) return fail_out(st);
    std::vector<float> zeros((size_t)off, 0.0f);
    if ((st = upload_vec(&r->g, zeros)) != NAVSIM_OK) return fail_out(st);
    if ((st = upload_vec(&r->m, zeros)) != NAVSIM_OK) return fail_out(st);
    if ((st = upload_vec(&r->v, zeros)) != NAVSIM_OK) return fail_out(st);
    if (hipMalloc((void **)&r->pb, (size_t)off * 2) != hipSuccess ||
        hipMalloc((void **)&r->pool_rows,
                  (size_t)M * c.num_bins * (kPoolCells + c.num_bins) * 2) != hipSuccess)
        return fail_out(fail(NAVSIM_E_OOM, "hipMalloc of the network failed"));
    if (launch_to_bf16(off, r->p, r->pb, nullptr) != hipSuccess ||
        launch_pool_rows(M, c.num_bins, r->pool, r->pool_rows, nullptr) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess)
        return fail_out(fail(NAVSIM_E_HIP, "initialising the proposer failed"));
    ReachParams &rp = r->rp;
    rp.maps = r->maps;
    rp.bits = r->bits;
    rp.free_cells = r->free_cells;
    rp.hop_bin = r->hop_bin;
    rp.bin_hi = r->bin_hi;
    rp.max_hops = maxh;
    rp.nbins = c.num_bins;
    rp.num_maps = M;
    rp.gmd = (double)h->cfg.goal_min_dist_m;
    rp.key0 = (uint32_t)(c.seed & 0xffffffffu);
    rp.key1 = (uint32_t)(c.seed >> 32);
    // the fixed workspace's device address on this device (the device is current)
    const hipError_t se = rp_scratch_address(r->device, &r->scratch);
    if (se != hipSuccess)
        return fail_out(fail(NAVSIM_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(se)));
    h->proposers++;
    *out = r;
    return NAVSIM_OK;
}

navsim_status navsim_rp_label(navsim_rp_t r, int32_t n, const int32_t *map, uint32_t first_sid,
                              int32_t *start, int32_t *goal, int32_t *hops, void *stream) {
    if (!r) return fail(NAVSIM_E_BAD_HANDLE, "proposer is NULL");
    if (n < 0 || (n > 0 && (!map || !start || !goal || !hops)))
        return fail(NAVSIM_E_INVALID_ARG, "n >= 0 and map, start, goal, hops are required");
    DeviceGuard dg(r->device);
    RP_HIP(launch_label(r->rp, n, map, first_sid, start, goal, hops, (hipStream_t)stream));
    return NAVSIM_OK;
}

navsim_status navsim_rp_train(navsim_rp_t r, int32_t num_pairs, const int32_t *pair_map,
                              const int32_t *pair_bin, const int32_t *pair_start,
                              const int32_t *pair_goal, int32_t steps, int32_t batch,
                              int32_t samples, float lr, float weight_decay, float *loss,
                              void *stream) {
    if (!r) return fail(NAVSIM_E_BAD_HANDLE, "proposer is NULL");
    if (num_pairs < 1 || !pair_map || !pair_bin || !pair_start || !pair_goal)
        return fail(NAVSIM_E_INVALID_ARG, "a non-empty pair set is required");
    if (steps < 0 || batch < 1 || batch > 65536 || samples < 1 || samples > 256)
        return fail(NAVSIM_E_INVALID_ARG, "steps >= 0, batch in 1..65536, samples in 1..256");
    if (!(lr > 0.0f) || !(weight_decay >= 0.0f))
        return fail(NAVSIM_E_INVALID_ARG, "lr > 0 and weight_decay >= 0");
    DeviceGuard dg(r->device);
    const hipStream_t s = (hipStream_t)stream;
    const int nz = r->cfg.noise_dim, nb = r->cfg.num_bins, Hd = r->cfg.hidden;
    const int R = batch * samples;
    RP_BUF(r->bmap, (size_t)batch * 4);
    RP_BUF(r->bbin, (size_t)batch * 4);
    RP_BUF(r->target, (size_t)batch * 5 * 4);
    RP_BUF(r->chosen, (size_t)batch * 4);
    RP_BUF(r->zc, (size_t)R * nz * 2);
    RP_BUF(r->ridx, (size_t)R * 4);
    RP_BUF(r->yc, (size_t)R * 5 * 4);
    RP_BUF(r->x, (size_t)batch * r->d0 * 2);
    RP_BUF(r->y, (size_t)batch * 5 * 4);
    RP_BUF(r->lrows, (size_t)batch * 4);
    RP_BUF(r->ctable, ctable_bytes(r));
    RP_BUF(r->hc[0], (size_t)R * Hd * 2);
    RP_BUF(r->hc[1], (size_t)R * Hd * 2);
    for (int t = 0; t < steps; ++t) {
        const uint32_t step = r->train_step++;
        navsim_status st = refresh_ctable(r, r->ctable.as<float>(), s);
        if (st != NAVSIM_OK) return st;
        BatchArgs ba;
        ba.batch = batch;
        ba.num_pairs = num_pairs;
        ba.num_maps = r->num_maps;
        ba.nbins = nb;
        ba.step = step;
        ba.pair_map = pair_map;
        ba.pair_bin = pair_bin;
        ba.pair_start = pair_start;
        ba.pair_goal = pair_goal;
        ba.maps = r->maps;
        ba.map = r->bmap.as<int32_t>();
        ba.bin = r->bbin.as<int32_t>();
        ba.target = r->target.as<float>();
        RP_HIP(launch_batch(ba, r->rp.key0, r->rp.key1, s));
        NoiseArgs na;
        na.n = batch;
        na.per = samples;
        na.nz = nz;
        na.nbins = nb;
        na.num_maps = r->num_maps;
        na.c0 = nullptr;
        na.c1 = nullptr;
        na.c1_const = step;
        na.stream = 9u;
        na.map = ba.map;
        na.bin = ba.bin;
        na.z = r->zc.as<uint16_t>();
        na.row_idx = r->ridx.as<int32_t>();
        RP_HIP(launch_noise(na, r->rp.key0, r->rp.key1, s));
        if ((st = forward_noise(r, R, na.z, na.row_idx, r->yc.as<float>(), r->ctable.as<float>(),
                                r->hc[0].as<uint16_t>(), r->hc[1].as<uint16_t>(), s)) != NAVSIM_OK)
            return st;
        SelectArgs sa;
        sa.batch = batch;
        sa.per = samples;
        sa.nz = nz;
        sa.nbins = nb;
        sa.y = r->yc.as<float>();
        sa.target = ba.target;
        sa.w = r->wloss;
        sa.z = na.z;
        sa.map = ba.map;
        sa.bin = ba.bin;
        sa.pool = r->pool;
        sa.x = r->x.as<uint16_t>();
        sa.chosen = r->chosen.as<int32_t>();
        RP_HIP(launch_select(sa, s));
        if ((st = forward_full(r, batch, sa.x, r->y.as<float>(), s)) != NAVSIM_OK) return st;
        if ((st = backward_full(r, batch, sa.x, r->y.as<float>(), ba.target,
                                r->lrows.as<float>(), s)) != NAVSIM_OK)
            return st;
        if ((st = adamw_step(r, r->g, lr, weight_decay, s)) != NAVSIM_OK) return st;
        if (loss) {
            RP_BUF(r->colsum, (size_t)((batch + 31) / 32 + 1) * 4);
            RP_HIP(launch_col_sum(batch, 1, r->lrows.as<float>(), r->colsum.as<float>(),
                                  loss + t, s));
        }
    }
    return NAVSIM_OK;
}

navsim_status navsim_rp_propose(navsim_rp_t r, int32_t n, const int32_t *map, const int32_t *bin,
                                const uint32_t *env, const uint32_t *episode, int32_t proposals,
                                int32_t max_tries, float *pose, int32_t *hops, int32_t *source,
                                int32_t *checks, float *y_out, void *stream) {
    navsim_status st = check_propose(r, n, map, bin, env, episode, proposals, max_tries, pose,
                                     hops, source, checks);
    if (st != NAVSIM_OK || n == 0) return st;
    DeviceGuard dg(r->device);
    ProposeWork w;
    if (proposals > 0) {
        const int64_t R = (int64_t)n * proposals;
        const int Hd = hidden_width(r);
        RP_BUF(r->ctable, ctable_bytes(r));
        RP_BUF(r->zp, (size_t)R * r->cfg.noise_dim * 2);
        RP_BUF(r->rp_idx, (size_t)R * 4);
        RP_BUF(r->yp, (size_t)R * 5 * 4);
        RP_BUF(r->hc[0], (size_t)R * Hd * 2);
        RP_BUF(r->hc[1], (size_t)R * Hd * 2);
        w = ProposeWork{r->ctable.as<float>(), r->zp.as<uint16_t>(), r->rp_idx.as<int32_t>(),
                        r->yp.as<float>(), r->hc[0].as<uint16_t>(), r->hc[1].as<uint16_t>()};
    }
    return propose_run(r, n, map, bin, env, episode, proposals, max_tries, pose, hops, source,
                       checks, y_out, w, (hipStream_t)stream);
}

navsim_status navsim_rp_propose_noalloc(navsim_rp_t r, int32_t n, const int32_t *map,
                                        const int32_t *bin, const uint32_t *env,
                                        const uint32_t *episode, int32_t proposals,
                                        int32_t max_tries, float *pose, int32_t *hops,
                                        int32_t *source, int32_t *checks, float *y_out,
                                        void *stream) {
    navsim_status st = check_propose(r, n, map, bin, env, episode, proposals, max_tries, pose,
                                     hops, source, checks);
    if (st != NAVSIM_OK) return st;
    if (!r->scratch) return fail(NAVSIM_E_STATE, "the proposer has no fixed workspace");
    const size_t need = noalloc_bytes(r, n, proposals);
    if (need > kRpScratchBytes)
        return fail(NAVSIM_E_INVALID_ARG,
                    "navsim_rp_propose_noalloc: %d requests x %d proposals need %zu workspace "
                    "bytes, more than the fixed %zu (use fewer requests per call)",
                    n, proposals, need, kRpScratchBytes);
    if (n == 0) return NAVSIM_OK;
    DeviceGuard dg(r->device);
    ProposeWork w;
    if (proposals > 0) {
        // carve the fixed workspace in the order noalloc_bytes() counts it
        const int64_t R = (int64_t)n * proposals;
        const int Hd = hidden_width(r);
        uint8_t *base = (uint8_t *)r->scratch;
        size_t off = 0;
        auto take = [&](size_t bytes) {
            uint8_t *q = base + off;
            off += align_up(bytes);
            return (void *)q;
        };
        w.ct = (float *)take(ctable_bytes(r));
        w.z = (uint16_t *)take((size_t)R * r->cfg.noise_dim * 2);
        w.row_idx = (int32_t *)take((size_t)R * 4);
        w.y = (float *)take((size_t)R * 5 * 4);
        w.hc0 = (uint16_t *)take((size_t)R * Hd * 2);
        w.hc1 = (uint16_t *)take((size_t)R * Hd * 2);
    }
    return propose_run(r, n, map, bin, env, episode, proposals, max_tries, pose, hops, source,
                       checks, y_out, w, (hipStream_t)stream);
}

navsim_status navsim_rp_forward(navsim_rp_t r, int32_t n, const uint16_t *x, float *y,
                                void *stream) {
    if (!r) return fail(NAVSIM_E_BAD_HANDLE, "proposer is NULL");
    if (n < 0 || (n > 0 && (!x || !y))) return fail(NAVSIM_E_INVALID_ARG, "x and y are required");
    DeviceGuard dg(r->device);
    return forward_full(r, n, x, y, (hipStream_t)stream);
}

navsim_status navsim_rp_loss_grad(navsim_rp_t r, int32_t n, const uint16_t *x,
                                  const float *target, float *loss_rows, float *grad,
                                  void *stream) {
    if (!r) return fail(NAVSIM_E_BAD_HANDLE, "proposer is NULL");
    if (n < 1 || !x || !target || !grad)
        return fail(NAVSIM_E_INVALID_ARG, "n >= 1 and x, target, grad are required");
    DeviceGuard dg(r->device);
    const hipStream_t s = (hipStream_t)stream;
    RP_BUF(r->y, (size_t)n * 5 * 4);
    navsim_status st = forward_full(r, n, x, r->y.as<float>(), s);
    if (st != NAVSIM_OK) return st;
    if ((st = backward_full(r, n, x, r->y.as<float>(), target, loss_rows, s)) != NAVSIM_OK)
        return st;
    RP_HIP(hipMemcpyAsync(grad, r->g, (size_t)r->nparams * 4, hipMemcpyDeviceToDevice, s));
    return NAVSIM_OK;
}

navsim_status navsim_rp_adamw(navsim_rp_t r, const float *grad, float lr, float weight_decay,
                              void *stream) {
    if (!r) return fail(NAVSIM_E_BAD_HANDLE, "proposer is NULL");
    if (!grad || !(lr > 0.0f) || !(weight_decay >= 0.0f))
        return fail(NAVSIM_E_INVALID_ARG, "grad, lr > 0, weight_decay >= 0 are required");
    DeviceGuard dg(r->device);
    return adamw_step(r, grad, lr, weight_decay, (hipStream_t)stream);
}

navsim_status navsim_rp_layout(navsim_rp_t r, int32_t *num_layers, int32_t *dims,
                               int64_t *offsets, int64_t *count) {
    if (!r) return fail(NAVSIM_E_BAD_HANDLE, "proposer is NULL");
    if (num_layers) *num_layers = r->L;
    if (count) *count = r->nparams;
    if (dims)
        for (int l = 0; l <= r->L; ++l) dims[l] = r->dims[l];
    if (offsets)
        for (int l = 0; l < r->L; ++l) {
            offsets[2 * l] = r->w_off[l];
            offsets[2 * l + 1] = r->b_off[l];
        }
    return NAVSIM_OK;
}

navsim_status navsim_rp_get_params(navsim_rp_t r, float *host, int64_t count) {
    if (!r) return fail(NAVSIM_E_BAD_HANDLE, "proposer is NULL");
    if (!host || count != r->nparams)
        return fail(NAVSIM_E_INVALID_ARG, "host buffer of %lld floats required",
                    (long long)r->nparams);
    DeviceGuard dg(r->device);
    NS_HIP(hipDeviceSynchronize());
    NS_HIP(hipMemcpy(host, r->p, (size_t)count * 4, hipMemcpyDeviceToHost));
    return NAVSIM_OK;
}

navsim_status navsim_rp_set_params(navsim_rp_t r, const float *host, int64_t count) {
    if (!r) return fail(NAVSIM_E_BAD_HANDLE, "proposer is NULL");
    if (!host || count != r->nparams)
        return fail(NAVSIM_E_INVALID_ARG, "host buffer of %lld floats required",
                    (long long)r->nparams);
    DeviceGuard dg(r->device);
    NS_HIP(hipDeviceSynchronize());
    NS_HIP(hipMemcpy(r->p, host, (size_t)count * 4, hipMemcpyHostToDevice));
    NS_HIP(launch_to_bf16(count, r->p, r->pb, nullptr));
    NS_HIP(hipDeviceSynchronize());
    r->param_version += 1;
    return NAVSIM_OK;
}

navsim_status navsim_rp_attach(navsim_rp_t r, const int32_t *bin, int32_t proposals,
                               int32_t max_tries, int32_t max_per_step) {
    if (!r) return fail(NAVSIM_E_BAD_HANDLE, "proposer is NULL");
    navsim_t h = r->h;
    const int N = h->cfg.num_envs, nb = r->cfg.num_bins;
    if (!bin) return fail(NAVSIM_E_INVALID_ARG, "bin (host int32 [num_envs]) is required");
    if (proposals < 0 || proposals > 4096 || max_tries < 0 || max_per_step < 1 ||
        max_per_step > N || (int64_t)max_per_step * proposals > (1 << 24))
        return fail(NAVSIM_E_INVALID_ARG,
                    "need proposals in 0..4096, max_tries >= 0, max_per_step in 1..num_envs and "
                    "max_per_step * proposals <= 2^24");
    for (int e = 0; e < N; ++e)
        if (bin[e] < -1 || bin[e] >= nb)
            return fail(NAVSIM_E_INVALID_ARG, "bin[%d] = %d is outside -1..%d", e, bin[e], nb - 1);
    if (h->hook.run && h->hook.ctx != r)
        return fail(NAVSIM_E_STATE, "another proposer is attached to this handle");
    DeviceGuard dg(r->device);
    if (dg.err != hipSuccess) return fail(NAVSIM_E_HIP, "hipSetDevice: %s", hipGetErrorString(dg.err));
    navsim_rp_s::Attach &A = r->at;
    // rounds of candidates after the head rounds (one tail workgroup each)
    const int W = propose_width(max_per_step);
    const int64_t rounds = ((int64_t)proposals + max_tries + W - 1) / W;
    const int tail_rounds = (int)std::max<int64_t>(0, rounds - kProposeHeadRounds);
    if ((int64_t)max_per_step * tail_rounds > (1 << 24))
        return fail(NAVSIM_E_INVALID_ARG, "max_per_step * candidate rounds must be at most 2^24");
    if (!(A.on && A.cap == max_per_step && A.props == proposals && A.tail_rounds >= tail_rounds)) {
        detach_rp(r);
        const size_t R = (size_t)max_per_step * (size_t)proposals, Hd = (size_t)r->cfg.hidden;
        const size_t parts[] = {(size_t)N * 4, (size_t)N * 4, (size_t)N * 4, (size_t)N,
                                (size_t)N * 20, (size_t)max_per_step * 4, (size_t)max_per_step * 4,
                                (size_t)max_per_step * 4, (size_t)max_per_step * 4, 256, 64,
                                proposals ? ctable_bytes(r) : 0, R * 20,
                                R * (size_t)r->cfg.noise_dim * 2, R * Hd * 2, R * Hd * 2, R * 4,
                                (size_t)max_per_step * 4, (size_t)max_per_step * 4,
                                (size_t)max_per_step * (size_t)tail_rounds * 16};
        constexpr int kParts = (int)(sizeof parts / sizeof parts[0]);
        size_t total = 0;
        for (size_t b : parts) total += align_up(b);
        if (hipMalloc(&A.block, total) != hipSuccess) {
            A.block = nullptr;
            return fail(NAVSIM_E_OOM, "hipMalloc of %zu bytes for in-step proposals failed", total);
        }
        uint8_t *q = (uint8_t *)A.block;
        void *ptrs[kParts];
        for (int k = 0; k < kParts; ++k) {
            ptrs[k] = q;
            q += align_up(parts[k]);
        }
        A.pend = (int32_t *)ptrs[17];
        A.best = (int32_t *)ptrs[18];
        A.tail = (int4 *)ptrs[19];
        A.tail_rounds = tail_rounds;
        A.bin = (int32_t *)ptrs[0];
        A.src = (int32_t *)ptrs[1];
        A.hops = (int32_t *)ptrs[2];
        A.defer = (uint8_t *)ptrs[3];
        A.pose = (float *)ptrs[4];
        A.r_env = (uint32_t *)ptrs[5];
        A.r_ep = (uint32_t *)ptrs[6];
        A.r_map = (int32_t *)ptrs[7];
        A.r_bin = (int32_t *)ptrs[8];
        A.n_dev = (int32_t *)ptrs[9];
        A.stats = (unsigned long long *)ptrs[10];
        A.ct = (float *)ptrs[11];
        A.y = (float *)ptrs[12];
        A.z = (uint16_t *)ptrs[13];
        A.hc0 = (uint16_t *)ptrs[14];
        A.hc1 = (uint16_t *)ptrs[15];
        A.ridx = (int32_t *)ptrs[16];
        A.cap = max_per_step;
        A.props = proposals;
        A.ct_version = ~0ull;
        NS_HIP(hipMemset(A.block, 0, total));
        NS_HIP(hipMemset(A.src, 0xff, (size_t)N * 4));
        NS_HIP(hipMemset(A.hops, 0xff, (size_t)N * 4));
    }
    NS_HIP(hipDeviceSynchronize());  // steps in flight may read the old bins
    NS_HIP(hipMemcpy(A.bin, bin, (size_t)N * 4, hipMemcpyHostToDevice));
    A.tries = max_tries;
    A.on = true;
    h->hook.bin = A.bin;
    h->hook.defer = A.defer;
    h->hook.pose = A.pose;
    h->hook.src = A.src;
    h->hook.run = rp_hook_run;
    h->hook.ctx = r;
    return NAVSIM_OK;
}

navsim_status navsim_rp_detach(navsim_rp_t r) {
    if (!r) return fail(NAVSIM_E_BAD_HANDLE, "proposer is NULL");
    DeviceGuard dg(r->device);
    detach_rp(r);
    return NAVSIM_OK;
}

navsim_status navsim_rp_attach_stats(navsim_rp_t r, int64_t *out, int32_t clear) {
    if (!r) return fail(NAVSIM_E_BAD_HANDLE, "proposer is NULL");
    if (!out) return fail(NAVSIM_E_INVALID_ARG, "out (host int64 [8]) is required");
    if (!r->at.on) return fail(NAVSIM_E_STATE, "the proposer is not attached");
    DeviceGuard dg(r->device);
    NS_HIP(hipDeviceSynchronize());
    unsigned long long v[8];
    NS_HIP(hipMemcpy(v, r->at.stats, sizeof v, hipMemcpyDeviceToHost));
    for (int k = 0; k < 8; ++k) out[k] = (int64_t)v[k];
    if (clear) NS_HIP(hipMemset(r->at.stats, 0, sizeof v));
    return NAVSIM_OK;
}

navsim_status navsim_rp_attach_outputs(navsim_rp_t r, int32_t *source, int32_t *hops,
                                       void *stream) {
    if (!r) return fail(NAVSIM_E_BAD_HANDLE, "proposer is NULL");
    if (!source || !hops) return fail(NAVSIM_E_INVALID_ARG, "source and hops are required");
    if (!r->at.on) return fail(NAVSIM_E_STATE, "the proposer is not attached");
    DeviceGuard dg(r->device);
    const size_t bytes = (size_t)r->h->cfg.num_envs * 4;
    const hipStream_t s = (hipStream_t)stream;
    NS_HIP(hipMemcpyAsync(source, r->at.src, bytes, hipMemcpyDeviceToDevice, s));
    NS_HIP(hipMemcpyAsync(hops, r->at.hops, bytes, hipMemcpyDeviceToDevice, s));
    return NAVSIM_OK;
}

navsim_status navsim_rp_destroy(navsim_rp_t r) {
    if (!r) return fail(NAVSIM_E_BAD_HANDLE, "proposer is NULL");
    {
        DeviceGuard dg(r->device);
        detach_rp(r);
        (void)hipDeviceSynchronize();
        free_rp(r);
    }
    if (r->h && r->h->proposers > 0) r->h->proposers--;
    delete r;
    return NAVSIM_OK;
}

}  // extern "C"
