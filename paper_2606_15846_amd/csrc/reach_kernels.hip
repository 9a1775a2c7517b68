// Reachability kernels of the learned reset proposal: breadth-first search on
// C-free bitsets staged in LDS, one workgroup per request.  Each search level
// dilates the frontier by one 4-neighbour move with word shifts (left/right
// within a row, carries across words) and row offsets (up/down), masks it with
// the C-free bits and the visited set, and stops as soon as the target bit
// appears, the frontier empties or the depth limit is reached.
#include <limits.h>
#include <math.h>

#include "mlp_internal.hpp"
#include "philox.hpp"
#include "reach_internal.hpp"

namespace navsim {
namespace {

constexpr double kPiR = 3.14159265358979323846;
constexpr double kTwo32 = 4294967296.0;

__device__ __forceinline__ bool cell_bit(const uint32_t *b, const ReachDesc &d, int cell) {
    const int i = cell % d.W, j = cell / d.W;
    return (b[j * d.wpr + (i >> 5)] >> (i & 31)) & 1u;
}

__device__ __forceinline__ void set_cell(uint32_t *b, const ReachDesc &d, int cell) {
    const int i = cell % d.W, j = cell / d.W;
    b[j * d.wpr + (i >> 5)] |= 1u << (i & 31);
}

__device__ __forceinline__ uint16_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ void stage_free(const ReachParams &rp, const ReachDesc &d, uint32_t *fb) {
    const uint32_t *g = rp.bits + d.bit_off;
    for (int w = threadIdx.x; w < d.words; w += blockDim.x) fb[w] = g[w];
}

// One search level: nx = (frontier moved by one step) & C-free & ~visited,
// visited |= nx, over the words of rows r0..r1 and word columns c0..c1 only
// (the caller's box holds every bit the level can set; nx, vis and fr are
// zero outside it).  Returns the OR of this thread's nx words.
__device__ uint32_t search_level(const ReachDesc &d, const uint32_t *fb, uint32_t *vis,
                                 const uint32_t *fr, uint32_t *nx, int r0, int r1, int c0,
                                 int c1) {
    uint32_t any = 0;
    const int wpr = d.wpr, nw = c1 - c0 + 1, total = (r1 - r0 + 1) * nw;
    const float inv_nw = 1.0f / (float)nw;
    for (int q = threadIdx.x; q < total; q += blockDim.x) {
        int rr = (int)((float)q * inv_nw);
        if (rr * nw > q) --rr;
        if ((rr + 1) * nw <= q) ++rr;
        const int r = r0 + rr, c = c0 + (q - rr * nw), w = r * wpr + c;
        const uint32_t f = fr[w];
        uint32_t g = (f << 1) | (f >> 1);
        if (c > 0) g |= fr[w - 1] >> 31;
        if (c + 1 < wpr) g |= fr[w + 1] << 31;
        if (r > 0) g |= fr[w - wpr];
        if (r + 1 < d.H) g |= fr[w + wpr];
        const uint32_t n = g & fb[w] & ~vis[w];
        nx[w] = n;
        vis[w] |= n;
        any |= n;
    }
    return any;
}

// Rows and word columns that level `level` (>= 1 moves from cell a) can reach.
struct SearchBox {
    int r0, r1, c0, c1;
};

__device__ __forceinline__ SearchBox level_box(const ReachDesc &d, int a, int level) {
    const int i = a % d.W, j = a / d.W;
    SearchBox b;
    b.r0 = max(j - level, 0);
    b.r1 = min(j + level, d.H - 1);
    b.c0 = max(i - level, 0) >> 5;
    b.c1 = min(i + level, d.W - 1) >> 5;
    return b;
}

// Clears vis, fr and nx and seeds vis and fr with cell a (which must be C-free).
__device__ void search_start(const ReachDesc &d, uint32_t *vis, uint32_t *fr, uint32_t *nx,
                             int a) {
    uint4 *v4 = reinterpret_cast<uint4 *>(vis), *f4 = reinterpret_cast<uint4 *>(fr),
          *n4 = reinterpret_cast<uint4 *>(nx);
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (int w = threadIdx.x; w < (d.words + 3) / 4; w += blockDim.x) {
        v4[w] = z;
        f4[w] = z;
        n4[w] = z;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        set_cell(vis, d, a);
        set_cell(fr, d, a);
    }
    __syncthreads();
}

// Hop count from C-free a to b within max_hops moves, else -1 (uniform
// across the workgroup).  A 4-neighbour path is at least as long as the
// Manhattan distance, so a farther b is rejected without a search, and level
// L only touches the box of cells within L moves of a.
__device__ int hops_to(const ReachDesc &d, const uint32_t *fb, uint32_t *vis, uint32_t *fr,
                       uint32_t *nx, int a, int b, int max_hops) {
    if (a == b) return 0;
    const int man = abs(a % d.W - b % d.W) + abs(a / d.W - b / d.W);
    if (man > max_hops) return -1;
    search_start(d, vis, fr, nx, a);
    for (int level = 0; level < max_hops; ++level) {
        const SearchBox bx = level_box(d, a, level + 1);
        const uint32_t any = search_level(d, fb, vis, fr, nx, bx.r0, bx.r1, bx.c0, bx.c1);
        const int more = __syncthreads_or(any != 0u);
        if (cell_bit(nx, d, b)) return level + 1;
        if (!more) return -1;
        uint32_t *t = fr;
        fr = nx;
        nx = t;
    }
    return -1;
}

__device__ __forceinline__ double centre_dist(const ReachDesc &d, int a, int b) {
    const double dx = (double)(b % d.W - a % d.W) * (double)d.s;
    const double dy = (double)(b / d.W - a / d.W) * (double)d.s;
    return sqrt(dx * dx + dy * dy);
}

// The exact check of (a, b) for bin k: hop count when valid, else -1.
__device__ int check_pair(const ReachParams &rp, const ReachDesc &d, const uint32_t *fb,
                          uint32_t *vis, uint32_t *fr, uint32_t *nx, int a, int b, int k) {
    if (a < 0 || b < 0 || !cell_bit(fb, d, a) || !cell_bit(fb, d, b)) return -1;
    if (centre_dist(d, a, b) < rp.gmd) return -1;
    const int h = hops_to(d, fb, vis, fr, nx, a, b, rp.bin_hi[k]);
    return (h >= 0 && rp.hop_bin[h] == k) ? h : -1;
}

// Nearest C-free cell to c: least |di| + |dj|, then least index; -1 if none.
__device__ int snap_cell(const ReachDesc &d, const uint32_t *fb, int c, int *s_min) {
    if (cell_bit(fb, d, c)) return c;
    const int i0 = c % d.W, j0 = c / d.W;
    for (int r = 1; r <= d.W + d.H; ++r) {
        __syncthreads();
        if (threadIdx.x == 0) *s_min = INT_MAX;
        __syncthreads();
        for (int q = threadIdx.x; q < 4 * r; q += blockDim.x) {
            const int side = q / r, t = q % r;
            int di, dj;
            if (side == 0) {
                di = r - t;
                dj = t;
            } else if (side == 1) {
                di = -t;
                dj = r - t;
            } else if (side == 2) {
                di = t - r;
                dj = -t;
            } else {
                di = t;
                dj = t - r;
            }
            const int i = i0 + di, j = j0 + dj;
            if (i >= 0 && i < d.W && j >= 0 && j < d.H && cell_bit(fb, d, j * d.W + i))
                atomicMin(s_min, j * d.W + i);
        }
        __syncthreads();
        const int m = *s_min;
        if (m != INT_MAX) return m;
    }
    return -1;
}

__device__ __forceinline__ int decode_axis(float y, int n) {
    const double v = (double)y * (double)n;
    if (v != v) return 0;
    const double f = floor(v);
    return f < 0.0 ? 0 : (f > (double)(n - 1) ? n - 1 : (int)f);
}

__device__ __forceinline__ float decode_heading(float y) {
    double t = (double)y;
    t = t != t ? 0.0 : (t < -1.0 ? -1.0 : (t > 1.0 ? 1.0 : t));
    return (float)(t * kPiR);
}

__device__ __forceinline__ float cell_x(const ReachDesc &d, int c) {
    return (float)(((double)(c % d.W) + 0.5) * (double)d.s);
}

__device__ __forceinline__ float cell_y(const ReachDesc &d, int c) {
    return (float)(((double)(c / d.W) + 0.5) * (double)d.s);
}

__global__ __launch_bounds__(kReachThreads) void label_kernel(ReachParams rp, const int32_t *map,
                                                              uint32_t first_sid, int32_t *start,
                                                              int32_t *goal, int32_t *hops) {
    extern __shared__ uint4 lds4[];  // 16-byte aligned: the searches clear it 16 bytes at a time
    uint32_t *lds = reinterpret_cast<uint32_t *>(lds4);
    __shared__ unsigned long long s_best[kReachMaxBins];
    const int i = blockIdx.x, tid = threadIdx.x;
    const int mk = map[i];
    const ReachDesc d = rp.maps[(mk >= 0 && mk < rp.num_maps) ? mk : 0];
    const uint32_t sid = first_sid + (uint32_t)i;
    if (d.free_cnt == 0 || mk < 0 || mk >= rp.num_maps) {
        if (tid < rp.nbins) {
            goal[(int64_t)i * rp.nbins + tid] = -1;
            hops[(int64_t)i * rp.nbins + tid] = -1;
        }
        if (tid == 0) start[i] = -1;
        return;
    }
    uint32_t *fb = lds, *vis = fb + kReachMaxWords, *fr = vis + kReachMaxWords,
             *nx = fr + kReachMaxWords;
    uint32_t c[4] = {sid, 0u, 0u, 6u};
    philox4x32_10(c, rp.key0, rp.key1);
    const int a = rp.free_cells[d.free_off + pick_of(c[0], d.free_cnt)];
    stage_free(rp, d, fb);
    if (tid < kReachMaxBins) s_best[tid] = ~0ull;
    search_start(d, vis, fr, nx, a);
    for (int level = 0; level < rp.max_hops; ++level) {
        const SearchBox bx = level_box(d, a, level + 1);
        const uint32_t any = search_level(d, fb, vis, fr, nx, bx.r0, bx.r1, bx.c0, bx.c1);
        const int h = level + 1;
        const int k = rp.hop_bin[h];
        if (k >= 0 && any) {
            // the words this thread wrote in search_level (same box, same
            // order), so no barrier is needed before reading them
            unsigned long long best = ~0ull;
            const int nw = bx.c1 - bx.c0 + 1, total = (bx.r1 - bx.r0 + 1) * nw;
            const float inv_nw = 1.0f / (float)nw;
            for (int qi = tid; qi < total; qi += blockDim.x) {
                int rr = (int)((float)qi * inv_nw);
                if (rr * nw > qi) --rr;
                if ((rr + 1) * nw <= qi) ++rr;
                const int row = bx.r0 + rr, wc = bx.c0 + (qi - rr * nw);
                uint32_t n = nx[row * d.wpr + wc];
                const int col0 = wc * 32;
                while (n) {
                    const int bit = __ffs(n) - 1;
                    n &= n - 1u;
                    const int cell = row * d.W + col0 + bit;
                    if (centre_dist(d, a, cell) < rp.gmd) continue;
                    uint32_t q[4] = {sid, (uint32_t)cell, 0u, 5u};
                    philox4x32_10(q, rp.key0, rp.key1);
                    const unsigned long long v = ((unsigned long long)q[0] << 32) |
                                                 ((unsigned long long)cell << 16) |
                                                 (unsigned long long)h;
                    best = v < best ? v : best;
                }
            }
            if (best != ~0ull) atomicMin(&s_best[k], best);
        }
        if (!__syncthreads_or(any != 0u)) break;
        uint32_t *t = fr;
        fr = nx;
        nx = t;
    }
    __syncthreads();
    if (tid < rp.nbins) {
        const unsigned long long v = s_best[tid];
        goal[(int64_t)i * rp.nbins + tid] = v == ~0ull ? -1 : (int32_t)((v >> 16) & 0xffffu);
        hops[(int64_t)i * rp.nbins + tid] = v == ~0ull ? -1 : (int32_t)(v & 0xffffu);
    }
    if (tid == 0) start[i] = a;
}

// ---------------------------------------------------------------------------
// Searches in one wavefront's registers, for maps whose rows take WPR words
// with WPR dividing 32 (W <= 32, 64, ..., 1024 cells): lane l holds words
// [32 l, 32 l + 32) of the row-major C-free bitset, i.e. 32 / WPR whole rows,
// so a row's left and right carries stay in the lane and only the rows above
// the lane's first and below its last come from lanes l - 1 and l + 1
// (cross-lane moves).  No LDS and no workgroup barrier per level: the four
// wavefronts of a workgroup check four candidates at once.

// Word j (uniform) of a lane's 32 registers, without dynamic register indexing.
// One breadth-first level of wave_hops: the next frontier nx from fr; a cell
// joins it iff a 4-neighbour is in fr and it is still in un (C-free, not
// reached yet), and then leaves un.  Returns whether any lane's nx is
// non-empty.  A word's horizontal neighbours come from two funnel shifts with
// the adjacent words of its row.
template <int WPR>
__device__ __forceinline__ bool wave_level(const uint32_t fr[32], uint32_t nx[32], uint32_t un[32],
                                           int lane) {
    uint32_t up[WPR], dn[WPR];
#pragma unroll
    for (int k = 0; k < WPR; ++k) {
        // rows above the lane's first: the last row of lane - 1; below its
        // last: the first row of lane + 1; none past the ends.  DPP wavefront
        // shifts by one lane (wave_shr:1, wave_shl:1), the lane past an end
        // reading 0: one full-rate move each, no LDS permute and no select
        up[k] = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)fr[32 - WPR + k], 0x138, 0xf, 0xf,
                                                      true);
        dn[k] = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)fr[k], 0x130, 0xf, 0xf, true);
    }
    (void)lane;
    uint32_t any = 0u;
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        const uint32_t prev = j % WPR != 0 ? fr[j % WPR != 0 ? j - 1 : 0] : 0u;
        const uint32_t next = j % WPR != WPR - 1 ? fr[j % WPR != WPR - 1 ? j + 1 : 0] : 0u;
        const uint32_t h = __builtin_amdgcn_alignbit(fr[j], prev, 31u) |
                           __builtin_amdgcn_alignbit(next, fr[j], 1u);
        const uint32_t v = (j >= WPR ? fr[j >= WPR ? j - WPR : 0] : up[j < WPR ? j : 0]) |
                           (j + WPR < 32 ? fr[j + WPR < 32 ? j + WPR : 0]
                                         : dn[j + WPR >= 32 ? j + WPR - 32 : 0]);
        nx[j] = (h | v) & un[j];
        un[j] ^= nx[j];
        any |= nx[j];
    }
    return __ballot(any != 0u) != 0ull;
}

// Hop count from a to b (both C-free, a != b) within max_hops moves, else -1
// (uniform across the wavefront); the same levels as hops_to.  Per lane: 32
// words of rows of WPR words; two frontier buffers used in turn (two levels
// per loop pass, so no frontier is copied).
template <int WPR>
__device__ int wave_hops(const uint32_t *fb, const ReachDesc &d, int a, int b, int max_hops,
                         int lane, int c, const int *s_won, const int *g_won) {
    const int wa = (a / d.W) * WPR + ((a % d.W) >> 5);
    const int wb = (b / d.W) * WPR + ((b % d.W) >> 5);
    const int la = wa >> 5, ja = wa & 31, lb = wb >> 5;
    // b is reached when its bit leaves un; its register index is the same on
    // every lane (one relative register move)
    const int jb = __builtin_amdgcn_readfirstlane(wb & 31);
    const uint32_t ba = 1u << ((a % d.W) & 31), bb = (b % d.W) & 31;
    // the C-free words come from the staged map in LDS (lane l holds words
    // 32 l .. 32 l + 31), read once per search rather than kept in registers
    uint32_t f0[32], f1[32], un[32];
    const int base = lane * 32;
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        const uint32_t seed = (lane == la && j == ja) ? ba : 0u;
        f0[j] = seed;
        un[j] = (base + j < d.words ? fb[base + j] : 0u) & ~seed;
    }
    for (int level = 1; level <= max_hops; level += 2) {
        // a lower candidate of the round (s_won, LDS) or of the request (g_won,
        // device memory: other workgroups' rounds) already passed: this one
        // cannot win (looked at every 8 levels)
        if ((level & 7) == 1) {
            if (s_won && __atomic_load_n(s_won, __ATOMIC_RELAXED) < c) return -1;
            if (g_won && __atomic_load_n(g_won, __ATOMIC_RELAXED) < c) return -1;
        }
        bool more = wave_level<WPR>(f0, f1, un, lane);
        if (!((__shfl(un[jb], lb) >> bb) & 1u)) return level;
        if (!more || level + 1 > max_hops) return -1;
        more = wave_level<WPR>(f1, f0, un, lane);
        if (!((__shfl(un[jb], lb) >> bb) & 1u)) return level + 1;
        if (!more) return -1;
    }
    return -1;
}

__device__ __forceinline__ bool lds_cell(const uint32_t *fb, const ReachDesc &d, int c) {
    return (fb[(c / d.W) * d.wpr + ((c % d.W) >> 5)] >> ((c % d.W) & 31)) & 1u;
}

// Nearest C-free cell to c (least |di| + |dj|, then least index; -1 if none),
// by one wavefront: the cells of ring r split over the lanes, a ballot and a
// lane minimum.
__device__ int wave_snap(const ReachDesc &d, const uint32_t *fb, int c, int lane) {
    if (lds_cell(fb, d, c)) return c;
    const int i0 = c % d.W, j0 = c / d.W;
    for (int r = 1; r <= d.W + d.H; ++r) {
        int best = INT_MAX;
        for (int q = lane; q < 4 * r; q += 64) {
            const int side = q / r, t = q % r;
            const int di = side == 0 ? r - t : (side == 1 ? -t : (side == 2 ? t - r : t));
            const int dj = side == 0 ? t : (side == 1 ? r - t : (side == 2 ? -t : t - r));
            const int i = i0 + di, j = j0 + dj;
            if (i >= 0 && i < d.W && j >= 0 && j < d.H && lds_cell(fb, d, j * d.W + i))
                best = min(best, j * d.W + i);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o));
        if (best != INT_MAX) return best;
    }
    return -1;
}

// The exact check of (a, b) for bin k by one wavefront (see check_pair).
template <int WPR>
__device__ int wave_check(const ReachParams &rp, const ReachDesc &d, const uint32_t *fb,
                          int a, int b, int k, int lane, int c = 0, const int *s_won = nullptr,
                          const int *g_won = nullptr) {
    if (a < 0 || b < 0 || !lds_cell(fb, d, a) || !lds_cell(fb, d, b)) return -1;
    if (centre_dist(d, a, b) < rp.gmd) return -1;
    const int hi = rp.bin_hi[k];
    int h;
    if (a == b) {
        h = 0;
    } else {
        const int man = abs(a % d.W - b % d.W) + abs(a / d.W - b / d.W);
        h = man > hi ? -1 : wave_hops<WPR>(fb, d, a, b, hi, lane, c, s_won, g_won);
    }
    return (h >= 0 && rp.hop_bin[h] == k) ? h : -1;
}

// Candidate c of request i: network draw c < props (decoded, snapped), else
// rejection attempt c - props.  Returns the pair and the heading.
__device__ void candidate(const ReachParams &rp, const ProposeArgs &pa, const ReachDesc &d,
                          const uint32_t *fb, int i, int c, int lane, int &a, int &b,
                          float &th) {
    if (c < pa.props) {
        const float *y = pa.y + ((int64_t)i * pa.props + c) * 5;
        const int a0 = decode_axis(y[1], d.H) * d.W + decode_axis(y[0], d.W);
        const int b0 = decode_axis(y[4], d.H) * d.W + decode_axis(y[3], d.W);
        a = wave_snap(d, fb, a0, lane);
        b = wave_snap(d, fb, b0, lane);
        th = decode_heading(y[2]);
    } else {
        uint32_t q[4] = {pa.env[i], pa.episode[i], (uint32_t)(c - pa.props), 7u};
        philox4x32_10(q, rp.key0, rp.key1);
        a = rp.free_cells[d.free_off + pick_of(q[0], d.free_cnt)];
        b = rp.free_cells[d.free_off + pick_of(q[1], d.free_cnt)];
        th = (float)((((double)q[2] + 0.5) / kTwo32) * (2.0 * kPiR) - kPiR);
    }
}

// Proposals with one candidate per wavefront: candidates W r .. W r + W - 1
// (W wavefronts) are checked together and the lowest valid one wins, the
// result of checking them in order; `checks` counts as the sequential search
// does.
// Outputs of request i (row o): pair (a, b) and heading th, the winning
// candidate win (-1: none valid), its hop count h; checks as the sequential
// search counts them.
__device__ void write_request(const ProposeArgs &pa, const ReachDesc &d, int o, int win, int la,
                              int lb, int lh, float lth, int total) {
    float *p = pa.pose + (int64_t)o * 5;
    p[0] = la >= 0 ? cell_x(d, la) : 0.0f;
    p[1] = la >= 0 ? cell_y(d, la) : 0.0f;
    p[2] = lth;
    p[3] = lb >= 0 ? cell_x(d, lb) : 0.0f;
    p[4] = lb >= 0 ? cell_y(d, lb) : 0.0f;
    const int checks = win >= 0 ? win + 1 : total;
    if (pa.hops) pa.hops[o] = win >= 0 ? lh : -1;
    pa.source[o] = win;
    if (pa.checks) pa.checks[o] = checks;
    if (pa.stats) {
        atomicAdd(&pa.stats[0], 1ull);
        atomicAdd(&pa.stats[win < 0 ? 3 : (win < pa.props ? 1 : 2)], 1ull);
        atomicAdd(&pa.stats[4], (unsigned long long)checks);
    }
}

// W candidates c0 .. c0 + W - 1 of request i, one per wavefront; returns the
// lowest valid one (-1: none), with its pair, hop count and heading in the
// *_out arguments (every thread); with none valid and the request's last
// candidate (a rejection attempt) in this round, that attempt's pair and
// heading go there instead (the pair that stands when nothing is valid).
template <int WPR, int W>
__device__ int check_round(const ReachParams &rp, const ProposeArgs &pa, const ReachDesc &d,
                           const uint32_t *fb, int i, int k, int c0, int total, int &a_out,
                           int &b_out, int &h_out, float &th_out, const int *g_won = nullptr) {
    __shared__ int s_ok[W], s_a[W], s_b[W], s_h[W];
    __shared__ float s_th[W];
    __shared__ int s_won;  // lowest candidate of the round found valid so far
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = c0 + wave;
    if (threadIdx.x == 0) s_won = INT_MAX;
    __syncthreads();
    int a = -1, b = -1, h = -1;
    float th = 0.0f;
    if (c < total) {
        candidate(rp, pa, d, fb, i, c, lane, a, b, th);
        // searches of higher candidates stop once a lower one has passed
        // (they cannot win); the winner and the check counts are unchanged
        h = wave_check<WPR>(rp, d, fb, a, b, k, lane, c, &s_won, g_won);
        if (h >= 0 && lane == 0) atomicMin(&s_won, c);
    }
    if (lane == 0) {
        s_ok[wave] = (c < total && h >= 0) ? c : INT_MAX;
        s_a[wave] = a;
        s_b[wave] = b;
        s_h[wave] = h;
        s_th[wave] = th;
    }
    __syncthreads();
    int best = INT_MAX, bw = -1;
    for (int w = 0; w < W; ++w)
        if (s_ok[w] < best) {
            best = s_ok[w];
            bw = w;
        }
    int win = -1;
    if (bw >= 0) {
        win = best;
        a_out = s_a[bw];
        b_out = s_b[bw];
        h_out = s_h[bw];
        th_out = s_th[bw];
    } else if (total - 1 >= c0 && total - 1 < c0 + W && total - 1 >= pa.props) {
        // none valid: the last rejection attempt's pair stands
        const int w = total - 1 - c0;
        a_out = s_a[w];
        b_out = s_b[w];
        th_out = s_th[w];
    }
    __syncthreads();
    return win;
}

template <int WPR, int W>
__device__ void propose_waves(const ReachParams &rp, const ProposeArgs &pa, const ReachDesc &d,
                              const uint32_t *fb, int i, int o, int k) {
    const int total = pa.props + (d.free_cnt > 0 ? pa.tries : 0);
    int win = -1, la = -1, lb = -1, lh = -1;
    float lth = 0.0f;
    int c0 = 0;
    for (int round = 0; c0 < total && win < 0; c0 += W, ++round) {
        if (pa.head_rounds > 0 && round == pa.head_rounds) {
            // the rest of this request's rounds go to the tail launch
            if (threadIdx.x == 0) {
                const int p = atomicAdd(pa.n_pend, 1);
                pa.pend[p] = i;
                pa.best[p] = INT_MAX;
            }
            return;
        }
        win = check_round<WPR, W>(rp, pa, d, fb, i, k, c0, total, la, lb, lh, lth);
    }
    if (threadIdx.x == 0) write_request(pa, d, o, win, la, lb, lh, lth, total);
}

// One workgroup of W wavefronts per request.
template <int W>
__global__ __launch_bounds__(64 * W) void propose_kernel(ReachParams rp, ProposeArgs pa) {
    extern __shared__ uint4 lds4[];  // 16-byte aligned: the searches clear it 16 bytes at a time
    uint32_t *lds = reinterpret_cast<uint32_t *>(lds4);
    __shared__ int s_min;
    const int i = blockIdx.x, tid = threadIdx.x;
    if (pa.n_dev && i >= *pa.n_dev) return;  // past the requests counted on the device
    const int o = pa.slot ? pa.slot[i] : i;    // output row
    const int mk = pa.map[i], k = pa.bin[i];
    if (mk < 0 || mk >= rp.num_maps || k < 0 || k >= rp.nbins) {  // rejected request
        if (tid < 5) pa.pose[(int64_t)o * 5 + tid] = 0.0f;
        if (tid == 0) {
            if (pa.hops) pa.hops[o] = -1;
            pa.source[o] = -1;
            if (pa.checks) pa.checks[o] = 0;
            if (pa.stats) {
                atomicAdd(&pa.stats[0], 1ull);
                atomicAdd(&pa.stats[3], 1ull);
            }
        }
        return;
    }
    const ReachDesc d = rp.maps[mk];
    uint32_t *fb = lds, *vis = fb + kReachMaxWords, *fr = vis + kReachMaxWords,
             *nx = fr + kReachMaxWords;
    stage_free(rp, d, fb);
    __syncthreads();
    if (d.wpr * d.H <= kReachMaxWords && 32 % d.wpr == 0) {
        switch (d.wpr) {  // rows of 1, 2, 4, ..., 32 words: searches in registers
            case 1: propose_waves<1, W>(rp, pa, d, fb, i, o, k); return;
            case 2: propose_waves<2, W>(rp, pa, d, fb, i, o, k); return;
            case 4: propose_waves<4, W>(rp, pa, d, fb, i, o, k); return;
            case 8: propose_waves<8, W>(rp, pa, d, fb, i, o, k); return;
            case 16: propose_waves<16, W>(rp, pa, d, fb, i, o, k); return;
            default: propose_waves<32, W>(rp, pa, d, fb, i, o, k); return;
        }
    }
    int checks = 0, src = -1, ra = -1, rb = -1, rh = -1;
    float th = 0.0f;
    for (int j = 0; j < pa.props && src < 0; ++j) {
        const float *y = pa.y + ((int64_t)i * pa.props + j) * 5;
        const int a0 = decode_axis(y[1], d.H) * d.W + decode_axis(y[0], d.W);
        const int b0 = decode_axis(y[4], d.H) * d.W + decode_axis(y[3], d.W);
        const int a = snap_cell(d, fb, a0, &s_min);
        const int b = snap_cell(d, fb, b0, &s_min);
        ++checks;
        const int h = check_pair(rp, d, fb, vis, fr, nx, a, b, k);
        if (h >= 0) {
            src = j;
            ra = a;
            rb = b;
            rh = h;
            th = decode_heading(y[2]);
        }
    }
    for (int t = 0; t < pa.tries && src < 0 && d.free_cnt > 0; ++t) {
        uint32_t c[4] = {pa.env[i], pa.episode[i], (uint32_t)t, 7u};
        philox4x32_10(c, rp.key0, rp.key1);
        const int a = rp.free_cells[d.free_off + pick_of(c[0], d.free_cnt)];
        const int b = rp.free_cells[d.free_off + pick_of(c[1], d.free_cnt)];
        ++checks;
        const int h = check_pair(rp, d, fb, vis, fr, nx, a, b, k);
        ra = a;
        rb = b;
        th = (float)((((double)c[2] + 0.5) / kTwo32) * (2.0 * kPiR) - kPiR);
        if (h >= 0) {
            src = pa.props + t;
            rh = h;
        }
    }
    if (tid == 0) {
        float *p = pa.pose + (int64_t)o * 5;
        p[0] = ra >= 0 ? cell_x(d, ra) : 0.0f;
        p[1] = ra >= 0 ? cell_y(d, ra) : 0.0f;
        p[2] = th;
        p[3] = rb >= 0 ? cell_x(d, rb) : 0.0f;
        p[4] = rb >= 0 ? cell_y(d, rb) : 0.0f;
        if (pa.hops) pa.hops[o] = rh;
        pa.source[o] = src;
        if (pa.checks) pa.checks[o] = checks;
        if (pa.stats) {
            atomicAdd(&pa.stats[0], 1ull);
            atomicAdd(&pa.stats[src < 0 ? 3 : (src < pa.props ? 1 : 2)], 1ull);
            atomicAdd(&pa.stats[4], (unsigned long long)checks);
        }
    }
}

__global__ __launch_bounds__(1024) void compact_kernel(CompactArgs a) {
    // each thread takes 16 consecutive envs per pass (one 16-byte load of
    // their flags; bins read only for the flagged ones), and a workgroup
    // prefix sum of the per-thread counts places them in env order
    __shared__ int s_wave[16];
    __shared__ int s_base;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) {
        s_base = 0;
        if (a.n_pend) *a.n_pend = 0;
    }
    __syncthreads();
    const bool vec = (reinterpret_cast<uintptr_t>(a.defer) & 15u) == 0u;
    for (int e0 = 0; e0 < a.N; e0 += 1024 * 16) {
        const int eb = e0 + tid * 16;
        uint32_t m = 0u;  // bit i: env eb + i asks for a pair
        if (vec && eb + 16 <= a.N) {
            const uint4 v = *reinterpret_cast<const uint4 *>(a.defer + eb);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if ((w[q] >> (8 * b)) & 0xffu) m |= 1u << (4 * q + b);
        } else {
            for (int i = 0; i < 16; ++i)
                if (eb + i < a.N && a.defer[eb + i] != 0) m |= 1u << i;
        }
        for (uint32_t r = m; r != 0u; r &= r - 1u) {
            const int i = (int)__builtin_ctz(r);
            if (a.bin[eb + i] < 0) m &= ~(1u << i);
        }
        const int cnt = __popc(m);
        int inc = cnt;  // inclusive prefix sum over the wavefront
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(inc, o);
            if (lane >= o) inc += t;
        }
        if (lane == 63) s_wave[wave] = inc;
        __syncthreads();
        int before = s_base, total = 0;
        for (int w = 0; w < 16; ++w) {
            const int c = s_wave[w];
            before += w < wave ? c : 0;
            total += c;
        }
        int pos = before + inc - cnt;
        for (uint32_t r = m; r != 0u; r &= r - 1u, ++pos) {
            const int e = eb + (int)__builtin_ctz(r);
            a.src[e] = -1;
            if (pos < a.cap) {
                a.env[pos] = (uint32_t)e;
                a.map[pos] = a.env_map[e];
                a.rbin[pos] = a.bin[e];
                a.episode[pos] = a.ep[e];
            }
        }
        __syncthreads();
        if (tid == 0) s_base += total;
        __syncthreads();
    }
    if (tid == 0) {
        const int count = s_base;
        *a.n_out = count < a.cap ? count : a.cap;
        if (a.stats) {
            atomicAdd(&a.stats[0], (unsigned long long)count);
            atomicAdd(&a.stats[1], (unsigned long long)(count > a.cap ? count - a.cap : 0));
        }
    }
}

__global__ void noise_kernel(NoiseArgs a, uint32_t key0, uint32_t key1) {
    const int nq = (a.nz + 3) / 4;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = a.n_dev ? min(a.n, *a.n_dev) : a.n;
    const int64_t rows = (int64_t)n * a.per;
    if (idx >= rows * nq) return;
    const int64_t r = idx / nq;
    const int q = (int)(idx % nq);
    const int i = (int)(r / a.per), j = (int)(r % a.per);
    uint32_t c[4] = {a.c0 ? a.c0[i] : (uint32_t)i, a.c1 ? a.c1[i] : a.c1_const,
                     ((uint32_t)j << 8) | (uint32_t)q, a.stream};
    philox4x32_10(c, key0, key1);
    for (int t = 0; t < 4; ++t) {
        const int col = 4 * q + t;
        if (col < a.nz) {
            const double u = ((double)c[t] + 0.5) / kTwo32;
            a.z[r * a.nz + col] = bf16_bits((float)(2.0 * u - 1.0));
        }
    }
    if (q == 0 && a.row_idx) {
        const int m = a.map[i], b = a.bin[i];
        a.row_idx[r] = (m >= 0 && m < a.num_maps && b >= 0 && b < a.nbins) ? m * a.nbins + b : 0;
    }
}

__global__ void pool_rows_kernel(int num_maps, int nbins, const float *pool, uint16_t *rows) {
    const int width = kPoolCells + nbins;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)num_maps * nbins * width) return;
    const int64_t row = idx / width;
    const int col = (int)(idx % width);
    const int m = (int)(row / nbins), b = (int)(row % nbins);
    const float v = col < kPoolCells ? pool[(int64_t)m * kPoolCells + col]
                                     : (col - kPoolCells == b ? 1.0f : 0.0f);
    rows[idx] = bf16_bits(v);
}

__global__ void batch_kernel(BatchArgs a, uint32_t key0, uint32_t key1) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.batch) return;
    uint32_t c[4] = {a.step, (uint32_t)i, 0u, 10u};
    philox4x32_10(c, key0, key1);
    const int p = pick_of(c[0], a.num_pairs);
    int m = a.pair_map[p], b = a.pair_bin[p];
    const bool ok_mb = m >= 0 && m < a.num_maps && b >= 0 && b < a.nbins;
    const ReachDesc d = a.maps[ok_mb ? m : 0];
    int s = a.pair_start[p], g = a.pair_goal[p];
    const int cells = d.W * d.H;
    float *t = a.target + (int64_t)i * 5;
    if (!ok_mb || s < 0 || s >= cells || g < 0 || g >= cells) {
        a.map[i] = 0;
        a.bin[i] = 0;
        for (int q = 0; q < 5; ++q) t[q] = 0.0f;
        return;
    }
    a.map[i] = m;
    a.bin[i] = b;
    t[0] = (float)(((double)(s % d.W) + 0.5) / (double)d.W);
    t[1] = (float)(((double)(s / d.W) + 0.5) / (double)d.H);
    t[2] = 0.0f;
    t[3] = (float)(((double)(g % d.W) + 0.5) / (double)d.W);
    t[4] = (float)(((double)(g / d.W) + 0.5) / (double)d.H);
}

__global__ __launch_bounds__(256) void select_kernel(SelectArgs a) {
    __shared__ int s_j;
    const int i = blockIdx.x, tid = threadIdx.x;
    if (tid == 0) {
        const float *t = a.target + (int64_t)i * 5;
        int bj = 0;
        float bd = 0.0f;
        for (int j = 0; j < a.per; ++j) {
            const float *y = a.y + ((int64_t)i * a.per + j) * 5;
            float dsum = 0.0f;
            for (int q = 0; q < 5; ++q) {
                const float e = y[q] - t[q];
                dsum += a.w[q] * (e * e);
            }
            if (j == 0 || dsum < bd) {
                bd = dsum;
                bj = j;
            }
        }
        s_j = bj;
        if (a.chosen) a.chosen[i] = bj;
    }
    __syncthreads();
    const int j = s_j;
    const int width = kPoolCells + a.nbins + a.nz;
    const int m = a.map[i], b = a.bin[i];
    uint16_t *x = a.x + (int64_t)i * width;
    const uint16_t *z = a.z + ((int64_t)i * a.per + j) * a.nz;
    for (int col = tid; col < width; col += blockDim.x) {
        uint16_t v;
        if (col < kPoolCells)
            v = bf16_bits(a.pool[(int64_t)m * kPoolCells + col]);
        else if (col < kPoolCells + a.nbins)
            v = bf16_bits(col - kPoolCells == b ? 1.0f : 0.0f);
        else
            v = z[col - kPoolCells - a.nbins];
        x[col] = v;
    }
}

unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

constexpr size_t kSearchLds = 4u * kReachMaxWords * sizeof(uint32_t);

}  // namespace

hipError_t launch_label(const ReachParams &rp, int n, const int32_t *map, uint32_t first_sid,
                        int32_t *start, int32_t *goal, int32_t *hops, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(label_kernel, dim3((unsigned)n), dim3(kReachThreads), kSearchLds, s, rp,
                       map, first_sid, start, goal, hops);
    return hipGetLastError();
}

// Tail rounds: every (pending request, round) is one work item, taken by the
// workgroups of a fixed grid in round-major order (all requests' first tail
// round, then their second, ...), so a request's rounds run at once on
// different workgroups.  A round's lowest valid candidate goes to its slot and
// into the request's best index (atomic minimum); a round that starts above a
// valid candidate already found is skipped (it cannot win).  Requests reach
// the pending list only from the register search, so the same path serves.
template <int W>
__global__ __launch_bounds__(64 * W) void propose_tail_kernel(ReachParams rp, ProposeArgs pa,
                                                              int tail_rounds) {
    extern __shared__ uint4 lds4[];
    uint32_t *fb = reinterpret_cast<uint32_t *>(lds4);
    const int np = *pa.n_pend;
    const int items = np * tail_rounds;
    for (int g = blockIdx.x; g < items; g += gridDim.x) {
        const int p = g % np, r = g / np;
        const int i = pa.pend[p];
        const int mk = pa.map[i], k = pa.bin[i];
        const ReachDesc d = rp.maps[mk];
        const int total = pa.props + (d.free_cnt > 0 ? pa.tries : 0);
        const int c0 = (pa.head_rounds + r) * W;
        // uniform across the workgroup: one read of best, then a barrier
        // before any thread moves on
        __shared__ int s_skip;
        if (threadIdx.x == 0) s_skip = c0 >= total || __atomic_load_n(&pa.best[p], __ATOMIC_RELAXED) < c0;
        __syncthreads();
        const bool skip = s_skip != 0;
        __syncthreads();
        if (skip) continue;
        stage_free(rp, d, fb);
        __syncthreads();
        int a = -1, b = -1, h = -1, win = -1;
        float th = 0.0f;
        const int *gw = &pa.best[p];
        switch (d.wpr) {
            case 1: win = check_round<1, W>(rp, pa, d, fb, i, k, c0, total, a, b, h, th, gw); break;
            case 2: win = check_round<2, W>(rp, pa, d, fb, i, k, c0, total, a, b, h, th, gw); break;
            case 4: win = check_round<4, W>(rp, pa, d, fb, i, k, c0, total, a, b, h, th, gw); break;
            case 8: win = check_round<8, W>(rp, pa, d, fb, i, k, c0, total, a, b, h, th, gw); break;
            case 16: win = check_round<16, W>(rp, pa, d, fb, i, k, c0, total, a, b, h, th, gw); break;
            default: win = check_round<32, W>(rp, pa, d, fb, i, k, c0, total, a, b, h, th, gw); break;
        }
        if (threadIdx.x == 0 && win >= 0) {
            pa.tail[(int64_t)p * tail_rounds + r] = make_int4(a, b, h, __float_as_int(th));
            atomicMin(&pa.best[p], win);
        }
        __syncthreads();  // the map in LDS is restaged by the next item
    }
}

// Outputs of the pending requests: the lowest valid candidate any tail round
// found, else the last rejection attempt's pair (as the sequential search).
__global__ void propose_final_kernel(ReachParams rp, ProposeArgs pa, int tail_rounds, int W) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= *pa.n_pend) return;
    const int i = pa.pend[p], o = pa.slot ? pa.slot[i] : i;
    const ReachDesc d = rp.maps[pa.map[i]];
    const int total = pa.props + (d.free_cnt > 0 ? pa.tries : 0);
    const int win = pa.best[p] == INT_MAX ? -1 : pa.best[p];
    int la = -1, lb = -1, lh = -1;
    float lth = 0.0f;
    if (win >= 0) {
        const int4 q = pa.tail[(int64_t)p * tail_rounds + win / W - pa.head_rounds];
        la = q.x;
        lb = q.y;
        lh = q.z;
        lth = __int_as_float(q.w);
    } else if (total - 1 >= pa.props) {
        uint32_t q[4] = {pa.env[i], pa.episode[i], (uint32_t)(total - 1 - pa.props), 7u};
        philox4x32_10(q, rp.key0, rp.key1);
        la = rp.free_cells[d.free_off + pick_of(q[0], d.free_cnt)];
        lb = rp.free_cells[d.free_off + pick_of(q[1], d.free_cnt)];
        lth = (float)((((double)q[2] + 0.5) / kTwo32) * (2.0 * kPiR) - kPiR);
    }
    write_request(pa, d, o, win, la, lb, lh, lth, total);
}

int propose_width(int n) { return n <= kProposeWideMax ? 8 : 4; }

hipError_t launch_propose_tail(const ReachParams &rp, const ProposeArgs &a, int tail_rounds,
                               hipStream_t s) {
    if (a.n <= 0 || tail_rounds <= 0) return hipSuccess;
    // a fixed grid: the pending count is only known on the device
    const unsigned g = (unsigned)std::min<int64_t>((int64_t)a.n * tail_rounds, 1024);
    const int W = propose_width(a.n);
    if (W == 8)
        hipLaunchKernelGGL(propose_tail_kernel<8>, dim3(g), dim3(512), kSearchLds, s, rp, a,
                           tail_rounds);
    else
        hipLaunchKernelGGL(propose_tail_kernel<4>, dim3(g), dim3(256), kSearchLds, s, rp, a,
                           tail_rounds);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(propose_final_kernel, dim3(nblocks(a.n, 256)), dim3(256), 0, s, rp, a,
                       tail_rounds, W);
    return hipGetLastError();
}

hipError_t launch_propose(const ReachParams &rp, const ProposeArgs &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    // few requests (a step's resets): 8 candidates at a time shortens the
    // slowest requests, which set the launch's time; many (a batch): 4, fewer
    // checks past the first valid candidate
    if (propose_width(a.n) == 8)
        hipLaunchKernelGGL(propose_kernel<8>, dim3((unsigned)a.n), dim3(512), kSearchLds, s, rp, a);
    else
        hipLaunchKernelGGL(propose_kernel<4>, dim3((unsigned)a.n), dim3(256), kSearchLds, s, rp, a);
    return hipGetLastError();
}

hipError_t launch_compact(const CompactArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_noise(const NoiseArgs &a, uint32_t key0, uint32_t key1, hipStream_t s) {
    const int64_t total = (int64_t)a.n * a.per * ((a.nz + 3) / 4);
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(noise_kernel, dim3(nblocks(total, 256)), dim3(256), 0, s, a, key0, key1);
    return hipGetLastError();
}

hipError_t launch_pool_rows(int num_maps, int nbins, const float *pool, uint16_t *rows,
                            hipStream_t s) {
    const int64_t total = (int64_t)num_maps * nbins * (kPoolCells + nbins);
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(pool_rows_kernel, dim3(nblocks(total, 256)), dim3(256), 0, s, num_maps,
                       nbins, pool, rows);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs &a, uint32_t key0, uint32_t key1, hipStream_t s) {
    if (a.batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_kernel, dim3(nblocks(a.batch, 256)), dim3(256), 0, s, a, key0, key1);
    return hipGetLastError();
}

hipError_t launch_select(const SelectArgs &a, hipStream_t s) {
    if (a.batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(select_kernel, dim3((unsigned)a.batch), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace navsim
