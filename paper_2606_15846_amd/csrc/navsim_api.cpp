// Host side of libnavsim.so: argument checking, map packing, free-cell lists,
// env grouping, device allocation and kernel launches.  The C ABI is declared
// and documented in include/navsim.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <set>
#include <new>
#include <string>
#include <vector>

#include "navsim.h"
#include "navsim_host.hpp"
#include "navsim_internal.hpp"

using namespace navsim;

namespace navsim {

thread_local std::string g_err;

navsim_status fail(navsim_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

}  // namespace navsim

namespace {

navsim_status check_config(const navsim_config *c) {
    if (!c) return fail(NAVSIM_E_INVALID_ARG, "cfg is NULL");
    if (c->abi_version != NAVSIM_ABI_VERSION)
        return fail(NAVSIM_E_INVALID_ARG, "abi_version %u, library has %u", c->abi_version,
                    NAVSIM_ABI_VERSION);
    if (c->num_envs < 1) return fail(NAVSIM_E_INVALID_ARG, "num_envs must be >= 1");
    if (c->num_beams < 1 || c->num_beams > kMaxBeams)
        return fail(NAVSIM_E_INVALID_ARG, "num_beams must be in 1..%d", kMaxBeams);
    if (c->num_sectors < 1 || c->num_beams % c->num_sectors != 0)
        return fail(NAVSIM_E_INVALID_ARG, "num_sectors must divide num_beams");
    if (!finite_pos(c->fov_rad)) return fail(NAVSIM_E_INVALID_ARG, "fov_rad must be > 0");
    if (!finite_pos(c->max_range_m) || c->max_range_m > 1.0e4f)
        return fail(NAVSIM_E_INVALID_ARG, "max_range_m must be in (0, 1e4]");
    if (!finite_pos(c->dt_s)) return fail(NAVSIM_E_INVALID_ARG, "dt_s must be > 0");
    if (c->horizon < 1) return fail(NAVSIM_E_INVALID_ARG, "horizon must be >= 1");
    if (!isfinite(c->goal_radius_m) || c->goal_radius_m < 0.0f)
        return fail(NAVSIM_E_INVALID_ARG, "goal_radius_m must be >= 0");
    if (!isfinite(c->c_progress) || !isfinite(c->r_success) || !isfinite(c->r_collision))
        return fail(NAVSIM_E_INVALID_ARG, "reward parameters must be finite");
    if (c->footprint == NAVSIM_DISC) {
        if (!finite_pos(c->radius_m)) return fail(NAVSIM_E_INVALID_ARG, "radius_m must be > 0");
    } else if (c->footprint == NAVSIM_RECT) {
        if (!finite_pos(c->length_m) || !finite_pos(c->width_m))
            return fail(NAVSIM_E_INVALID_ARG, "length_m and width_m must be > 0");
    } else {
        return fail(NAVSIM_E_INVALID_ARG, "footprint must be NAVSIM_DISC or NAVSIM_RECT");
    }
    if (!isfinite(c->v_min) || !isfinite(c->v_max) || c->v_min > c->v_max)
        return fail(NAVSIM_E_INVALID_ARG, "need finite v_min <= v_max");
    if (!isfinite(c->w_min) || !isfinite(c->w_max) || c->w_min > c->w_max)
        return fail(NAVSIM_E_INVALID_ARG, "need finite w_min <= w_max");
    if (!isfinite(c->goal_min_dist_m) || c->goal_min_dist_m < 0.0f)
        return fail(NAVSIM_E_INVALID_ARG, "goal_min_dist_m must be >= 0");
    if (c->reset_max_tries < 1 || c->reset_max_tries > 1024)
        return fail(NAVSIM_E_INVALID_ARG, "reset_max_tries must be in 1..1024");
    return NAVSIM_OK;
}

// Angle of beam k of K to the heading: K equal steps from -pi over a full
// circle, K points spanning [-fov/2, fov/2] otherwise.
double beam_angle(float fov_rad, int K, int k) {
    const double pi = 3.14159265358979323846;
    const double fov = (double)fov_rad;
    if (fov >= 2.0 * pi - 1e-6) return -pi + (double)k * (2.0 * pi / (double)K);
    if (K == 1) return 0.0;
    return -0.5 * fov + (double)k * (fov / (double)(K - 1));
}

double circumradius(int footprint, float radius, float length, float width) {
    if (footprint == NAVSIM_DISC) return (double)radius;
    const double hl = 0.5 * (double)length, hb = 0.5 * (double)width;
    return sqrt(hl * hl + hb * hb);
}

// Host copy of the disc predicate used for the free-cell lists (same closed-box
// rule as the kernels: strictly closer than r, out of bounds occupied).
bool disc_clear_host(const uint8_t *occ, int W, int H, double s, double x, double y, double r) {
    const long i0 = (long)floor((x - r) / s), i1 = (long)floor((x + r) / s);
    const long j0 = (long)floor((y - r) / s), j1 = (long)floor((y + r) / s);
    const double r2 = r * r;
    for (long j = j0; j <= j1; ++j)
        for (long i = i0; i <= i1; ++i) {
            const bool filled = i < 0 || j < 0 || i >= W || j >= H || occ[(size_t)j * W + i] != 0;
            if (!filled) continue;
            const double bx0 = (double)i * s, bx1 = (double)(i + 1) * s;
            const double by0 = (double)j * s, by1 = (double)(j + 1) * s;
            const double cx = x < bx0 ? bx0 : (x > bx1 ? bx1 : x);
            const double cy = y < by0 ? by0 : (y > by1 ? by1 : y);
            const double ex = x - cx, ey = y - cy;
            if (ex * ex + ey * ey < r2) return false;
        }
    return true;
}

void drop_graph(navsim_s *h) {
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
    h->graph_steps = 0;
}

void free_device(navsim_s *h) {
    drop_graph(h);
    void *ptrs[] = {h->bits, h->maps, h->free_cells, h->env_map, h->perm, h->tiles};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    h->bits = nullptr;
    h->maps = nullptr;
    h->free_cells = nullptr;
    h->env_map = nullptr;
    h->perm = nullptr;
    h->tiles = nullptr;
}

template <typename T>
navsim_status upload(T **dst, const std::vector<T> &src) {
    const size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
    if (hipMalloc((void **)dst, bytes) != hipSuccess)
        return fail(NAVSIM_E_OOM, "hipMalloc of %zu bytes failed", bytes);
    if (!src.empty()) NS_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return NAVSIM_OK;
}


// LDS walk slots per chunk for workgroups of `threads` threads, given the
// device's LDS per workgroup (lds_block) and per CU (lds_cu).  Automatic (slots
// 0): within the share of a CU's LDS that lets the register budget's 16
// wavefronts per CU run together, beam table in LDS if at least 512 slots (or
// a whole tile's) still fit beside it, else in device memory; maps too large
// for that share get up to max(share, 64 KiB) as below.  Otherwise at most
// `slots` slots in lds_block, keeping the beam table in LDS when a full tile's
// rays still fit next to it.
int choose_ray_cap(int max_words, const navsim_config &c, int tile_envs, int threads, int slots,
                   int lds_block, int lds_cu, int cell_bytes, bool &beams_lds) {
    const int m = c.num_sectors, K = c.num_beams;
    const int share =
        std::min(lds_block, (int)((int64_t)lds_cu * (threads / 64) / kFusedWavesPerCu));
    int budget = lds_block;
    if (slots == 0) {
        const int full = ((tile_envs + 1) * K + 63) & ~63;
        for (const bool b : {true, false}) {
            const int cap = fused_ray_cap(max_words, m, tile_envs, K, b, share, cell_bytes);
            if (cap > 0 && (cap >= 512 || cap >= full)) {
                beams_lds = b;
                return cap;
            }
        }
        budget = std::min(lds_block, std::max(share, 65536));
    }
    int cap;
    const int with = fused_ray_cap(max_words, m, tile_envs, K, true, budget, cell_bytes);
    if (with >= tile_envs * K) {
        beams_lds = true;
        cap = with;
    } else {
        const int without = fused_ray_cap(max_words, m, tile_envs, K, false, budget, cell_bytes);
        beams_lds = without <= with;
        cap = beams_lds ? with : without;
    }
    if (cap > 0 && slots > 0) cap = std::min(cap, std::max(256, (slots + 63) & ~63));
    return cap;
}

// LDS words of the staged bitmaps: the largest bitmap, and for the run walk on
// the bitmap and its transpose (walk 5, exact traversal) the largest
// transposed one after it.
int staged_words(int max_words, int max_words_t, int walk, int scan_mode) {
    return max_words + ((scan_mode == NAVSIM_SCAN_TRAVERSAL && walk == 5) ? max_words_t : 0);
}

// LDS layout of the fused step for one launch shape and scan mode.  The claim
// walks (walk 3, 4, 5; exact traversal only) keep no ray slots; the chunked
// walks (and the march) use ray_cap slots.  walk 2 and 4 stage the map's
// byte-per-cell copy, walk 5 the transposed bitmap.  Fails with UNSUPPORTED
// when nothing fits.
struct FusedShape {
    int ray_cap = 0, cell_bytes = 0, claim = 0, resident = 0;
    bool beams_lds = true;
};

navsim_status fused_shape(const navsim_s *h, int max_words_row, int max_words_t, int tile_envs,
                          int threads, int slots, int walk, int scan_mode, FusedShape &out) {
    const navsim_config &c = h->cfg;
    const int m = c.num_sectors, K = c.num_beams;
    const int max_words = staged_words(max_words_row, max_words_t, walk, scan_mode);
    out.claim = scan_mode == NAVSIM_SCAN_TRAVERSAL && walk >= 3;
    // the run walk packs a hit's position in the transposed bitmap in 19 bits
    if (max_words > max_words_row && (int64_t)max_words_t * 32 >= (1 << 19))
        return fail(NAVSIM_E_UNSUPPORTED, "walk 5: a transposed bitmap of %d words is too large",
                    max_words_t);
    out.cell_bytes =
        (scan_mode == NAVSIM_SCAN_TRAVERSAL && (walk == 2 || walk == 4)) ? max_words_row * 32 : 0;
    if (out.cell_bytes && fused_static_lds(tile_envs, threads) != 0)
        return fail(NAVSIM_E_UNSUPPORTED,
                    "the byte walk needs a fused kernel without static LDS (tile_envs %d, "
                    "threads %d)",
                    tile_envs, threads);
    if (out.claim) {
        const size_t share = std::min<size_t>(
            (size_t)h->lds_block, (size_t)h->lds_cu * (threads / 64) / kFusedWavesPerCu);
        const size_t with = fused_lds_bytes(max_words, m, tile_envs, K, 0, out.cell_bytes);
        const size_t without = fused_lds_bytes(max_words, m, tile_envs, 0, 0, out.cell_bytes);
        if (without > (size_t)h->lds_block)
            return fail(NAVSIM_E_UNSUPPORTED,
                        "launch shape (tile_envs %d, threads %d, walk %d) does not fit LDS",
                        tile_envs, threads, walk);
        out.beams_lds = with <= (size_t)h->lds_block && (with <= share || without > share);
        out.ray_cap = 256;  // unused by the claim walk
    } else {
        out.ray_cap = choose_ray_cap(max_words, c, tile_envs, threads, slots, h->lds_block,
                                     h->lds_cu, out.cell_bytes, out.beams_lds);
        if (out.ray_cap == 0)
            return fail(NAVSIM_E_UNSUPPORTED,
                        "launch shape (tile_envs %d, threads %d, walk %d) and the largest map, "
                        "%d beams, %d sectors do not fit the LDS of one workgroup (%d bytes)",
                        tile_envs, threads, walk, K, m, h->lds_block);
    }
    out.resident = fused_resident_groups(max_words, m, tile_envs, threads, K, out.beams_lds,
                                         out.claim ? 0 : out.ray_cap, out.cell_bytes);
    if (out.resident <= 0) return fail(NAVSIM_E_HIP, "occupancy query of the fused step failed");
    return NAVSIM_OK;
}

void apply_shape(navsim_s *h, const FusedShape &f) {
    h->ray_cap = f.ray_cap;
    h->cell_bytes = f.cell_bytes;
    h->claim = f.claim;
    h->resident = f.resident;
    h->beams_lds = f.beams_lds;
}

// Envs grouped by map (stable in env order) into tiles of up to tile_envs envs,
// one fused workgroup each.
// A ray's fixed cost in units of one cell visit: claiming it, setting up its
// walk, its range and pooling (~360 VALU lane-slots per ray against ~10 per
// visited cell in the C4 counters, ~35 visits), plus its partial last window
// and the lanes that idle as rays end.  C4's step time is flat for 50 to 250
// and 1 % slower with the bare cell count.
constexpr double kRayCostCells = 64.0;

// Scan work of one env on a map, for scheduling only: K times (the mean
// number of cells a ray walks + a ray's fixed cost), from a few rays cast on
// the host (up to 128 free cells, 16 directions each, first occupied or
// outside cell or r_max).
double map_scan_work(const uint8_t *occ, int W, int H, double s, double rmax, int K,
                     const int32_t *free_cells, int free_cnt) {
    if (free_cnt <= 0) return (double)K;
    const int samples = std::min(free_cnt, 128), stride = std::max(1, free_cnt / samples);
    const double rc = rmax / s;
    double cells = 0.0;
    int rays = 0;
    for (int q = 0; q < samples; ++q) {
        const int c = free_cells[(int64_t)q * stride];
        const double x0 = (c % W) + 0.5, y0 = (c / W) + 0.5;
        for (int a = 0; a < 16; ++a) {
            const double th = (a + 0.25) * (2.0 * M_PI / 16.0);
            const double dx = cos(th), dy = sin(th);
            int i = (int)x0, j = (int)y0, n = 0;
            const int si = dx > 0 ? 1 : -1, sj = dy > 0 ? 1 : -1;
            const double tdx = fabs(1.0 / dx), tdy = fabs(1.0 / dy);
            double tx = (dx > 0 ? (i + 1 - x0) : (x0 - i)) * tdx;
            double ty = (dy > 0 ? (j + 1 - y0) : (y0 - j)) * tdy;
            for (;;) {
                if (tx < ty) {
                    if (tx > rc) break;
                    i += si;
                    tx += tdx;
                } else {
                    if (ty > rc) break;
                    j += sj;
                    ty += tdy;
                }
                ++n;
                if (i < 0 || j < 0 || i >= W || j >= H || occ[(size_t)j * W + i]) break;
            }
            cells += n;
            ++rays;
        }
    }
    return (double)K * (kRayCostCells + cells / rays);
}

// Launch order for the XCDs' own L2 caches.  The dispatcher hands workgroup i
// to XCD i mod kXcds, so the tiles at positions x, x + kXcds, x + 2 kXcds, ...
// all run on XCD x; placing a map's tiles there lets that XCD's L2 fetch the
// map's bitmaps from HBM once instead of every XCD fetching them.  Maps go to
// XCDs in descending total work, each to the least-loaded XCD with room for
// all of its tiles (each XCD takes exactly its share of positions; a map is
// split only when no XCD has room), and each XCD runs its own tiles heaviest
// first.  Results do not depend on the order; small launches (fewer than two
// tiles per XCD, or fewer maps than XCDs) keep the plain heaviest-first order.
// Multiply-shift constants of a map's two small divisions (MapDesc), checked
// over the whole operand range once per distinct divisor.
int ceil_log2(uint32_t x) {
    int s = 0;
    while ((1u << s) < x) ++s;
    return s;
}

bool magic_for(uint32_t d, int bits, uint32_t &magic, int32_t &shift) {
    shift = bits + ceil_log2(d);
    magic = (uint32_t)(((1ull << shift) + d - 1) / d);
    static std::mutex mu;
    static std::set<std::pair<uint32_t, int>> checked;  // divisors already verified
    std::lock_guard<std::mutex> lock(mu);
    if (checked.count({d, bits})) return true;
    for (uint64_t x = 0; x < (1ull << bits); ++x)
        if ((uint32_t)((x * magic) >> shift) != (uint32_t)(x / d)) return false;
    checked.insert({d, bits});
    return true;
}

bool set_quotient_magic(MapDesc &d, int sectors) {
    return magic_for((uint32_t)d.K, 18, d.k_magic, d.k_shift) &&
           magic_for((uint32_t)(d.K / sectors), 12, d.per_magic, d.per_shift);
}

void order_tiles_by_xcd(std::vector<Tile> &tiles, const std::vector<double> &map_weight) {
    const int T = (int)tiles.size();
    std::vector<int> maps;  // in first-seen order of the heaviest-first list
    std::vector<double> work(map_weight.size(), 0.0);
    std::vector<int> ntile(map_weight.size(), 0);
    for (const Tile &t : tiles) {
        if (ntile[t.map]++ == 0) maps.push_back(t.map);
        work[t.map] += map_weight[t.map] * t.count;
    }
    if (T < 2 * kXcds || (int)maps.size() < kXcds) return;
    std::stable_sort(maps.begin(), maps.end(),
                     [&](int a, int b) { return work[a] > work[b]; });
    std::vector<int> room(kXcds), xcd_of(map_weight.size(), -1);
    std::vector<double> load(kXcds, 0.0);
    for (int x = 0; x < kXcds; ++x) room[x] = T / kXcds + (x < T % kXcds ? 1 : 0);
    std::vector<std::vector<Tile>> per(kXcds);
    std::vector<std::vector<Tile>> by_map(map_weight.size());
    for (const Tile &t : tiles) by_map[t.map].push_back(t);  // heaviest first within a map
    for (const int m : maps) {
        std::vector<Tile> &mt = by_map[m];
        size_t next = 0;
        while (next < mt.size()) {
            const int need = (int)(mt.size() - next);
            int best = -1;
            for (int x = 0; x < kXcds; ++x)  // least loaded with room for the rest
                if (room[x] >= need && (best < 0 || load[x] < load[best])) best = x;
            if (best < 0)  // none: the XCD with the most room takes what fits
                for (int x = 0; x < kXcds; ++x)
                    if (room[x] > 0 && (best < 0 || room[x] > room[best])) best = x;
            const int take = std::min(need, room[best]);
            for (int k = 0; k < take; ++k, ++next) {
                per[best].push_back(mt[next]);
                load[best] += map_weight[m] * mt[next].count;
            }
            room[best] -= take;
        }
    }
    for (int x = 0; x < kXcds; ++x)
        std::stable_sort(per[x].begin(), per[x].end(), [&](const Tile &a, const Tile &b) {
            return map_weight[a.map] * a.count > map_weight[b.map] * b.count;
        });
    for (int i = 0; i < T; ++i) tiles[i] = per[i % kXcds][i / kXcds];
}

// Envs grouped by map into tiles, launched heaviest first (longest-processing-
// time order) by the tiles' estimated scan work (envs x the map's work per
// env); tiles of equal weight keep their order, so a map's full tiles stay
// together.  balance = 0: tiles of tile_envs envs (a map's last one smaller).
// balance = 1: each map gets enough tiles that every tile's estimated work is
// about equal, at least target_tiles in all (the workgroups that run at once),
// at most tile_envs envs per tile; a map's envs split into near-equal tiles.
void build_tiles(const std::vector<int32_t> &env_map, int tile_envs,
                 const std::vector<double> &map_weight, int balance, int target_tiles,
                 std::vector<int32_t> &perm, std::vector<Tile> &tiles) {
    const int N = (int)env_map.size();
    perm.resize(N);
    for (int e = 0; e < N; ++e) perm[e] = e;
    std::stable_sort(perm.begin(), perm.end(),
                     [&](int32_t a, int32_t b) { return env_map[a] < env_map[b]; });
    tiles.clear();
    // maps in use: [first, first + count) of perm
    std::vector<int> mfirst, mcount, mid;
    for (int i = 0; i < N;) {
        int j = i;
        while (j < N && env_map[perm[j]] == env_map[perm[i]]) ++j;
        mid.push_back(env_map[perm[i]]);
        mfirst.push_back(i);
        mcount.push_back(j - i);
        i = j;
    }
    const int nm = (int)mid.size();
    std::vector<int> ntiles(nm);
    int total = 0;
    for (int q = 0; q < nm; ++q) {
        ntiles[q] = (mcount[q] + tile_envs - 1) / tile_envs;
        total += ntiles[q];
    }
    if (balance) {
        // one more tile, each time, to the map whose tiles carry the most work
        while (total < target_tiles) {
            int best = -1;
            double load = 0.0;
            for (int q = 0; q < nm; ++q) {
                if (ntiles[q] >= mcount[q]) continue;  // one env per tile already
                const double l = map_weight[mid[q]] * (double)mcount[q] / ntiles[q];
                if (l > load) {
                    load = l;
                    best = q;
                }
            }
            if (best < 0) break;
            ++ntiles[best];
            ++total;
        }
    }
    for (int q = 0; q < nm; ++q) {
        const int n = mcount[q], T = ntiles[q];
        if (balance) {
            for (int t = 0, at = 0; t < T; ++t) {
                const int c = n / T + (t < n % T ? 1 : 0);
                tiles.push_back(Tile{mid[q], mfirst[q] + at, c, 0});
                at += c;
            }
        } else {
            for (int at = 0; at < n; at += tile_envs)
                tiles.push_back(Tile{mid[q], mfirst[q] + at, std::min(tile_envs, n - at), 0});
        }
    }
    std::stable_sort(tiles.begin(), tiles.end(), [&](const Tile &a, const Tile &b) {
        return map_weight[a.map] * a.count > map_weight[b.map] * b.count;
    });
    order_tiles_by_xcd(tiles, map_weight);
}

navsim_status run(navsim_t h, const StepParams &p, int kernel, hipStream_t s) {
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return fail(NAVSIM_E_HIP, "hipSetDevice: %s", hipGetErrorString(g.err));
    const hipError_t e =
        kernel == NAVSIM_KERNEL_PLAIN ? launch_plain(p, s) : launch_fused(p, h->tile_envs, s);
    if (e != hipSuccess) return fail(NAVSIM_E_HIP, "kernel launch: %s", hipGetErrorString(e));
    return NAVSIM_OK;
}

// After a fused launch that deferred resets: the attached proposer writes a
// pair for every deferred env it serves, then one masked reset pass applies
// them (the free-space sampler for the rest) and writes their reset rows.
navsim_status finish_deferred(navsim_t h, float *obs, uint8_t *fallback, hipStream_t s) {
    navsim_status st = h->hook.run(h->hook.ctx, s);
    if (st != NAVSIM_OK) return st;
    StepParams q = make_step_params(h);
    q.mode = 1;
    q.mask = h->hook.defer;
    q.pose = h->hook.pose;
    q.pose_src = h->hook.src;
    q.obs = obs;
    q.d_fb = fallback;
    return run(h, q, NAVSIM_KERNEL_FUSED, s);
}

navsim_status step_common(navsim_t h, const float *act, float *obs, float *reward,
                          uint8_t *terminated, uint8_t *truncated, float *final_obs,
                          const navsim_debug *dbg, int32_t kernel, void *stream) {
    if (!h) return fail(NAVSIM_E_BAD_HANDLE, "handle is NULL");
    if (!h->loaded) return fail(NAVSIM_E_STATE, "navsim_load_maps has not been called");
    if (!h->initialized) return fail(NAVSIM_E_STATE, "navsim_reset (mask NULL) must come first");
    if (!act || !obs || !reward || !terminated || !truncated)
        return fail(NAVSIM_E_INVALID_ARG, "act, obs, reward, terminated, truncated are required");
    if (kernel != NAVSIM_KERNEL_FUSED && kernel != NAVSIM_KERNEL_PLAIN)
        return fail(NAVSIM_E_INVALID_ARG, "unknown kernel %d", kernel);
    StepParams p = make_step_params(h);
    p.mode = 0;
    p.act = act;
    p.obs = obs;
    p.reward = reward;
    p.term = terminated;
    p.trunc = truncated;
    p.final_obs = final_obs;
    if (dbg) {
        p.d_ranges = dbg->ranges;
        p.d_hits = dbg->hits;
        p.d_visits = dbg->visits;
        p.d_coll = dbg->collision;
        p.d_goal = dbg->goal;
        p.d_reset = dbg->reset;
        p.d_fb = dbg->fallback;
    }
    if (!h->hook.run) return run(h, p, kernel, (hipStream_t)stream);
    if (kernel != NAVSIM_KERNEL_FUSED)
        return fail(NAVSIM_E_UNSUPPORTED, "learned resets (navsim_rp_attach) run with the fused step only");
    p.defer_bin = h->hook.bin;
    p.defer_out = h->hook.defer;
    navsim_status st = run(h, p, kernel, (hipStream_t)stream);
    if (st != NAVSIM_OK) return st;
    return finish_deferred(h, obs, dbg ? dbg->fallback : nullptr, (hipStream_t)stream);
}

// Every launch parameter (buffers, maps, settings) is part of a captured
// rollout's key; StepParams starts zeroed, so its bytes compare.
bool same_outputs(const StepParams &a, const StepParams &b) {
    return memcmp(&a, &b, sizeof a) == 0;
}

// Step `i` of a rollout: outputs advanced by i rows of each buffer.
StepParams rollout_step(const StepParams &p0, int i, int64_t N, int row) {
    StepParams p = p0;
    p.step_off = i;
    if (p.act_out) p.act_out += (int64_t)i * N * 2;
    p.obs += (int64_t)i * N * row;
    p.reward += (int64_t)i * N;
    p.term += (int64_t)i * N;
    p.trunc += (int64_t)i * N;
    if (p.final_obs) p.final_obs += (int64_t)i * N * row;
    return p;
}

navsim_status launch_steps(navsim_t h, const StepParams &p0, int steps, int kernel,
                           hipStream_t s) {
    const int64_t N = h->cfg.num_envs;
    const int row = h->cfg.num_sectors + 4;
    for (int i = 0; i < steps; ++i) {
        const StepParams p = rollout_step(p0, i, N, row);
        const hipError_t e =
            kernel == NAVSIM_KERNEL_PLAIN ? launch_plain(p, s) : launch_fused(p, h->tile_envs, s);
        if (e != hipSuccess) return fail(NAVSIM_E_HIP, "kernel launch: %s", hipGetErrorString(e));
    }
    return NAVSIM_OK;
}

// Captures the rollout's step launches once into an executable graph; later
// calls with the same buffers, step count, kernel and launch shape replay it.
navsim_status rollout_graph(navsim_t h, const StepParams &p0, int steps, int kernel) {
    if (h->graph && h->graph_steps == steps && h->graph_kernel == kernel &&
        h->graph_tile_envs == h->tile_envs && same_outputs(h->graph_params, p0))
        return NAVSIM_OK;
    drop_graph(h);
    if (!h->capture_stream)
        NS_HIP(hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking));
    NS_HIP(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
    const navsim_status st = launch_steps(h, p0, steps, kernel, h->capture_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(h->capture_stream, &graph);
    if (st != NAVSIM_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(NAVSIM_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess)
        return fail(NAVSIM_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
    h->graph = exec;
    h->graph_params = p0;
    h->graph_steps = steps;
    h->graph_kernel = kernel;
    h->graph_tile_envs = h->tile_envs;
    return NAVSIM_OK;
}

}  // namespace

// Launch parameters of the handle's current maps, state and settings.
StepParams navsim::make_step_params(const navsim_s *h) {
    const navsim_config &c = h->cfg;
    StepParams p;
    memset(&p, 0, sizeof p);
    p.N = c.num_envs;
    p.K = c.num_beams;  // the largest per-map beam count
    p.m = c.num_sectors;
    p.horizon = c.horizon;
    p.tries = c.reset_max_tries;
    p.rmax = c.max_range_m;
    p.dt = c.dt_s;
    p.goal_r = c.goal_radius_m;
    p.c1 = c.c_progress;
    p.r_succ = c.r_success;
    p.r_coll = c.r_collision;
    p.vlo = c.v_min;
    p.vhi = c.v_max;
    p.wlo = c.w_min;
    p.whi = c.w_max;
    p.gmd = c.goal_min_dist_m;
    p.key0 = (uint32_t)(c.seed & 0xffffffffu);
    p.key1 = (uint32_t)(c.seed >> 32);
    p.st = h->st;
    p.env_map = h->env_map;
    p.maps = h->maps;
    p.bits = h->bits;
    p.free_cells = h->free_cells;
    p.beams = h->beams;
    p.perm = h->perm;
    p.tiles = h->tiles;
    p.num_tiles = h->num_tiles;
    p.num_maps = h->num_maps;
    p.max_words = staged_words(h->max_words, h->max_words_t, h->walk_mode, h->scan_mode);
    p.tbits_off = p.max_words > h->max_words ? h->max_words : 0;
    p.refill_at = h->refill_at;
    p.groups = h->groups;
    p.ray_cap = h->ray_cap;
    p.beams_lds = h->beams_lds ? 1 : 0;
    p.scan_mode = h->scan_mode;
    p.walk_mode = h->walk_mode;
    p.cell_bytes = h->cell_bytes;
    p.claim = h->claim;
    p.queue = h->persist ? h->queue : nullptr;
    p.chunk = h->persist;
    p.resident = h->resident;
    p.wg_threads = h->wg_threads;
    p.march_kmax = h->march_kmax;
    p.march_h = h->march_h;
    return p;
}

extern "C" {

const char *navsim_last_error(void) { return g_err.c_str(); }

navsim_status navsim_create(const navsim_config *cfg, int hip_device, navsim_t *out) {
    if (!out) return fail(NAVSIM_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    const navsim_status s = check_config(cfg);
    if (s != NAVSIM_OK) return s;
    int ndev = 0;
    NS_HIP(hipGetDeviceCount(&ndev));
    if (hip_device < 0 || hip_device >= ndev)
        return fail(NAVSIM_E_INVALID_ARG, "hip_device %d not in 0..%d", hip_device, ndev - 1);
    DeviceGuard g(hip_device);
    if (g.err != hipSuccess) return fail(NAVSIM_E_HIP, "hipSetDevice: %s", hipGetErrorString(g.err));
    navsim_s *h = new (std::nothrow) navsim_s();
    if (!h) return fail(NAVSIM_E_OOM, "host allocation failed");
    h->cfg = *cfg;
    h->device = hip_device;
    const size_t N = (size_t)cfg->num_envs;
    if (hipMalloc(&h->state_buf, 40 * N) != hipSuccess) {
        delete h;
        return fail(NAVSIM_E_OOM, "hipMalloc of the env state failed");
    }
    if (hipMemset(h->state_buf, 0, 40 * N) != hipSuccess) {
        (void)hipFree(h->state_buf);
        delete h;
        return fail(NAVSIM_E_HIP, "hipMemset of the env state failed");
    }
    if (hipMalloc(&h->step_ctr, 2 * sizeof(uint32_t)) != hipSuccess) {
        (void)hipFree(h->state_buf);
        delete h;
        return fail(NAVSIM_E_OOM, "hipMalloc of the step counter failed");
    }
    // LDS limits of the device (gfx950: 160 KiB per CU, and per workgroup)
    if (hipDeviceGetAttribute(&h->lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock,
                              hip_device) != hipSuccess ||
        hipDeviceGetAttribute(&h->lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                              hip_device) != hipSuccess) {
        (void)hipFree(h->step_ctr);
        (void)hipFree(h->state_buf);
        delete h;
        return fail(NAVSIM_E_HIP, "LDS size query failed");
    }
    h->lds_block = std::max(h->lds_block, 65536);
    h->lds_cu = std::max(h->lds_cu, h->lds_block);
    // the tile queue starts at zero; every persistent launch leaves it there
    if (hipMalloc(&h->queue, 2 * sizeof(int32_t)) != hipSuccess ||
        hipMemset(h->queue, 0, 2 * sizeof(int32_t)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        if (h->queue) (void)hipFree(h->queue);
        (void)hipFree(h->step_ctr);
        (void)hipFree(h->state_buf);
        delete h;
        return fail(NAVSIM_E_HIP, "tile queue allocation failed");
    }
    float *f = (float *)h->state_buf;
    h->st.x = f;
    h->st.y = f + N;
    h->st.th = f + 2 * N;
    h->st.v = f + 3 * N;
    h->st.w = f + 4 * N;
    h->st.gx = f + 5 * N;
    h->st.gy = f + 6 * N;
    h->st.dprev = f + 7 * N;
    h->st.t = (int32_t *)(f + 8 * N);
    h->st.ep = (uint32_t *)(f + 9 * N);
    *out = h;
    return NAVSIM_OK;
}

navsim_status navsim_load_maps(navsim_t h, int32_t num_maps, const int32_t *width,
                               const int32_t *height, const float *res_m, const uint8_t *occ,
                               const int32_t *env_map) {
    return navsim_load_maps_ex(h, num_maps, width, height, res_m, occ, env_map, nullptr);
}

navsim_status navsim_load_maps_ex(navsim_t h, int32_t num_maps, const int32_t *width,
                                  const int32_t *height, const float *res_m, const uint8_t *occ,
                                  const int32_t *env_map, const navsim_map_profile *profiles) {
    if (!h) return fail(NAVSIM_E_BAD_HANDLE, "handle is NULL");
    if (num_maps < 1 || !width || !height || !res_m || !occ || !env_map)
        return fail(NAVSIM_E_INVALID_ARG, "num_maps >= 1 and all arrays are required");
    const int N = h->cfg.num_envs;
    const navsim_config &cfg = h->cfg;
    std::vector<navsim_map_profile> prof((size_t)num_maps);
    for (int k = 0; k < num_maps; ++k) {
        if (profiles) {
            prof[k] = profiles[k];
        } else {
            prof[k].num_beams = cfg.num_beams;
            prof[k].footprint = cfg.footprint;
            prof[k].radius_m = cfg.radius_m;
            prof[k].length_m = cfg.length_m;
            prof[k].width_m = cfg.width_m;
        }
        const navsim_map_profile &q = prof[k];
        if (q.num_beams < 1 || q.num_beams > cfg.num_beams || q.num_beams % cfg.num_sectors != 0)
            return fail(NAVSIM_E_INVALID_ARG,
                        "map %d: num_beams %d must be in 1..%d and a multiple of num_sectors", k,
                        q.num_beams, cfg.num_beams);
        if (q.footprint == NAVSIM_DISC) {
            if (!finite_pos(q.radius_m)) return fail(NAVSIM_E_INVALID_ARG, "map %d: radius_m", k);
        } else if (q.footprint == NAVSIM_RECT) {
            if (!finite_pos(q.length_m) || !finite_pos(q.width_m))
                return fail(NAVSIM_E_INVALID_ARG, "map %d: length_m and width_m", k);
        } else {
            return fail(NAVSIM_E_INVALID_ARG, "map %d: footprint", k);
        }
    }
    std::vector<int64_t> occ_off(num_maps + 1, 0);
    for (int k = 0; k < num_maps; ++k) {
        if (width[k] < 1 || height[k] < 1 || width[k] > 4096 || height[k] > 4096)
            return fail(NAVSIM_E_INVALID_ARG, "map %d: size %dx%d out of range", k, width[k],
                        height[k]);
        if (!finite_pos(res_m[k])) return fail(NAVSIM_E_INVALID_ARG, "map %d: res must be > 0", k);
        {
            const navsim_map_profile &q = prof[k];
            const double rc = circumradius(q.footprint, q.radius_m, q.length_m, q.width_m);
            const double win = floor(2.0 * rc / (double)res_m[k]) + 2.0;
            if (win > (double)kMaxFootprintCells)
                return fail(NAVSIM_E_UNSUPPORTED,
                            "map %d: the footprint's candidate window, %.0f cells per side "
                            "(circumscribed radius %.4f m at %.4f m cells), exceeds %d", k, win,
                            rc, (double)res_m[k], kMaxFootprintCells);
        }
        const int64_t wpr = (width[k] + 2 * kPad + 31) / 32;
        if (wpr * (int64_t)(height[k] + 2 * kPad) > kMaxMapWords)
            return fail(NAVSIM_E_UNSUPPORTED,
                        "map %d: padded bitmap of %lld words exceeds the %d-word LDS budget", k,
                        (long long)(wpr * (height[k] + 2 * kPad)), kMaxMapWords);
        if (width[k] + height[k] + 2 * kPad > 8191)
            return fail(NAVSIM_E_UNSUPPORTED, "map %d: width + height must be at most %d", k,
                        8191 - 2 * kPad);
        occ_off[k + 1] = occ_off[k] + (int64_t)width[k] * height[k];
    }
    std::vector<int> used(num_maps, 0);
    for (int e = 0; e < N; ++e) {
        if (env_map[e] < 0 || env_map[e] >= num_maps)
            return fail(NAVSIM_E_INVALID_ARG, "env_map[%d] = %d not in 0..%d", e, env_map[e],
                        num_maps - 1);
        used[env_map[e]] = 1;
    }

    // padded bitmaps, beam tables (one per distinct beam count), free-cell lists
    std::vector<MapDesc> descs(num_maps);
    std::vector<double2> beams;
    std::map<int, int32_t> beam_off;
    std::vector<uint32_t> bits;
    std::vector<int32_t> free_cells;
    int max_words = 4, max_words_t = 4;
    for (int k = 0; k < num_maps; ++k) {
        const int W = width[k], H = height[k];
        const uint8_t *m = occ + occ_off[k];
        MapDesc &d = descs[k];
        d.w = W;
        d.h = H;
        d.wpr = (W + 2 * kPad + 31) / 32;
        d.words = ((d.wpr * (H + 2 * kPad)) + 3) & ~3;
        d.word_off = (int64_t)bits.size();
        d.res = res_m[k];
        d.K = prof[k].num_beams;
        d.footprint = prof[k].footprint;
        d.radius = prof[k].radius_m;
        d.len = prof[k].length_m;
        d.wid = prof[k].width_m;
        d.rc = circumradius(d.footprint, d.radius, d.len, d.wid);
        if (!set_quotient_magic(d, cfg.num_sectors))
            return fail(NAVSIM_E_UNSUPPORTED, "map %d: no exact quotient constants for %d beams", k,
                        d.K);
        auto it = beam_off.find(d.K);
        if (it == beam_off.end()) {
            it = beam_off.emplace(d.K, (int32_t)beams.size()).first;
            for (int b = 0; b < d.K; ++b) {
                const double a = beam_angle(cfg.fov_rad, d.K, b);
                beams.push_back(make_double2(cos(a), sin(a)));
            }
        }
        d.beam_off = it->second;
        bits.resize(bits.size() + d.words, 0xffffffffu);
        uint32_t *b = bits.data() + d.word_off;
        for (int iy = 0; iy < H; ++iy) {
            uint32_t *row = b + (size_t)(iy + kPad) * d.wpr;
            for (int wd = 0; wd < d.wpr; ++wd) row[wd] = 0u;
            for (int c = 0; c < d.wpr * 32; ++c) {
                const int ix = c - kPad;
                const bool filled = ix < 0 || ix >= W || m[(size_t)iy * W + ix] != 0;
                if (filled) row[c >> 5] |= 1u << (c & 31);
            }
        }
        max_words = std::max(max_words, d.words);
        // transposed copy: line c = ix + kPad holds the padded column, bit r =
        // iy + kPad; the same ring of occupied cells
        d.wpr_t = (H + 2 * kPad + 31) / 32;
        d.words_t = ((d.wpr_t * (W + 2 * kPad)) + 3) & ~3;
        d.word_off_t = (int64_t)bits.size();
        bits.resize(bits.size() + d.words_t, 0xffffffffu);
        uint32_t *bt = bits.data() + d.word_off_t;
        for (int ix = 0; ix < W; ++ix) {
            uint32_t *line = bt + (size_t)(ix + kPad) * d.wpr_t;
            for (int wd = 0; wd < d.wpr_t; ++wd) line[wd] = 0u;
            for (int r = 0; r < d.wpr_t * 32; ++r) {
                const int iy = r - kPad;
                const bool filled = iy < 0 || iy >= H || m[(size_t)iy * W + ix] != 0;
                if (filled) line[r >> 5] |= 1u << (r & 31);
            }
        }
        max_words_t = std::max(max_words_t, d.words_t);
        d.free_off = (int64_t)free_cells.size();
        const double s = (double)res_m[k];
        for (int iy = 0; iy < H; ++iy)
            for (int ix = 0; ix < W; ++ix) {
                const float cx = (float)(((double)ix + 0.5) * s);
                const float cy = (float)(((double)iy + 0.5) * s);
                if (disc_clear_host(m, W, H, s, (double)cx, (double)cy, d.rc))
                    free_cells.push_back(iy * W + ix);
            }
        d.free_cnt = (int32_t)((int64_t)free_cells.size() - d.free_off);
        if (used[k] && d.free_cnt == 0)
            return fail(NAVSIM_E_NO_FREE_SPACE, "map %d has no cell where the footprint fits", k);
    }

    FusedShape shape;
    {
        DeviceGuard g(h->device);
        const navsim_status fs = fused_shape(h, max_words, max_words_t, h->tile_envs, h->wg_threads,
                                             h->ray_slots, h->walk_mode, h->scan_mode, shape);
        if (fs != NAVSIM_OK) return fs;
    }
    std::vector<int32_t> host_env_map(env_map, env_map + N);
    std::vector<double> map_weight(num_maps);
    for (int k = 0; k < num_maps; ++k)
        map_weight[k] = used[k] ? map_scan_work(occ + occ_off[k], width[k], height[k],
                                                (double)res_m[k], (double)cfg.max_range_m,
                                                descs[k].K, free_cells.data() + descs[k].free_off,
                                                descs[k].free_cnt)
                                : 0.0;
    std::vector<int32_t> perm;
    std::vector<Tile> tiles;
    build_tiles(host_env_map, h->tile_envs, map_weight, h->balance, shape.resident, perm, tiles);

    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return fail(NAVSIM_E_HIP, "hipSetDevice: %s", hipGetErrorString(g.err));
    free_device(h);
    if (h->beams) (void)hipFree(h->beams);
    h->beams = nullptr;
    h->loaded = false;
    h->initialized = false;
    navsim_status s;
    if ((s = upload(&h->beams, beams)) != NAVSIM_OK) return s;
    std::vector<int32_t> em(env_map, env_map + N);
    if ((s = upload(&h->bits, bits)) != NAVSIM_OK) return s;
    if ((s = upload(&h->maps, descs)) != NAVSIM_OK) return s;
    if ((s = upload(&h->free_cells, free_cells)) != NAVSIM_OK) return s;
    if ((s = upload(&h->env_map, em)) != NAVSIM_OK) return s;
    if ((s = upload(&h->perm, perm)) != NAVSIM_OK) return s;
    if ((s = upload(&h->tiles, tiles)) != NAVSIM_OK) return s;
    h->num_maps = num_maps;
    h->num_tiles = (int)tiles.size();
    h->max_words = max_words;
    h->max_words_t = max_words_t;
    apply_shape(h, shape);
    h->host_env_map.swap(host_env_map);
    h->host_map_weight.swap(map_weight);
    h->host_occ.assign(occ, occ + occ_off[num_maps]);
    h->host_occ_off = occ_off;
    h->host_w.assign(width, width + num_maps);
    h->host_h.assign(height, height + num_maps);
    h->host_res.assign(res_m, res_m + num_maps);
    h->host_rc.resize(num_maps);
    h->host_free_off.resize(num_maps);
    h->host_free_cnt.resize(num_maps);
    for (int k = 0; k < num_maps; ++k) {
        h->host_rc[k] = descs[k].rc;
        h->host_free_off[k] = descs[k].free_off;
        h->host_free_cnt[k] = descs[k].free_cnt;
    }
    h->host_free.swap(free_cells);
    h->loaded = true;
    return NAVSIM_OK;
}

navsim_status navsim_reset(navsim_t h, const uint8_t *mask, float *obs, void *hip_stream) {
    if (!h) return fail(NAVSIM_E_BAD_HANDLE, "handle is NULL");
    if (!h->loaded) return fail(NAVSIM_E_STATE, "navsim_load_maps has not been called");
    if (!obs) return fail(NAVSIM_E_INVALID_ARG, "obs is required");
    if (mask && !h->initialized)
        return fail(NAVSIM_E_STATE, "the first reset must cover all envs (mask NULL)");
    StepParams p = make_step_params(h);
    p.mode = 1;
    p.mask = mask;
    p.obs = obs;
    p.defer_bin = h->hook.bin;
    p.defer_out = h->hook.defer;
    navsim_status s = run(h, p, NAVSIM_KERNEL_FUSED, (hipStream_t)hip_stream);
    if (s == NAVSIM_OK && h->hook.run) s = finish_deferred(h, obs, nullptr, (hipStream_t)hip_stream);
    if (s == NAVSIM_OK) h->initialized = true;
    return s;
}

navsim_status navsim_reset_to(navsim_t h, const uint8_t *mask, const float *pose, float *obs,
                              void *hip_stream) {
    if (!h) return fail(NAVSIM_E_BAD_HANDLE, "handle is NULL");
    if (!h->loaded) return fail(NAVSIM_E_STATE, "navsim_load_maps has not been called");
    if (!pose || !obs) return fail(NAVSIM_E_INVALID_ARG, "pose and obs are required");
    if (mask && !h->initialized)
        return fail(NAVSIM_E_STATE, "the first reset must cover all envs (mask NULL)");
    StepParams p = make_step_params(h);
    p.mode = 1;
    p.mask = mask;
    p.pose = pose;
    p.obs = obs;
    const navsim_status s = run(h, p, NAVSIM_KERNEL_FUSED, (hipStream_t)hip_stream);
    if (s == NAVSIM_OK) h->initialized = true;
    return s;
}

navsim_status navsim_step(navsim_t h, const float *act, float *obs, float *reward,
                          uint8_t *terminated, uint8_t *truncated, float *final_obs,
                          void *hip_stream) {
    return step_common(h, act, obs, reward, terminated, truncated, final_obs, nullptr,
                       NAVSIM_KERNEL_FUSED, hip_stream);
}

navsim_status navsim_step_plain(navsim_t h, const float *act, float *obs, float *reward,
                                uint8_t *terminated, uint8_t *truncated, float *final_obs,
                                void *hip_stream) {
    return step_common(h, act, obs, reward, terminated, truncated, final_obs, nullptr,
                       NAVSIM_KERNEL_PLAIN, hip_stream);
}

navsim_status navsim_step_debug(navsim_t h, const float *act, float *obs, float *reward,
                                uint8_t *terminated, uint8_t *truncated, float *final_obs,
                                const navsim_debug *dbg, int32_t kernel, void *hip_stream) {
    return step_common(h, act, obs, reward, terminated, truncated, final_obs, dbg, kernel,
                       hip_stream);
}

navsim_status navsim_get_state(navsim_t h, void *host_soa, size_t bytes, void *hip_stream) {
    if (!h) return fail(NAVSIM_E_BAD_HANDLE, "handle is NULL");
    if (!host_soa || bytes != NAVSIM_STATE_BYTES(h->cfg.num_envs))
        return fail(NAVSIM_E_INVALID_ARG, "need a host buffer of exactly %zu bytes",
                    NAVSIM_STATE_BYTES(h->cfg.num_envs));
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return fail(NAVSIM_E_HIP, "hipSetDevice: %s", hipGetErrorString(g.err));
    NS_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
    NS_HIP(hipMemcpy(host_soa, h->state_buf, bytes, hipMemcpyDeviceToHost));
    return NAVSIM_OK;
}

navsim_status navsim_set_state(navsim_t h, const void *host_soa, size_t bytes, void *hip_stream) {
    if (!h) return fail(NAVSIM_E_BAD_HANDLE, "handle is NULL");
    if (!host_soa || bytes != NAVSIM_STATE_BYTES(h->cfg.num_envs))
        return fail(NAVSIM_E_INVALID_ARG, "need a host buffer of exactly %zu bytes",
                    NAVSIM_STATE_BYTES(h->cfg.num_envs));
    if (!h->loaded) return fail(NAVSIM_E_STATE, "navsim_load_maps has not been called");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return fail(NAVSIM_E_HIP, "hipSetDevice: %s", hipGetErrorString(g.err));
    NS_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
    NS_HIP(hipMemcpy(h->state_buf, host_soa, bytes, hipMemcpyHostToDevice));
    h->initialized = true;
    return NAVSIM_OK;
}

navsim_status navsim_rollout(navsim_t h, int32_t steps, uint64_t first_step, float *act,
                             float *obs, float *reward, uint8_t *terminated, uint8_t *truncated,
                             float *final_obs, int32_t kernel, int32_t flags, void *stream) {
    if (!h) return fail(NAVSIM_E_BAD_HANDLE, "handle is NULL");
    if (!h->loaded) return fail(NAVSIM_E_STATE, "navsim_load_maps has not been called");
    if (!h->initialized) return fail(NAVSIM_E_STATE, "navsim_reset (mask NULL) must come first");
    if (steps < 1 || steps > 4096) return fail(NAVSIM_E_INVALID_ARG, "steps must be in 1..4096");
    if (!obs || !reward || !terminated || !truncated)
        return fail(NAVSIM_E_INVALID_ARG, "obs, reward, terminated, truncated are required");
    if (kernel != NAVSIM_KERNEL_FUSED && kernel != NAVSIM_KERNEL_PLAIN)
        return fail(NAVSIM_E_INVALID_ARG, "unknown kernel %d", kernel);
    if (flags & ~NAVSIM_ROLLOUT_GRAPH) return fail(NAVSIM_E_INVALID_ARG, "unknown flags 0x%x", flags);
    if (h->hook.run)
        return fail(NAVSIM_E_UNSUPPORTED,
                    "rollouts use the in-kernel sampler: detach the reset proposer first");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return fail(NAVSIM_E_HIP, "hipSetDevice: %s", hipGetErrorString(g.err));
    StepParams p = make_step_params(h);
    p.mode = 0;
    p.act = nullptr;
    p.step_ctr = h->step_ctr;
    p.act_out = act;
    p.obs = obs;
    p.reward = reward;
    p.term = terminated;
    p.trunc = truncated;
    p.final_obs = final_obs;
    const hipStream_t s = (hipStream_t)stream;
    if (flags & NAVSIM_ROLLOUT_GRAPH) {
        const navsim_status st = rollout_graph(h, p, steps, kernel);
        if (st != NAVSIM_OK) return st;
    }
    hipError_t e = launch_set_step(h->step_ctr, first_step, s);
    if (e != hipSuccess) return fail(NAVSIM_E_HIP, "kernel launch: %s", hipGetErrorString(e));
    if (!(flags & NAVSIM_ROLLOUT_GRAPH)) return launch_steps(h, p, steps, kernel, s);
    e = hipGraphLaunch(h->graph, s);
    if (e != hipSuccess) return fail(NAVSIM_E_HIP, "hipGraphLaunch: %s", hipGetErrorString(e));
    return NAVSIM_OK;
}

navsim_status navsim_set_scan(navsim_t h, int32_t mode, float step_m) {
    if (!h) return fail(NAVSIM_E_BAD_HANDLE, "handle is NULL");
    if (mode != NAVSIM_SCAN_TRAVERSAL && mode != NAVSIM_SCAN_MARCH)
        return fail(NAVSIM_E_INVALID_ARG, "unknown scan mode %d", mode);
    int kmax = 0;
    if (mode == NAVSIM_SCAN_MARCH) {
        if (!finite_pos(step_m)) return fail(NAVSIM_E_INVALID_ARG, "step_m must be > 0");
        const double hh = (double)step_m, rmax = (double)h->cfg.max_range_m;
        const double q = floor(rmax / hh);
        if (q > (double)(1 << 20))
            return fail(NAVSIM_E_INVALID_ARG, "max_range_m / step_m must be <= 2^20");
        kmax = (int)q;
        while ((double)(kmax + 1) * hh <= rmax) ++kmax;
        while (kmax > 0 && (double)kmax * hh > rmax) --kmax;
    }
    FusedShape shape;
    if (h->loaded) {
        DeviceGuard g(h->device);
        const navsim_status fs = fused_shape(h, h->max_words, h->max_words_t, h->tile_envs, h->wg_threads,
                                             h->ray_slots, h->walk_mode, mode, shape);
        if (fs != NAVSIM_OK) return fs;
    }
    {
        DeviceGuard g(h->device);
        drop_graph(h);
    }
    if (h->loaded) apply_shape(h, shape);
    h->scan_mode = mode;
    h->march_h = mode == NAVSIM_SCAN_MARCH ? (double)step_m : 0.0;
    h->march_kmax = kmax;
    return NAVSIM_OK;
}

navsim_status navsim_set_tuning(navsim_t h, const navsim_tuning *t) {
    if (!h) return fail(NAVSIM_E_BAD_HANDLE, "handle is NULL");
    if (!t) return fail(NAVSIM_E_INVALID_ARG, "tuning is NULL");
    if (!fused_tile_envs_supported(t->tile_envs))
        return fail(NAVSIM_E_INVALID_ARG, "tile_envs must be 1, 2, 4, 8, 16 or 32");
    if (t->refill_at < 0 || t->refill_at > 63)
        return fail(NAVSIM_E_INVALID_ARG, "refill_at must be in 0..63");
    if (t->groups < 1 || t->groups > 64) return fail(NAVSIM_E_INVALID_ARG, "groups must be in 1..64");
    if (t->ray_slots < 0 || (t->ray_slots > 0 && t->ray_slots < 256))
        return fail(NAVSIM_E_INVALID_ARG, "ray_slots must be 0 or >= 256");
    if (t->walk < 0 || t->walk > 5) return fail(NAVSIM_E_INVALID_ARG, "walk must be in 0..5");
    if (t->persist < 0 || t->persist > 64)
        return fail(NAVSIM_E_INVALID_ARG, "persist must be in 0..64");
    if (!fused_threads_supported(t->threads))
        return fail(NAVSIM_E_INVALID_ARG, "threads must be 256, 512 or 1024");
    if (t->tile_envs * 16 > t->threads)
        return fail(NAVSIM_E_INVALID_ARG, "tile_envs %d needs at least %d threads", t->tile_envs,
                    t->tile_envs * 16);
    if (t->balance != 0 && t->balance != 1)
        return fail(NAVSIM_E_INVALID_ARG, "balance must be 0 or 1");
    {
        DeviceGuard g(h->device);
        drop_graph(h);
    }
    FusedShape shape;
    if (h->loaded) {
        DeviceGuard g(h->device);
        const navsim_status fs = fused_shape(h, h->max_words, h->max_words_t, t->tile_envs, t->threads,
                                             t->ray_slots, t->walk, h->scan_mode, shape);
        if (fs != NAVSIM_OK) return fs;
    }
    if (h->loaded) {
        std::vector<int32_t> perm;
        std::vector<Tile> tiles;
        build_tiles(h->host_env_map, t->tile_envs, h->host_map_weight, t->balance, shape.resident,
                    perm, tiles);
        DeviceGuard g(h->device);
        if (g.err != hipSuccess) return fail(NAVSIM_E_HIP, "hipSetDevice: %s", hipGetErrorString(g.err));
        NS_HIP(hipDeviceSynchronize());
        (void)hipFree(h->perm);
        (void)hipFree(h->tiles);
        h->perm = nullptr;
        h->tiles = nullptr;
        navsim_status s;
        if ((s = upload(&h->perm, perm)) != NAVSIM_OK) return s;
        if ((s = upload(&h->tiles, tiles)) != NAVSIM_OK) return s;
        h->num_tiles = (int)tiles.size();
    }
    h->tile_envs = t->tile_envs;
    h->refill_at = t->refill_at;
    h->groups = t->groups;
    h->ray_slots = t->ray_slots;
    h->walk_mode = t->walk;
    h->persist = t->persist;
    h->wg_threads = t->threads;
    h->balance = t->balance;
    if (h->loaded) apply_shape(h, shape);
    return NAVSIM_OK;
}

navsim_status navsim_get_tuning(navsim_t h, navsim_tuning *t) {
    if (!h) return fail(NAVSIM_E_BAD_HANDLE, "handle is NULL");
    if (!t) return fail(NAVSIM_E_INVALID_ARG, "tuning is NULL");
    t->tile_envs = h->tile_envs;
    t->refill_at = h->refill_at;
    t->groups = h->groups;
    t->ray_slots = h->ray_slots;
    t->walk = h->walk_mode;
    t->persist = h->persist;
    t->threads = h->wg_threads;
    t->balance = h->balance;
    return NAVSIM_OK;
}

navsim_status navsim_destroy(navsim_t h) {
    if (!h) return fail(NAVSIM_E_BAD_HANDLE, "handle is NULL");
    if (h->proposers > 0)
        return fail(NAVSIM_E_STATE, "%d reset proposer(s) still use this handle: destroy them first",
                    h->proposers);
    {
        DeviceGuard g(h->device);
        free_device(h);
        if (h->beams) (void)hipFree(h->beams);
        if (h->state_buf) (void)hipFree(h->state_buf);
        if (h->step_ctr) (void)hipFree(h->step_ctr);
        if (h->queue) (void)hipFree(h->queue);
        if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
    }
    delete h;
    return NAVSIM_OK;
}

}  // extern "C"
