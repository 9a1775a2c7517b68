// Internal types shared by the host API (navsim_api.cpp) and the kernels
// (navsim_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "navsim.h"

namespace navsim {

// Padded bitmap layout.  A map of W x H cells is stored with a ring of kPad
// occupied cells on every side: row r = iy + kPad in 0..H + 2 kPad - 1,
// column c = ix + kPad, bit c & 31 of word r * wpr + (c >> 5), with
// 32 * wpr >= W + 2 kPad; every bit at c >= W + kPad is set.  Leaving the map
// reads as occupied, and a walk that starts inside the map can look up to kPad
// cells ahead without leaving the stored rows.
constexpr int kPad = 4;
constexpr int kMaxMapWords = 12288;  // largest padded bitmap staged in LDS (48 KiB)
constexpr int kMaxBeams = 4096;
// Largest footprint window, in cells per side: floor(2 rc / s) + 2 for the
// circumscribed radius rc at cell size s bounds the candidate cells of the
// disc, of every heading of the rectangle and of the goal disc.  Maps whose
// profile exceeds it are rejected at load.
constexpr int kMaxFootprintCells = 128;
// Default launch shape of the fused step (a good choice on every workload
// measured; the autotuner refines it per workload)
constexpr int kDefaultTileEnvs = 8;   // envs per fused workgroup
constexpr int kDefaultRefillAt = 40;  // refill idle lanes once at most this many are busy
constexpr int kDefaultGroups = 8;     // 4-cell groups walked between refill checks
constexpr int kDefaultWalk = 3;       // claim walk on the bitmap (any map size)

struct MapDesc {
    int32_t w, h;
    int32_t wpr;        // words per padded row
    int32_t words;      // padded words, rounded up to a multiple of 4
    int64_t word_off;   // start in the bit pool (multiple of 4 words)
    int64_t free_off;   // start of this map's free-cell list
    int32_t free_cnt;
    float res;
    // robot/sensor profile of envs on this map
    int32_t K;          // beams
    int32_t beam_off;   // start of this map's beam table
    int32_t footprint;  // NAVSIM_DISC / NAVSIM_RECT
    float radius, len, wid;
    double rc;          // circumradius of the footprint
    // the same bitmap transposed (line c = padded column, bit r = padded row;
    // kPad occupied ring, every bit at r >= H + kPad set), for walk 5
    int32_t wpr_t;       // words per padded column
    int32_t words_t;     // padded words, rounded up to a multiple of 4
    int64_t word_off_t;  // start in the bit pool (multiple of 4 words)
    // exact quotients by multiply and shift: floor(x / K) = x k_magic >> k_shift
    // for x < 2^18 (a claim index), floor(b / per) = b per_magic >> per_shift
    // for b < 2^12 (a beam; per = K / sectors), with magic = ceil(2^shift / d)
    // and shift = 18 (12) + ceil(log2 d), so that x d <= 2^shift
    uint32_t k_magic, per_magic;
    int32_t k_shift, per_shift;
};

// A group of up to tile_envs envs that share one map (one fused workgroup).
struct Tile {
    int32_t map, first, count, pad;
};

struct DevState {
    float *x, *y, *th, *v, *w, *gx, *gy, *dprev;
    int32_t *t;
    uint32_t *ep;
};

// Everything a step or reset launch needs, passed by value.
struct StepParams {
    int32_t N, K, m, horizon, tries, mode;  // K: largest beam count; mode 0 step, 1 reset
    int32_t refill_at, groups;  // fused walk: refill threshold, 4-cell groups per check
    int32_t walk_mode;          // fused walk: 0 groups of 4 cells, 1 runs, 2 groups on bytes,
                                // 3 claim walk (setup and finish per claimed ray), 4 on bytes,
                                // 5 claim walk over runs on the bitmap and its transpose
    int32_t cell_bytes;         // walk 2, 4: LDS bytes of the byte-per-cell map copy (else 0)
    int32_t claim;              // claim walk in use (walk 3, 4 with the exact traversal)
    int32_t *queue;             // persistent workgroups: {next tile, finished groups}, or null
    int32_t chunk;              // persistent workgroups: tiles taken at a time
    int32_t resident;           // persistent workgroups: how many stay resident on the device
    int32_t wg_threads;         // fused step: threads per workgroup (256, 512, 1024)
    int32_t ray_cap;            // rays walked per chunk (LDS slots)
    int32_t beams_lds;          // stage the beam table in LDS
    int32_t scan_mode;          // 0 exact traversal, 1 fixed-step march
    int32_t march_kmax;         // march: last sample index with k h <= r_max
    double march_h;             // march: sample spacing, metres
    float rmax, dt, goal_r, c1, r_succ, r_coll;
    float vlo, vhi, wlo, whi, gmd;
    uint32_t key0, key1;
    DevState st;
    const int32_t *env_map;
    const MapDesc *maps;
    const uint32_t *bits;
    const int32_t *free_cells;
    const double2 *beams;  // (cos, sin) of each beam's angle to the heading
    const int32_t *perm;   // env ids grouped by map
    const Tile *tiles;
    int32_t num_tiles, num_maps, max_words;  // max_words: LDS words of the staged bitmaps
    int32_t tbits_off;  // walk 5: LDS word offset of the staged transposed bitmap (else 0)
    // inputs / outputs
    const float *act;          // normalised actions [N][2], or null in a rollout
    const uint32_t *step_ctr;  // rollout: device {lo, hi} of the first step index
    int32_t step_off;          // rollout: this step's offset from that index
    float *act_out;            // rollout: the drawn actions [N][2] (may be null)
    const uint8_t *mask;
    const float *pose;         // reset to given poses [N][5] (x, y, heading, goal x, goal y), or null
    const int32_t *pose_src;   // with pose: env e takes row e only when pose_src[e] >= 0, else
                               // the free-space sampler (null: every masked env takes its row)
    const int32_t *defer_bin;  // envs whose episode ends with defer_bin[e] >= 0 are not reset
                               // here (null: none); a later reset pass gives them their pair
    uint8_t *defer_out;        // [N]: 1 where the env ended and deferred its reset, else 0
    float *obs, *reward, *final_obs;
    uint8_t *term, *trunc;
    // diagnostics (may be null)
    float *d_ranges;
    int32_t *d_hits, *d_visits;
    uint8_t *d_coll, *d_goal, *d_reset, *d_fb;
};

size_t fused_lds_bytes(int max_words, int m, int tile_envs, int K, int ray_cap, int cell_bytes);
int fused_ray_cap(int max_words, int m, int tile_envs, int K, bool beams_lds, int budget,
                  int cell_bytes);
// Wavefronts per CU that the fused step's register budget allows (4 per SIMD).
constexpr int kFusedWavesPerCu = 16;
constexpr int kXcds = 8;  // gfx950: 8 XCDs of 32 CUs, each with its own L2
// Workgroups of the fused step that fit on the current device at once (0 on error).
int fused_resident_groups(int max_words, int m, int tile_envs, int threads, int K, bool beams_lds,
                          int ray_cap, int cell_bytes);
bool fused_tile_envs_supported(int tile_envs);
bool fused_threads_supported(int threads);
// Static LDS bytes of the fused kernel for a shape (-1 on error).  The byte
// walk needs 0: its map copy must start at LDS address 0.
int fused_static_lds(int tile_envs, int threads);
hipError_t launch_fused(const StepParams &p, int tile_envs, hipStream_t s);
hipError_t launch_plain(const StepParams &p, hipStream_t s);
hipError_t launch_set_step(uint32_t *ctr, uint64_t first_step, hipStream_t s);

}  // namespace navsim
