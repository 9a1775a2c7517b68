// Internal types shared by the host API (navsim_api.cpp) and the kernels
// (navsim_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "navsim.h"

namespace navsim {

// Largest padded bitmap (in 32-bit words) the fused step stages in LDS.
constexpr int kMaxMapWords = 12288;  // 48 KiB
constexpr int kMaxBeams = 4096;
constexpr int kWavesPerGroup = 4;    // envs per workgroup in the fused step

// Per-map table entry in device memory.  A map of W x H cells is stored with a
// one-cell ring of occupied padding: row r = iy + 1 in 0..H+1, column
// c = ix + 1 in 0..W+1, bit c & 31 of word r * wpr + (c >> 5); every bit at
// c >= W + 1 is set, so leaving the map reads as occupied.
struct MapDesc {
    int32_t w, h;
    int32_t wpr;       // words per padded row, 32 * wpr >= W + 2
    int32_t words;     // padded words, rounded up to a multiple of 4
    int64_t word_off;  // start in the bit pool (multiple of 4 words)
    int64_t free_off;  // start of this map's free-cell list
    int32_t free_cnt;
    float res;
};

// A group of up to kWavesPerGroup envs that share one map (fused step).
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
    int32_t N, K, m, horizon, footprint, tries, full_circle, mode;  // mode 0 step, 1 reset
    float rmax, dt, goal_r, c1, r_succ, r_coll, radius, len, wid;
    float vlo, vhi, wlo, whi, gmd;
    uint32_t key0, key1;
    double rc;  // circumradius of the footprint
    DevState st;
    const int32_t *env_map;
    const MapDesc *maps;
    const uint32_t *bits;
    const int32_t *free_cells;
    const double2 *beams;  // (cos, sin) of each beam's angle to the heading
    const int32_t *perm;   // env ids grouped by map
    const Tile *tiles;
    int32_t num_tiles, max_words;
    // inputs / outputs
    const float *act;
    const uint8_t *mask;
    float *obs, *reward, *final_obs;
    uint8_t *term, *trunc;
    // diagnostics (may be null)
    float *d_ranges;
    int32_t *d_hits, *d_visits;
    uint8_t *d_coll, *d_goal, *d_reset, *d_fb;
};

hipError_t launch_fused(const StepParams &p, hipStream_t s);
hipError_t launch_plain(const StepParams &p, hipStream_t s);

}  // namespace navsim
