// Reachability kernels of the learned reset proposal (library internal):
// geodesic search on C-free bitsets, labelled pairs, the exact pair check,
// proposals with the rejection sampler behind them, and the network's inputs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace navsim {

constexpr int kReachMaxWords = 2048;  // C-free bitset words per map (e.g. 256 x 256 cells)
constexpr int kReachMaxBins = 16;
constexpr int kReachThreads = 256;
// propose_kernel: one candidate check per wavefront, 8 at a time for launches
// of at most this many requests, else 4
constexpr int kProposeWideMax = 2048;
// in-step proposals: rounds a request's own workgroup checks before its other
// rounds go to the tail launch, all at once
constexpr int kProposeHeadRounds = 1;
constexpr int kPoolCells = 1024;      // 32 x 32 pooled occupancy

// One map's C-free bitset: row j, column i is bit i & 31 of word
// j * wpr + (i >> 5); bits at i >= W are 0.
struct ReachDesc {
    int32_t W, H, wpr, words;
    int64_t bit_off;   // into the bitset array
    int64_t free_off;  // into the C-free cell list
    int32_t free_cnt;
    float s;           // cell size, metres
};

struct ReachParams {
    const ReachDesc *maps;
    const uint32_t *bits;
    const int32_t *free_cells;
    const int8_t *hop_bin;   // bin of each hop count 0..max_hops, -1 outside
    const int32_t *bin_hi;   // largest hop count of each bin
    int32_t max_hops, nbins, num_maps;
    double gmd;              // least start-goal distance between cell centres
    uint32_t key0, key1;     // Philox key
};

// Labelling: request i uses map map[i] and start id first_sid + i.
hipError_t launch_label(const ReachParams &rp, int n, const int32_t *map, uint32_t first_sid,
                        int32_t *start, int32_t *goal, int32_t *hops, hipStream_t s);

// Proposals: request i (map, bin, env, episode) tries the network's `props`
// outputs y[(i props + j) 5 ..] in order (decoded, snapped to C-free cells,
// checked), then rejection attempts 0 .. tries - 1.
struct ProposeArgs {
    int n, props, tries;
    const int32_t *map, *bin;
    const uint32_t *env, *episode;
    const float *y;
    float *pose;
    int32_t *hops, *source, *checks;
    // optional: requests = min(n, *n_dev) read on the device; outputs of
    // request i at row slot[i] (else i); per-call totals added to stats
    // {requests, from the network, from rejection, none valid, checks}
    const int32_t *n_dev = nullptr;
    const int32_t *slot = nullptr;
    unsigned long long *stats = nullptr;
    // optional two-phase search: a request with no valid candidate in its
    // first head_rounds rounds (0: no limit) is appended to pend (count
    // *n_pend, best[p] = INT_MAX) instead of written; the tail launch checks
    // its remaining rounds all at once (round slots in tail) and the final
    // launch writes it
    int head_rounds = 0;
    int32_t *pend = nullptr, *n_pend = nullptr, *best = nullptr;
    int4 *tail = nullptr;
};
// Candidates checked together per request (one per wavefront).
int propose_width(int n);
hipError_t launch_propose(const ReachParams &rp, const ProposeArgs &a, hipStream_t s);
// The rounds head_rounds .. head_rounds + tail_rounds - 1 of the pending
// requests (a.n = the most there can be), then their outputs.
hipError_t launch_propose_tail(const ReachParams &rp, const ProposeArgs &a, int tail_rounds,
                               hipStream_t s);

// Noise inputs: row r = i * per + j of z (bfloat16, nz columns) draws
// Philox(c0[i], c1[i] or c1_const, (j << 8) | q, stream) words for
// q = 0 .. ceil(nz / 4) - 1, z = 2 u - 1 with u = (w + 1/2) 2^-32.
// row_idx[r] = map[i] * nbins + bin[i].
struct NoiseArgs {
    int n, per, nz, nbins, num_maps;  // row_idx = 0 for a request with map or bin out of range
    const uint32_t *c0;  // per request (null: c0 = i)
    const uint32_t *c1;  // per request (null: c1_const)
    uint32_t c1_const, stream;
    const int32_t *map, *bin;
    uint16_t *z;
    int32_t *row_idx;
    const int32_t *n_dev = nullptr;  // optional: requests = min(n, *n_dev) read on the device
};
hipError_t launch_noise(const NoiseArgs &a, uint32_t key0, uint32_t key1, hipStream_t s);

// Requests of the envs that deferred their reset in a step: in env order,
// env e with defer[e] != 0 and bin[e] >= 0 is request i (the first `cap`
// only): env[i] = e, map[i] = env_map[e], bin[i] = bin[e], episode[i] =
// ep[e]; src[e] = -1 for every such env (the proposal call then overwrites
// the ones it serves); *n_out = min(count, cap); stats[0] += count,
// stats[1] += count beyond cap.  One workgroup.
struct CompactArgs {
    int N, cap;
    const uint8_t *defer;
    const int32_t *bin, *env_map;
    const uint32_t *ep;
    uint32_t *env, *episode;
    int32_t *map, *rbin, *src, *n_out;
    unsigned long long *stats;
    int32_t *n_pend = nullptr;  // cleared here for the proposal launches that follow
};
hipError_t launch_compact(const CompactArgs &a, hipStream_t s);

// Rows [pool(map) | one-hot(bin)] of every (map, bin), bfloat16, width
// 1024 + nbins (the constant part of the first layer's input).
hipError_t launch_pool_rows(int num_maps, int nbins, const float *pool, uint16_t *rows,
                            hipStream_t s);

// Training batch of step t: target i draws pair (w0 P) >> 32, w = Philox(t, i,
// 0, 10); writes its map and bin, the float targets ((a_x + 1/2) / W,
// (a_y + 1/2) / H, 0, (b_x + 1/2) / W, (b_y + 1/2) / H).
struct BatchArgs {
    int batch, num_pairs, num_maps, nbins;  // a pair out of range trains as map 0, bin 0, zeros
    uint32_t step;
    const int32_t *pair_map, *pair_bin, *pair_start, *pair_goal;
    const ReachDesc *maps;
    int32_t *map, *bin;
    float *target;
};
hipError_t launch_batch(const BatchArgs &a, uint32_t key0, uint32_t key1, hipStream_t s);

// IMLE choice: for target i the candidate j < per with the smallest
// sum_d w_d (y - t)^2 (first on ties); writes the training input row
// [pool(map) | one-hot(bin) | z of that candidate].
struct SelectArgs {
    int batch, per, nz, nbins;
    const float *y;        // [batch per][5]
    const float *target;   // [batch][5]
    const float *w;        // [5]
    const uint16_t *z;     // [batch per][nz]
    const int32_t *map, *bin;
    const float *pool;     // [maps][1024]
    uint16_t *x;           // [batch][1024 + nbins + nz]
    int32_t *chosen;
};
hipError_t launch_select(const SelectArgs &a, hipStream_t s);

}  // namespace navsim
