/*
 * Learned reset proposal for libnavsim (C ABI, version 1).
 *
 * The paper resets finished environments to collision-free start and goal
 * poses drawn from free space (section 2.2.3).  This extension asks for a
 * pair at a given path-length difficulty and answers it with a small network
 * whose every proposal is checked exactly, with the plain rejection sampler
 * behind it.  Definitions (this library's reading; the paper has none):
 *
 *   C-free cell      a cell whose centre passes the clearance test of the
 *                    map's circumscribed robot disc (the cells of the
 *                    free-cell list navsim_load_maps builds);
 *   geodesic hops    h(a, b): fewest 4-neighbour moves from C-free cell a to
 *                    C-free cell b through C-free cells; distance h * s;
 *   bins             num_bins equal half-open intervals of [d_lo_m, d_hi_m):
 *                    bin k holds d with d_lo + k w <= d < d_lo + (k + 1) w,
 *                    w = (d_hi - d_lo) / num_bins, d = h * s in double;
 *   valid pair       (a, b) for bin k: both C-free, cell centres at least
 *                    goal_min_dist_m apart, h(a, b) * s in bin k;
 *   rejection        for env e in episode ep, attempt t draws Philox4x32-10
 *                    (key = seed, counter (e, ep, t, 7)) words w0..w3: start
 *                    = C-free cell number (w0 n) >> 32 of the map's list
 *                    (n cells), goal likewise from w1, heading
 *                    (w2 + 1/2) 2^-32 2 pi - pi; the first valid attempt wins;
 *   network          input [32 x 32 max-pooled occupancy | one-hot bin |
 *                    noise z], leaky-ReLU hidden layers, output (start x,
 *                    start y, heading, goal x, goal y) with positions as
 *                    fractions of the map's width / height and heading / pi;
 *                    bfloat16 weights and activations, float accumulation;
 *   proposal         output -> cells floor(x W), floor(y H) (clamped),
 *                    each moved to the nearest C-free cell (least |di|+|dj|,
 *                    then least index), heading clamp(y2, -1, 1) pi; then the
 *                    exact check above.
 * Maps used with a proposer need W, H >= 32 and H ceil(W / 32) <= 2048.
 */
#ifndef NAVSIM_RESET_PROPOSAL_H
#define NAVSIM_RESET_PROPOSAL_H

#include <stddef.h>
#include <stdint.h>

#include "navsim.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct navsim_rp_s *navsim_rp_t;

typedef struct {
    int32_t num_bins;       /* 1..16 (8)                                         */
    float d_lo_m, d_hi_m;   /* 0 <= d_lo < d_hi (1, 12)                          */
    int32_t noise_dim;      /* noise inputs, 1..64 (16)                          */
    int32_t hidden;         /* hidden width, 16..1024, multiple of 16 (256)      */
    int32_t hidden_layers;  /* 1..4 (3)                                          */
    float leaky_slope;      /* > 0 (0.01)                                        */
    uint64_t seed;          /* weight init, noise, batch draws, rejection draws */
} navsim_rp_config;

/* Proposer for the maps currently loaded in h (it keeps its own tables; load
 * new maps = create a new proposer).  Weights: uniform in +-1/sqrt(fan_in),
 * biases 0.  h must outlive the proposer (navsim_destroy(h) fails with STATE
 * while a proposer created on it is alive).  Errors: INVALID_ARG (config),
 * STATE (no maps), UNSUPPORTED (a map outside the size limits above), OOM,
 * HIP. */
navsim_status navsim_rp_create(navsim_t h, const navsim_rp_config *cfg, navsim_rp_t *out);

/* Labelled pairs (device arrays): row i draws start id first_sid + i on map
 * map[i]: start = C-free cell number (w0 n) >> 32, w = Philox(sid, 0, 0, 6);
 * for each bin k the goal is, among cells b that make a valid pair with the
 * start for bin k, the one with the smallest (word 0 of Philox(sid, b, 0, 5),
 * b); goal[i nb + k] = hops[i nb + k] = -1 when bin k has none.
 * start int32 [n], goal / hops int32 [n][num_bins]. */
navsim_status navsim_rp_label(navsim_rp_t rp, int32_t n, const int32_t *map, uint32_t first_sid,
                              int32_t *start, int32_t *goal, int32_t *hops, void *hip_stream);

/* `steps` training steps on a device pair set (map, bin, start cell, goal
 * cell: int32 [num_pairs] each).  Step t (the proposer's own counter) draws
 * `batch` pairs (Philox(t, i, 0, 10)), scores `samples` noise draws per pair
 * (Philox(t, i, (j << 8) | q, 9)) through the network and keeps the closest
 * (implicit maximum likelihood: sum over start x, y, goal x, y of the squared
 * error), then one AdamW step (b1 0.9, b2 0.999, eps 1e-8, weight decay on
 * weights only) on the mean squared error of the kept draws.  loss: device
 * float [steps] = sum over the batch of that error (NULL = not written). */
navsim_status navsim_rp_train(navsim_rp_t rp, int32_t num_pairs, const int32_t *pair_map,
                              const int32_t *pair_bin, const int32_t *pair_start,
                              const int32_t *pair_goal, int32_t steps, int32_t batch,
                              int32_t samples, float lr, float weight_decay, float *loss,
                              void *hip_stream);

/* Start/goal pairs for n requests (device arrays map, bin int32 [n]; env,
 * episode uint32 [n]).  Request i tries `proposals` network draws (noise
 * Philox(env, episode, (j << 8) | q, 8)) in order, then rejection attempts
 * 0 .. max_tries - 1.  Outputs (device): pose float [n][5] (start x, y,
 * heading, goal x, y: cell centres in metres, ready for navsim_reset_to),
 * hops int32 [n], source int32 [n] (j < proposals: network draw j;
 * proposals + t: rejection attempt t; -1: nothing valid, pose = the last
 * rejection attempt's pair, zeros when none ran), checks int32 [n] (exact
 * checks run), y_out float [n][proposals][5] the network's raw outputs (may
 * be NULL).  proposals = 0 is the rejection sampler alone; n * proposals
 * <= 2^24. */
navsim_status navsim_rp_propose(navsim_rp_t rp, int32_t n, const int32_t *map, const int32_t *bin,
                                const uint32_t *env, const uint32_t *episode, int32_t proposals,
                                int32_t max_tries, float *pose, int32_t *hops, int32_t *source,
                                int32_t *checks, float *y_out, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call, arguments, outputs and kernels as navsim_rp_propose, with every
 * workspace it needs (the constant first-layer table, noise inputs, network
 * outputs and two hidden activations) carved from one fixed 16 MiB array per
 * device that the library's code object holds until the process ends; it
 * calls no hipMalloc or hipFree.  Workspace bytes, each part rounded up to
 * 256: maps x num_bins x hidden x 4 + R x (2 noise_dim + 4 + 20 + 4 hidden)
 * with R = n x proposals (0 when proposals = 0: the rejection sampler alone
 * uses none); e.g. 64 maps, 8 bins, hidden 256, noise 16: up to ~15,000
 * draws per call.  Errors: as navsim_rp_propose, and INVALID_ARG when the
 * workspace would exceed 16 MiB (nothing is launched).  Every call on a
 * device shares that device's array and leaves its contents there (nothing in
 * it needs to start at zero): calls that overlap on one device, on different
 * streams or from different threads, race and must be serialised by the
 * caller. */
navsim_status navsim_rp_propose_noalloc(navsim_rp_t rp, int32_t n, const int32_t *map,
                                        const int32_t *bin, const uint32_t *env,
                                        const uint32_t *episode, int32_t proposals,
                                        int32_t max_tries, float *pose, int32_t *hops,
                                        int32_t *source, int32_t *checks, float *y_out,
                                        void *hip_stream);

/* Learned resets inside the step (the sparse reset of section 2.2.3, with
 * difficulty): after this call, every env e with bin[e] in 0..num_bins-1
 * (host int32 [num_envs]; -1 = the free-space sampler as before) whose
 * episode ends in navsim_step, or that navsim_reset resets, takes its new
 * start/goal pair from this proposer, in the same call and on the same
 * stream: the fused launch writes its flags, reward and final observation but
 * leaves its reset for later; the first max_per_step such envs in env order
 * become requests (env e, its map, bin[e], its episode counter), each tries
 * `proposals` network draws and then max_tries rejection attempts exactly as
 * navsim_rp_propose does (every pair passes the exact check: C-free start
 * and goal, geodesic hop count in the bin, centre distance >= the goal
 * minimum); a masked reset pass then sets every deferred env's state (v = w
 * = 0, t = 0, episode counter + 1) and its reset observation in obs, from
 * its pair, or from the free-space sampler (the pose navsim_step would have
 * drawn) when its request found no valid pair or did not fit under
 * max_per_step.  No allocation, host synchronisation or memset happens in
 * the step.  navsim_step_plain and the rollout calls return UNSUPPORTED while
 * a proposer is attached.  Calling it again replaces the bins (and the other
 * settings); the handle's maps must be the ones the proposer was created
 * for.  Errors: INVALID_ARG (a bin outside -1..num_bins-1, proposals outside
 * 0..4096, max_tries < 0, max_per_step outside 1..num_envs,
 * max_per_step x proposals > 2^24), STATE (another proposer is attached),
 * OOM, HIP.  Synchronises the device. */
navsim_status navsim_rp_attach(navsim_rp_t rp, const int32_t *bin, int32_t proposals,
                               int32_t max_tries, int32_t max_per_step);

/* Back to the free-space sampler for every env; frees the in-step buffers
 * (synchronises the device).  navsim_rp_destroy detaches too. */
navsim_status navsim_rp_detach(navsim_rp_t rp);

/* Totals since attach (or the last clear), host int64 [8]: deferred resets,
 * deferred resets past max_per_step, requests, pairs from the network, pairs
 * from rejection attempts, requests with no valid pair, exact checks run,
 * 0.  clear != 0 zeroes them.  STATE when not attached.  Synchronises. */
navsim_status navsim_rp_attach_stats(navsim_rp_t rp, int64_t *out, int32_t clear);

/* Per env, of the last step or reset: source (device int32 [num_envs]; for an
 * env that deferred its reset: the draw that gave its pair as in
 * navsim_rp_propose, or -1 for the free-space sampler; other rows keep older
 * values) and hops (device int32 [num_envs], the pair's hop count where
 * source >= 0).  Copies on hip_stream.  STATE when not attached. */
navsim_status navsim_rp_attach_outputs(navsim_rp_t rp, int32_t *source, int32_t *hops,
                                       void *hip_stream);

/* Network on explicit inputs: x bfloat16 bits [n][d0] (d0 = 1024 + num_bins
 * + noise_dim), y float [n][5] (device). */
navsim_status navsim_rp_forward(navsim_rp_t rp, int32_t n, const uint16_t *x, float *y,
                                void *hip_stream);

/* Loss sum_d w_d (y - t)^2 per row (w = 1, 1, 0, 1, 1) and the gradient of
 * its mean over the n rows into grad (device float, parameter layout).
 * loss_rows float [n] may be NULL. */
navsim_status navsim_rp_loss_grad(navsim_rp_t rp, int32_t n, const uint16_t *x,
                                  const float *target, float *loss_rows, float *grad,
                                  void *hip_stream);

/* One AdamW step with the given gradient (device float, parameter layout). */
navsim_status navsim_rp_adamw(navsim_rp_t rp, const float *grad, float lr, float weight_decay,
                              void *hip_stream);

/* Parameter layout: dims[0..L] (L = hidden_layers + 1), for layer l the
 * weight [dims[l+1]][dims[l]] at offsets[2 l] and bias [dims[l+1]] at
 * offsets[2 l + 1] of the flat float vector of *count parameters.  Pass NULL
 * arrays to query L and count first. */
navsim_status navsim_rp_layout(navsim_rp_t rp, int32_t *num_layers, int32_t *dims,
                               int64_t *offsets, int64_t *count);

/* Copy the float master parameters to / from host memory (count floats). */
navsim_status navsim_rp_get_params(navsim_rp_t rp, float *host, int64_t count);
navsim_status navsim_rp_set_params(navsim_rp_t rp, const float *host, int64_t count);

navsim_status navsim_rp_destroy(navsim_rp_t rp);

#ifdef __cplusplus
}
#endif
#endif
