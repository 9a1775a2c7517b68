/*
 * navsim: batched bitmap navigation step for AMD Instinct MI355X (gfx950).
 *
 * C ABI of libnavsim.so.  Implements the data-parallel environment step of
 * FlashNav (arXiv 2606.15846, section 2.2): thousands of independent
 * goal-conditioned navigation environments on occupancy bitmaps, advanced
 * together by one step call.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every call returns a navsim_status (0 = NAVSIM_OK, < 0 = error).  On error
 *   navsim_last_error() returns a message for the calling thread.
 * - Argument errors are reported synchronously, before anything is enqueued;
 *   output buffers are then untouched.
 * - "device" pointers are HIP device allocations on the handle's device (for
 *   example torch tensors' data pointers), contiguous, with the stated layout.
 *   "host" pointers are ordinary process memory, read during the call only.
 * - Calls that take `hip_stream` (a hipStream_t; NULL = the null stream)
 *   enqueue their work on that stream and return without waiting.  The caller
 *   keeps device buffers alive until the stream has consumed them.  Faults of
 *   enqueued work surface at the next synchronisation.
 * - A handle is used by one thread at a time; different handles are
 *   independent.  Calls on one handle that overlap on different streams race.
 *
 * Environment layout (the navigation MDP of section 2.1)
 * ------------------------------------------------------
 * Per env the library keeps, in device memory, float32 pose x, y, theta (m,
 * m, rad in [-pi, pi]), commanded velocity v, w, goal gx, gy, previous goal
 * distance d_prev, int32 step counter t and uint32 episode counter.
 * Observation row (eq. 1, raw pooled ranges; the reciprocal transform of
 * eq. 2 has a trainable parameter and belongs to the policy):
 *     obs[e] = [ l_1 .. l_m , d_goal , phi_goal , v , w ]   (m + 4 floats)
 * l_j = min range over sector j (eq. 6): sectors are contiguous blocks of K/m
 * beams.  Beam k's angle to the heading is -pi + k 2pi/K for a full circle,
 * -fov/2 + k fov/(K-1) otherwise.  phi_goal is the goal bearing in the robot
 * frame, in (-pi, pi].
 */
#ifndef NAVSIM_H
#define NAVSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NAVSIM_ABI_VERSION 1u

typedef struct navsim_s *navsim_t;

typedef enum {
    NAVSIM_OK = 0,
    NAVSIM_E_INVALID_ARG = -1,    /* bad pointer, size or parameter value          */
    NAVSIM_E_BAD_HANDLE = -2,     /* NULL or destroyed handle                       */
    NAVSIM_E_STATE = -3,          /* call order: step before load_maps/reset        */
    NAVSIM_E_NO_FREE_SPACE = -4,  /* a map used by some env has no collision-free cell */
    NAVSIM_E_OOM = -5,            /* device or host allocation failed               */
    NAVSIM_E_HIP = -6,            /* a HIP runtime call failed (message has details) */
    NAVSIM_E_UNSUPPORTED = -7     /* valid but beyond this library's limits         */
} navsim_status;

enum { NAVSIM_DISC = 0, NAVSIM_RECT = 1 };

/* Robot preset and episode parameters (section 2.2.1 presets; appendix B,
 * tables 7-9 for the paper's values). */
typedef struct {
    uint32_t abi_version;        /* must equal NAVSIM_ABI_VERSION                        */
    int32_t num_envs;            /* N >= 1                                                */
    int32_t num_beams;           /* K, 1..4096                                            */
    int32_t num_sectors;         /* m, K % m == 0                                         */
    float fov_rad;               /* >= 2pi - 1e-6 means a full circle                     */
    float max_range_m;           /* r_max > 0 (eq. 5)                                     */
    float dt_s;                  /* integration step > 0                                  */
    int32_t horizon;             /* truncation after this many steps (table 7: 200)       */
    float goal_radius_m;         /* goal reached when d < this (table 7: 0.2)             */
    float c_progress;            /* eq. 3 progress coefficient c_1 (table 7: 2)           */
    float r_success;             /* eq. 3 goal reward (table 7: +10)                      */
    float r_collision;           /* eq. 3 collision reward (table 7: -10)                 */
    int32_t footprint;           /* NAVSIM_DISC or NAVSIM_RECT                            */
    float radius_m;              /* disc radius                                           */
    float length_m, width_m;     /* rectangle, long side along the heading                */
    float v_min, v_max;          /* linear velocity for normalised action -1 / +1          */
    float w_min, w_max;          /* angular velocity for normalised action -1 / +1         */
    float goal_min_dist_m;       /* reset: minimum start-goal distance                    */
    int32_t reset_max_tries;     /* reset: rejection attempts before the free-cell list, 1..1024 */
    uint64_t seed;               /* key of the reset sampler's counter-based generator     */
} navsim_config;

/* Create a simulator for cfg on HIP device hip_device.  Allocates the env
 * state on that device (state starts zeroed; call navsim_load_maps and
 * navsim_reset before stepping).  *out receives the handle. */
navsim_status navsim_create(const navsim_config *cfg, int hip_device, navsim_t *out);

/* Load the occupancy bitmaps (section 2.2.1) and the env-to-map assignment.
 * All pointers are host memory, copied during the call (synchronous).
 *   width, height [num_maps]  cells per row / rows, >= 1; the map with its
 *                             4-cell padding ring, (height + 8) * ceil((width + 8)
 *                             / 32) 32-bit words, must fit 48 KiB of LDS (for
 *                             example 512 x 700 cells); larger maps give
 *                             NAVSIM_E_UNSUPPORTED
 *   res_m [num_maps]          cell size in metres (> 0); cell (ix, iy) covers
 *                             [ix s, (ix+1) s) x [iy s, (iy+1) s)
 *   occ                       maps concatenated, each row-major [height][width],
 *                             iy-major, byte 0 = free, nonzero = occupied;
 *                             everything outside the map counts as occupied
 *   env_map [num_envs]        map id of each env, 0..num_maps-1
 * Errors: NAVSIM_E_NO_FREE_SPACE if a used map has no cell where the footprint's
 * circumscribed disc fits (the reset sampler could not succeed);
 * NAVSIM_E_UNSUPPORTED if a map's footprint window, floor(2 rc / res) + 2 cells
 * per side for the circumscribed radius rc, exceeds 128 cells (for example the
 * 0.80 x 0.41 m rectangle fits down to 0.0071 m cells: 91 cells at 0.01 m);
 * NAVSIM_E_UNSUPPORTED also guards the step's exact multiply-shift quotients
 * by a map's beam count and beams per sector, which are checked here over
 * their whole operand range (they hold for every beam count up to the limit). */
navsim_status navsim_load_maps(navsim_t h, int32_t num_maps, const int32_t *width,
                               const int32_t *height, const float *res_m, const uint8_t *occ,
                               const int32_t *env_map);

/* Robot and sensor of the envs on one map: lets maps of different beam counts
 * and footprints run in the same step (the configuration's beam count is then
 * the largest, and the stride of per-ray diagnostics). */
typedef struct {
    int32_t num_beams;        /* K for this map: 1..cfg.num_beams, multiple of num_sectors */
    int32_t footprint;        /* NAVSIM_DISC or NAVSIM_RECT                                */
    float radius_m, length_m, width_m;
} navsim_map_profile;

/* navsim_load_maps with one profile per map (host array [num_maps]; NULL = the
 * configuration's beam count and footprint for every map). */
navsim_status navsim_load_maps_ex(navsim_t h, int32_t num_maps, const int32_t *width,
                                  const int32_t *height, const float *res_m, const uint8_t *occ,
                                  const int32_t *env_map, const navsim_map_profile *profiles);

/* Sparse reset (section 2.2.3): every env with mask[e] != 0 (mask NULL = all)
 * gets a new collision-free start pose and goal from its map's free space,
 * zero velocity, t = 0, and its reset observation written to obs row e.  Rows
 * of envs not reset are left untouched.  The first reset must use mask NULL.
 *   mask  device uint8 [N] or NULL
 *   obs   device float32 [N][m+4] */
navsim_status navsim_reset(navsim_t h, const uint8_t *mask, float *obs, void *hip_stream);

/* navsim_reset to caller-given poses: every env with mask[e] != 0 (mask NULL =
 * all) gets start (x, y, heading) and goal (x, y) from row e of `pose`
 * (device float32 [N][5]: x, y, heading, goal x, goal y in metres / radians),
 * v = w = 0, t = 0, its episode counter + 1, and the reset observation in its
 * obs row (device float32 [N][m+4]).  The poses are not checked: callers pass
 * verified ones (navsim_rp_propose writes such rows).  Same errors as
 * navsim_reset. */
navsim_status navsim_reset_to(navsim_t h, const uint8_t *mask, const float *pose, float *obs,
                              void *hip_stream);

/* One environment step for all N envs, the step data path of eq. 7:
 * action -> pose -> ranges -> (collision, reward, termination) -> O_{t+1}
 * -> reset observation where the episode ended.
 *   act         device float32 [N][2], normalised (a_v, a_w); clipped to [-1, 1],
 *               NaN treated as 0; v = v_min + (a_v + 1)/2 (v_max - v_min), w alike
 *   obs         device float32 [N][m+4]: O_{t+1}, or the reset observation for envs
 *               whose episode ended in this step
 *   reward      device float32 [N]   eq. 3 for the transition just taken
 *   terminated  device uint8 [N]     goal reached or collision
 *   truncated   device uint8 [N]     t reached the horizon with neither event
 *   final_obs   device float32 [N][m+4] or NULL: O_{t+1} of envs that ended
 *               (rows of other envs untouched)
 * One launch on hip_stream: a workgroup per tile of envs that share a map
 * stages the map's bitmap in LDS, steps each env on a group of 16 lanes
 * (ballots for collision and reset attempts), walks all of the tile's rays
 * (new poses and reset poses) with every lane, pools sectors in LDS and writes
 * the observation rows.  With a reset proposer attached (navsim_rp_attach in
 * navsim_reset_proposal.h), envs with a requested difficulty bin take their
 * new pair from it instead: the fused launch defers their reset, the
 * proposer's kernels pick and verify the pairs, and one masked reset launch
 * applies them (all on hip_stream). */
navsim_status navsim_step(navsim_t h, const float *act, float *obs, float *reward,
                          uint8_t *terminated, uint8_t *truncated, float *final_obs,
                          void *hip_stream);

/* Same contract and results as navsim_step, computed by the plain mapping: one
 * GPU thread per env, beams in sequence, bitmap read from device memory.  Kept
 * as the comparison point for the fused step. */
navsim_status navsim_step_plain(navsim_t h, const float *act, float *obs, float *reward,
                                uint8_t *terminated, uint8_t *truncated, float *final_obs,
                                void *hip_stream);

/* Optional per-step diagnostics.  Every pointer may be NULL (= not written). */
typedef struct {
    float *ranges;      /* device float32 [N][K]: range of each beam at the pre-reset pose */
    int32_t *hits;      /* device int32 [N][K]: hit cell iy*W+ix, -1 none within r_max,
                           -2 map boundary                                              */
    int32_t *visits;    /* device int32 [N][K]: cells whose occupancy the ray read      */
    uint8_t *collision; /* device uint8 [N]                                            */
    uint8_t *goal;      /* device uint8 [N]                                            */
    uint8_t *reset;     /* device uint8 [N]: env was reset in this step                */
    uint8_t *fallback;  /* device uint8 [N]: bit 0 start, bit 1 goal came from the
                           free-cell list                                              */
} navsim_debug;

enum { NAVSIM_KERNEL_FUSED = 0, NAVSIM_KERNEL_PLAIN = 1 };

/* navsim_step (kernel = NAVSIM_KERNEL_FUSED) or navsim_step_plain
 * (NAVSIM_KERNEL_PLAIN) that also writes the diagnostics in *dbg (host struct
 * of device pointers; NULL = none). */
navsim_status navsim_step_debug(navsim_t h, const float *act, float *obs, float *reward,
                                uint8_t *terminated, uint8_t *truncated, float *final_obs,
                                const navsim_debug *dbg, int32_t kernel, void *hip_stream);

/* Rollout: `steps` consecutive steps (1..4096) of every env with synthetic
 * normalised actions drawn on the device, for throughput runs and data
 * collection under random actions (section 3 measures under random actions;
 * the generator is this library's): env e at step n = first_step + i uses
 * Philox4x32-10 with key = seed and counter (e, n mod 2^32, n div 2^32, 4),
 * a_j = 2 u_j - 1 with u_j = (w_j + 1/2) 2^-32 from words 0 and 1, rounded to
 * float32.  Step i is exactly navsim_step (or navsim_step_plain, by `kernel`)
 * with those actions, so results equal a loop of single steps bitwise.
 * Device outputs, row i = step i:
 *   act        float32 [steps][N][2]     drawn actions (NULL = not written)
 *   obs        float32 [steps][N][m+4]   as navsim_step
 *   reward     float32 [steps][N]
 *   terminated uint8   [steps][N]
 *   truncated  uint8   [steps][N]
 *   final_obs  float32 [steps][N][m+4]   (NULL = not written)
 * flags: NAVSIM_ROLLOUT_GRAPH captures the step launches once into a HIP graph
 * (kept in the handle: replayed while buffers, steps, kernel and launch shape
 * stay the same, captured again otherwise; dropped by navsim_set_tuning and
 * navsim_load_maps) and launches that graph on hip_stream; without it each
 * step is launched on hip_stream.  The rollout's first step index lives in
 * device memory, set on hip_stream before the steps: two rollouts of one
 * handle in flight on different streams race.  Errors: as navsim_step, and
 * NAVSIM_E_HIP when capture or instantiation fails. */
enum { NAVSIM_ROLLOUT_GRAPH = 1 };
navsim_status navsim_rollout(navsim_t h, int32_t steps, uint64_t first_step, float *act,
                             float *obs, float *reward, uint8_t *terminated, uint8_t *truncated,
                             float *final_obs, int32_t kernel, int32_t flags, void *hip_stream);

/* Range query of both step mappings.  NAVSIM_SCAN_TRAVERSAL (default): the
 * exact first occupied or out-of-bounds cell along each beam (integer grid
 * traversal), range = its entry distance.  NAVSIM_SCAN_MARCH: the paper's
 * fixed-step query (section 2.2.2, table 7: 0.03 m): samples at tau = k step_m,
 * k = 0, 1, ... while tau <= r_max; the first sample whose cell floor(p / s)
 * (double precision) is occupied or outside the map ends the beam at
 * range = tau, else range = r_max; visits = samples evaluated.  It can step
 * over a cell the beam only clips.  Errors: INVALID_ARG (unknown mode,
 * step_m <= 0, r_max / step_m > 2^20).  Drops a captured rollout graph. */
enum { NAVSIM_SCAN_TRAVERSAL = 0, NAVSIM_SCAN_MARCH = 1 };
navsim_status navsim_set_scan(navsim_t h, int32_t mode, float step_m);

/* Launch shape of the fused step.  Results never depend on it (bitwise); it
 * only moves work between lanes, wavefronts and workgroups. */
typedef struct {
    int32_t tile_envs;  /* envs per workgroup (they share one staged map): 1, 2, 4, 8, 16, 32
                           (at most this many with balance = 1)                            */
    int32_t refill_at;  /* a wavefront hands new rays to its idle lanes once at most this
                           many of its 64 lanes are still walking, 0..63                  */
    int32_t groups;     /* 4-cell groups a lane walks between refill checks, 1..64        */
    int32_t ray_slots;  /* LDS ray slots per workgroup (each 16 B): 0 = automatic (the
                           tile's rays plus one reset scan, or as many as fit in the LDS
                           share that lets 1024 / threads workgroups run per CU, i.e. 40 KiB
                           at 256 threads on a 160 KiB CU; up to max(share, 64 KiB) for
                           maps too large for that); else at most this many (>= 256,
                           rounded up to 64) within the device's LDS per workgroup.  Fewer
                           slots: less LDS, more workgroups per CU, more chunks per tile  */
    int32_t walk;       /* 0: cells in groups of 4; 1: runs of cells between minor-axis
                           steps (32 cells per test along x); 2: cells in groups of 4 read
                           from a one-byte-per-cell copy of the map staged next to the
                           bitmap (32x its LDS; no address arithmetic or bit extraction per
                           cell); 3: as 0, but each lane sets up the rays it claims and
                           pools each ray when done (no LDS ray slots, no chunks; ray_slots
                           is ignored); 4: as 3 on the byte copy; 5: as 3, testing up to
                           31 cells of a run between minor-axis steps at once, x-major rays
                           in the bitmap and y-major rays in its transpose staged beside it
                           (2x the bitmap's LDS; UNSUPPORTED for a transposed bitmap of
                           16384 words or more).  3, 4 and 5 apply to the exact traversal;
                           the fixed-step march keeps its chunked walk.  Same cells, same
                           results                                                        */
    int32_t persist;    /* 0: one workgroup per tile; c in 1..64: only as many workgroups
                           as stay resident, each taking c consecutive tiles at a time from
                           a device counter and keeping its staged map while the tiles'
                           map does not change                                             */
    int32_t threads;    /* threads per workgroup, 256, 512 or 1024 (at least 16 per env of
                           a tile): the tile's envs share this many lanes (and one ray
                           pool); automatic ray slots grow with it (the CU's LDS split
                           between 1024 / threads workgroups)                              */
    int32_t balance;    /* 0: tiles of tile_envs envs; 1: each map gets as many tiles as
                           make every tile's estimated scan work (envs x beams x the mean
                           cells a ray walks on that map, sampled on the host at load) about
                           equal, at least as many tiles in all as workgroups run at once,
                           at most tile_envs envs each.  Tiles always launch heaviest first */
} navsim_tuning;

/* Set the fused step's launch shape (defaults: 8, 40, 8, 0, 3, 0, 256, 0).  Changing tile_envs
 * after navsim_load_maps waits for the device and re-groups the envs; returns
 * NAVSIM_E_UNSUPPORTED if the larger tile would not fit LDS. */
navsim_status navsim_set_tuning(navsim_t h, const navsim_tuning *t);

/* Current launch shape. */
navsim_status navsim_get_tuning(navsim_t h, navsim_tuning *t);

/* Host copy of the env state (checkpoint), SoA, N entries each, in this order:
 * float32 x, y, theta, v, w, gx, gy, d_prev; int32 t; uint32 episode
 * (10 * 4 * N bytes).  Waits for hip_stream before copying. */
#define NAVSIM_STATE_BYTES(n) ((size_t)(n) * 40u)
navsim_status navsim_get_state(navsim_t h, void *host_soa, size_t bytes, void *hip_stream);

/* Replace the env state from a host blob in the navsim_get_state layout
 * (restores a checkpoint; also counts as the first reset).  Synchronous. */
navsim_status navsim_set_state(navsim_t h, const void *host_soa, size_t bytes, void *hip_stream);

/* Free all device and host memory of the handle.  Using h afterwards, or
 * destroying it twice, is undefined.  Errors: STATE while reset proposers
 * created on h (navsim_rp_create) are alive: destroy them first. */
navsim_status navsim_destroy(navsim_t h);

/* Message for the last failed call on this thread ("" if none). */
const char *navsim_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NAVSIM_H */
