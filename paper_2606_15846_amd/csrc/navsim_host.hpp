// Library-internal host declarations shared by the C ABI sources: the handle
// behind navsim_t, error reporting and the device guard.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include <string>
#include <vector>

#include "navsim.h"
#include "navsim_internal.hpp"

namespace navsim {

// Records the message returned by navsim_last_error() and returns s.
navsim_status fail(navsim_status s, const char *fmt, ...);

#define NS_HIP(call)                                                                        \
    do {                                                                                    \
        hipError_t _e = (call);                                                             \
        if (_e != hipSuccess)                                                               \
            return ::navsim::fail(NAVSIM_E_HIP, "%s: %s", #call, hipGetErrorString(_e));    \
    } while (0)

// Makes the handle's device current for the duration of a call and restores
// the caller's device afterwards.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

inline bool finite_pos(float v) { return isfinite(v) && v > 0.0f; }

}  // namespace navsim

struct navsim_s {
    navsim_config cfg;
    int device = 0;
    bool loaded = false;
    bool initialized = false;
    // device memory
    void *state_buf = nullptr;
    navsim::DevState st{};
    double2 *beams = nullptr;
    uint32_t *bits = nullptr;
    navsim::MapDesc *maps = nullptr;
    int32_t *free_cells = nullptr;
    int32_t *env_map = nullptr;
    int32_t *perm = nullptr;
    navsim::Tile *tiles = nullptr;
    int num_maps = 0, num_tiles = 0, max_words = 0;
    int max_words_t = 0;  // largest transposed bitmap (staged beside the bitmap by walk 5)
    int tile_envs = navsim::kDefaultTileEnvs, refill_at = navsim::kDefaultRefillAt, groups = navsim::kDefaultGroups;
    int ray_cap = 0;
    int ray_slots = 0;  // requested cap on ray_cap (0 = automatic)
    int walk_mode = navsim::kDefaultWalk;  // fused walk (see navsim_tuning.walk)
    bool beams_lds = true;
    int persist = 0;    // persistent workgroups: tiles per grab (0 = one workgroup per tile)
    int wg_threads = 256;  // fused step: threads per workgroup
    int balance = 0;       // tiles sized per map by estimated scan work
    int cell_bytes = 0;    // walk 2, 4: LDS bytes of the byte-per-cell map copy
    int claim = 0;         // walk 3, 4 with the exact traversal: claim walk, no ray slots
    int lds_block = 65536, lds_cu = 65536;  // device LDS bytes per workgroup and per CU
    int resident = 0;   // workgroups of the fused step resident at once on the device
    int32_t *queue = nullptr;  // device {next tile, finished workgroups}, zero between launches
    int scan_mode = 0;       // 0 exact traversal, 1 fixed-step march
    int march_kmax = 0;
    double march_h = 0.03;
    std::vector<int32_t> host_env_map;  // kept to rebuild the tiles when tile_envs changes
    std::vector<double> host_map_weight;  // per-map scan work estimate (tile launch order)
    // host copies of the loaded maps (reset proposals build their own tables)
    std::vector<uint8_t> host_occ;
    std::vector<int64_t> host_occ_off;
    std::vector<int32_t> host_w, host_h;
    std::vector<float> host_res;
    std::vector<double> host_rc;
    std::vector<int32_t> host_free;
    std::vector<int64_t> host_free_off;
    std::vector<int32_t> host_free_cnt;
    // rollouts: first step index on the device, and the last captured rollout
    uint32_t *step_ctr = nullptr;
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    navsim::StepParams graph_params{};  // parameters of step 0 of the captured rollout
    int graph_steps = 0, graph_kernel = -1, graph_tile_envs = 0;
    // learned resets inside the step (navsim_rp_attach): envs with a requested
    // bin defer their reset in the fused launch, run() writes a verified pair
    // for each (or leaves it to the free-space sampler), and a masked reset
    // pass applies them
    struct ResetHook {
        const int32_t *bin = nullptr;  // device [N] requested bin per env, -1 none
        uint8_t *defer = nullptr;      // device [N] the env deferred its reset in this call
        const float *pose = nullptr;   // device [N][5] pairs written by run()
        const int32_t *src = nullptr;  // device [N] >= 0 where run() wrote a pair
        navsim_status (*run)(void *ctx, hipStream_t s) = nullptr;
        void *ctx = nullptr;
    } hook;
    int proposers = 0;  // live navsim_rp handles created on this handle
};


namespace navsim {
// Launch parameters of the handle's current maps, state and settings (all
// optional inputs and outputs null).
StepParams make_step_params(const navsim_s *h);
}  // namespace navsim
