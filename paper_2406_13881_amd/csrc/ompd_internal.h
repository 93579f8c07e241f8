// Host-side internal types of libompd.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ompd.h"
#include "ompd_device.h"

struct ServingState;

struct ompd_ctx {
    int device = 0;
    hipDeviceProp_t prop{};
    int n_cu = 1;
    int lds_max = 64 * 1024;
    uint64_t budget = 0;
    int64_t wall_khz = 100000;     // device wall-clock rate (s_memrealtime)
    int32_t wait_ticks = 0;        // bound of a kernel wait without progress, in wall-clock ticks
    char* static_scratch = nullptr;   // this device's copy of the allocation-free entry point's scratch
    std::mutex mu;                 // serialises API calls
    ServingState* srv = nullptr;   // created on first submit
    std::mutex srv_mu;
};

// Launch sizes of one solve: slots of the result ring, each phase kernel's
// LDS bytes and grid, and the grid of the pass kernels.
struct LaunchDims {
    int ring_slots = 16;
    bool split = true;           // one kernel per phase and pass (else the per-tile kernel)
    size_t lds[ompd::N_PHASES] = {0, 0, 0, 0, 0, 0};
    int grid[ompd::N_PHASES] = {1, 1, 1, 1, 1, 1};
    bool refine = false;         // some CFG runs the loop-entry refinement (phase and pass launched)
    int grid_edge = 1;
    size_t lds_tile = 0;         // the per-tile kernel: LDS of its largest phase
    int grid_tile = 1;
    int n_level = 0;             // level tiles: the last n_level entries of the tile array
    size_t lds_level = 0;        // LDS of a level workgroup (the largest level CFG's column state)
    int grid_level = 1;
};

// Tunable launch configuration of a plan; results never depend on it.
struct PlanConfig {
    size_t lds_bytes = 0;   // bytes of the result ring per phase workgroup (0 = default)
    int wg_per_cu = 0;      // phase workgroups per CU (0 = as many as fit)
    bool split = true;      // one kernel per phase and pass (else one per-tile kernel)
    bool use_graph = true;  // replay a captured HIP graph
    // schedule per size bucket (ompd_sched_bucket): -1 the default rule, else SCHED_WALK or
    // SCHED_LEVEL; CFGs whose schedule the plan's flags name keep it
    int bucket_sched[OMPD_SCHED_BUCKETS] = {-1, -1, -1, -1, -1};
    int only_bucket = -1;   // autotuning: solve only the CFGs of this bucket (-1: all)
};
// Size bucket of a CFG for the schedule choice: blocks below 256, 1,024, 4,096, 16,384, or more.
inline int ompd_sched_bucket(int n_blocks)
{
    return n_blocks < 256 ? 0 : n_blocks < 1024 ? 1 : n_blocks < 4096 ? 2 : n_blocks < 16384 ? 3 : 4;
}

struct ompd_plan {
    ompd_ctx* ctx = nullptr;
    int n = 0;
    uint32_t flags = 0;
    PlanConfig cfg;
    std::vector<ompd::DevCfg> h_cfgs;
    std::vector<ompd_result> res;
    std::vector<int32_t> h_info;
    int32_t* d_info = nullptr;            // [n][INFO_WORDS]: every CFG's status words, gathered for one copy
    ompd::DevCfg* d_cfgs = nullptr;
    std::vector<ompd::Tile> h_tiles;
    ompd::Tile* d_tiles = nullptr;
    int n_tiles = 0;
    ompd::EdgeItem* d_items = nullptr;
    int n_items = 0;
    int32_t* d_counter = nullptr;
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    int max_nb = 2;
    LaunchDims dims;
    size_t lds_prep = 0;
    hipGraph_t g_prep = nullptr, g_solve = nullptr;
    hipGraphExec_t gx_prep = nullptr, gx_solve = nullptr;
    hipStream_t last_stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
    bool profile = false;          // launch directly and time every kernel
    hipEvent_t evk[ompd::N_SOLVE_KERNELS] = {};   // after each solve kernel (profile runs)
};

int ompd_fail(int code, const std::string& msg);
// The message for CFG i's info words (status, and for OMPD_E_DEVICE which wait gave up).
std::string ompd_status_message(int i, const int32_t* info);

struct ScratchOff {
    size_t aveout, mayp, later, flg, eag, both, nu, ave, ie, ig, avf, vk, bnd, pp, pi, pe, tmp, recf, recb, stf, stb,
        lorder, loff, fp, info;
};
size_t ompd_cfg_scratch(const ompd_cfg& g, const ompd_result& r, ScratchOff& o);
void ompd_fill_devcfg(const ompd_cfg& g, const ompd_result& r, char* base, const ScratchOff& o, uint32_t flags,
                      int32_t wait_ticks, ompd::DevCfg& d, uint64_t* bnd_host, uint64_t* bnd_dev = nullptr);
// Blocks from which a CFG takes the level schedule when the caller names none
// (in a launch that fills the GPU the walk's throughput wins below this; a
// 16,386-block CFG runs 3.6x faster on levels), and the most blocks a CFG on
// the level schedule may have (its column's state, 8 bytes per block, must
// fit a workgroup's LDS; larger CFGs take the walk whatever the caller asks).
constexpr int OMPD_LEVEL_MIN_BLOCKS = 12288;
constexpr int OMPD_LEVEL_MAX_BLOCKS = 20000;
int ompd_default_sched(int n_blocks, int n_vars);
// A level tile keeps a whole column of its CFG in LDS, so a CU runs one at a time: the level
// schedule has the lower latency per CFG but the lower throughput per CU.  When the CFGs that
// the default rule put on it have more level tiles than this many rounds of the CUs take, they
// go back to the walk (the launch is throughput-bound then).  Serving C2-shaped requests: 3
// rounds gave a p50 of 243-453 ms at half load, 5 rounds 189 ms at the same capacity (~146
// requests/s), 8 rounds 149 ms but a capacity of 133 requests/s.
constexpr int OMPD_LEVEL_ROUNDS = 5;
// ... and a launch with at most n_cu / OMPD_IDLE_FRACTION walk tiles moves the CFGs that the rule
// put on the walk to the level schedule (one round of level tiles at most): alone, a CFG usually
// finishes sooner there.
constexpr int OMPD_IDLE_FRACTION = 4;
void ompd_settle_sched(ompd::DevCfg* h, int n, int n_cu);
// Default bound of a kernel wait without progress (the longest legitimate wait is one step of
// the other wavefront, microseconds).
constexpr int64_t OMPD_WAIT_DEFAULT_NS = 2000000000ll;
// Launch shape of a set of CFGs: tiles (longest first), edge-step items and grids.
struct Shape {
    std::vector<ompd::Tile> tiles;
    std::vector<ompd::EdgeItem> items;
    LaunchDims dims;
    size_t lds_prep = 0;
};
int ompd_make_shape(ompd_ctx* ctx, const std::vector<ompd::DevCfg>& cfgs, const PlanConfig& pc, Shape& sh);
int ompd_launch_prep(const ompd::DevCfg* d_cfgs, int n, int32_t* d_counter, size_t lds, int ring_slots, hipStream_t s);
int ompd_launch_solve(const ompd::DevCfg* d_cfgs, const ompd::Tile* d_tiles, int n_tiles, const ompd::EdgeItem* d_items,
                      int n_items, int32_t* d_counter, const LaunchDims& dims, hipStream_t s,
                      hipEvent_t* after = nullptr);
int ompd_plan_build(ompd_ctx* ctx, const ompd_cfg* cfgs, ompd_result* res, int32_t n, uint32_t flags,
                    const PlanConfig& pc, ompd_plan** out);
int ompd_plan_retile(ompd_plan* p, const PlanConfig& pc);
int ompd_plan_run_locked(ompd_plan* p, hipStream_t s);
int ompd_plan_collect(ompd_plan* p, int32_t* per_cfg);
int ompd_batch_locked(ompd_ctx* ctx, const ompd_cfg* cfgs, ompd_result* res, int32_t n, uint32_t flags,
                      hipStream_t s);
void ompd_serving_shutdown(ompd_ctx* ctx);
