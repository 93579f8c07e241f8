// Host runtime of libompd: contexts, resident plans (scratch arena, tiles,
// captured HIP graph), the host-pointer batch path and the autotuner.
// The serving loop lives in ompd_serving.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ompd.h"
#include "ompd_device.h"
#include "ompd_internal.h"

namespace ompd {
extern "C" __global__ void ompd_k_prep(const DevCfg*, int, int32_t*, int);
extern "C" __global__ void ompd_k_nu(const DevCfg*, const Tile*, int, int32_t*, int);
extern "C" __global__ void ompd_k_ave(const DevCfg*, const Tile*, int, int32_t*, int);
extern "C" __global__ void ompd_k_mayp(const DevCfg*, const Tile*, int, int32_t*, int);
extern "C" __global__ void ompd_k_later(const DevCfg*, const Tile*, int, int32_t*, int);
extern "C" __global__ void ompd_k_avf(const DevCfg*, const Tile*, int, int32_t*, int);
extern "C" __global__ void ompd_k_post_ave(const DevCfg*, const Tile*, const EdgeItem*, int, int32_t*);
extern "C" __global__ void ompd_k_post_mayp(const DevCfg*, const Tile*, const EdgeItem*, int, int32_t*);
extern "C" __global__ void ompd_k_post_later(const DevCfg*, const Tile*, const EdgeItem*, int, int32_t*);
extern "C" __global__ void ompd_k_post_avf(const DevCfg*, const Tile*, const EdgeItem*, int, int32_t*);
extern "C" __global__ void ompd_k_live(const DevCfg*, const Tile*, int, int32_t*, int);
extern "C" __global__ void ompd_k_post_live(const DevCfg*, const Tile*, const EdgeItem*, int, int32_t*);
extern "C" __global__ void ompd_k_lv_live(const DevCfg*, const Tile*, int, int32_t*);
extern "C" __global__ void ompd_k_varkind(const DevCfg*, const Tile*, int, int32_t*);
extern "C" __global__ void ompd_k_solve(const DevCfg*, const Tile*, int, int32_t*, int);
extern "C" __global__ void ompd_k_lv_nu(const DevCfg*, const Tile*, int, int32_t*);
extern "C" __global__ void ompd_k_lv_ave(const DevCfg*, const Tile*, int, int32_t*);
extern "C" __global__ void ompd_k_lv_mayp(const DevCfg*, const Tile*, int, int32_t*);
extern "C" __global__ void ompd_k_lv_later(const DevCfg*, const Tile*, int, int32_t*);
extern "C" __global__ void ompd_k_lv_avf(const DevCfg*, const Tile*, int, int32_t*);
static const void* const k_levels[N_PHASES] = {(const void*)ompd_k_lv_nu, (const void*)ompd_k_lv_ave,
                                               (const void*)ompd_k_lv_mayp, (const void*)ompd_k_lv_later,
                                               (const void*)ompd_k_lv_avf, (const void*)ompd_k_lv_live};
static const void* const k_phases[N_PHASES] = {(const void*)ompd_k_nu, (const void*)ompd_k_ave,
                                               (const void*)ompd_k_mayp, (const void*)ompd_k_later,
                                               (const void*)ompd_k_avf, (const void*)ompd_k_live};
// threads of a phase workgroup: the compute and the helper wavefront
constexpr int PHASE_THREADS = 128;
}  // namespace ompd

using namespace ompd;

static thread_local std::string g_err;

// Scratch of the allocation-free batch entry point (ompd_analyze_batch_noalloc):
// every device the library runs on holds its own copy, from the first context
// on it until the process ends.  Host code never passes this name to a kernel
// or a copy: it uses the device address that hipGetSymbolAddress returns for
// the current device (ompd_ctx::static_scratch).
constexpr size_t OMPD_STATIC_SCRATCH_BYTES = (size_t)OMPD_NOALLOC_SCRATCH_MIB << 20;
static __device__ __align__(256) char scratch[OMPD_STATIC_SCRATCH_BYTES];
static std::mutex g_scratch_mu[64];   // one caller at a time per device (the scratch is shared)

int ompd_fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define CK(x)                                                                                   \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess)                                                                   \
            return ompd_fail(OMPD_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_));    \
    } while (0)

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
static void drop_graphs(ompd_plan* p);

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" int ompd_ctx_create(ompd_ctx** out, int device_ordinal, uint64_t budget)
{
    if (!out) return ompd_fail(OMPD_E_INVAL, "out is NULL");
    int ndev = 0;
    CK(hipGetDeviceCount(&ndev));
    if (device_ordinal < 0 || device_ordinal >= ndev) return ompd_fail(OMPD_E_DEVICE, "no such device");
    ompd_ctx* c = new ompd_ctx();
    c->device = device_ordinal;
    c->budget = budget ? budget : (64ull << 30);
    hipError_t e = hipSetDevice(device_ordinal);
    if (e == hipSuccess) e = hipGetDeviceProperties(&c->prop, device_ordinal);
    if (e != hipSuccess) {
        delete c;
        return ompd_fail(OMPD_E_DEVICE, hipGetErrorString(e));
    }
    c->n_cu = c->prop.multiProcessorCount;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device_ordinal) == hipSuccess && khz > 0)
        c->wall_khz = khz;
    (void)hipGetLastError();
    c->wait_ticks = (int32_t)std::min<int64_t>(OMPD_WAIT_DEFAULT_NS / 1000 * c->wall_khz / 1000, INT32_MAX);
    // this device's address of the static scratch (the device is current)
    void* sp = nullptr;
    e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !sp) {
        delete c;
        return ompd_fail(OMPD_E_DEVICE, std::string("static scratch address: ") + hipGetErrorString(e));
    }
    c->static_scratch = (char*)sp;
    size_t lds_max = c->prop.maxSharedMemoryPerMultiProcessor;
    if (!lds_max) lds_max = c->prop.sharedMemPerBlock;
    lds_max = std::min<size_t>(lds_max ? lds_max : 64 * 1024, 160 * 1024);
    // dynamic LDS limit per kernel = device limit minus the kernel's static LDS
    int dyn = (int)lds_max;
    for (const void* k : {k_phases[0], k_phases[1], k_phases[2], k_phases[3], k_phases[4], k_phases[5],
                          (const void*)ompd_k_prep, (const void*)ompd_k_solve, k_levels[0], k_levels[1], k_levels[2],
                          k_levels[3], k_levels[4], k_levels[5]}) {
        hipFuncAttributes fa{};
        int st = 0;
        if (hipFuncGetAttributes(&fa, k) == hipSuccess) st = (int)fa.sharedSizeBytes;
        int want = (int)lds_max - st;
        if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, want) != hipSuccess) {
            (void)hipGetLastError();
            want = std::min(want, 64 * 1024 - st);
        }
        dyn = std::min(dyn, want);
    }
    (void)hipGetLastError();
    c->lds_max = dyn;
    *out = c;
    return OMPD_OK;
}

extern "C" int ompd_set_wait_limit(ompd_ctx* c, int64_t ns)
{
    if (!c) return ompd_fail(OMPD_E_INVAL, "ctx is NULL");
    if (ns < 0) return ompd_fail(OMPD_E_INVAL, "wait limit is negative");
    std::lock_guard<std::mutex> lk(c->mu);
    if (ns == 0) ns = OMPD_WAIT_DEFAULT_NS;
    const int64_t t = ns / 1000 * c->wall_khz / 1000 + (ns % 1000) * c->wall_khz / 1000000;
    c->wait_ticks = (int32_t)std::max<int64_t>(1, std::min<int64_t>(t, INT32_MAX));
    return OMPD_OK;
}

extern "C" void ompd_ctx_destroy(ompd_ctx* c)
{
    if (!c) return;
    ompd_serving_shutdown(c);
    delete c;
}

extern "C" const char* ompd_last_error(const ompd_ctx*) { return g_err.c_str(); }

extern "C" int ompd_device_info(ompd_ctx* c, int32_t* n_cu, int32_t* lds_bytes, int64_t* mem_bytes)
{
    if (!c) return ompd_fail(OMPD_E_INVAL, "ctx is NULL");
    if (n_cu) *n_cu = c->n_cu;
    if (lds_bytes) *lds_bytes = c->lds_max;
    if (mem_bytes) *mem_bytes = (int64_t)c->prop.totalGlobalMem;
    return OMPD_OK;
}

// ---------------------------------------------------------------------------
// tile rules
// ---------------------------------------------------------------------------
// Cut one CFG into tiles: ceil(wd / TILE_WORDS) runs of words, split evenly.
static void make_tiles(int ci, int nv, std::vector<Tile>& out)
{
    int wd = (nv + 63) / 64;
    int t = tiles_of(wd);
    if (wd == 0) {
        out.push_back(Tile{ci, 0, 0, 0});
        return;
    }
    int s0 = 0;
    for (int k = 0; k < t; ++k) {
        int n = wd / t + (k < wd % t ? 1 : 0);
        out.push_back(Tile{ci, s0, n, k});
        s0 += n;
    }
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
static int check_cfg_host(const ompd_cfg& g, int i)
{
    char buf[160];
    auto bad = [&](const char* why) {
        snprintf(buf, sizeof buf, "cfg %d: %s", i, why);
        return ompd_fail(OMPD_E_INVAL, buf);
    };
    if (g.n_blocks < 2) return bad("n_blocks < 2");
    if (g.n_edges < 0 || g.n_vars < 0) return bad("negative size");
    if (g.entry < 0 || g.entry >= g.n_blocks || g.exit < 0 || g.exit >= g.n_blocks || g.entry == g.exit)
        return bad("entry/exit out of range");
    if (!g.succ_ptr || !g.space) return bad("succ_ptr/space missing");
    if (g.n_edges > 0 && (!g.succ_idx || !g.edge_kind)) return bad("succ_idx/edge_kind missing");
    if (g.n_vars > 0 && (!g.read_bits || !g.write_bits)) return bad("read/write bits missing");
    if (g.call_summary && (g.n_summaries <= 0 || !g.summaries)) return bad("call summaries missing");
    return OMPD_OK;
}

// Scratch of one CFG, offsets relative to its base (each 256-aligned).
size_t ompd_cfg_scratch(const ompd_cfg& g, const ompd_result& r, ScratchOff& o)
{
    size_t total = 0;
    auto take = [&](size_t bytes) { size_t x = total; total += align256(bytes); return x; };
    size_t wd = (size_t)(g.n_vars + 63) / 64;
    size_t bv = (size_t)g.n_blocks * wd * 8, ev = (size_t)g.n_edges * wd * 8;
    o.aveout = take(2 * bv);
    o.mayp = take(2 * bv);
    o.later = take(2 * bv);
    o.eag = take(2 * ev);
    o.both = take(ev);
    o.flg = take((size_t)tiles_of((int)wd) * 4 * (size_t)g.n_blocks * 8);
    o.nu = (r.nu_host && r.nu_dev) ? SIZE_MAX : take(2 * bv);
    o.ave = (r.ave_host && r.ave_dev) ? SIZE_MAX : take(2 * bv);
    o.ie = (r.ins_entry_to_host && r.ins_entry_to_dev) ? SIZE_MAX : take(2 * bv);
    o.ig = (r.ins_edge_to_host && r.ins_edge_to_dev) ? SIZE_MAX : take(2 * ev);
    o.avf = (!r.avf_host == !r.avf_dev) ? SIZE_MAX : take(2 * bv);
    o.vk = r.var_kind ? take(4 * wd * 8) : SIZE_MAX;
    o.fp = take(wd * 8 + 8);
    o.bnd = take(4 * wd * 8);
    o.pp = take(4 * ((size_t)g.n_blocks + 1));
    o.pi = take(4 * (size_t)std::max(g.n_edges, 1));
    o.pe = take(4 * (size_t)std::max(g.n_edges, 1));
    o.tmp = take(4 * ((size_t)g.n_blocks + 1));
    o.recf = take(32 * (size_t)g.n_blocks);
    o.recb = take(32 * (size_t)g.n_blocks);
    o.stf = take(32 * (size_t)g.n_blocks);
    o.stb = take(32 * (size_t)g.n_blocks);
    o.lorder = take(4 * (size_t)g.n_blocks);
    o.loff = take(4 * ((size_t)g.n_blocks + 1));
    o.info = take(4 * INFO_WORDS);
    return total;
}

// The schedule of a CFG when the caller names none: the level schedule for
// large CFGs, whose levels hold enough blocks to keep a workgroup busy.
int ompd_default_sched(int n_blocks, int n_vars)
{
    (void)n_vars;
    return n_blocks >= OMPD_LEVEL_MIN_BLOCKS ? SCHED_LEVEL : SCHED_WALK;
}

void ompd_settle_sched(DevCfg* h, int n, int n_cu)
{
    auto by_rule = [&](const DevCfg& d) { return d.sched == SCHED_LEVEL && d.sched_rule; };
    int64_t tiles = 0;
    for (int i = 0; i < n; ++i)
        if (by_rule(h[i])) tiles += 2 * (int64_t)h[i].wd + 1;
    if (tiles > (int64_t)OMPD_LEVEL_ROUNDS * n_cu) {
        for (int i = 0; i < n; ++i)
            if (by_rule(h[i])) h[i].sched = SCHED_WALK;
        return;
    }
    // A launch whose walk tiles leave most CUs idle is bound by its longest tile's dependent
    // steps, not by throughput: there the level schedule (a wavefront per 32-bit column, the
    // blocks of a level in parallel) usually finishes a CFG sooner (40 C3 CFGs alone: 0.16-0.9x
    // the walk's time, a few small ones up to 1.1x), so the CFGs the rule put on the walk move to
    // it while one round of level tiles holds them all.
    int64_t walk = 0, level = 0;
    for (int i = 0; i < n; ++i) {
        if (h[i].sched == SCHED_LEVEL) level += 2 * (int64_t)h[i].wd + 1;
        else walk += tiles_of(h[i].wd);
    }
    if (walk == 0 || walk * OMPD_IDLE_FRACTION > n_cu) return;
    for (int i = 0; i < n; ++i) {
        if (h[i].sched != SCHED_WALK || !h[i].sched_rule || h[i].nb > OMPD_LEVEL_MAX_BLOCKS) continue;
        const int64_t t = 2 * (int64_t)h[i].wd + 1;
        if (level + t > n_cu) continue;
        h[i].sched = SCHED_LEVEL;
        level += t;
    }
}

// Fill the kernels' descriptor of one CFG whose scratch starts at `base`.
// Default boundary values (for NULL boundaries) are written to bnd_host
// ([4*wd] words: entry valid H, D, exit live H, D), to be copied by the
// caller to bnd_dev (default: base + o.bnd), where the descriptor points.
void ompd_fill_devcfg(const ompd_cfg& g, const ompd_result& r, char* base, const ScratchOff& o, uint32_t flags,
                      int32_t wait_ticks, DevCfg& d, uint64_t* bnd_host, uint64_t* bnd_dev)
{
    int wd = (g.n_vars + 63) / 64;
    memset(&d, 0, sizeof d);
    d.wait_ticks = wait_ticks > 0 ? wait_ticks : 1;
    d.nb = g.n_blocks; d.ne = g.n_edges; d.nv = g.n_vars; d.entry = g.entry; d.exit = g.exit; d.wd = wd;
    d.n_sums = g.call_summary ? g.n_summaries : 0;
    d.placement = ((flags & OMPD_F_PLACEMENT_EAGER) ? PL_EAGER : 0) | ((flags & OMPD_F_SUMMARY) ? PL_SUMMARY : 0) |
                  ((flags & OMPD_F_PLACEMENT_LAZY) ? PL_LAZY : 0) | ((flags & OMPD_F_PLACEMENT_REFINE) ? PL_REFINE : 0);
    d.sweep_cap = (int)((flags >> 16) & 0xFFFFu);
    d.sched = (flags & OMPD_F_SCHED_LEVEL) ? SCHED_LEVEL
            : (flags & OMPD_F_SCHED_WALK) ? SCHED_WALK
            : ompd_default_sched(g.n_blocks, g.n_vars);
    d.sched_rule = !(flags & (OMPD_F_SCHED_LEVEL | OMPD_F_SCHED_WALK));
    if (g.n_blocks > OMPD_LEVEL_MAX_BLOCKS) d.sched = SCHED_WALK;
    d.succ_ptr = g.succ_ptr; d.succ_idx = g.succ_idx; d.kind = g.edge_kind; d.space = g.space;
    d.R = g.read_bits; d.W = g.write_bits;
    uint64_t* bnd = bnd_dev ? bnd_dev : (uint64_t*)(base + o.bnd);
    d.ev_h = g.entry_valid_host ? g.entry_valid_host : bnd;
    d.ev_d = g.entry_valid_dev ? g.entry_valid_dev : bnd + wd;
    d.lx_h = g.exit_live_host ? g.exit_live_host : bnd + 2 * wd;
    d.lx_d = g.exit_live_dev ? g.exit_live_dev : bnd + 3 * wd;
    d.call = g.call_summary; d.sums = g.summaries;
    d.scalar = g.scalar;
    d.fp = (uint64_t*)(base + o.fp);
    d.fpc = r.fp_clause;
    size_t bvw = (size_t)g.n_blocks * wd, evw = (size_t)g.n_edges * wd;
    auto at = [&](size_t off) { return off == SIZE_MAX ? (uint64_t*)nullptr : (uint64_t*)(base + off); };
    uint64_t *nu = at(o.nu), *ave = at(o.ave), *ie = at(o.ie), *ig = at(o.ig), *avf = at(o.avf);
    // a requested half is written in place; a missing half goes to scratch
    d.nu_h = r.nu_host ? r.nu_host : nu;               d.nu_d = r.nu_dev ? r.nu_dev : nu + bvw;
    d.ave_h = r.ave_host ? r.ave_host : ave;           d.ave_d = r.ave_dev ? r.ave_dev : ave + bvw;
    d.ie_h = r.ins_entry_to_host ? r.ins_entry_to_host : ie;
    d.ie_d = r.ins_entry_to_dev ? r.ins_entry_to_dev : ie + bvw;
    d.ig_h = r.ins_edge_to_host ? r.ins_edge_to_host : ig;
    d.ig_d = r.ins_edge_to_dev ? r.ins_edge_to_dev : ig + evw;
    if (r.avf_host || r.avf_dev) {
        d.avf_h = r.avf_host ? r.avf_host : avf;
        d.avf_d = r.avf_dev ? r.avf_dev : avf + bvw;
    }
    d.var_kind = r.var_kind; d.after_dev = r.after_dev; d.before_dev = r.before_dev;
    uint64_t* ao = at(o.aveout);
    uint64_t* mp = at(o.mayp);
    uint64_t* la = at(o.later);
    d.aveout_h = ao; d.aveout_d = ao + bvw; d.mayp_h = mp; d.mayp_d = mp + bvw;
    d.later_h = la; d.later_d = la + bvw;
    uint64_t* ea = at(o.eag);
    d.eag_h = ea; d.eag_d = ea + evw; d.both = at(o.both);
    d.flg = at(o.flg);
    d.vk_acc = at(o.vk);
    d.pred_ptr = (int32_t*)(base + o.pp); d.pred_idx = (int32_t*)(base + o.pi);
    d.pred_eid = (int32_t*)(base + o.pe); d.tmp = (int32_t*)(base + o.tmp);
    d.rec_f = (int32_t*)(base + o.recf); d.rec_b = (int32_t*)(base + o.recb);
    d.step_f = (int32_t*)(base + o.stf); d.step_b = (int32_t*)(base + o.stb);
    d.lorder = (int32_t*)(base + o.lorder); d.loff = (int32_t*)(base + o.loff);
    d.info = (int32_t*)(base + o.info);
    if (bnd_host && wd > 0) {
        uint64_t last = (g.n_vars & 63) ? ((1ull << (g.n_vars & 63)) - 1) : ~0ull;
        for (int w = 0; w < 4 * wd; ++w) bnd_host[w] = 0;
        for (int w = 0; w < wd; ++w) {
            uint64_t m = (w == wd - 1) ? last : ~0ull;
            bnd_host[w] = m;            // entry valid on the host
            bnd_host[2 * wd + w] = m;   // live on the host after exit
        }
    }
}

// Default result ring of one phase workgroup (recently computed blocks, STATE_BYTES each).
constexpr size_t RING_BYTES_DEFAULT = 64 * STATE_BYTES;

// Tiles for a set of CFGs, longest first, the edge-step items and the launch
// sizes that go with them under a configuration.
int ompd_make_shape(ompd_ctx* ctx, const std::vector<DevCfg>& cfgs, const PlanConfig& pc, Shape& sh)
{
    std::vector<Tile>& tiles = sh.tiles;
    tiles.clear();
    sh.items.clear();
    auto in_plan = [&](int i) { return pc.only_bucket < 0 || ompd_sched_bucket(cfgs[i].nb) == pc.only_bucket; };
    for (int i = 0; i < (int)cfgs.size(); ++i)
        if (in_plan(i)) make_tiles(i, cfgs[i].nv, tiles);
    // a tile's work ~ its blocks times the sweeps, which grow with the CFG: longest first
    std::stable_sort(tiles.begin(), tiles.end(),
                     [&](const Tile& a, const Tile& b) { return cfgs[a.cfg].nb > cfgs[b.cfg].nb; });
    // level tiles (after the walk tiles): each 32-bit column of a CFG on the level schedule, and
    // its flag column (s0 = -1)
    std::vector<Tile> lt;
    int lv_nb = 0;
    for (int i = 0; i < (int)cfgs.size(); ++i) {
        if (cfgs[i].sched != SCHED_LEVEL || !in_plan(i)) continue;
        lv_nb = std::max(lv_nb, cfgs[i].nb);
        lt.push_back(Tile{i, -1, 0, 0});
        for (int hc = 0; hc < 2 * cfgs[i].wd; ++hc) lt.push_back(Tile{i, hc, 1, 0});
    }
    std::stable_sort(lt.begin(), lt.end(), [&](const Tile& a, const Tile& b) { return cfgs[a.cfg].nb > cfgs[b.cfg].nb; });
    sh.dims.n_level = (int)lt.size();
    tiles.insert(tiles.end(), lt.begin(), lt.end());
    // pass items: runs of up to PASS_WORDS words (the passes need no LDS, so a full wavefront of
    // words each), 64-block chunks, longest CFGs first
    {
        std::vector<int> order(cfgs.size());
        for (int i = 0; i < (int)order.size(); ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cfgs[a].nb > cfgs[b].nb; });
        for (int i : order) {
            const int wd = cfgs[i].wd;
            if (wd <= 0 || !in_plan(i)) continue;
            const int runs = (wd + PASS_WORDS - 1) / PASS_WORDS;
            for (int r = 0; r < runs; ++r) {
                const int s0 = (int)((int64_t)wd * r / runs), s1 = (int)((int64_t)wd * (r + 1) / runs);
                for (int b0 = 0; b0 < cfgs[i].nb; b0 += 64) sh.items.push_back(EdgeItem{i, s0, s1 - s0, b0});
            }
        }
    }
    // result ring: a power of two of STATE_BYTES slots in [8, 64], as large as every phase's LDS allows
    const size_t want = pc.lds_bytes ? pc.lds_bytes : RING_BYTES_DEFAULT;
    int rs = 8;
    while (rs < 64 && (size_t)(2 * rs) * STATE_BYTES <= want) rs *= 2;
    while (rs > 1 && phase_lds(PH_LATER, rs) > (size_t)ctx->lds_max) rs /= 2;
    LaunchDims& dm = sh.dims;
    dm.ring_slots = rs;
    sh.lds_prep = 0;
    // each phase kernel: as many workgroups as it keeps resident
    for (int ph = 0; ph < N_PHASES; ++ph) {
        dm.lds[ph] = phase_lds(ph, rs);
        int n = 0;
        CK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_phases[ph], PHASE_THREADS, dm.lds[ph]));
        n = std::max(1, n);
        if (pc.wg_per_cu > 0) n = std::min(n, pc.wg_per_cu);
        dm.grid[ph] = std::max(1, std::min((int)tiles.size(), n * ctx->n_cu));
    }
    dm.split = pc.split;
    dm.lds_tile = 0;
    for (int ph = 0; ph < N_PHASES; ++ph) dm.lds_tile = std::max(dm.lds_tile, dm.lds[ph]);
    dm.refine = false;
    for (int i = 0; i < (int)cfgs.size(); ++i) dm.refine |= in_plan(i) && refines(cfgs[i].placement);
    {
        int n = 0;
        CK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)ompd_k_solve, PHASE_THREADS, dm.lds_tile));
        n = std::max(1, n);
        if (pc.wg_per_cu > 0) n = std::min(n, pc.wg_per_cu);
        dm.grid_tile = std::max(1, std::min((int)tiles.size(), n * ctx->n_cu));
    }
    dm.lds_level = align256(8 * (size_t)lv_nb);
    if (dm.n_level) {
        if (dm.lds_level > (size_t)ctx->lds_max)
            return ompd_fail(OMPD_E_INVAL, "a CFG on the level schedule has more blocks than LDS holds");
        int n = 0;
        CK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_levels[PH_LATER], LEVEL_THREADS, dm.lds_level));
        dm.grid_level = std::max(1, std::min(dm.n_level, std::max(1, n) * ctx->n_cu));
    }
    if (dm.n_level) dm.split = true;   // the per-tile kernel does not run level tiles
    int pe = 1;
    CK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&pe, (const void*)ompd_k_post_ave, 64, 0));
    dm.grid_edge = std::max(1, std::min((int)std::max<size_t>(sh.items.size(), tiles.size()), std::max(1, pe) * ctx->n_cu));
    return OMPD_OK;
}

int ompd_plan_build(ompd_ctx* ctx, const ompd_cfg* cfgs, ompd_result* res, int32_t n, uint32_t flags,
                    const PlanConfig& pc, ompd_plan** out)
{
    if (!ctx || !out || n < 0 || (n > 0 && !cfgs)) return ompd_fail(OMPD_E_INVAL, "bad arguments");
    for (int i = 0; i < n; ++i) {
        int rc = check_cfg_host(cfgs[i], i);
        if (rc) return rc;
    }
    CK(hipSetDevice(ctx->device));
    ompd_plan* p = new ompd_plan();
    p->ctx = ctx;
    p->n = n;
    p->flags = flags;
    p->cfg = pc;
    if (flags & OMPD_F_TILE_KERNEL) p->cfg.split = false;
    if (const uint32_t r = (flags >> 8) & 7u) p->cfg.lds_bytes = (size_t)(4u << r) * STATE_BYTES;   // 8 .. 64 slots
    p->res.assign(res, res + n);
    p->h_cfgs.resize(n);

    std::vector<ScratchOff> off(n);
    std::vector<size_t> base(n);
    size_t total = 0;
    int max_nb = 2;
    for (int i = 0; i < n; ++i) {
        base[i] = total;
        total += ompd_cfg_scratch(cfgs[i], res[i], off[i]);
        max_nb = std::max(max_nb, cfgs[i].n_blocks);
    }
    size_t counter_off = total;
    total += 256;
    // default boundaries of every CFG, side by side (one upload)
    std::vector<size_t> boff(n);
    size_t bnd_words = 0;
    for (int i = 0; i < n; ++i) {
        boff[i] = bnd_words;
        bnd_words += 4 * (size_t)((cfgs[i].n_vars + 63) / 64);
    }
    const size_t bnd_off = total;
    total += (8 * bnd_words + 255) & ~(size_t)255;
    p->scratch_bytes = total;
    hipError_t e = hipMalloc(&p->scratch, std::max<size_t>(total, 256));
    if (e != hipSuccess) {
        delete p;
        return ompd_fail(OMPD_E_NOMEM, std::string("scratch allocation: ") + hipGetErrorString(e));
    }
    char* S = (char*)p->scratch;
    p->d_counter = (int32_t*)(S + counter_off);
    std::vector<uint64_t> bnd(std::max<size_t>(bnd_words, 1), 0);
    uint64_t* bnd_dev = (uint64_t*)(S + bnd_off);
    for (int i = 0; i < n; ++i)
        ompd_fill_devcfg(cfgs[i], res[i], S + base[i], off[i], flags, ctx->wait_ticks, p->h_cfgs[i], bnd.data() + boff[i],
                         bnd_dev + boff[i]);
    if (bnd_words) {
        e = hipMemcpy(bnd_dev, bnd.data(), 8 * bnd_words, hipMemcpyHostToDevice);
        if (e != hipSuccess) { ompd_plan_destroy(p); return ompd_fail(OMPD_E_DEVICE, hipGetErrorString(e)); }
    }
    p->max_nb = max_nb;
    e = hipMalloc(&p->d_cfgs, sizeof(DevCfg) * std::max(n, 1));
    if (e == hipSuccess && n > 0)
        e = hipMemcpy(p->d_cfgs, p->h_cfgs.data(), sizeof(DevCfg) * n, hipMemcpyHostToDevice);
    if (e != hipSuccess) { ompd_plan_destroy(p); return ompd_fail(OMPD_E_DEVICE, hipGetErrorString(e)); }
    p->h_info.assign((size_t)n * INFO_WORDS, 0);
    e = hipMalloc(&p->d_info, 4 * INFO_WORDS * (size_t)std::max(n, 1));
    if (e != hipSuccess) { ompd_plan_destroy(p); return ompd_fail(OMPD_E_NOMEM, hipGetErrorString(e)); }
    int rc = ompd_plan_retile(p, p->cfg);
    if (rc) { ompd_plan_destroy(p); return rc; }
    CK(hipEventCreate(&p->ev0));
    CK(hipEventCreate(&p->ev1));
    CK(hipEventCreate(&p->ev2));
    *out = p;
    return OMPD_OK;
}

// (Re)build tiles and launch shapes for a configuration (drops captured graphs).
int ompd_plan_retile(ompd_plan* p, const PlanConfig& pc)
{
    ompd_ctx* ctx = p->ctx;
    // the schedule of each CFG the plan's flags leave open: the bucket's choice, else the rule
    if (!(p->flags & (OMPD_F_SCHED_LEVEL | OMPD_F_SCHED_WALK))) {
        bool changed = false;
        for (int i = 0; i < p->n; ++i) {
            DevCfg& d = p->h_cfgs[i];
            const int want = pc.bucket_sched[ompd_sched_bucket(d.nb)];
            int sc = want < 0 ? ompd_default_sched(d.nb, d.nv) : want;
            if (d.nb > OMPD_LEVEL_MAX_BLOCKS) sc = SCHED_WALK;
            d.sched_rule = want < 0;
            if (d.sched != sc) { d.sched = sc; changed = true; }
        }
        std::vector<int> before(p->n);
        for (int i = 0; i < p->n; ++i) before[i] = p->h_cfgs[i].sched;
        ompd_settle_sched(p->h_cfgs.data(), p->n, ctx->n_cu);
        for (int i = 0; i < p->n; ++i) changed |= before[i] != p->h_cfgs[i].sched;
        if (changed && p->d_cfgs)
            CK(hipMemcpy(p->d_cfgs, p->h_cfgs.data(), sizeof(DevCfg) * p->n, hipMemcpyHostToDevice));
    }
    Shape sh;
    int rc = ompd_make_shape(ctx, p->h_cfgs, pc, sh);
    if (rc) return rc;
    p->cfg = pc;
    p->dims = sh.dims;
    p->lds_prep = sh.lds_prep;
    p->h_tiles = sh.tiles;
    p->n_tiles = (int)sh.tiles.size();
    p->n_items = (int)sh.items.size();
    if (p->d_tiles) { (void)hipFree(p->d_tiles); p->d_tiles = nullptr; }
    if (p->d_items) { (void)hipFree(p->d_items); p->d_items = nullptr; }
    CK(hipMalloc(&p->d_tiles, sizeof(Tile) * std::max(p->n_tiles, 1)));
    CK(hipMalloc(&p->d_items, sizeof(EdgeItem) * std::max(p->n_items, 1)));
    if (p->n_tiles)
        CK(hipMemcpy(p->d_tiles, sh.tiles.data(), sizeof(Tile) * p->n_tiles, hipMemcpyHostToDevice));
    if (p->n_items)
        CK(hipMemcpy(p->d_items, sh.items.data(), sizeof(EdgeItem) * p->n_items, hipMemcpyHostToDevice));
    drop_graphs(p);
    return OMPD_OK;
}

int ompd_launch_prep(const DevCfg* d_cfgs, int n, int32_t* d_counter, size_t lds, int ring_slots, hipStream_t s)
{
    if (n <= 0) return OMPD_OK;
    hipLaunchKernelGGL(ompd_k_prep, dim3(n), dim3(256), lds, s, d_cfgs, n, d_counter, ring_slots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return ompd_fail(OMPD_E_DEVICE, std::string("prep launch (lds ") + std::to_string(lds) + "): " +
                                            hipGetErrorString(e));
    return OMPD_OK;
}

int ompd_launch_solve(const DevCfg* d_cfgs, const Tile* d_tiles, int n_tiles, const EdgeItem* d_items, int n_items,
                      int32_t* d_counter, const LaunchDims& dm, hipStream_t s, hipEvent_t* after)
{
    if (n_tiles <= 0) return OMPD_OK;
    // the walk tiles, then the level tiles
    const int n_level = dm.n_level;
    n_tiles -= n_level;
    const Tile* d_ltiles = d_tiles + n_tiles;
    const int rs = dm.ring_slots, grid_edge = dm.grid_edge;
    int k = 0;
    auto mark = [&]() { if (after) (void)hipEventRecord(after[k], s); ++k; };
    if (!dm.split) {
        // every phase and pass of a tile in one persistent kernel
        hipLaunchKernelGGL(ompd_k_solve, dim3(dm.grid_tile), dim3(PHASE_THREADS), dm.lds_tile, s, d_cfgs, d_tiles,
                           n_tiles, d_counter, rs);
        mark();
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return ompd_fail(OMPD_E_DEVICE, std::string("solve launch (ring slots ") + std::to_string(rs) + "): " +
                                                hipGetErrorString(e));
        return OMPD_OK;
    }
    // (a phase or pass that no CFG needs is not launched; its profile mark is still taken)
    auto phase = [&](int ph, bool launch) {
        if (launch && n_tiles > 0) {
            void* args[] = {(void*)&d_cfgs, (void*)&d_tiles, (void*)&n_tiles, (void*)&d_counter, (void*)&rs};
            (void)hipLaunchKernel(k_phases[ph], dim3(dm.grid[ph]), dim3(PHASE_THREADS), args, dm.lds[ph], s);
        }
        if (launch && n_level > 0) {
            void* args[] = {(void*)&d_cfgs, (void*)&d_ltiles, (void*)&n_level, (void*)&d_counter};
            (void)hipLaunchKernel(k_levels[ph], dim3(dm.grid_level), dim3(LEVEL_THREADS), args, dm.lds_level, s);
        }
        mark();
    };
    auto pass = [&](const void* fn, bool launch) {
        if (launch && n_items > 0) {
            void* args[] = {(void*)&d_cfgs, (void*)&d_tiles, (void*)&d_items, (void*)&n_items, (void*)&d_counter};
            (void)hipLaunchKernel(fn, dim3(grid_edge), dim3(64), args, 0, s);
        }
        mark();
    };
    phase(PH_NU, true);
    phase(PH_AVE, true);
    pass((const void*)ompd_k_post_ave, true);
    phase(PH_MAYP, true);
    pass((const void*)ompd_k_post_mayp, true);
    phase(PH_LATER, true);
    pass((const void*)ompd_k_post_later, true);
    phase(PH_LIVE, dm.refine);
    pass((const void*)ompd_k_post_live, dm.refine);
    phase(PH_AVF, true);
    pass((const void*)ompd_k_post_avf, true);
    hipLaunchKernelGGL(ompd_k_varkind, dim3(grid_edge), dim3(64), 0, s, d_cfgs, d_tiles, n_tiles, d_counter);
    mark();
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return ompd_fail(OMPD_E_DEVICE, std::string("solve launch (ring slots ") + std::to_string(rs) + "): " +
                                            hipGetErrorString(e));
    return OMPD_OK;
}

static int launch_prep(ompd_plan* p, hipStream_t s)
{
    return ompd_launch_prep((const DevCfg*)p->d_cfgs, p->n, p->d_counter, p->lds_prep, p->dims.ring_slots, s);
}

static int launch_solve(ompd_plan* p, hipStream_t s)
{
    return ompd_launch_solve((const DevCfg*)p->d_cfgs, (const Tile*)p->d_tiles, p->n_tiles,
                             (const EdgeItem*)p->d_items, p->n_items, p->d_counter, p->dims, s);
}

// Capture one launch function into an executable graph (nullptr if capture
// is not available here).
static hipGraphExec_t capture(ompd_plan* p, int (*fn)(ompd_plan*, hipStream_t), hipGraph_t* keep)
{
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    int rc = (e == hipSuccess) ? fn(p, cs) : OMPD_E_DEVICE;
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    (void)hipGetLastError();
    if (e != hipSuccess || e2 != hipSuccess || rc != OMPD_OK || !g) {
        if (g) (void)hipGraphDestroy(g);
        return nullptr;
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphDestroy(g);
        return nullptr;
    }
    *keep = g;
    return x;
}

static void drop_graphs(ompd_plan* p)
{
    if (p->gx_prep) (void)hipGraphExecDestroy(p->gx_prep);
    if (p->gx_solve) (void)hipGraphExecDestroy(p->gx_solve);
    if (p->g_prep) (void)hipGraphDestroy(p->g_prep);
    if (p->g_solve) (void)hipGraphDestroy(p->g_solve);
    p->gx_prep = p->gx_solve = nullptr;
    p->g_prep = p->g_solve = nullptr;
}

// Enqueue one solve: HIP events on the caller's stream around the ingest
// kernel and around the persistent solve (events stay outside the graphs).
static int launch_all(ompd_plan* p, hipStream_t s)
{
    (void)hipGetLastError();
    if (p->cfg.use_graph && !p->gx_prep) {
        p->gx_prep = capture(p, launch_prep, &p->g_prep);
        p->gx_solve = capture(p, launch_solve, &p->g_solve);
        if (!p->gx_prep || !p->gx_solve) {
            drop_graphs(p);
            p->cfg.use_graph = false;   // capture unavailable: launch directly
        }
    }
    CK(hipEventRecord(p->ev0, s));
    if (p->profile) {
        // direct launches with an event after every kernel, all on the caller's stream
        int rc = launch_prep(p, s);
        if (rc) return rc;
        CK(hipEventRecord(p->ev1, s));
        rc = ompd_launch_solve((const DevCfg*)p->d_cfgs, (const Tile*)p->d_tiles, p->n_tiles,
                               (const EdgeItem*)p->d_items, p->n_items, p->d_counter, p->dims, s, p->evk);
        if (rc) return rc;
        CK(hipEventRecord(p->ev2, s));
        return OMPD_OK;
    }
    if (p->cfg.use_graph) CK(hipGraphLaunch(p->gx_prep, s));
    else { int rc = launch_prep(p, s); if (rc) return rc; }
    CK(hipEventRecord(p->ev1, s));
    if (p->cfg.use_graph) CK(hipGraphLaunch(p->gx_solve, s));
    else { int rc = launch_solve(p, s); if (rc) return rc; }
    CK(hipEventRecord(p->ev2, s));
    return OMPD_OK;
}

extern "C" int ompd_plan_create(ompd_ctx* ctx, const ompd_cfg* cfgs, ompd_result* res, int32_t n, uint32_t flags,
                                ompd_plan** out)
{
    if (!(flags & OMPD_F_DEVICE_PTRS)) return ompd_fail(OMPD_E_INVAL, "plans need OMPD_F_DEVICE_PTRS");
    if (!ctx) return ompd_fail(OMPD_E_INVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    PlanConfig pc;
    return ompd_plan_build(ctx, cfgs, res, n, flags, pc, out);
}

int ompd_plan_run_locked(ompd_plan* p, hipStream_t s)
{
    CK(hipSetDevice(p->ctx->device));
    p->last_stream = s;
    return launch_all(p, s);
}

extern "C" int ompd_plan_run(ompd_plan* p, void* stream)
{
    if (!p) return ompd_fail(OMPD_E_INVAL, "plan is NULL");
    std::lock_guard<std::mutex> lk(p->ctx->mu);
    return ompd_plan_run_locked(p, (hipStream_t)stream);
}

std::string ompd_status_message(int i, const int32_t* inf)
{
    const int st = inf[INFO_STATUS];
    char buf[320];
    if (st == OMPD_E_DEVICE && inf[INFO_PM_PHASE] > 0) {
        static const char* const ph[5] = {"next use", "eager validity", "pending copies", "delayed placement",
                                          "final validity"};
        static const char* const what[5] = {"?", "inputs of a step (in_ready)", "a free ring slot (consumed)",
                                            "stored states (flushed)", "a produced step (produced, helper)"};
        const int k = inf[INFO_PM_PHASE] - 1, w = inf[INFO_PM_WHAT];
        snprintf(buf, sizeof buf,
                 "cfg %d: a kernel wait gave up (phase %s, tile %d of the CFG, waiting for %s: counter at %d, "
                 "needed %d, after %d wall-clock ticks)",
                 i, (k >= 0 && k < 5) ? ph[k] : "?", inf[INFO_PM_TILE], (w >= 0 && w < 5) ? what[w] : "?",
                 inf[INFO_PM_SEEN], inf[INFO_PM_TARGET], inf[INFO_PM_TICKS]);
    } else
        snprintf(buf, sizeof buf, "cfg %d: %s", i,
                 st == OMPD_E_INVAL ? "malformed CFG" : st == OMPD_E_NOCONVERGE ? "sweep cap reached" : "device error");
    return buf;
}

// The status words of every CFG of a launch (each in its own scratch) into one array, so that
// they come back in one copy instead of one per CFG.
__global__ void __launch_bounds__(256) ompd_k_info(const DevCfg* __restrict__ cfgs, int n, int32_t* __restrict__ out)
{
    const int total = n * INFO_WORDS;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x)
        out[t] = cfgs[t / INFO_WORDS].info[t % INFO_WORDS];
}

static int gather_info(const DevCfg* d_cfgs, int n, int32_t* d_out, int32_t* h_out, hipStream_t s)
{
    if (n <= 0) return OMPD_OK;
    const int total = n * INFO_WORDS;
    hipLaunchKernelGGL(ompd_k_info, dim3(std::min((total + 255) / 256, 1024)), dim3(256), 0, s, d_cfgs, n, d_out);
    CK(hipGetLastError());
    CK(hipMemcpyAsync(h_out, d_out, 4 * (size_t)total, hipMemcpyDeviceToHost, s));
    return OMPD_OK;
}

int ompd_plan_collect(ompd_plan* p, int32_t* per_cfg)
{
    CK(hipSetDevice(p->ctx->device));
    CK(hipStreamSynchronize(p->last_stream));
    if (p->n == 0) return OMPD_OK;
    // info words live per CFG inside the scratch arena
    int rg = gather_info(p->d_cfgs, p->n, p->d_info, p->h_info.data(), p->last_stream);
    if (rg) return rg;
    CK(hipStreamSynchronize(p->last_stream));
    int first = OMPD_OK;
    for (int i = 0; i < p->n; ++i) {
        const int32_t* inf = &p->h_info[(size_t)i * INFO_WORDS];
        int st = inf[INFO_STATUS];
        if (per_cfg) per_cfg[i] = st;
        for (int k = 0; k < 6; ++k) p->res[i].sweeps[k] = inf[INFO_SWEEPS + k];
        if (st && first == OMPD_OK) {
            first = st;
            g_err = ompd_status_message(i, inf);
        }
    }
    return first;
}

extern "C" int ompd_plan_status(ompd_plan* p, int32_t* per_cfg)
{
    if (!p) return ompd_fail(OMPD_E_INVAL, "plan is NULL");
    std::lock_guard<std::mutex> lk(p->ctx->mu);
    return ompd_plan_collect(p, per_cfg);
}

extern "C" int ompd_plan_last_ms(ompd_plan* p, float* total_ms, float* solve_ms)
{
    if (!p) return ompd_fail(OMPD_E_INVAL, "plan is NULL");
    CK(hipEventSynchronize(p->ev2));
    float a = 0, b = 0;
    CK(hipEventElapsedTime(&a, p->ev0, p->ev2));
    CK(hipEventElapsedTime(&b, p->ev1, p->ev2));
    if (total_ms) *total_ms = a;
    if (solve_ms) *solve_ms = b;
    return OMPD_OK;
}

extern "C" int ompd_plan_profile(ompd_plan* p, int32_t enable)
{
    if (!p) return ompd_fail(OMPD_E_INVAL, "plan is NULL");
    std::lock_guard<std::mutex> lk(p->ctx->mu);
    if (enable && !p->evk[0])
        for (hipEvent_t& e : p->evk) CK(hipEventCreate(&e));
    p->profile = enable != 0;
    return OMPD_OK;
}

extern "C" int ompd_plan_kernel_ms(ompd_plan* p, float* ms, int32_t capacity, int32_t* n_kernels)
{
    if (!p || !ms) return ompd_fail(OMPD_E_INVAL, "bad arguments");
    if (!p->profile) return ompd_fail(OMPD_E_INVAL, "profiling is off for this plan");
    CK(hipEventSynchronize(p->ev2));
    const int n = 1 + (p->dims.split ? N_SOLVE_KERNELS : 1);
    if (n_kernels) *n_kernels = n;
    hipEvent_t marks[2 + N_SOLVE_KERNELS] = {p->ev0, p->ev1};
    for (int k = 0; k < N_SOLVE_KERNELS; ++k) marks[2 + k] = p->evk[k];
    for (int k = 0; k < n && k < capacity; ++k) {
        float x = 0;
        CK(hipEventElapsedTime(&x, marks[k], marks[k + 1]));
        ms[k] = x;
    }
    return OMPD_OK;
}

extern "C" int ompd_plan_configure(ompd_plan* p, int64_t lds_bytes, int32_t wg_per_cu)
{
    if (!p || lds_bytes < 0 || wg_per_cu < 0) return ompd_fail(OMPD_E_INVAL, "bad plan configuration");
    std::lock_guard<std::mutex> lk(p->ctx->mu);
    PlanConfig c = p->cfg;
    c.lds_bytes = (size_t)lds_bytes;
    c.wg_per_cu = wg_per_cu;
    c.use_graph = true;
    return ompd_plan_retile(p, c);
}

extern "C" int ompd_plan_split_kernels(ompd_plan* p, int32_t split)
{
    if (!p) return ompd_fail(OMPD_E_INVAL, "plan is NULL");
    std::lock_guard<std::mutex> lk(p->ctx->mu);
    PlanConfig c = p->cfg;
    c.split = split != 0;
    c.use_graph = true;
    return ompd_plan_retile(p, c);
}

extern "C" int ompd_plan_describe(ompd_plan* p, char* buf, int32_t len)
{
    if (!p || !buf || len <= 0) return ompd_fail(OMPD_E_INVAL, "bad arguments");
    long lanes = 0;
    for (size_t i = 0; i + p->dims.n_level < p->h_tiles.size(); ++i) lanes += p->h_tiles[i].nw;
    int level_cfgs = 0;
    for (const DevCfg& d : p->h_cfgs) level_cfgs += d.sched == SCHED_LEVEL;
    snprintf(buf, len,
             "{\"cfgs\": %d, \"tiles\": %d, \"words\": %ld, \"ring_slots\": %d, \"split\": %d, \"grid_tile\": %d, "
             "\"grid_phases\": [%d, %d, %d, %d, %d], "
             "\"lds_bytes\": %zu, \"wg_per_cu\": %d, \"graph\": %d, \"graph_captured\": %d, "
             "\"scratch_bytes\": %zu, \"bucket_sched\": [%d, %d, %d, %d, %d], \"level_cfgs\": %d, "
             "\"level_tiles\": %d, \"lds_level\": %zu}",
             p->n, p->n_tiles - p->dims.n_level, lanes, p->dims.ring_slots, (int)p->dims.split, p->dims.grid_tile,
             p->dims.grid[0], p->dims.grid[1], p->dims.grid[2],
             p->dims.grid[3], p->dims.grid[4], p->cfg.lds_bytes, p->cfg.wg_per_cu,
             p->cfg.use_graph ? 1 : 0, p->gx_solve ? 1 : 0, p->scratch_bytes, p->cfg.bucket_sched[0],
             p->cfg.bucket_sched[1], p->cfg.bucket_sched[2], p->cfg.bucket_sched[3], p->cfg.bucket_sched[4],
             level_cfgs, p->dims.n_level, p->dims.lds_level);
    return OMPD_OK;
}

extern "C" void ompd_plan_destroy(ompd_plan* p)
{
    if (!p) return;
    (void)hipSetDevice(p->ctx->device);
    if (p->last_stream || p->gx_prep) (void)hipDeviceSynchronize();
    drop_graphs(p);
    if (p->d_tiles) (void)hipFree(p->d_tiles);
    if (p->d_items) (void)hipFree(p->d_items);
    if (p->d_cfgs) (void)hipFree(p->d_cfgs);
    if (p->d_info) (void)hipFree(p->d_info);
    if (p->scratch) (void)hipFree(p->scratch);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    if (p->ev2) (void)hipEventDestroy(p->ev2);
    for (hipEvent_t e : p->evk)
        if (e) (void)hipEventDestroy(e);
    delete p;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
// Time the plan under configuration c: `trials` runs after one that warms up the graph.
static int time_config(ompd_plan* p, const PlanConfig& c, hipStream_t s, int trials, float& avg)
{
    int rc = ompd_plan_retile(p, c);
    if (rc) return rc;
    float tot = 0;
    for (int t = 0; t < trials + 1; ++t) {
        rc = ompd_plan_run_locked(p, s);
        if (rc) return rc;
        CK(hipEventSynchronize(p->ev2));
        float ms = 0;
        CK(hipEventElapsedTime(&ms, p->ev0, p->ev2));
        if (t > 0) tot += ms;
    }
    avg = tot / trials;
    return OMPD_OK;
}

extern "C" int ompd_plan_autotune(ompd_plan* p, void* stream, int32_t trials, float* best_ms)
{
    if (!p) return ompd_fail(OMPD_E_INVAL, "plan is NULL");
    std::lock_guard<std::mutex> lk(p->ctx->mu);
    hipStream_t s = (hipStream_t)stream;
    trials = std::max(1, trials);
    PlanConfig base = p->cfg;
    base.only_bucket = -1;
    // 1. the schedule of each size bucket, its CFGs timed alone under both schedules
    if (!(p->flags & (OMPD_F_SCHED_LEVEL | OMPD_F_SCHED_WALK))) {
        int count[OMPD_SCHED_BUCKETS] = {0}, small[OMPD_SCHED_BUCKETS] = {0};
        for (const DevCfg& d : p->h_cfgs) {
            const int b = ompd_sched_bucket(d.nb);
            ++count[b];
            small[b] += d.nb <= OMPD_LEVEL_MAX_BLOCKS;
        }
        for (int b = 0; b < OMPD_SCHED_BUCKETS; ++b) {
            if (!count[b]) continue;
            float best = 1e30f;
            int pick = SCHED_WALK;
            for (int sc : {(int)SCHED_WALK, (int)SCHED_LEVEL}) {
                if (sc == SCHED_LEVEL && small[b] == 0) continue;
                PlanConfig c = base;
                c.bucket_sched[b] = sc;
                c.only_bucket = b;
                float ms = 0;
                if (time_config(p, c, s, trials, ms) != OMPD_OK) continue;
                if (ms < best) { best = ms; pick = sc; }
            }
            base.bucket_sched[b] = pick;
        }
    }
    // the buckets were timed alone, where the lower latency wins; on the whole plan the throughput
    // may favour the default rule instead: keep whichever runs the plan faster
    if (!(p->flags & (OMPD_F_SCHED_LEVEL | OMPD_F_SCHED_WALK))) {
        PlanConfig rule = base;
        for (int b = 0; b < OMPD_SCHED_BUCKETS; ++b) rule.bucket_sched[b] = -1;
        float t_pick = 0, t_rule = 0;
        if (time_config(p, base, s, trials, t_pick) == OMPD_OK && time_config(p, rule, s, trials, t_rule) == OMPD_OK &&
            t_rule < t_pick)
            base = rule;
    }
    // 2. the launch configuration of the whole plan with those schedules
    PlanConfig best = base;
    float best_t = 1e30f;
    for (size_t lds : {(size_t)16 * STATE_BYTES, (size_t)32 * STATE_BYTES, (size_t)64 * STATE_BYTES}) {
        for (int wpc : {0, 4}) {
            PlanConfig c = base;
            c.lds_bytes = lds;
            c.wg_per_cu = wpc;
            float ms = 0;
            if (time_config(p, c, s, trials, ms) != OMPD_OK) continue;
            if (ms < best_t) { best_t = ms; best = c; }
        }
    }
    int rc = ompd_plan_retile(p, best);
    if (rc) return rc;
    if (best_t >= 1e30f) return ompd_fail(OMPD_E_DEVICE, "autotune: no configuration ran");
    if (best_ms) *best_ms = best_t;
    return OMPD_OK;
}

extern "C" int ompd_plan_set_schedule(ompd_plan* p, const int32_t* per_bucket)
{
    if (!p || !per_bucket) return ompd_fail(OMPD_E_INVAL, "bad arguments");
    for (int b = 0; b < OMPD_SCHED_BUCKETS; ++b)
        if (per_bucket[b] < -1 || per_bucket[b] > 1) return ompd_fail(OMPD_E_INVAL, "schedule must be -1, 0 or 1");
    std::lock_guard<std::mutex> lk(p->ctx->mu);
    PlanConfig c = p->cfg;
    for (int b = 0; b < OMPD_SCHED_BUCKETS; ++b) c.bucket_sched[b] = per_bucket[b];
    c.only_bucket = -1;
    c.use_graph = true;
    return ompd_plan_retile(p, c);
}

// ---------------------------------------------------------------------------
// host-pointer batch path (and the device-pointer one-shot path)
// ---------------------------------------------------------------------------
namespace {
struct Staged {
    std::vector<ompd_cfg> dcfg;
    std::vector<ompd_result> dres;
    void* dmem = nullptr;
    size_t bytes = 0;
    // output copies back: (device offset, host pointer, bytes)
    struct Back { size_t off; void* host; size_t bytes; };
    std::vector<Back> back;
    ~Staged() { if (dmem) (void)hipFree(dmem); }
};
}  // namespace

static int stage_inputs(const ompd_cfg* cfgs, ompd_result* res, int n, Staged& st, hipStream_t s)
{
    // layout: inputs then outputs, each 256-aligned
    std::vector<uint8_t> host;
    size_t total = 0;
    auto reserve = [&](size_t bytes) { size_t o = total; total += align256(bytes); return o; };
    struct In { size_t sp, si, kd, spc, R, W, evh, evd, lxh, lxd, call, sums, sc; };
    struct OutO { size_t nu_h, nu_d, ave_h, ave_d, avf_h, avf_d, ie_d, ie_h, ig_d, ig_h, vk, ad, bd, fpc; };
    std::vector<In> in(n);
    std::vector<OutO> oo(n);
    for (int i = 0; i < n; ++i) {
        const ompd_cfg& g = cfgs[i];
        const ompd_result& r = res[i];
        size_t wd = (size_t)(g.n_vars + 63) / 64;
        size_t bv = (size_t)g.n_blocks * wd * 8, ev = (size_t)g.n_edges * wd * 8;
        In& a = in[i];
        a.sp = reserve(4 * ((size_t)g.n_blocks + 1));
        a.si = reserve(4 * (size_t)g.n_edges);
        a.kd = reserve((size_t)g.n_edges);
        a.spc = reserve((size_t)g.n_blocks);
        a.R = reserve(bv);
        a.W = reserve(bv);
        a.evh = g.entry_valid_host ? reserve(wd * 8) : SIZE_MAX;
        a.evd = g.entry_valid_dev ? reserve(wd * 8) : SIZE_MAX;
        a.lxh = g.exit_live_host ? reserve(wd * 8) : SIZE_MAX;
        a.lxd = g.exit_live_dev ? reserve(wd * 8) : SIZE_MAX;
        a.call = g.call_summary ? reserve(4 * (size_t)g.n_blocks) : SIZE_MAX;
        a.sums = g.call_summary ? reserve((size_t)g.n_summaries * 16 * wd * 8) : SIZE_MAX;
        a.sc = g.scalar ? reserve(wd * 8) : SIZE_MAX;
        (void)r;
        (void)ev;
    }
    size_t in_bytes = total;
    for (int i = 0; i < n; ++i) {
        const ompd_cfg& g = cfgs[i];
        const ompd_result& r = res[i];
        size_t wd = (size_t)(g.n_vars + 63) / 64;
        size_t bv = (size_t)g.n_blocks * wd * 8, ev = (size_t)g.n_edges * wd * 8;
        OutO& o = oo[i];
        auto opt = [&](const void* ptr, size_t bytes) { return ptr ? reserve(bytes) : SIZE_MAX; };
        o.nu_h = opt(r.nu_host, bv); o.nu_d = opt(r.nu_dev, bv);
        o.ave_h = opt(r.ave_host, bv); o.ave_d = opt(r.ave_dev, bv);
        o.avf_h = (r.avf_host || r.avf_dev) ? reserve(bv) : SIZE_MAX;
        o.avf_d = (r.avf_host || r.avf_dev) ? reserve(bv) : SIZE_MAX;
        o.ie_d = opt(r.ins_entry_to_dev, bv); o.ie_h = opt(r.ins_entry_to_host, bv);
        o.ig_d = opt(r.ins_edge_to_dev, ev); o.ig_h = opt(r.ins_edge_to_host, ev);
        o.vk = opt(r.var_kind, (size_t)g.n_vars); o.ad = opt(r.after_dev, g.n_blocks); o.bd = opt(r.before_dev, g.n_blocks);
        o.fpc = opt(r.fp_clause, bv);
    }
    st.bytes = total;
    hipError_t e = hipMalloc(&st.dmem, std::max<size_t>(total, 256));
    if (e != hipSuccess) return ompd_fail(OMPD_E_NOMEM, std::string("device staging: ") + hipGetErrorString(e));
    host.assign(in_bytes, 0);
    char* D = (char*)st.dmem;
    st.dcfg.resize(n);
    st.dres.resize(n);
    for (int i = 0; i < n; ++i) {
        const ompd_cfg& g = cfgs[i];
        const ompd_result& r = res[i];
        size_t wd = (size_t)(g.n_vars + 63) / 64;
        size_t bv = (size_t)g.n_blocks * wd * 8, ev = (size_t)g.n_edges * wd * 8;
        const In& a = in[i];
        auto put = [&](size_t o, const void* src, size_t bytes) { if (bytes && src) memcpy(host.data() + o, src, bytes); };
        put(a.sp, g.succ_ptr, 4 * ((size_t)g.n_blocks + 1));
        put(a.si, g.succ_idx, 4 * (size_t)g.n_edges);
        put(a.kd, g.edge_kind, (size_t)g.n_edges);
        put(a.spc, g.space, (size_t)g.n_blocks);
        put(a.R, g.read_bits, bv);
        put(a.W, g.write_bits, bv);
        if (a.evh != SIZE_MAX) put(a.evh, g.entry_valid_host, wd * 8);
        if (a.evd != SIZE_MAX) put(a.evd, g.entry_valid_dev, wd * 8);
        if (a.lxh != SIZE_MAX) put(a.lxh, g.exit_live_host, wd * 8);
        if (a.lxd != SIZE_MAX) put(a.lxd, g.exit_live_dev, wd * 8);
        if (a.call != SIZE_MAX) put(a.call, g.call_summary, 4 * (size_t)g.n_blocks);
        if (a.sums != SIZE_MAX) put(a.sums, g.summaries, (size_t)g.n_summaries * 16 * wd * 8);
        if (a.sc != SIZE_MAX) put(a.sc, g.scalar, wd * 8);
        ompd_cfg d = g;
        d.succ_ptr = (const int32_t*)(D + a.sp);
        d.succ_idx = (const int32_t*)(D + a.si);
        d.edge_kind = (const uint8_t*)(D + a.kd);
        d.space = (const uint8_t*)(D + a.spc);
        d.read_bits = (const uint64_t*)(D + a.R);
        d.write_bits = (const uint64_t*)(D + a.W);
        d.entry_valid_host = a.evh != SIZE_MAX ? (const uint64_t*)(D + a.evh) : nullptr;
        d.entry_valid_dev = a.evd != SIZE_MAX ? (const uint64_t*)(D + a.evd) : nullptr;
        d.exit_live_host = a.lxh != SIZE_MAX ? (const uint64_t*)(D + a.lxh) : nullptr;
        d.exit_live_dev = a.lxd != SIZE_MAX ? (const uint64_t*)(D + a.lxd) : nullptr;
        d.call_summary = a.call != SIZE_MAX ? (const int32_t*)(D + a.call) : nullptr;
        d.summaries = a.sums != SIZE_MAX ? (const uint64_t*)(D + a.sums) : nullptr;
        d.scalar = a.sc != SIZE_MAX ? (const uint64_t*)(D + a.sc) : nullptr;
        st.dcfg[i] = d;
        const OutO& o = oo[i];
        ompd_result dr;
        memset(&dr, 0, sizeof dr);
        auto outp = [&](size_t off, void* hp, size_t bytes) -> void* {
            if (off == SIZE_MAX) return nullptr;
            if (hp) st.back.push_back({off, hp, bytes});
            return D + off;
        };
        dr.nu_host = (uint64_t*)outp(o.nu_h, r.nu_host, bv);
        dr.nu_dev = (uint64_t*)outp(o.nu_d, r.nu_dev, bv);
        dr.ave_host = (uint64_t*)outp(o.ave_h, r.ave_host, bv);
        dr.ave_dev = (uint64_t*)outp(o.ave_d, r.ave_dev, bv);
        dr.avf_host = (uint64_t*)outp(o.avf_h, r.avf_host, bv);
        dr.avf_dev = (uint64_t*)outp(o.avf_d, r.avf_dev, bv);
        dr.ins_entry_to_dev = (uint64_t*)outp(o.ie_d, r.ins_entry_to_dev, bv);
        dr.ins_entry_to_host = (uint64_t*)outp(o.ie_h, r.ins_entry_to_host, bv);
        dr.ins_edge_to_dev = (uint64_t*)outp(o.ig_d, r.ins_edge_to_dev, ev);
        dr.ins_edge_to_host = (uint64_t*)outp(o.ig_h, r.ins_edge_to_host, ev);
        dr.var_kind = (uint8_t*)outp(o.vk, r.var_kind, (size_t)g.n_vars);
        dr.after_dev = (uint8_t*)outp(o.ad, r.after_dev, (size_t)g.n_blocks);
        dr.before_dev = (uint8_t*)outp(o.bd, r.before_dev, (size_t)g.n_blocks);
        dr.fp_clause = (uint64_t*)outp(o.fpc, r.fp_clause, bv);
        st.dres[i] = dr;
    }
    if (in_bytes) CK(hipMemcpyAsync(st.dmem, host.data(), in_bytes, hipMemcpyHostToDevice, s));
    CK(hipStreamSynchronize(s));
    return OMPD_OK;
}

int ompd_batch_locked(ompd_ctx* ctx, const ompd_cfg* cfgs, ompd_result* res, int32_t n, uint32_t flags,
                      hipStream_t s)
{
    if (n < 0 || (n > 0 && (!cfgs || !res))) return ompd_fail(OMPD_E_INVAL, "bad arguments");
    CK(hipSetDevice(ctx->device));
    for (int i = 0; i < n; ++i) {
        int rc = check_cfg_host(cfgs[i], i);
        if (rc) return rc;
    }
    PlanConfig pc;
    pc.use_graph = false;
    if (flags & OMPD_F_DEVICE_PTRS) {
        ompd_plan* p = nullptr;
        int rc = ompd_plan_build(ctx, cfgs, res, n, flags, pc, &p);
        if (rc) return rc;
        rc = ompd_plan_run_locked(p, s);
        if (rc == OMPD_OK) rc = ompd_plan_collect(p, nullptr);
        for (int i = 0; i < n; ++i) memcpy(res[i].sweeps, p->res[i].sweeps, sizeof res[i].sweeps);
        ompd_plan_destroy(p);
        return rc;
    }
    Staged st;
    int rc = stage_inputs(cfgs, res, n, st, s);
    if (rc) return rc;
    ompd_plan* p = nullptr;
    rc = ompd_plan_build(ctx, st.dcfg.data(), st.dres.data(), n, flags | OMPD_F_DEVICE_PTRS, pc, &p);
    if (rc) return rc;
    rc = ompd_plan_run_locked(p, s);
    int rc2 = (rc == OMPD_OK) ? ompd_plan_collect(p, nullptr) : rc;
    if (rc == OMPD_OK) {
        for (int i = 0; i < n; ++i) memcpy(res[i].sweeps, p->res[i].sweeps, sizeof res[i].sweeps);
        // copy outputs back (also for invalid CFGs: their buffers hold unspecified values)
        std::vector<uint8_t> host(st.bytes);
        hipError_t e = hipMemcpy(host.data(), st.dmem, st.bytes, hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc2 = ompd_fail(OMPD_E_DEVICE, hipGetErrorString(e));
        else
            for (const auto& b : st.back) memcpy(b.host, host.data() + b.off, b.bytes);
    }
    ompd_plan_destroy(p);
    return rc2;
}

extern "C" int ompd_analyze_batch(ompd_ctx* ctx, const ompd_cfg* cfgs, ompd_result* res, int32_t n, uint32_t flags,
                                  void* stream)
{
    if (!ctx) return ompd_fail(OMPD_E_INVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    return ompd_batch_locked(ctx, cfgs, res, n, flags, (hipStream_t)stream);
}

extern "C" int ompd_analyze_batch_noalloc(ompd_ctx* ctx, const ompd_cfg* cfgs, ompd_result* res, int32_t n,
                                          uint32_t flags, void* stream)
{
    if (!ctx) return ompd_fail(OMPD_E_INVAL, "ctx is NULL");
    if (!(flags & OMPD_F_DEVICE_PTRS)) return ompd_fail(OMPD_E_INVAL, "noalloc: needs OMPD_F_DEVICE_PTRS");
    if (n < 0 || (n > 0 && (!cfgs || !res))) return ompd_fail(OMPD_E_INVAL, "bad arguments");
    std::lock_guard<std::mutex> lk(ctx->mu);
    std::lock_guard<std::mutex> sk(g_scratch_mu[ctx->device & 63]);
    if (!ctx->static_scratch) return ompd_fail(OMPD_E_DEVICE, "noalloc: no static scratch on this device");
    CK(hipSetDevice(ctx->device));
    for (int i = 0; i < n; ++i) {
        int rc = check_cfg_host(cfgs[i], i);
        if (rc) return rc;
    }
    if (n == 0) return OMPD_OK;
    hipStream_t s = (hipStream_t)stream;
    PlanConfig pc;
    pc.use_graph = false;
    if (flags & OMPD_F_TILE_KERNEL) pc.split = false;
    if (const uint32_t r = (flags >> 8) & 7u) pc.lds_bytes = (size_t)(4u << r) * STATE_BYTES;
    // layout of the static scratch: each CFG's solver scratch, the work counters, the default
    // boundaries, then the launch tables (descriptors, tiles, pass items) and the gathered
    // status words
    char* S = ctx->static_scratch;
    std::vector<ScratchOff> off(n);
    std::vector<size_t> base(n), boff(n);
    size_t total = 0, bnd_words = 0;
    for (int i = 0; i < n; ++i) {
        base[i] = total;
        total += ompd_cfg_scratch(cfgs[i], res[i], off[i]);
        boff[i] = bnd_words;
        bnd_words += 4 * (size_t)((cfgs[i].n_vars + 63) / 64);
    }
    const size_t counter_off = total;
    total += 256;
    const size_t bnd_off = total;
    total += align256(8 * bnd_words);
    std::vector<uint64_t> bnd(std::max<size_t>(bnd_words, 1), 0);
    std::vector<DevCfg> h(n);
    for (int i = 0; i < n; ++i)
        ompd_fill_devcfg(cfgs[i], res[i], S + base[i], off[i], flags, ctx->wait_ticks, h[i], bnd.data() + boff[i],
                         (uint64_t*)(S + bnd_off) + boff[i]);
    ompd_settle_sched(h.data(), n, ctx->n_cu);
    Shape sh;
    int rc = ompd_make_shape(ctx, h, pc, sh);
    if (rc) return rc;
    const size_t cfg_off = total;
    total += align256(sizeof(DevCfg) * n);
    const size_t tile_off = total;
    total += align256(sizeof(Tile) * std::max<size_t>(sh.tiles.size(), 1));
    const size_t item_off = total;
    total += align256(sizeof(EdgeItem) * std::max<size_t>(sh.items.size(), 1));
    const size_t info_off = total;
    total += align256(4 * INFO_WORDS * (size_t)n);
    if (total > OMPD_STATIC_SCRATCH_BYTES) {
        char buf[200];
        snprintf(buf, sizeof buf, "noalloc: the batch needs %zu bytes of scratch, the static scratch holds %zu",
                 total, OMPD_STATIC_SCRATCH_BYTES);
        return ompd_fail(OMPD_E_NOMEM, buf);
    }
    // nothing here needs zeroed memory: the ingest kernel clears the counters and status words
    if (bnd_words) CK(hipMemcpyAsync(S + bnd_off, bnd.data(), 8 * bnd_words, hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(S + cfg_off, h.data(), sizeof(DevCfg) * n, hipMemcpyHostToDevice, s));
    if (!sh.tiles.empty())
        CK(hipMemcpyAsync(S + tile_off, sh.tiles.data(), sizeof(Tile) * sh.tiles.size(), hipMemcpyHostToDevice, s));
    if (!sh.items.empty())
        CK(hipMemcpyAsync(S + item_off, sh.items.data(), sizeof(EdgeItem) * sh.items.size(), hipMemcpyHostToDevice,
                          s));
    const DevCfg* dc = (const DevCfg*)(S + cfg_off);
    int32_t* counter = (int32_t*)(S + counter_off);
    rc = ompd_launch_prep(dc, n, counter, sh.lds_prep, sh.dims.ring_slots, s);
    if (rc == OMPD_OK)
        rc = ompd_launch_solve(dc, (const Tile*)(S + tile_off), (int)sh.tiles.size(), (const EdgeItem*)(S + item_off),
                               (int)sh.items.size(), counter, sh.dims, s);
    std::vector<int32_t> info((size_t)n * INFO_WORDS, 0);
    if (rc == OMPD_OK) rc = gather_info(dc, n, (int32_t*)(S + info_off), info.data(), s);
    CK(hipStreamSynchronize(s));   // the host tables above stay alive until the copies are done
    if (rc) return rc;
    int first = OMPD_OK;
    for (int i = 0; i < n; ++i) {
        const int32_t* inf = &info[(size_t)i * INFO_WORDS];
        for (int k = 0; k < 6; ++k) res[i].sweeps[k] = inf[INFO_SWEEPS + k];
        if (inf[INFO_STATUS] && first == OMPD_OK) {
            first = inf[INFO_STATUS];
            g_err = ompd_status_message(i, inf);
        }
    }
    return first;
}

extern "C" int ompd_analyze_cfg(ompd_ctx* ctx, const ompd_cfg* cfg, ompd_result* res, uint32_t flags, void* stream)
{
    if (!ctx || !cfg || !res) return ompd_fail(OMPD_E_INVAL, "bad arguments");
    std::lock_guard<std::mutex> lk(ctx->mu);
    return ompd_batch_locked(ctx, cfg, res, 1, flags, (hipStream_t)stream);
}
