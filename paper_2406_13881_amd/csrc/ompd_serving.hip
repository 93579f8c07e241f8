// Serving loop of libompd: continuous batching of analysis requests.
//
// submit() admits a request when its device footprint (inputs, outputs and
// solver scratch) fits the context's device-memory budget and its inputs fit
// the pinned staging pool; otherwise it returns OMPD_E_BUSY.  A step's launch
// tables live in a fixed region of the stream it runs on, outside both pools,
// so a free stream can always launch a step, however full the pools are.  A launcher
// thread groups the admitted requests into steps — everything admitted since
// the last step — and launches each step (uploads, ingest kernel, persistent
// solve) on the next of several streams, so requests that arrive while
// others run are solved concurrently with them.  A completion thread copies
// results back, records completion times and frees the memory, which lets
// waiting requests in.  Each request's CFG stays resident on the device for
// all phases and sweeps of its solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <unordered_map>

#include "ompd_internal.h"
#include "ompd_pool.h"

using namespace ompd;

namespace {

using ompd_pool::a256;
using ompd_pool::Pool;

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Back {
    size_t dev_off;
    void* host;
    size_t bytes;
};

struct Req {
    ompd_ticket id = 0;
    uint32_t flags = 0;
    ompd_result* user = nullptr;
    size_t dev_off = 0, dev_bytes = 0, pin_off = 0, pin_bytes = 0;
    size_t in_bytes = 0, scratch_off = 0;
    ompd_cfg dcfg{};
    ompd_result dres{};
    ScratchOff so{};
    std::vector<Back> back;
    size_t tab_bytes = 0;   // what the request adds to a step's launch tables
    int status = 0;
    std::string msg;   // what went wrong, when status != 0
    int state = 0;   // 0 admitted, 1 running, 2 done
    int64_t t_submit = 0, t_done = 0;
};

struct Step {
    std::vector<Req*> reqs;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    size_t info_pin_off = 0;
    int launch_rc = 0;
};

}  // namespace

struct ServingState {
    ompd_ctx* ctx = nullptr;
    char* dev_base = nullptr;
    char* pin_base = nullptr;
    Pool dev, pin;
    // launch tables: one region per stream, device and pinned (outside the pools)
    static constexpr size_t TAB_REGION = 8u << 20;
    char* tab_dev = nullptr;
    char* tab_pin = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_busy;
    std::vector<hipEvent_t> events;
    hipStream_t d2h = nullptr;
    std::mutex mu;
    std::condition_variable cv_launch, cv_done, cv_complete;
    std::deque<Req*> pending;
    std::deque<Step*> inflight;
    std::unordered_map<ompd_ticket, Req*> reqs;
    ompd_ticket next_id = 1;
    bool stop = false;
    std::thread launcher, completer;
    int64_t admitted = 0, completed = 0;
    int max_steps = 4;
    int max_step_reqs = 256;
    // While another step runs, a new one waits until min_step_reqs requests are pending or the
    // oldest has waited max_wait_ns: fewer, larger steps keep the few hardware queues busy with
    // many tiles each instead of a request or two.
    int min_step_reqs = 32;
    int64_t max_wait_ns = 20 * 1000 * 1000;
    size_t max_reqs = 4096;
};

static void complete_step(ServingState* S, Step* st);

static void launcher_main(ServingState* S)
{
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        auto ready = [&] {
            if (S->stop) return true;
            if (S->pending.empty()) return false;
            int n_free = 0, n_busy = 0;
            for (int b : S->stream_busy) ++(b ? n_busy : n_free);
            if (n_free == 0) return false;
            if (n_busy == 0 || (int)S->pending.size() >= S->min_step_reqs) return true;
            return now_ns() - S->pending.front()->t_submit >= S->max_wait_ns;
        };
        while (!ready()) S->cv_launch.wait_for(lk, std::chrono::milliseconds(1));
        if (S->stop && S->pending.empty()) break;
        if (S->stop) break;
        int si = -1;
        for (int i = 0; i < (int)S->stream_busy.size(); ++i)
            if (!S->stream_busy[i]) { si = i; break; }
        if (si < 0) continue;
        // the pending requests, front first, as far as the stream's table region holds them
        std::deque<size_t> tb;
        for (size_t i = 0; i < S->pending.size() && (int)i < S->max_step_reqs; ++i) tb.push_back(S->pending[i]->tab_bytes);
        const int take = ompd_pool::take_step(tb, ServingState::TAB_REGION, S->max_step_reqs);
        Step* st = new Step();
        for (int i = 0; i < take; ++i) {
            st->reqs.push_back(S->pending.front());
            S->pending.pop_front();
        }
        const int k = (int)st->reqs.size();
        std::vector<DevCfg> h(k);
        for (int i = 0; i < k; ++i) {
            Req* r = st->reqs[i];
            ompd_fill_devcfg(r->dcfg, r->dres, S->dev_base + r->dev_off + r->scratch_off, r->so, r->flags,
                             S->ctx->wait_ticks, h[i], nullptr);
        }
        ompd_settle_sched(h.data(), k, S->ctx->n_cu);
        PlanConfig pc;
        Shape sh;
        int rc = ompd_make_shape(S->ctx, h, pc, sh);
        const std::vector<Tile>& tiles = sh.tiles;
        const ompd_pool::TableBytes tab = ompd_pool::table_bytes(k, tiles.size(), sh.items.size(), sizeof(DevCfg),
                                                                 sizeof(Tile), sizeof(EdgeItem), 4 * INFO_WORDS);
        const size_t cfg_bytes = tab.cfg, tile_bytes = tab.tiles + tab.items, item_bytes = tab.items;
        if (rc == OMPD_OK && (tab.device() > ServingState::TAB_REGION || tab.pinned() > ServingState::TAB_REGION))
            rc = ompd_fail(OMPD_E_NOMEM, "serving: step tables exceed their region");   // excluded at submit
        S->stream_busy[si] = 1;
        st->stream = S->streams[si];
        st->done = S->events[si];
        for (Req* r : st->reqs) r->state = 1;
        lk.unlock();
        if (rc == OMPD_OK) {
            char* pin = S->tab_pin + (size_t)si * ServingState::TAB_REGION;
            memcpy(pin, h.data(), sizeof(DevCfg) * k);
            if (!tiles.empty()) memcpy(pin + cfg_bytes, tiles.data(), sizeof(Tile) * tiles.size());
            if (!sh.items.empty())
                memcpy(pin + cfg_bytes + (tile_bytes - item_bytes), sh.items.data(), sizeof(EdgeItem) * sh.items.size());
            char* dtab = S->tab_dev + (size_t)si * ServingState::TAB_REGION;
            hipStream_t s = st->stream;
            hipError_t e = hipSuccess;
            for (Req* r : st->reqs)
                if (e == hipSuccess && r->in_bytes)
                    e = hipMemcpyAsync(S->dev_base + r->dev_off, S->pin_base + r->pin_off, r->in_bytes,
                                       hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(dtab, pin, cfg_bytes + tile_bytes, hipMemcpyHostToDevice, s);
            int32_t* counter = (int32_t*)(dtab + cfg_bytes + tile_bytes);
            if (e != hipSuccess) rc = OMPD_E_DEVICE;
            if (rc == OMPD_OK) rc = ompd_launch_prep((const DevCfg*)dtab, k, counter, sh.lds_prep, sh.dims.ring_slots, s);
            if (rc == OMPD_OK)
                rc = ompd_launch_solve((const DevCfg*)dtab, (const Tile*)(dtab + cfg_bytes), (int)tiles.size(),
                                       (const EdgeItem*)(dtab + cfg_bytes + (tile_bytes - item_bytes)),
                                       (int)sh.items.size(), counter, sh.dims, s);
            // per-request status words back to pinned memory
            st->info_pin_off = (size_t)si * ServingState::TAB_REGION + cfg_bytes + tile_bytes;
            for (int i = 0; i < k && rc == OMPD_OK; ++i)
                if (hipMemcpyAsync(S->tab_pin + st->info_pin_off + 4 * INFO_WORDS * (size_t)i, h[i].info,
                                   4 * INFO_WORDS, hipMemcpyDeviceToHost, s) != hipSuccess)
                    rc = OMPD_E_DEVICE;
            if (hipEventRecord(st->done, s) != hipSuccess && rc == OMPD_OK) rc = OMPD_E_DEVICE;
        }
        st->launch_rc = rc;
        lk.lock();
        S->inflight.push_back(st);
        S->cv_complete.notify_all();
    }
}

static void completer_main(ServingState* S)
{
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_complete.wait(lk, [&] { return S->stop || !S->inflight.empty(); });
        if (S->inflight.empty()) {
            if (S->stop) break;
            continue;
        }
        Step* st = S->inflight.front();
        S->inflight.pop_front();
        lk.unlock();
        if (st->launch_rc == OMPD_OK) (void)hipEventSynchronize(st->done);
        complete_step(S, st);
        lk.lock();
    }
}

static void complete_step(ServingState* S, Step* st)
{
    for (size_t i = 0; i < st->reqs.size(); ++i) {
        Req* r = st->reqs[i];
        int status = st->launch_rc;
        if (status == OMPD_OK) {
            const int32_t* info = (const int32_t*)(S->tab_pin + st->info_pin_off) + INFO_WORDS * i;
            status = info[INFO_STATUS];
            if (status) r->msg = "request " + std::to_string(r->id) + ", " + ompd_status_message(0, info);
            if (r->user)
                for (int k = 0; k < 6; ++k) r->user->sweeps[k] = info[INFO_SWEEPS + k];
            for (const Back& b : r->back)
                if (hipMemcpyAsync(b.host, S->dev_base + r->dev_off + b.dev_off, b.bytes, hipMemcpyDeviceToHost,
                                   S->d2h) != hipSuccess)
                    status = OMPD_E_DEVICE;
            if (hipStreamSynchronize(S->d2h) != hipSuccess) status = OMPD_E_DEVICE;
        }
        r->status = status;
    }
    std::lock_guard<std::mutex> g(S->mu);
    int64_t t = now_ns();
    for (Req* r : st->reqs) {
        S->dev.release(r->dev_off, r->dev_bytes);
        S->pin.release(r->pin_off, r->pin_bytes);
        r->state = 2;
        r->t_done = t;
        S->completed++;
    }
    for (size_t i = 0; i < S->streams.size(); ++i)
        if (S->streams[i] == st->stream) S->stream_busy[i] = 0;
    delete st;
    S->cv_launch.notify_all();
    S->cv_done.notify_all();
}

static int serving_init(ompd_ctx* ctx)
{
    std::lock_guard<std::mutex> g(ctx->srv_mu);
    if (ctx->srv) return OMPD_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return ompd_fail(OMPD_E_DEVICE, "hipSetDevice");
    ServingState* S = new ServingState();
    S->ctx = ctx;
    size_t dev_bytes = ctx->budget;
    size_t pin_bytes = std::min<size_t>(std::max<size_t>(ctx->budget / 8, 64ull << 20), 8ull << 30);
    if (hipMalloc((void**)&S->dev_base, dev_bytes) != hipSuccess) {
        delete S;
        return ompd_fail(OMPD_E_NOMEM, "serving: device pool allocation failed");
    }
    if (hipHostMalloc((void**)&S->pin_base, pin_bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(S->dev_base);
        delete S;
        return ompd_fail(OMPD_E_NOMEM, "serving: pinned pool allocation failed");
    }
    S->dev.init(dev_bytes);
    S->pin.init(pin_bytes);
    const size_t tab_total = (size_t)S->max_steps * ServingState::TAB_REGION;
    if (hipMalloc((void**)&S->tab_dev, tab_total) != hipSuccess) {
        (void)hipFree(S->dev_base);
        (void)hipHostFree(S->pin_base);
        delete S;
        return ompd_fail(OMPD_E_NOMEM, "serving: table region allocation failed");
    }
    if (hipHostMalloc((void**)&S->tab_pin, tab_total, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(S->tab_dev);
        (void)hipFree(S->dev_base);
        (void)hipHostFree(S->pin_base);
        delete S;
        return ompd_fail(OMPD_E_NOMEM, "serving: pinned table region allocation failed");
    }
    S->streams.resize(S->max_steps);
    S->events.resize(S->max_steps);
    S->stream_busy.assign(S->max_steps, 0);
    for (int i = 0; i < S->max_steps; ++i) {
        if (hipStreamCreateWithFlags(&S->streams[i], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&S->events[i], hipEventDisableTiming) != hipSuccess)
            return ompd_fail(OMPD_E_DEVICE, "serving: stream creation failed");
    }
    if (hipStreamCreateWithFlags(&S->d2h, hipStreamNonBlocking) != hipSuccess)
        return ompd_fail(OMPD_E_DEVICE, "serving: stream creation failed");
    S->launcher = std::thread(launcher_main, S);
    S->completer = std::thread(completer_main, S);
    ctx->srv = S;
    return OMPD_OK;
}

void ompd_serving_shutdown(ompd_ctx* ctx)
{
    ServingState* S = ctx->srv;
    if (!S) return;
    {
        // let admitted work finish, then stop both threads
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_done.wait(lk, [&] { return S->pending.empty() && S->inflight.empty() &&
                                         std::all_of(S->stream_busy.begin(), S->stream_busy.end(),
                                                     [](int b) { return b == 0; }); });
        S->stop = true;
    }
    S->cv_launch.notify_all();
    S->cv_complete.notify_all();
    S->launcher.join();
    S->completer.join();
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
    for (hipEvent_t e : S->events) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(S->d2h);
    (void)hipFree(S->dev_base);
    (void)hipHostFree(S->pin_base);
    (void)hipFree(S->tab_dev);
    (void)hipHostFree(S->tab_pin);
    for (auto& kv : S->reqs) delete kv.second;
    delete S;
    ctx->srv = nullptr;
}

extern "C" int ompd_submit(ompd_ctx* ctx, const ompd_cfg* cfg, ompd_result* res, uint32_t flags, ompd_ticket* out)
{
    if (!ctx || !cfg || !res || !out) return ompd_fail(OMPD_E_INVAL, "bad arguments");
    if (flags & OMPD_F_DEVICE_PTRS) return ompd_fail(OMPD_E_INVAL, "submit takes host pointers");
    const ompd_cfg& g = *cfg;
    if (g.n_blocks < 2 || g.n_edges < 0 || g.n_vars < 0 || g.entry < 0 || g.entry >= g.n_blocks || g.exit < 0 ||
        g.exit >= g.n_blocks || g.entry == g.exit || !g.succ_ptr || !g.space ||
        (g.n_edges > 0 && (!g.succ_idx || !g.edge_kind)) || (g.n_vars > 0 && (!g.read_bits || !g.write_bits)) ||
        (g.call_summary && (g.n_summaries <= 0 || !g.summaries)))
        return ompd_fail(OMPD_E_INVAL, "malformed request");
    int rc = serving_init(ctx);
    if (rc) return rc;
    ServingState* S = ctx->srv;
    Req* r = new Req();
    r->flags = flags;
    r->user = res;
    // device layout: inputs (boundaries always materialised), outputs, scratch
    const size_t nb = g.n_blocks, ne = g.n_edges, nv = g.n_vars, wd = (nv + 63) / 64;
    const size_t bv = nb * wd * 8, ev = ne * wd * 8;
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off += a256(b); return o; };
    size_t o_sp = take(4 * (nb + 1)), o_si = take(4 * ne), o_kd = take(ne), o_spc = take(nb);
    size_t o_R = take(bv), o_W = take(bv), o_bnd = take(4 * wd * 8);
    size_t o_call = g.call_summary ? take(4 * nb) : SIZE_MAX;
    size_t o_sums = g.call_summary ? take((size_t)g.n_summaries * 16 * wd * 8) : SIZE_MAX;
    size_t o_sc = g.scalar ? take(wd * 8) : SIZE_MAX;
    r->in_bytes = off;
    size_t o_out[14];
    const size_t out_sz[14] = {bv, bv, bv, bv, bv, bv, bv, bv, ev, ev, nv, nb, nb, bv};
    for (int i = 0; i < 14; ++i) o_out[i] = take(out_sz[i]);
    ompd_result full{};
    uint64_t** op[10] = {&full.nu_host, &full.nu_dev, &full.ave_host, &full.ave_dev, &full.avf_host, &full.avf_dev,
                         &full.ins_entry_to_host, &full.ins_entry_to_dev, &full.ins_edge_to_host, &full.ins_edge_to_dev};
    for (int i = 0; i < 10; ++i) *op[i] = (uint64_t*)1;   // non-NULL: only sizes the scratch here
    full.var_kind = (uint8_t*)1; full.after_dev = (uint8_t*)1; full.before_dev = (uint8_t*)1;
    full.fp_clause = (uint64_t*)1;
    r->scratch_off = off;
    off += ompd_cfg_scratch(g, full, r->so);
    r->dev_bytes = off;
    r->pin_bytes = r->in_bytes;
    {
        // its share of a step's launch tables: descriptor, tiles, pass items, status words
        const size_t tiles = (size_t)tiles_of((int)wd) + 2 * wd + 1;   // walk tiles, level tiles
        const size_t items = wd ? ((wd + PASS_WORDS - 1) / PASS_WORDS) * ((nb + 63) / 64) : 0;
        r->tab_bytes = ompd_pool::request_table_bytes(tiles, items, sizeof(DevCfg), sizeof(Tile), sizeof(EdgeItem),
                                                      4 * INFO_WORDS);
        if (r->tab_bytes + ompd_pool::TABLE_SLACK > ServingState::TAB_REGION) {
            delete r;
            return ompd_fail(OMPD_E_INVAL, "serving: request too large for a step's launch tables");
        }
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->reqs.size() >= S->max_reqs) { delete r; return ompd_fail(OMPD_E_BUSY, "serving: too many requests"); }
        if (!S->dev.alloc(r->dev_bytes, r->dev_off)) {
            delete r;
            return ompd_fail(OMPD_E_BUSY, "serving: device-memory budget full");
        }
        if (!S->pin.alloc(r->pin_bytes, r->pin_off)) {
            S->dev.release(r->dev_off, r->dev_bytes);
            delete r;
            return ompd_fail(OMPD_E_BUSY, "serving: staging pool full");
        }
        r->id = S->next_id++;
    }
    // stage the inputs (and default boundaries) in pinned memory
    char* P = S->pin_base + r->pin_off;
    auto put = [&](size_t o, const void* src, size_t n) { if (n && src) memcpy(P + o, src, n); };
    put(o_sp, g.succ_ptr, 4 * (nb + 1));
    put(o_si, g.succ_idx, 4 * ne);
    put(o_kd, g.edge_kind, ne);
    put(o_spc, g.space, nb);
    put(o_R, g.read_bits, bv);
    put(o_W, g.write_bits, bv);
    if (wd) {
        uint64_t* bnd = (uint64_t*)(P + o_bnd);
        uint64_t last = (nv & 63) ? ((1ull << (nv & 63)) - 1) : ~0ull;
        for (size_t w = 0; w < wd; ++w) {
            uint64_t m = (w == wd - 1) ? last : ~0ull;
            bnd[w] = g.entry_valid_host ? g.entry_valid_host[w] : m;
            bnd[wd + w] = g.entry_valid_dev ? g.entry_valid_dev[w] : 0;
            bnd[2 * wd + w] = g.exit_live_host ? g.exit_live_host[w] : m;
            bnd[3 * wd + w] = g.exit_live_dev ? g.exit_live_dev[w] : 0;
        }
    }
    if (o_call != SIZE_MAX) {
        put(o_call, g.call_summary, 4 * nb);
        put(o_sums, g.summaries, (size_t)g.n_summaries * 16 * wd * 8);
    }
    if (o_sc != SIZE_MAX) put(o_sc, g.scalar, wd * 8);
    char* D = S->dev_base + r->dev_off;
    ompd_cfg d = g;
    d.succ_ptr = (const int32_t*)(D + o_sp);
    d.succ_idx = (const int32_t*)(D + o_si);
    d.edge_kind = (const uint8_t*)(D + o_kd);
    d.space = (const uint8_t*)(D + o_spc);
    d.read_bits = (const uint64_t*)(D + o_R);
    d.write_bits = (const uint64_t*)(D + o_W);
    d.entry_valid_host = (const uint64_t*)(D + o_bnd);
    d.entry_valid_dev = d.entry_valid_host + wd;
    d.exit_live_host = d.entry_valid_host + 2 * wd;
    d.exit_live_dev = d.entry_valid_host + 3 * wd;
    d.call_summary = o_call != SIZE_MAX ? (const int32_t*)(D + o_call) : nullptr;
    d.summaries = o_sums != SIZE_MAX ? (const uint64_t*)(D + o_sums) : nullptr;
    d.scalar = o_sc != SIZE_MAX ? (const uint64_t*)(D + o_sc) : nullptr;
    r->dcfg = d;
    ompd_result& dr = r->dres;
    void* user_ptr[14] = {res->nu_host, res->nu_dev, res->ave_host, res->ave_dev, res->avf_host, res->avf_dev,
                          res->ins_entry_to_host, res->ins_entry_to_dev, res->ins_edge_to_host, res->ins_edge_to_dev,
                          res->var_kind, res->after_dev, res->before_dev, res->fp_clause};
    uint64_t** dp[10] = {&dr.nu_host, &dr.nu_dev, &dr.ave_host, &dr.ave_dev, &dr.avf_host, &dr.avf_dev,
                         &dr.ins_entry_to_host, &dr.ins_entry_to_dev, &dr.ins_edge_to_host, &dr.ins_edge_to_dev};
    for (int i = 0; i < 10; ++i) *dp[i] = (uint64_t*)(D + o_out[i]);
    dr.var_kind = (uint8_t*)(D + o_out[10]);
    dr.after_dev = (uint8_t*)(D + o_out[11]);
    dr.before_dev = (uint8_t*)(D + o_out[12]);
    dr.fp_clause = (uint64_t*)(D + o_out[13]);
    for (int i = 0; i < 14; ++i)
        if (user_ptr[i] && out_sz[i]) r->back.push_back(Back{o_out[i], user_ptr[i], out_sz[i]});
    r->t_submit = now_ns();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->reqs[r->id] = r;
        S->pending.push_back(r);
        S->admitted++;
    }
    S->cv_launch.notify_all();
    *out = r->id;
    return OMPD_OK;
}

static int poll_locked(ServingState* S, ompd_ticket t, int* done, int64_t* done_ns)
{
    auto it = S->reqs.find(t);
    if (it == S->reqs.end()) return ompd_fail(OMPD_E_UNKNOWN_TICKET, "unknown ticket");
    Req* r = it->second;
    if (r->state != 2) {
        *done = 0;
        return OMPD_OK;
    }
    *done = r->status ? r->status : 1;
    if (done_ns) *done_ns = r->t_done;
    if (r->status) (void)ompd_fail(r->status, r->msg.empty() ? "request failed" : r->msg);
    S->reqs.erase(it);
    delete r;
    return OMPD_OK;
}

extern "C" int ompd_poll(ompd_ctx* ctx, ompd_ticket t, int* done)
{
    return ompd_poll_ex(ctx, t, done, nullptr);
}

extern "C" int ompd_poll_ex(ompd_ctx* ctx, ompd_ticket t, int* done, int64_t* done_ns)
{
    if (!ctx || !done) return ompd_fail(OMPD_E_INVAL, "bad arguments");
    ServingState* S = ctx->srv;
    if (!S) return ompd_fail(OMPD_E_UNKNOWN_TICKET, "unknown ticket");
    std::lock_guard<std::mutex> lk(S->mu);
    return poll_locked(S, t, done, done_ns);
}

extern "C" int ompd_wait(ompd_ctx* ctx, ompd_ticket t, int64_t timeout_ns, int* done)
{
    if (!ctx || !done) return ompd_fail(OMPD_E_INVAL, "bad arguments");
    ServingState* S = ctx->srv;
    if (!S) return ompd_fail(OMPD_E_UNKNOWN_TICKET, "unknown ticket");
    std::unique_lock<std::mutex> lk(S->mu);
    auto ready = [&] {
        auto it = S->reqs.find(t);
        return it == S->reqs.end() || it->second->state == 2;
    };
    if (timeout_ns < 0) S->cv_done.wait(lk, ready);
    else if (!S->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), ready)) {
        *done = 0;
        return ompd_fail(OMPD_E_TIMEOUT, "wait timed out");
    }
    return poll_locked(S, t, done, nullptr);
}

extern "C" int ompd_serving_stats(ompd_ctx* ctx, int64_t* admitted, int64_t* completed, int64_t* in_flight,
                                  int64_t* bytes_in_use)
{
    if (!ctx) return ompd_fail(OMPD_E_INVAL, "bad arguments");
    ServingState* S = ctx->srv;
    if (!S) {
        if (admitted) *admitted = 0;
        if (completed) *completed = 0;
        if (in_flight) *in_flight = 0;
        if (bytes_in_use) *bytes_in_use = 0;
        return OMPD_OK;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (admitted) *admitted = S->admitted;
    if (completed) *completed = S->completed;
    if (in_flight) *in_flight = S->admitted - S->completed;
    if (bytes_in_use) *bytes_in_use = (int64_t)S->dev.used;
    return OMPD_OK;
}
