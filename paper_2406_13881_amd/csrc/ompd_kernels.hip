// HIP kernels (gfx950) for the OMPDart data-flow solve.
//
// ompd_k_prep  (one 256-thread workgroup per CFG): ingest and normalise —
//   validates the CSR and the boundary rules, builds the predecessor CSR
//   (with the successor-edge id of every predecessor link), assigns every
//   block a level = longest path from a level-0 block over forward edges
//   (u -> v with u < v), and bucket-sorts blocks by level.
//
// ompd_k_solve (persistent, one wavefront per tile): a tile is one CFG and a
//   range of bit-slices (8, 16 or 32 variables per slice).  The tile runs
//   every phase of the method on its variables:
//     next use (backward may), validity with eager copies (forward must),
//     pending copies (forward may), delayed placement (forward AND/OR) and
//     its materialisation, validity after placement (forward must), the
//     reachability facts behind the map/update labels, and the per-variable
//     map kind (Table II).
//   Each phase iterates Gauss-Seidel sweeps over the levels: within a level
//   the 64 lanes evaluate (block, slice) items in parallel, levels go in
//   order (reverse order for the backward phase), and the iterated vector
//   of the phase stays in LDS.  A sweep that changes nothing ends the phase
//   (wavefront vote); every phase is monotone on a finite lattice, so the
//   chaotic order reaches the unique fixed point and the result does not
//   depend on the schedule.
//
// All arithmetic is integer AND / OR / ANDN; variables never interact, so
// any slicing of the variable axis is exact.
#include <hip/hip_runtime.h>

#include "ompd_device.h"

#define OMPD_E_INVAL_ (-1)
#define OMPD_E_NOCONVERGE_ (-4)

namespace ompd {

// Views of generic pointers as global-memory pointers: loads and stores
// through them compile to global_load/global_store, which only count
// against vmcnt, so a wait for LDS does not also drain outstanding
// global prefetches (flat accesses would count against both).
#define GAS __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const GAS T* G(const T* p) { return (const GAS T*)p; }
template <typename T>
__device__ __forceinline__ GAS T* G(T* p) { return (GAS T*)p; }

__device__ __forceinline__ void set_status(int32_t* info, int32_t code)
{
    atomicCAS(&info[INFO_STATUS], 0, code);
}

// Inclusive prefix sum of a[0..n) in global memory by one workgroup.
__device__ void block_scan_inclusive(int32_t* a, int n, int32_t* sh)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int carry = 0;
    for (int base = 0; base < n; base += blockDim.x) {
        int i = base + threadIdx.x;
        int x = (i < n) ? a[i] : 0;
        for (int d = 1; d < 64; d <<= 1) {
            int y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        if (lane == 63) sh[wv] = x;
        __syncthreads();
        int off = carry, tot = 0;
        for (int j = 0; j < nw; ++j) {
            if (j < wv) off += sh[j];
            tot += sh[j];
        }
        __syncthreads();
        if (i < n) a[i] = x + off;
        carry += tot;
    }
    __syncthreads();
}

// --------------------------------------------------------------------------
// ingest / normalise
// --------------------------------------------------------------------------
extern "C" __global__ void __launch_bounds__(256)
ompd_k_prep(const DevCfg* __restrict__ cfgs, int n_cfgs, int32_t* __restrict__ solve_counter)
{
    extern __shared__ __align__(16) int32_t plds[];
    __shared__ int s_err;
    __shared__ int s_max;
    __shared__ int32_t s_scan[16];
    const int ci = blockIdx.x;
    if (ci == 0 && threadIdx.x == 0) *solve_counter = 0;
    if (ci >= n_cfgs) return;
    const DevCfg c = cfgs[ci];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nb = c.nb, ne = c.ne, wd = c.wd;
    if (tid == 0) { s_err = 0; s_max = 0; }
    for (int i = tid; i < INFO_WORDS; i += nt) c.info[i] = 0;
    __syncthreads();

    // validation, stage 1: pointers, kinds, spaces
    int err = 0;
    if (tid == 0 && (c.succ_ptr[0] != 0 || c.succ_ptr[nb] != ne)) err = 1;
    for (int b = tid; b < nb; b += nt) {
        int a = c.succ_ptr[b], z = c.succ_ptr[b + 1];
        if (z < a || a < 0 || z > ne) err = 1;
        if (c.space[b] > 1) err = 1;
    }
    for (int e = tid; e < ne; e += nt)
        if (c.kind[e] > 2) err = 1;
    if (tid == 0 && (c.space[c.entry] != 0 || c.space[c.exit] != 0)) err = 1;
    if (err) atomicOr(&s_err, 1);
    __syncthreads();
    if (s_err) { if (tid == 0) c.info[INFO_STATUS] = OMPD_E_INVAL_; return; }

    // stage 2: successor targets, ENTRY/EXIT rules, bit rows, boundaries, calls
    if (tid == 0 && c.succ_ptr[c.exit + 1] != c.succ_ptr[c.exit]) err = 1;
    for (int e = tid; e < ne; e += nt) {
        int q = c.succ_idx[e];
        if (q < 0 || q >= nb || q == c.entry) err = 1;
        else if (q == c.exit && c.kind[e] != 0) err = 1;
    }
    for (int e = c.succ_ptr[c.entry] + tid; e < c.succ_ptr[c.entry + 1]; e += nt)
        if (c.kind[e] == 1) err = 1;
    for (int b = tid; b < nb; b += nt)
        if (c.succ_ptr[b + 1] - c.succ_ptr[b] > (int)REC_COUNT) err = 1;
    if (wd > 0) {
        const uint64_t last = (c.nv & 63) ? ((1ull << (c.nv & 63)) - 1ull) : ~0ull;
        for (int w = tid; w < wd; w += nt) {
            uint64_t m = (w == wd - 1) ? last : ~0ull;
            if (c.R[(size_t)c.entry * wd + w] | c.W[(size_t)c.entry * wd + w] |
                c.R[(size_t)c.exit * wd + w] | c.W[(size_t)c.exit * wd + w]) err = 1;
            uint64_t eh = c.ev_h[w], ed = c.ev_d[w];
            if ((eh | ed | c.lx_h[w] | c.lx_d[w]) & ~m) err = 1;
            if (((eh | ed) & m) != m) err = 1;
        }
        for (int b = tid; b < nb; b += nt)
            if ((c.R[(size_t)b * wd + wd - 1] | c.W[(size_t)b * wd + wd - 1]) & ~last) err = 1;
    }
    if (c.call) {
        for (int b = tid; b < nb; b += nt) {
            int k = c.call[b];
            if (k >= 0 && (k >= c.n_sums || c.space[b] != 0 || b == c.entry || b == c.exit)) err = 1;
        }
    }
    if (err) atomicOr(&s_err, 1);
    __syncthreads();
    if (s_err) { if (tid == 0) c.info[INFO_STATUS] = OMPD_E_INVAL_; return; }

    // predecessor CSR
    int32_t* pp = c.pred_ptr;
    for (int b = tid; b <= nb; b += nt) pp[b] = 0;
    __syncthreads();
    for (int e = tid; e < ne; e += nt) atomicAdd(&pp[c.succ_idx[e] + 1], 1);
    __syncthreads();
    block_scan_inclusive(pp + 1, nb, s_scan);
    for (int b = tid; b < nb; b += nt) c.tmp[b] = pp[b];
    __syncthreads();
    for (int b = tid; b < nb; b += nt)
        for (int e = c.succ_ptr[b]; e < c.succ_ptr[b + 1]; ++e) {
            int q = c.succ_idx[e];
            int pos = atomicAdd(&c.tmp[q], 1);
            c.pred_idx[pos] = b;
            c.pred_eid[pos] = e;
        }
    __syncthreads();

    // levels: longest path over forward edges, chunk by chunk in id order;
    // inside a chunk, Jacobi rounds until no level changes
    int32_t* lvl = plds;
    for (int c0 = 0; c0 < nb; c0 += nt) {
        const int b = c0 + tid;
        const bool act = b < nb;
        int a = act ? pp[b] : 0, z = act ? pp[b + 1] : 0;
        int f0 = -1, f1 = -1, f2 = -1, f3 = -1, nf = 0, extra = 0;
        for (int j = a; j < z; ++j) {
            int p = c.pred_idx[j];
            if (p >= b) continue;
            if (nf == 0) f0 = p; else if (nf == 1) f1 = p; else if (nf == 2) f2 = p; else if (nf == 3) f3 = p; else extra = 1;
            ++nf;
        }
        if (act) lvl[b] = 0;
        __syncthreads();
        for (;;) {
            int L = 0;
            if (act) {
                if (f0 >= 0) L = max(L, lvl[f0] + 1);
                if (f1 >= 0) L = max(L, lvl[f1] + 1);
                if (f2 >= 0) L = max(L, lvl[f2] + 1);
                if (f3 >= 0) L = max(L, lvl[f3] + 1);
                if (extra)
                    for (int j = a; j < z; ++j) {
                        int p = c.pred_idx[j];
                        if (p < b) L = max(L, lvl[p] + 1);
                    }
            }
            int ch = act && (L != lvl[b]);
            __syncthreads();
            if (ch) lvl[b] = L;
            if (!__syncthreads_or(ch)) break;
        }
    }
    int mx = 0;
    for (int b = tid; b < nb; b += nt) mx = max(mx, lvl[b]);
    atomicMax(&s_max, mx);
    __syncthreads();
    const int nL = s_max + 1;
    int32_t* hist = c.tmp;   // free again after the predecessor scatter; nL <= nb
    for (int l = tid; l < nL; l += nt) hist[l] = 0;
    __syncthreads();
    for (int b = tid; b < nb; b += nt) atomicAdd(&hist[lvl[b]], 1);
    __syncthreads();
    for (int l = tid; l < nL; l += nt) c.level_ptr[l + 1] = hist[l];
    if (tid == 0) c.level_ptr[0] = 0;
    __syncthreads();
    block_scan_inclusive(c.level_ptr + 1, nL, s_scan);
    for (int l = tid; l < nL; l += nt) hist[l] = c.level_ptr[l];
    __syncthreads();
    for (int b = tid; b < nb; b += nt) {
        int pos = atomicAdd(&hist[lvl[b]], 1);
        c.level_blk[pos] = b;
    }
    __syncthreads();
    // level-ordered records: block, flags, first two predecessors / successors
    // with their edge ids (LOOP_ENTRY in bit 31), and the CSR start of the rest
    int4* RF = reinterpret_cast<int4*>(c.rec_f);
    int4* RB = reinterpret_cast<int4*>(c.rec_b);
    for (int pos = tid; pos < nb; pos += nt) {
        const int b = c.level_blk[pos];
        uint32_t fl = (b == c.entry ? REC_ENTRY : 0u) | (b == c.exit ? REC_EXIT : 0u) | (c.space[b] ? REC_DEV : 0u) |
                      ((c.call && c.call[b] >= 0) ? REC_CALL : 0u);
        int a = pp[b], cnt = pp[b + 1] - a;
        int e0 = cnt > 0 ? c.pred_eid[a] : 0, e1 = cnt > 1 ? c.pred_eid[a + 1] : 0;
        int4 r0, r1;
        r0.x = b;
        r0.y = (int)((uint32_t)cnt | fl);
        r0.z = cnt > 0 ? c.pred_idx[a] : 0;
        r0.w = cnt > 1 ? c.pred_idx[a + 1] : 0;
        r1.x = (int)((uint32_t)e0 | ((cnt > 0 && c.kind[e0] == 2) ? 0x80000000u : 0u));
        r1.y = (int)((uint32_t)e1 | ((cnt > 1 && c.kind[e1] == 2) ? 0x80000000u : 0u));
        r1.z = a;
        r1.w = lvl[b];
        RF[2 * pos] = r0;
        RF[2 * pos + 1] = r1;
        a = c.succ_ptr[b];
        cnt = c.succ_ptr[b + 1] - a;
        r0.y = (int)((uint32_t)cnt | fl);
        r0.z = cnt > 0 ? c.succ_idx[a] : 0;
        r0.w = cnt > 1 ? c.succ_idx[a + 1] : 0;
        r1.x = a;
        r1.y = a + 1;
        r1.z = a;
        r1.w = lvl[b];
        RB[2 * pos] = r0;
        RB[2 * pos + 1] = r1;
    }
    if (tid == 0) c.info[INFO_NLEVELS] = nL;
}

// --------------------------------------------------------------------------
// solve
// --------------------------------------------------------------------------
// Level-ordered record of one block (32 bytes): its first two neighbours
// (predecessors for forward phases, successors for the backward phase) with
// their edge ids inline, so one load per item replaces the chain
// level list -> CSR pointer -> CSR entry.
//   meta = neighbour count (24 bits) | ENTRY<<24 | EXIT<<25 | DEVICE<<26 | CALL<<27
//   e0/e1 = successor-CSR edge id | LOOP_ENTRY<<31
//   ovf = start of the full neighbour list in the CSR (for neighbours 2..)
//   lvl = the block's level
template <typename T>
struct Tv {
    const DevCfg& c;
    int s0, RW;
    __device__ __forceinline__ size_t row(int b, int k) const { return (size_t)b * RW + s0 + k; }
    __device__ __forceinline__ T ld(const uint64_t* p, int b, int k) const
    {
        return G(reinterpret_cast<const T*>(p))[row(b, k)];
    }
    __device__ __forceinline__ void st(uint64_t* p, int b, int k, T v) const
    {
        G(reinterpret_cast<T*>(p))[row(b, k)] = v;
    }
    __device__ __forceinline__ T vec(const uint64_t* p, int k) const
    {
        return G(reinterpret_cast<const T*>(p))[s0 + k];
    }
    __device__ __forceinline__ T sum(int ci, int r, int k) const
    {
        return G(reinterpret_cast<const T*>(c.sums))[((size_t)ci * SUM_ROWS + r) * RW + s0 + k];
    }
};

template <typename T>
__device__ __forceinline__ T ones() { return (T)~(T)0; }

// Per-item data fetched one step ahead of its use (everything a sweep needs
// that does not change while the phase iterates).
template <typename T>
struct Item {
    int b, k, lvl;
    uint32_t meta;
    int n0, n1;
    uint32_t e0, e1;
    int ovf;
    T vm;        // valid-variable mask of the item's slice
    T x[12];
};

template <typename T>
__device__ __forceinline__ bool solve_tile(const DevCfg& c, int s0, int ns, uint8_t* lds)
{
    constexpr int BITS = 8 * (int)sizeof(T);
    const int lane = threadIdx.x;
    const int nb = c.nb;
    const int RW = c.wd * (64 / BITS);
    const int nsi = ns > 0 ? ns : 1;
    const int lg = 31 - __clz(nsi);          // nsi is a power of two
    const bool data = ns > 0;
    T* SH = reinterpret_cast<T*>(lds);
    T* SD = SH + (size_t)nb * nsi;
    uint8_t* FL = lds + ((2 * (size_t)nb * nsi * sizeof(T) + 15) & ~(size_t)15);
    uint32_t* ACC = reinterpret_cast<uint32_t*>(FL + ((nb + 15) & ~15));
    const int nL = G(c.info)[INFO_NLEVELS];
    const GAS int32_t* __restrict__ lp = G(c.level_ptr);
    const GAS int32_t* __restrict__ RF = G(c.rec_f);
    const GAS int32_t* __restrict__ RB = G(c.rec_b);
    const GAS int32_t* __restrict__ sp = G(c.succ_ptr);
    const GAS int32_t* __restrict__ si = G(c.succ_idx);
    const GAS int32_t* __restrict__ pi = G(c.pred_idx);
    const GAS int32_t* __restrict__ pe = G(c.pred_eid);
    const GAS uint8_t* __restrict__ kind = G(c.kind);
    const GAS uint8_t* __restrict__ space = G(c.space);
    const GAS int32_t* __restrict__ callv = G(c.call);
    const Tv<T> tv{c, s0, RW};
    const int cap = c.sweep_cap > 0 ? c.sweep_cap : 2 * nb + 2;
    constexpr uint32_t M_ENTRY = REC_ENTRY, M_EXIT = REC_EXIT, M_DEV = REC_DEV, M_CALL = REC_CALL;

    auto vmask = [&](int k) -> T {
        long lo = (long)(s0 + k) * BITS;
        if (lo + BITS <= c.nv) return ones<T>();
        if (lo >= c.nv) return (T)0;
        return (T)((1u << (unsigned)(c.nv - lo)) - 1u);
    };
    auto sidx = [&](int b, int k) -> int { return (b << lg) + k; };
    // USE_s(b): a read in block b when b lies in space s; at EXIT the liveness after the region
    auto use = [&](int s, int b, int k) -> T {
        if (b == c.exit) return tv.vec(s ? c.lx_d : c.lx_h, k);
        T r = tv.ld(c.R, b, k);
        return ((int)space[b] == s) ? r : (T)0;
    };
    // USE'_s(b): a call whose callee may touch the variable stops pending copies like a read
    auto use_stop = [&](int s, int b, int k, bool call) -> T {
        T u = use(s, b, k);
        if (call) {
            int ci = callv[b];
            u |= tv.sum(ci, s ? SUM_MAYR_D : SUM_MAYR_H, k) | tv.sum(ci, SUM_MAYW_H, k) | tv.sum(ci, SUM_MAYW_D, k);
        }
        return u;
    };
    auto wr = [&](int s, int b, int k) -> T {
        if (b == c.exit) return (T)0;
        return ((int)space[b] == s) ? tv.ld(c.W, b, k) : (T)0;
    };
    // validity transfer: write here -> valid here; write in the other space -> stale here;
    // a call applies the callee's exit-validity table T_s[valid after own accesses][next use after the call]
    auto valid_out = [&](int s, int b, int k, T in, T w, bool dev, bool call, T vm) -> T {
        T a1 = (dev == (s == 1)) ? (T)(in | w) : (T)(in & ~w);
        if (call) {
            int ci = callv[b];
            const uint64_t* nus = s ? c.nu_d : c.nu_h;
            T l = 0;
            for (int e = sp[b]; e < sp[b + 1]; ++e) l |= tv.ld(nus, si[e], k);
            int base = s ? SUM_TD : SUM_TH;
            T t00 = tv.sum(ci, base + 0, k), t01 = tv.sum(ci, base + 1, k);
            T t10 = tv.sum(ci, base + 2, k), t11 = tv.sum(ci, base + 3, k);
            a1 = (T)((~a1 & ~l & t00) | (~a1 & l & t01) | (a1 & ~l & t10) | (a1 & l & t11));
        }
        return (T)(a1 & vm);
    };
    // i-th neighbour (pred or succ) of an item beyond the two inline ones
    auto nb_pred = [&](const Item<T>& it, int j, int& p, int& e) {
        if (j == 0) { p = it.n0; e = (int)it.e0; return; }
        if (j == 1) { p = it.n1; e = (int)it.e1; return; }
        p = pi[it.ovf + j];
        e = pe[it.ovf + j];
        e |= (kind[e] == 2) ? (int)0x80000000 : 0;
    };
    auto nb_succ = [&](const Item<T>& it, int j) -> int {
        if (j == 0) return it.n0;
        if (j == 1) return it.n1;
        return si[it.ovf + j];
    };

    // Pipelined sweep over the levels: the records and constants of the next
    // step are loaded while the current step computes from LDS.
    // The (position, slice) items of a sweep, in level order, are cut into
    // chunks of 64 consecutive items; a chunk usually spans several narrow
    // levels, which the wavefront evaluates one after another as masked
    // passes.  Chunks are loaded two ahead of their use, so one global round
    // trip serves several levels and overlaps with the work of two chunks.
    const int n_items = nb << lg;
    const int n_chunks = (n_items + 63) >> 6;
    auto sweep = [&](bool backward, auto&& fetch, auto&& compute) -> bool {
        const GAS int32_t* __restrict__ REC = backward ? RB : RF;
        auto load = [&](int ch) -> Item<T> {
            Item<T> it;
            it.k = -1;
            if (ch < 0 || ch >= n_chunks) return it;
            int i = (ch << 6) + lane;
            if (i < n_items) {
                const GAS int32_t* r = REC + 8 * (size_t)(i >> lg);
                it.b = r[0]; it.meta = (uint32_t)r[1]; it.n0 = r[2]; it.n1 = r[3];
                it.e0 = (uint32_t)r[4]; it.e1 = (uint32_t)r[5]; it.ovf = r[6]; it.lvl = r[7];
                it.k = i & (nsi - 1);
                it.vm = vmask(it.k);
                fetch(it);
            }
            return it;
        };
        const int step = backward ? -1 : 1;
        int ch = backward ? n_chunks - 1 : 0;
        bool changed = false;
        Item<T> cur = load(ch), nx1 = load(ch + step);
        for (int t = 0; t < n_chunks; ++t, ch += step) {
            Item<T> nx2 = load(ch + 2 * step);
            // levels present in this chunk (items are in level order)
            const int last = min(63, n_items - 1 - (ch << 6));
            const int lo = __shfl(cur.lvl, 0, 64), hi = __shfl(cur.lvl, last, 64);
            if (!backward) {
                for (int l = lo; l <= hi; ++l)
                    if (cur.k >= 0 && cur.lvl == l) changed |= compute(cur);
            } else {
                for (int l = hi; l >= lo; --l)
                    if (cur.k >= 0 && cur.lvl == l) changed |= compute(cur);
            }
            cur = nx1;
            nx1 = nx2;
        }
        return changed;
    };
    auto run_phase = [&](int phase, bool backward, auto&& fetch, auto&& compute) -> bool {
        int sweeps = 0;
        for (;;) {
            bool changed = sweep(backward, fetch, compute);
            ++sweeps;
            if (__ballot(changed) == 0ull) break;
            if (sweeps >= cap) {
                if (lane == 0) set_status(c.info, OMPD_E_NOCONVERGE_);
                return false;
            }
        }
        if (lane == 0) atomicMax(&c.info[INFO_SWEEPS + phase], sweeps);   // flat atomic: once per phase
        return true;
    };
    // Streaming pass over all items in level order (outputs), also pipelined.
    auto for_all = [&](auto&& fetch, auto&& f) {
        const int n = nb << lg;
        auto load = [&](int c0) -> Item<T> {
            Item<T> it;
            int i = c0 + lane;
            it.k = -1;
            if (i < n) {
                const GAS int32_t* r = RF + 8 * (size_t)(i >> lg);
                it.b = r[0]; it.meta = (uint32_t)r[1]; it.n0 = r[2]; it.n1 = r[3];
                it.e0 = (uint32_t)r[4]; it.e1 = (uint32_t)r[5]; it.ovf = r[6];
                it.k = i & (nsi - 1);
                it.vm = vmask(it.k);
                fetch(it);
            }
            return it;
        };
        Item<T> cur = load(0);
        for (int c0 = 0; c0 < n; c0 += 64) {
            Item<T> nxt;
            nxt.k = -1;
            if (c0 + 64 < n) nxt = load(c0 + 64);
            if (cur.k >= 0) f(cur);
            cur = nxt;
        }
    };
    auto no_fetch = [](Item<T>&) {};

    // ---------------------------------------------------------------- init
    for (int i = lane; i < (nb << lg); i += 64) { SH[i] = 0; SD[i] = 0; }
    for (int b = lane; b < nb; b += 64) {
        int dev = space[b] ? 1 : 0;
        FL[b] = (uint8_t)((b == c.exit ? 1 : 0) | (dev << 1) | (b == c.entry ? 4 : 0) | (dev << 3));
    }
    for (int i = lane; i < 3 * nsi; i += 64) ACC[i] = 0;
    __syncthreads();

    // ---------------------------------------------------------------- next use (backward, may)
    // NUin_s(b) = gen_s | (pass_s & OR over successors NUin_s(q)), with gen = USE_s and
    // pass = ~W for a plain block, gen = USE_s | (~W & NU0_s), pass = ~W & NU1_s for a call,
    // gen = the liveness after the region and pass = 0 at EXIT.
    // Flags bits 0/1: reaches EXIT / reaches a DEVICE block (before_dev).
    if (!run_phase(PH_NU, true,
            [&](Item<T>& it) {
                if (!data) return;
                const int b = it.b, k = it.k;
                if (it.meta & M_EXIT) {
                    it.x[0] = tv.vec(c.lx_h, k); it.x[1] = tv.vec(c.lx_d, k);
                    it.x[2] = 0; it.x[3] = 0;
                    return;
                }
                T r = tv.ld(c.R, b, k), w = tv.ld(c.W, b, k);
                T uH = (it.meta & M_DEV) ? (T)0 : r, uD = (it.meta & M_DEV) ? r : (T)0;
                if (it.meta & M_CALL) {
                    int ci = callv[b];
                    it.x[0] = uH | (~w & tv.sum(ci, SUM_NU0_H, k));
                    it.x[1] = uD | (~w & tv.sum(ci, SUM_NU0_D, k));
                    it.x[2] = ~w & tv.sum(ci, SUM_NU1_H, k);
                    it.x[3] = ~w & tv.sum(ci, SUM_NU1_D, k);
                } else {
                    it.x[0] = uH; it.x[1] = uD; it.x[2] = ~w; it.x[3] = ~w;
                }
            },
            [&](Item<T>& it) -> bool {
                const int b = it.b, k = it.k;
                const int cnt = (int)(it.meta & REC_COUNT);
                bool ch = false;
                if (data) {
                    T oH = 0, oD = 0;
                    for (int j = 0; j < cnt; ++j) {
                        int q = nb_succ(it, j);
                        oH |= SH[sidx(q, k)];
                        oD |= SD[sidx(q, k)];
                    }
                    T m = it.vm;
                    T vH = (it.x[0] | (it.x[2] & oH)) & m;
                    T vD = (it.x[1] | (it.x[3] & oD)) & m;
                    int li = sidx(b, k);
                    if (vH != SH[li]) { SH[li] = vH; ch = true; }
                    if (vD != SD[li]) { SD[li] = vD; ch = true; }
                }
                if (k == 0) {
                    uint8_t f = FL[b], g = 0;
                    for (int j = 0; j < cnt; ++j) g |= FL[nb_succ(it, j)];
                    uint8_t nf = (uint8_t)(f | (g & 3));
                    if (nf != f) { FL[b] = nf; ch = true; }
                }
                return ch;
            }))
        return false;
    if (data)
        for_all(no_fetch, [&](const Item<T>& it) {
            tv.st(c.nu_h, it.b, it.k, SH[sidx(it.b, it.k)]);
            tv.st(c.nu_d, it.b, it.k, SD[sidx(it.b, it.k)]);
        });
    __syncthreads();

    // ---------------------------------------------------------------- validity with eager copies
    // AVEin_s(q) = NUin_s(q) | AND over preds AVEout_s(p); AVEin(ENTRY) = boundary.
    // Flags bits 2/3: reached from ENTRY / reached from a DEVICE block (after_dev).
    auto fetch_gen_w = [&](Item<T>& it, const uint64_t* gh, const uint64_t* gd) {
        if (!data) return;
        if (it.meta & M_ENTRY) {
            it.x[0] = tv.vec(c.ev_h, it.k); it.x[1] = tv.vec(c.ev_d, it.k);
        } else {
            it.x[0] = tv.ld(gh, it.b, it.k); it.x[1] = tv.ld(gd, it.b, it.k);
        }
        it.x[2] = (it.meta & M_EXIT) ? (T)0 : tv.ld(c.W, it.b, it.k);
    };
    auto ave_in = [&](const Item<T>& it, T& iH, T& iD) {
        const int k = it.k;
        if (it.meta & M_ENTRY) {
            iH = it.x[0]; iD = it.x[1];
        } else {
            T mH = ones<T>(), mD = ones<T>();
            const int cnt = (int)(it.meta & REC_COUNT);
            for (int j = 0; j < cnt; ++j) {
                int p, e;
                nb_pred(it, j, p, e);
                mH &= SH[sidx(p, k)];
                mD &= SD[sidx(p, k)];
            }
            iH = it.x[0] | mH;
            iD = it.x[1] | mD;
        }
        T m = it.vm;
        iH &= m; iD &= m;
    };
    for (int i = lane; i < (nb << lg); i += 64) { SH[i] = ones<T>(); SD[i] = ones<T>(); }
    if (!run_phase(PH_AVE, false,
            [&](Item<T>& it) { fetch_gen_w(it, c.nu_h, c.nu_d); },
            [&](Item<T>& it) -> bool {
                const int q = it.b, k = it.k;
                bool ch = false;
                if (data) {
                    T iH, iD;
                    ave_in(it, iH, iD);
                    const bool dev = it.meta & M_DEV, call = it.meta & M_CALL;
                    T oH = valid_out(0, q, k, iH, it.x[2], dev, call, it.vm), oD = valid_out(1, q, k, iD, it.x[2], dev, call, it.vm);
                    int li = sidx(q, k);
                    if (oH != SH[li]) { SH[li] = oH; ch = true; }
                    if (oD != SD[li]) { SD[li] = oD; ch = true; }
                }
                if (k == 0) {
                    uint8_t f = FL[q], g = 0;
                    const int cnt = (int)(it.meta & REC_COUNT);
                    for (int j = 0; j < cnt; ++j) {
                        int p, e;
                        nb_pred(it, j, p, e);
                        g |= FL[p];
                    }
                    uint8_t nf = (uint8_t)(f | (g & 12));
                    if (nf != f) { FL[q] = nf; ch = true; }
                }
                return ch;
            }))
        return false;
    if (data)
        for_all([&](Item<T>& it) { fetch_gen_w(it, c.nu_h, c.nu_d); },
                [&](const Item<T>& it) {
                    T iH, iD;
                    ave_in(it, iH, iD);
                    tv.st(c.ave_h, it.b, it.k, iH);
                    tv.st(c.ave_d, it.b, it.k, iD);
                    tv.st(c.aveout_h, it.b, it.k, SH[sidx(it.b, it.k)]);
                    tv.st(c.aveout_d, it.b, it.k, SD[sidx(it.b, it.k)]);
                });
    {
        bool bad = false;
        for (int b = lane; b < nb; b += 64) {
            uint8_t f = FL[b];
            if ((f & 5) != 5) bad = true;
            if (s0 == 0) {
                if (c.after_dev) G(c.after_dev)[b] = (f >> 3) & 1;
                if (c.before_dev) G(c.before_dev)[b] = (f >> 1) & 1;
            }
        }
        if (__ballot(bad) != 0ull) {
            if (lane == 0) set_status(c.info, OMPD_E_INVAL_);
            return false;
        }
    }
    __syncthreads();

    // Constants of the two placement phases, per item: NU_s(q) in x0/x1, the stop
    // masks USE'_s(q) | WR_s(q) in x2/x3, AVEout_s of the two inline predecessors in
    // x4..x7 and (delay phase) their MAYPout_s in x8..x11.  EAG_s(e=p->q) = NU_s(q) & ~AVEout_s(p).
    auto fetch_place = [&](Item<T>& it, bool with_mayp) {
        const int b = it.b, k = it.k;
        const bool call = it.meta & M_CALL;
        it.x[0] = tv.ld(c.nu_h, b, k);
        it.x[1] = tv.ld(c.nu_d, b, k);
        it.x[2] = use_stop(0, b, k, call) | wr(0, b, k);
        it.x[3] = use_stop(1, b, k, call) | wr(1, b, k);
        const int cnt = (int)(it.meta & REC_COUNT);
        if (cnt > 0) {
            it.x[4] = tv.ld(c.aveout_h, it.n0, k); it.x[5] = tv.ld(c.aveout_d, it.n0, k);
            if (with_mayp) { it.x[8] = tv.ld(c.mayp_h, it.n0, k); it.x[9] = tv.ld(c.mayp_d, it.n0, k); }
        }
        if (cnt > 1) {
            it.x[6] = tv.ld(c.aveout_h, it.n1, k); it.x[7] = tv.ld(c.aveout_d, it.n1, k);
            if (with_mayp) { it.x[10] = tv.ld(c.mayp_h, it.n1, k); it.x[11] = tv.ld(c.mayp_d, it.n1, k); }
        }
    };
    // AVEout / MAYPout of predecessor j (inline for j < 2)
    auto pred_vals = [&](const Item<T>& it, int j, int p, T& aH, T& aD, T& mH, T& mD, bool with_mayp) {
        if (j == 0) {
            aH = it.x[4]; aD = it.x[5];
            if (with_mayp) { mH = it.x[8]; mD = it.x[9]; }
        } else if (j == 1) {
            aH = it.x[6]; aD = it.x[7];
            if (with_mayp) { mH = it.x[10]; mD = it.x[11]; }
        } else {
            aH = tv.ld(c.aveout_h, p, it.k); aD = tv.ld(c.aveout_d, p, it.k);
            if (with_mayp) { mH = tv.ld(c.mayp_h, p, it.k); mD = tv.ld(c.mayp_d, p, it.k); }
        }
    };

    if (c.placement == 0) {
        // ------------------------------------------------------------ pending copies (forward, may)
        // MAYP_s(e) = (EAG_s(e) | MAYPout_s(p)) & ~LE(e); MAYPout_s(q) = OR_e MAYP_s(e) & ~USE'_s(q) & ~WR_s(q)
        for (int i = lane; i < (nb << lg); i += 64) { SH[i] = 0; SD[i] = 0; }
        if (data) {
            if (!run_phase(PH_MAYP, false,
                    [&](Item<T>& it) { if (!(it.meta & M_ENTRY)) fetch_place(it, false); },
                    [&](Item<T>& it) -> bool {
                        if (it.meta & M_ENTRY) return false;
                        const int q = it.b, k = it.k;
                        T mH = 0, mD = 0;
                        const int cnt = (int)(it.meta & REC_COUNT);
                        for (int j = 0; j < cnt; ++j) {
                            int p, e;
                            nb_pred(it, j, p, e);
                            T nle = (e < 0) ? (T)0 : ones<T>();
                            T aH, aD, u0, u1;
                            pred_vals(it, j, p, aH, aD, u0, u1, false);
                            mH |= ((it.x[0] & ~aH) | SH[sidx(p, k)]) & nle;
                            mD |= ((it.x[1] & ~aD) | SD[sidx(p, k)]) & nle;
                        }
                        T m = it.vm;
                        T vH = mH & ~it.x[2] & m, vD = mD & ~it.x[3] & m;
                        bool ch = false;
                        int li = sidx(q, k);
                        if (vH != SH[li]) { SH[li] = vH; ch = true; }
                        if (vD != SD[li]) { SD[li] = vD; ch = true; }
                        return ch;
                    }))
                return false;
            for_all(no_fetch, [&](const Item<T>& it) {
                tv.st(c.mayp_h, it.b, it.k, SH[sidx(it.b, it.k)]);
                tv.st(c.mayp_d, it.b, it.k, SD[sidx(it.b, it.k)]);
            });
        }
        __syncthreads();

        // ------------------------------------------------------------ delayed placement (forward, LFP)
        // LATER_s(e) = EAG_s(e) | LATERout_s(p); L'_s(e) = LATER_s(e) & ~LE(e)
        // FV_x(e) = (AVEout_x(p) | EAG_x(e)) & ~MAYP_x(e)
        // N'_s(e) = (FV_s(e) & FV_o(e)) | (LATER_s(e) & LE(e))
        // LATERin_s(q) = AND_e (L'_s | N'_s) & OR_e L'_s; LATERout_s(q) = LATERin_s(q) & ~USE'_s(q) & ~WR_s(q)
        auto later_in = [&](const Item<T>& it, T& lH, T& lD) {
            const int k = it.k;
            T allH = ones<T>(), allD = ones<T>(), anyH = 0, anyD = 0;
            const int cnt = (int)(it.meta & REC_COUNT);
            for (int j = 0; j < cnt; ++j) {
                int p, e;
                nb_pred(it, j, p, e);
                T le = (e < 0) ? ones<T>() : (T)0;
                T aH, aD, mpH, mpD;
                pred_vals(it, j, p, aH, aD, mpH, mpD, true);
                T eH = it.x[0] & ~aH, eD = it.x[1] & ~aD;
                T fvH = (aH | eH) & ~((eH | mpH) & ~le);
                T fvD = (aD | eD) & ~((eD | mpD) & ~le);
                T latH = eH | SH[sidx(p, k)], latD = eD | SD[sidx(p, k)];
                T lpH = latH & ~le, lpD = latD & ~le;
                T both = fvH & fvD;
                allH &= lpH | both | (latH & le);
                allD &= lpD | both | (latD & le);
                anyH |= lpH;
                anyD |= lpD;
            }
            T m = it.vm;
            lH = allH & anyH & m;
            lD = allD & anyD & m;
        };
        for (int i = lane; i < (nb << lg); i += 64) { SH[i] = 0; SD[i] = 0; }
        if (data) {
            if (!run_phase(PH_LATER, false,
                    [&](Item<T>& it) { if (!(it.meta & M_ENTRY)) fetch_place(it, true); },
                    [&](Item<T>& it) -> bool {
                        if (it.meta & M_ENTRY) return false;
                        T lH, lD;
                        later_in(it, lH, lD);
                        T vH = lH & ~it.x[2], vD = lD & ~it.x[3];
                        bool ch = false;
                        int li = sidx(it.b, it.k);
                        if (vH != SH[li]) { SH[li] = vH; ch = true; }
                        if (vD != SD[li]) { SD[li] = vD; ch = true; }
                        return ch;
                    }))
                return false;
            // materialise: INS_ENTRY_s(q) = LATERin_s(q) & USE'_s(q);
            //              INS_EDGE_s(e=p->q) = LATER_s(e) & (LE(e) | ~LATERin_s(q))
            for_all([&](Item<T>& it) { fetch_place(it, true); },
                    [&](const Item<T>& it) {
                        const int q = it.b, k = it.k;
                        T lH = 0, lD = 0;
                        if (!(it.meta & M_ENTRY)) later_in(it, lH, lD);
                        const bool call = it.meta & M_CALL;
                        tv.st(c.ie_h, q, k, lH & use_stop(0, q, k, call));
                        tv.st(c.ie_d, q, k, lD & use_stop(1, q, k, call));
                        T m = it.vm;
                        const int cnt = (int)(it.meta & REC_COUNT);
                        for (int j = 0; j < cnt; ++j) {
                            int p, e;
                            nb_pred(it, j, p, e);
                            T le = (e < 0) ? ones<T>() : (T)0;
                            T aH, aD, u0, u1;
                            pred_vals(it, j, p, aH, aD, u0, u1, false);
                            T latH = (it.x[0] & ~aH) | SH[sidx(p, k)];
                            T latD = (it.x[1] & ~aD) | SD[sidx(p, k)];
                            int eid = e & 0x7FFFFFFF;
                            tv.st(c.ig_h, eid, k, latH & (le | ~lH) & m);
                            tv.st(c.ig_d, eid, k, latD & (le | ~lD) & m);
                        }
                    });
        }
    } else if (data) {
        // eager placement only: every EAG is materialised on its edge
        for_all([&](Item<T>& it) { fetch_place(it, false); },
                [&](const Item<T>& it) {
                    const int k = it.k;
                    tv.st(c.ie_h, it.b, k, (T)0);
                    tv.st(c.ie_d, it.b, k, (T)0);
                    T m = it.vm;
                    const int cnt = (int)(it.meta & REC_COUNT);
                    for (int j = 0; j < cnt; ++j) {
                        int p, e;
                        nb_pred(it, j, p, e);
                        T aH, aD, u0, u1;
                        pred_vals(it, j, p, aH, aD, u0, u1, false);
                        int eid = e & 0x7FFFFFFF;
                        tv.st(c.ig_h, eid, k, it.x[0] & ~aH & m);
                        tv.st(c.ig_d, eid, k, it.x[1] & ~aD & m);
                    }
                });
    }
    __syncthreads();

    // ---------------------------------------------------------------- validity after placement
    // AVFin_s(q) = INS_ENTRY_s(q) | AND_e (AVFout_s(p) | INS_EDGE_s(e))
    // x0/x1: INS_ENTRY (or the boundary at ENTRY), x2: W, x4..x7: INS_EDGE of the inline in-edges
    auto fetch_avf = [&](Item<T>& it) {
        fetch_gen_w(it, c.ie_h, c.ie_d);
        const int cnt = (int)(it.meta & REC_COUNT);
        if (cnt > 0) {
            int e = (int)(it.e0 & 0x7FFFFFFFu);
            it.x[4] = tv.ld(c.ig_h, e, it.k); it.x[5] = tv.ld(c.ig_d, e, it.k);
        }
        if (cnt > 1) {
            int e = (int)(it.e1 & 0x7FFFFFFFu);
            it.x[6] = tv.ld(c.ig_h, e, it.k); it.x[7] = tv.ld(c.ig_d, e, it.k);
        }
    };
    auto edge_ins = [&](const Item<T>& it, int j, int e, T& gH, T& gD) {
        if (j == 0) { gH = it.x[4]; gD = it.x[5]; }
        else if (j == 1) { gH = it.x[6]; gD = it.x[7]; }
        else {
            int eid = e & 0x7FFFFFFF;
            gH = tv.ld(c.ig_h, eid, it.k); gD = tv.ld(c.ig_d, eid, it.k);
        }
    };
    auto avf_in = [&](const Item<T>& it, T& iH, T& iD) {
        const int k = it.k;
        if (it.meta & M_ENTRY) {
            iH = it.x[0]; iD = it.x[1];
        } else {
            T mH = ones<T>(), mD = ones<T>();
            const int cnt = (int)(it.meta & REC_COUNT);
            for (int j = 0; j < cnt; ++j) {
                int p, e;
                nb_pred(it, j, p, e);
                T gH, gD;
                edge_ins(it, j, e, gH, gD);
                mH &= SH[sidx(p, k)] | gH;
                mD &= SD[sidx(p, k)] | gD;
            }
            iH = it.x[0] | mH;
            iD = it.x[1] | mD;
        }
        T m = it.vm;
        iH &= m; iD &= m;
    };
    if (data) {
        for (int i = lane; i < (nb << lg); i += 64) { SH[i] = ones<T>(); SD[i] = ones<T>(); }
        if (!run_phase(PH_AVF, false, fetch_avf,
                [&](Item<T>& it) -> bool {
                    T iH, iD;
                    avf_in(it, iH, iD);
                    const bool dev = it.meta & M_DEV, call = it.meta & M_CALL;
                    T oH = valid_out(0, it.b, it.k, iH, it.x[2], dev, call, it.vm);
                    T oD = valid_out(1, it.b, it.k, iD, it.x[2], dev, call, it.vm);
                    bool ch = false;
                    int li = sidx(it.b, it.k);
                    if (oH != SH[li]) { SH[li] = oH; ch = true; }
                    if (oD != SD[li]) { SD[li] = oD; ch = true; }
                    return ch;
                }))
            return false;
        // outputs, and the per-variable map kind (Table II):
        // map(to) copy into D: on p->q with !after_dev(p), before q with no after_dev predecessor;
        // map(from) copy into H: on p->q or before q with !before_dev(q).
        for_all(fetch_avf, [&](const Item<T>& it) {
            const int q = it.b, k = it.k;
            if (c.avf_h) {
                T iH, iD;
                avf_in(it, iH, iD);
                tv.st(c.avf_h, q, k, iH);
                tv.st(c.avf_d, q, k, iD);
            }
            if (c.var_kind) {
                T to = 0, from = 0, dev = 0;
                const bool before_q = (FL[q] >> 1) & 1;
                bool pred_after = false;
                const int cnt = (int)(it.meta & REC_COUNT);
                for (int j = 0; j < cnt; ++j) {
                    int p, e;
                    nb_pred(it, j, p, e);
                    T gH, gD;
                    edge_ins(it, j, e, gH, gD);
                    bool after_p = (FL[p] >> 3) & 1;
                    pred_after |= after_p;
                    if (!after_p) to |= gD;
                    if (!before_q) from |= gH;
                }
                if (!(it.meta & M_ENTRY)) {
                    if (!pred_after) to |= it.x[1];
                    if (!before_q) from |= it.x[0];
                }
                if ((it.meta & M_DEV) && !(it.meta & M_EXIT)) dev = tv.ld(c.R, q, k) | it.x[2];
                if (to) atomicOr(&ACC[k], (uint32_t)to);
                if (from) atomicOr(&ACC[nsi + k], (uint32_t)from);
                if (dev) atomicOr(&ACC[2 * nsi + k], (uint32_t)dev);
            }
        });
        __syncthreads();
        if (c.var_kind) {
            for (int v = lane; v < ns * BITS; v += 64) {
                long gv = (long)s0 * BITS + v;
                if (gv >= c.nv) continue;
                int k = v / BITS, bit = v % BITS;
                uint32_t to = (ACC[k] >> bit) & 1u, from = (ACC[nsi + k] >> bit) & 1u, dv = (ACC[2 * nsi + k] >> bit) & 1u;
                G(c.var_kind)[gv] = (uint8_t)(to | (from << 1) | ((dv && !to && !from) ? 4u : 0u));
            }
        }
    }
    return true;
}

extern "C" __global__ void __launch_bounds__(64)
ompd_k_solve(const DevCfg* __restrict__ cfgs, const Tile* __restrict__ tiles, int n_tiles, int32_t* __restrict__ counter)
{
    extern __shared__ __align__(16) uint8_t slds[];
    for (;;) {
        int t = 0;
        if (threadIdx.x == 0) t = atomicAdd(counter, 1);
        t = __builtin_amdgcn_readfirstlane(__shfl(t, 0, 64));
        if (t >= n_tiles) break;
        const Tile tl = tiles[t];
        const DevCfg c = cfgs[tl.cfg];
        if (G(c.info)[INFO_STATUS] != 0) continue;
        if (tl.tbits == 32) solve_tile<uint32_t>(c, tl.s0, tl.ns, slds);
        else if (tl.tbits == 16) solve_tile<uint16_t>(c, tl.s0, tl.ns, slds);
        else solve_tile<uint8_t>(c, tl.s0, tl.ns, slds);
        __syncthreads();
    }
}

}  // namespace ompd
