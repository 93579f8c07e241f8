// HIP kernels (gfx950) for the OMPDart data-flow solve.
//
// ompd_k_prep  (one 256-thread workgroup per CFG): ingest and normalise --
//   validates the CSR and the boundary rules, builds the predecessor CSR
//   (with the successor-edge id of every predecessor link) and writes one
//   32-byte record per block for each direction (flags, first two
//   neighbours with their edge ids, CSR start of the rest, call index).
//
// ompd_k_solve (persistent, one wavefront per tile): a tile is one CFG and a
//   run of up to 63 64-bit words of its variables.  The tile runs every
//   phase of the method on its variables:
//     next use (backward may), validity with eager copies (forward must),
//     pending copies (forward may), delayed placement (forward AND/OR) and
//     its materialisation, validity after placement (forward must), the
//     reachability facts behind the map/update labels, and the per-variable
//     map kind (Table II).
//
// All arithmetic is integer AND / OR / ANDN; variables never interact, so
// any split of the variable axis is exact.
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
    __shared__ int s_err;
    __shared__ int32_t s_scan[16];
    const int ci = blockIdx.x;
    if (ci == 0 && threadIdx.x < 8) solve_counter[threadIdx.x] = 0;   // one tile counter per phase
    if (ci >= n_cfgs) return;
    const DevCfg c = cfgs[ci];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nb = c.nb, ne = c.ne, wd = c.wd;
    if (tid == 0) s_err = 0;
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
            if (!(c.placement & 2) && ((eh | ed) & m) != m) err = 1;   // a summary evaluation may leave gaps
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

    // id-ordered records: flags, first two predecessors / successors with
    // their edge ids (LOOP_ENTRY in bit 31), the CSR start of the rest and
    // the call-summary index
    int4* RF = reinterpret_cast<int4*>(c.rec_f);
    int4* RB = reinterpret_cast<int4*>(c.rec_b);
    for (int b = tid; b < nb; b += nt) {
        uint32_t fl = (b == c.entry ? REC_ENTRY : 0u) | (b == c.exit ? REC_EXIT : 0u) | (c.space[b] ? REC_DEV : 0u) |
                      ((c.call && c.call[b] >= 0) ? REC_CALL : 0u);
        const int ci = c.call ? c.call[b] : -1;
        int a = pp[b], cnt = pp[b + 1] - a;
        int e0 = cnt > 0 ? c.pred_eid[a] : 0, e1 = cnt > 1 ? c.pred_eid[a + 1] : 0;
        int4 r0, r1;
        r0.x = (int)((uint32_t)cnt | fl);
        r0.y = cnt > 0 ? c.pred_idx[a] : 0;
        r0.z = cnt > 1 ? c.pred_idx[a + 1] : 0;
        r0.w = (int)((uint32_t)e0 | ((cnt > 0 && c.kind[e0] == 2) ? 0x80000000u : 0u));
        r1.x = (int)((uint32_t)e1 | ((cnt > 1 && c.kind[e1] == 2) ? 0x80000000u : 0u));
        r1.y = a;
        r1.z = ci;
        r1.w = 0;
        RF[2 * b] = r0;
        RF[2 * b + 1] = r1;
        a = c.succ_ptr[b];
        cnt = c.succ_ptr[b + 1] - a;
        r0.x = (int)((uint32_t)cnt | fl);
        r0.y = cnt > 0 ? c.succ_idx[a] : 0;
        r0.z = cnt > 1 ? c.succ_idx[a + 1] : 0;
        r0.w = a;
        r1.x = a + 1;
        r1.y = a;
        r1.z = ci;
        r1.w = 0;
        RB[2 * b] = r0;
        RB[2 * b + 1] = r1;
    }
}

// --------------------------------------------------------------------------
// solve
// --------------------------------------------------------------------------
// One wavefront solves one tile: a CFG and a run of up to 63 consecutive
// 64-bit words of its variable axis.  Lane l owns word s0 + l of every row;
// in the two phases that compute the CFG's reachability facts, lane nw (the
// flag lane) carries them as a pseudo-variable word whose inputs are
// synthesised so that the same equations compute them:
//   next use, host channel, bit 0 : the block reaches EXIT
//   next use, device channel, bit 1: a DEVICE block is reachable from here
//   eager validity, host channel, bit 0: the block is NOT reached from ENTRY
//   eager validity, host channel, bit 1: no DEVICE block reaches the block
// The CFG structure is the same for every lane, so the walk over blocks is
// scalar control flow (records and neighbour lists come through the scalar
// cache) and the lanes only do the bit arithmetic.
//
// A phase is a sequence of Gauss-Seidel sweeps in block-id order (reverse
// order for the backward phase).  The value of the block just computed stays
// in registers, the last RS blocks sit in an LDS ring (read one step ahead),
// and every other neighbour value comes from the phase's state rows in
// global memory, which also hold the previous sweep's values of blocks not
// yet visited.  The global inputs of block b+D are loaded right after block
// b is computed (D slots of registers), so a step does not wait for memory.
// Every phase is monotone on a finite lattice, so any visiting order reaches
// the same fixed point, and each block's value only moves one way between
// sweeps: a sweep changed nothing exactly when the popcount of the state
// is unchanged.  Outputs derived from a phase's state are written on every
// sweep; the last sweep writes the fixed point.
typedef uint64_t u64;
#define CAS __attribute__((address_space(4)))

struct Rec {
    uint32_t meta;      // neighbour count | ENTRY | EXIT | DEVICE | CALL
    int32_t n0, n1;     // first two neighbours
    uint32_t e0, e1;    // their edge ids | LOOP_ENTRY << 31 (predecessor records)
    int32_t ovf;        // CSR start of the neighbour list
    int32_t ci;         // call-summary index or -1
    int32_t pad;
};

template <typename T>
__device__ __forceinline__ const CAS T* K(const T* p) { return (const CAS T*)p; }

// Record b of a record array, through the scalar cache (b is wave-uniform).
__device__ __forceinline__ Rec ldrec(const int32_t* base, int b)
{
    const CAS int32_t* q = K(base) + 8 * (size_t)b;
    Rec r;
    r.meta = (uint32_t)q[0]; r.n0 = q[1]; r.n1 = q[2]; r.e0 = (uint32_t)q[3];
    r.e1 = (uint32_t)q[4]; r.ovf = q[5]; r.ci = q[6]; r.pad = q[7];
    return r;
}

__device__ __forceinline__ u64 tsel(u64 a1, u64 l, u64 t00, u64 t01, u64 t10, u64 t11)
{
    return (~a1 & ~l & t00) | (~a1 & l & t01) | (a1 & ~l & t10) | (a1 & l & t11);
}

__device__ __forceinline__ uint32_t popc2(u64 a, u64 b) { return (uint32_t)(__popcll(a) + __popcll(b)); }

// State rows of the iterated vector of one phase, per lane: data lanes
// address [nb][wd] rows at their word, the flag lane its own [nb] column.
struct Rows {
    GAS u64* h;
    GAS u64* d;
    int str;
    __device__ __forceinline__ u64 ldh(int b) const { return h[(size_t)b * str]; }
    __device__ __forceinline__ u64 ldd(int b) const { return d[(size_t)b * str]; }
    __device__ __forceinline__ void st(int b, u64 x, u64 y) const
    {
        h[(size_t)b * str] = x;
        d[(size_t)b * str] = y;
    }
};

// Per-block inputs loaded D steps ahead: phase inputs and the state of at
// most one far neighbour (more than RS blocks back, or not yet visited).
template <int NX>
struct Slot {
    u64 x[NX];
    u64 fh, fd;
};

template <int PH>
__device__ __forceinline__ void solve_phase(const DevCfg& c, int s0, int nw, int fslot, u64* ring, int ring_words)
{
    constexpr bool with_flags = PH == PH_NU || PH == PH_AVE;   // phases with the flag lane
    constexpr bool BWD = PH == PH_NU;
    constexpr int D = (PH == PH_NU || PH == PH_AVE) ? 8 : (PH == PH_MAYP ? 6 : 5);   // load-ahead depth
    constexpr int NX = PH == PH_NU ? 2 : PH == PH_AVE ? 3 : PH == PH_MAYP ? 6 : PH == PH_LATER ? 8 : 7;
    const int lane = threadIdx.x;
    const int nb = c.nb, wd = c.wd;
    // a tile without variables (nw = 0) has only flag lanes (they compute the same facts)
    const bool dat = lane < nw, flg = with_flags && (lane == nw || nw == 0), act = dat || flg;
    const int w = s0 + (dat ? lane : 0);
    // Every lane runs every step (no divergence around the walk, so records stay scalar loads
    // and waits stay precise): lanes past the tile shadow word s0 and store the same values.
    int RS = 1;
    while (RS < 64 && (size_t)4 * RS * 64 <= (size_t)ring_words) RS *= 2;   // slots of 2*64 words
    // valid-variable mask of the lane's word (shadow lanes share word s0's; the flag lane uses bits 0-1)
    const u64 vm = flg ? 3ull : ((w == wd - 1 && (c.nv & 63)) ? ((1ull << (c.nv & 63)) - 1ull) : ~0ull);
    const int cap = c.sweep_cap > 0 ? c.sweep_cap : 2 * nb + 2;
    const int32_t* REC = BWD ? c.rec_b : c.rec_f;
    const CAS int32_t* PI = K(c.pred_idx);
    const CAS int32_t* PE = K(c.pred_eid);
    const CAS int32_t* SI = K(c.succ_idx);
    const CAS uint8_t* KD = K(c.kind);
    GAS u64* FLG = G(c.flg) + (size_t)fslot * 4 * nb;   // flag lane: next use H, D, eager validity H, D
    const size_t wo = (size_t)w;
    // data arrays of a CFG without variables may be empty: loads then read a flag word instead
    auto arr = [&](const u64* a) -> const GAS u64* { return wd ? G(a) : (const GAS u64*)FLG; };
    auto row = [&](const u64* a, int b) -> u64 { return arr(a)[(size_t)b * wd + wo]; };
    auto vec = [&](const u64* a) -> u64 { return arr(a)[wo]; };
    auto sum = [&](int ci, int r) -> u64 { return arr(c.sums)[((size_t)ci * SUM_ROWS + r) * wd + wo]; };
    auto rows_of = [&](u64* h, u64* d, int fl) -> Rows {
        Rows r;
        if (flg) { r.h = FLG + (size_t)fl * nb; r.d = FLG + (size_t)(fl + 1) * nb; r.str = 1; }
        else { r.h = G(h) + wo; r.d = G(d) + wo; r.str = wd; }
        return r;
    };
    u64* rg = ring + lane;
    auto ring_h = [&](int b) -> u64& { return rg[(size_t)(b & (RS - 1)) * 128]; };
    auto ring_d = [&](int b) -> u64& { return rg[(size_t)(b & (RS - 1)) * 128 + 64]; };

    // neighbour j of a record (j >= 2 from the CSR); edge id with LOOP_ENTRY in bit 31
    auto nbr_f = [&](const Rec& r, int j, int& p, uint32_t& e) {
        if (j == 0) { p = r.n0; e = r.e0; return; }
        if (j == 1) { p = r.n1; e = r.e1; return; }
        p = PI[r.ovf + j];
        int ee = PE[r.ovf + j];
        e = (uint32_t)ee | (KD[ee] == 2 ? 0x80000000u : 0u);
    };
    auto nbr_b = [&](const Rec& r, int j) -> int {
        if (j == 0) return r.n0;
        if (j == 1) return r.n1;
        return SI[r.ovf + j];
    };
    auto nbr = [&](const Rec& r, int j) -> int {
        if constexpr (BWD) return nbr_b(r, j);
        else { int p; uint32_t e; nbr_f(r, j, p, e); return p; }
    };
    // distance of neighbour p from block b in walk order (1 = the block just before)
    auto dist = [&](int b, int p) -> int { return BWD ? (p - b) : (b - p); };
    // loaded with the slot (D steps ahead): not yet visited, or visited before both the ring
    // and the slot window; at compute time 1 = registers, 2..RS = ring (read a step ahead),
    // RS+1..D = read then
    const int FARD = RS > D ? RS : D;
    auto is_far = [&](int d) -> bool { return d <= 0 || d > FARD; };
    // neighbour state from memory: the previous sweep's row (or the initial value in sweep 0)
    // for a block not yet visited, this sweep's row for one visited more than RS steps ago
    auto far_val = [&](const Rows& S, int p, int d, int sweep, u64 init, u64& h, u64& dd) {
        if (d <= 0 && sweep == 0) { h = init; dd = init; }
        else { h = S.ldh(p); dd = S.ldd(p); }
    };

    // One sweep.  pre(b, r, x) loads the block's own inputs into x;
    // comp(b, r, x, nh, nd, ph, pd, sweep, vh, vd) computes the new state and writes outputs.
    auto walk = [&](const Rows& S, u64 init, int sweep, uint32_t& pc, auto&& pre, auto&& comp) {
        constexpr int dir = BWD ? -1 : 1;
        auto blk = [&](int i) -> int { return BWD ? nb - 1 - i : i; };
        Slot<NX> sl[D];
        auto load = [&](int b, Slot<NX>& s) {
            const Rec r = ldrec(REC, b);
            const int cnt = (int)(r.meta & REC_COUNT);
            // the first far neighbour (a fixed number of loads per slot: the block's own row otherwise)
            const int d0 = cnt > 0 ? dist(b, r.n0) : 1, d1 = cnt > 1 ? dist(b, r.n1) : 1;
            const bool f0 = cnt > 0 && is_far(d0), f1 = !f0 && cnt > 1 && is_far(d1);
            const int fp = f0 ? r.n0 : f1 ? r.n1 : b, fd = f0 ? d0 : f1 ? d1 : 1;
            const u64 lh = S.ldh(fp), ld = S.ldd(fp);
            const bool use_init = (f0 || f1) && fd <= 0 && sweep == 0;
            s.fh = use_init ? init : lh;
            s.fd = use_init ? init : ld;
            pre(b, r, s.x);
        };
        for (int k = 0; k < D && k < nb; ++k) load(blk(k), sl[k]);
        u64 ph = init, pd = init;                   // state of the block computed last
        u64 ch_[2] = {init, init}, cd_[2] = {init, init};   // ring values of the current block's neighbours
        for (int i0 = 0; i0 < nb; i0 += D) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const int i = i0 + k;
                if (i < nb) {
                    const int b = blk(i);
                    const Rec r = ldrec(REC, b);
                    const int cnt = (int)(r.meta & REC_COUNT);
                    // ring values of the next block's neighbours, read while this block computes
                    u64 nh_[2] = {0, 0}, nd_[2] = {0, 0};
                    if (i + 1 < nb) {
                        const Rec rn = ldrec(REC, b + dir);
                        const int cn = (int)(rn.meta & REC_COUNT);
                        for (int j = 0; j < 2 && j < cn; ++j) {
                            const int p = j == 0 ? rn.n0 : rn.n1, d = dist(b + dir, p);
                            if (d >= 2 && d <= RS) { nh_[j] = ring_h(p); nd_[j] = ring_d(p); }
                        }
                    }
                    u64 vh_[2], vd_[2];
                    bool far_used = false;
                    for (int j = 0; j < 2; ++j) {
                        vh_[j] = 0; vd_[j] = 0;
                        if (j >= cnt) continue;
                        const int p = j == 0 ? r.n0 : r.n1, d = dist(b, p);
                        if (d == 1) { vh_[j] = ph; vd_[j] = pd; }
                        else if (d >= 2 && d <= RS) { vh_[j] = ch_[j]; vd_[j] = cd_[j]; }
                        else if (is_far(d) && !far_used) { vh_[j] = sl[k].fh; vd_[j] = sl[k].fd; far_used = true; }
                        else far_val(S, p, d, sweep, init, vh_[j], vd_[j]);
                    }
                    u64 vh, vd;
                    comp(b, r, sl[k].x, vh_, vd_, ph, pd, sweep, vh, vd);
                    pc += popc2(vh, vd);
                    S.st(b, vh, vd);
                    if (RS >= 2) { ring_h(b) = vh; ring_d(b) = vd; }
                    ph = vh; pd = vd;
                    ch_[0] = nh_[0]; ch_[1] = nh_[1]; cd_[0] = nd_[0]; cd_[1] = nd_[1];
                    if (i + D < nb) load(blk(i + D), sl[k]);
                }
            }
        }
    };
    // a neighbour beyond the first two, at compute time
    auto extra = [&](const Rows& S, int b, int p, int sweep, u64 init, u64 ph, u64 pd, u64& h, u64& d) {
        const int dd = dist(b, p);
        if (dd == 1) { h = ph; d = pd; }
        else if (dd >= 2 && dd <= RS) { h = ring_h(p); d = ring_d(p); }
        else far_val(S, p, dd, sweep, init, h, d);
    };
    auto run_phase = [&](const Rows& S, u64 init, auto&& pre, auto&& comp) -> bool {
        int sweeps = 0;
        uint32_t last = (uint32_t)nb * 2u * (uint32_t)__popcll(init);
        for (;;) {
            uint32_t pc = 0;
            walk(S, init, sweeps, pc, pre, comp);
            ++sweeps;
            const bool ch = act && pc != last;
            last = pc;
            if (__ballot(ch) == 0ull) break;
            if (sweeps >= cap) {
                if (lane == 0) set_status(c.info, OMPD_E_NOCONVERGE_);
                return false;
            }
        }
        if (lane == 0) atomicMax(&c.info[INFO_SWEEPS + PH], sweeps);
        __threadfence_block();
        return true;
    };
    // NUout of a call block: OR over its successors' next use (final)
    auto nu_after = [&](int b, u64& lh, u64& ld) {
        const Rec rb = ldrec(c.rec_b, b);
        const int cnt = (int)(rb.meta & REC_COUNT);
        lh = 0; ld = 0;
        for (int j = 0; j < cnt; ++j) {
            int q = nbr_b(rb, j);
            lh |= row(c.nu_h, q);
            ld |= row(c.nu_d, q);
        }
    };
    // validity transfer of block b (a call applies the callee's exit-validity
    // tables to the validity after the block's own accesses and the next use after the call)
    auto valid_out = [&](int b, const Rec& r, u64 ih, u64 id, u64 wr, u64& oh, u64& od) {
        const bool dev = r.meta & REC_DEV;
        u64 ah = dev ? (ih & ~wr) : (ih | wr);
        u64 ad = dev ? (id | wr) : (id & ~wr);
        if (r.meta & REC_CALL) {
            u64 lh, ld;
            nu_after(b, lh, ld);
            const int ci = r.ci;   // the flag lane passes through (identity tables)
            const u64 th = tsel(ah, lh, sum(ci, SUM_TH + 0), sum(ci, SUM_TH + 1), sum(ci, SUM_TH + 2), sum(ci, SUM_TH + 3));
            const u64 td = tsel(ad, ld, sum(ci, SUM_TD + 0), sum(ci, SUM_TD + 1), sum(ci, SUM_TD + 2), sum(ci, SUM_TD + 3));
            ah = flg ? ah : th;
            ad = flg ? ad : td;
        }
        oh = ah & vm;
        od = ad & vm;
    };

    // ------------------------------------------------------------ next use (backward, may)
    // NUin_s(b) = USE_s(b) | (~W(b) & OR over successors NUin_s(q)); a call block
    // replaces the pass term by ~W & (NU0_s | (NU1_s & OR ...)); NUin(EXIT) = live after.
    if constexpr (PH == PH_NU) {
        const Rows S = rows_of(c.nu_h, c.nu_d, 0);
        // x0 = R, x1 = W (flag lane: R = 2, W = 2 at DEVICE blocks)
        auto pre = [&](int b, const Rec& r, u64* x) {
            const u64 rr = row(c.R, b), ww = row(c.W, b);
            x[0] = flg ? 2ull : rr;
            x[1] = flg ? ((r.meta & REC_DEV) ? 2ull : 0ull) : ww;
        };
        auto comp = [&](int b, const Rec& r, const u64* x, const u64* nh, const u64* nd, u64 ph, u64 pd, int sweep,
                        u64& vh, u64& vd) {
            if (r.meta & REC_EXIT) {
                const u64 lh = vec(c.lx_h), ld = vec(c.lx_d);
                vh = flg ? 1ull : lh;
                vd = flg ? 0ull : ld;
                return;
            }
            const int cnt = (int)(r.meta & REC_COUNT);
            u64 oh = nh[0] | nh[1], od = nd[0] | nd[1];
            for (int j = 2; j < cnt; ++j) {
                u64 h, d;
                extra(S, b, nbr_b(r, j), sweep, 0ull, ph, pd, h, d);
                oh |= h; od |= d;
            }
            const bool dev = r.meta & REC_DEV;
            const u64 rr = x[0], ww = x[1];
            if (r.meta & REC_CALL) {
                const int ci = r.ci;   // the flag lane passes through (NU0 = 0, NU1 = all ones)
                const u64 ch = sum(ci, SUM_NU0_H) | (sum(ci, SUM_NU1_H) & oh);
                const u64 cd = sum(ci, SUM_NU0_D) | (sum(ci, SUM_NU1_D) & od);
                oh = flg ? oh : ch;
                od = flg ? od : cd;
            }
            vh = (dev ? 0ull : rr) | (~ww & oh);
            vd = (dev ? rr : 0ull) | (~ww & od);
        };
        run_phase(S, 0ull, pre, comp);
        return;
    }

    // ------------------------------------------------------------ validity with eager copies (forward, must)
    // AVEin_s(q) = NUin_s(q) | AND over preds AVEout_s(p); AVEin(ENTRY) = boundary.
    if constexpr (PH == PH_AVE) {
        const Rows S = rows_of(c.aveout_h, c.aveout_d, 2);
        const u64 init = ~0ull & vm;
        // x0/x1 = NU (flag lane: 0), x2 = W (flag lane: 2 at DEVICE blocks)
        auto pre = [&](int b, const Rec& r, u64* x) {
            const u64 nh = row(c.nu_h, b), nd = row(c.nu_d, b), ww = row(c.W, b);
            x[0] = flg ? 0ull : nh;
            x[1] = flg ? 0ull : nd;
            x[2] = flg ? ((r.meta & REC_DEV) ? 2ull : 0ull) : ww;
        };
        auto comp = [&](int b, const Rec& r, const u64* x, const u64* nh, const u64* nd, u64 ph, u64 pd, int sweep,
                        u64& vh, u64& vd) {
            u64 ih, id;
            if (r.meta & REC_ENTRY) {
                const u64 eh = vec(c.ev_h), ed = vec(c.ev_d);
                ih = flg ? 2ull : eh;
                id = flg ? 0ull : ed;
            } else {
                const int cnt = (int)(r.meta & REC_COUNT);
                // meet over the predecessors (all ones over none: a block no edge enters)
                u64 mh = cnt == 0 ? ~0ull : cnt > 1 ? (nh[0] & nh[1]) : nh[0];
                u64 md = cnt == 0 ? ~0ull : cnt > 1 ? (nd[0] & nd[1]) : nd[0];
                for (int j = 2; j < cnt; ++j) {
                    int p; uint32_t e;
                    nbr_f(r, j, p, e);
                    u64 h, d;
                    extra(S, b, p, sweep, init, ph, pd, h, d);
                    mh &= h; md &= d;
                }
                ih = x[0] | mh;
                id = x[1] | md;
            }
            ih &= vm; id &= vm;
            if (dat) { G(c.ave_h)[(size_t)b * wd + wo] = ih; G(c.ave_d)[(size_t)b * wd + wo] = id; }
            valid_out(b, r, ih, id, x[2], vh, vd);
        };
        if (!run_phase(S, init, pre, comp)) return;
        // reachability: every block reached from ENTRY and reaching EXIT
        bool bad = false;
        for (int b = lane; b < nb; b += 64) {
            u64 fnu = FLG[b], fave = FLG[(size_t)2 * nb + b], fnud = FLG[(size_t)nb + b];
            if (!(fnu & 1) || (fave & 1)) bad = true;
            if (s0 == 0) {
                if (c.after_dev) G(c.after_dev)[b] = (uint8_t)(((fave >> 1) & 1) ^ 1);
                if (c.before_dev) G(c.before_dev)[b] = (uint8_t)((fnud >> 1) & 1);
            }
        }
        if (__ballot(bad) != 0ull && lane == 0) set_status(c.info, OMPD_E_INVAL_);
        return;
    }
    if (nw == 0) return;   // no variables: only the reachability facts

    // USE'_s(b) (a call whose callee may touch the variable stops pending copies like a read)
    // and the stop masks USE'_s | WR_s of a block, from R, W (and the live-after vectors at EXIT)
    auto use_wr = [&](int b, const Rec& r, u64 rr, u64 ww, u64& uh, u64& ud, u64& sh, u64& sd) {
        const bool dev = r.meta & REC_DEV;
        if (r.meta & REC_EXIT) { uh = vec(c.lx_h); ud = vec(c.lx_d); sh = uh; sd = ud; return; }
        uh = dev ? 0ull : rr;
        ud = dev ? rr : 0ull;
        if (r.meta & REC_CALL) {
            const int ci = r.ci;
            u64 mw = sum(ci, SUM_MAYW_H) | sum(ci, SUM_MAYW_D);
            uh |= sum(ci, SUM_MAYR_H) | mw;
            ud |= sum(ci, SUM_MAYR_D) | mw;
        }
        sh = uh | (dev ? 0ull : ww);
        sd = ud | (dev ? ww : 0ull);
    };
    auto erow = [&](const u64* a, uint32_t e) -> u64 { return G(a)[(size_t)(e & 0x7FFFFFFFu) * wd + wo]; };

    // -------------------------------------------------------- pending copies (forward, may)
    // MAYP_s(e) = (EAG_s(e) | MAYPout_s(p)) & ~LE(e), EAG_s(e=p->q) = NU_s(q) & ~AVEout_s(p);
    // MAYPout_s(q) = OR_e MAYP_s(e) & ~USE'_s(q) & ~WR_s(q)
    if constexpr (PH == PH_MAYP) {
        if (c.placement & 1) return;
        const Rows S = rows_of(c.mayp_h, c.mayp_d, 0);
        // x0 = R, x1 = W, x2..x5 = EAG_H/D of the two inline in-edges
        auto pre = [&](int b, const Rec& r, u64* x) {
            x[0] = row(c.R, b); x[1] = row(c.W, b);
            const int cnt = (int)(r.meta & REC_COUNT);
            const uint32_t e0 = cnt > 0 ? r.e0 : 0u, e1 = cnt > 1 ? r.e1 : 0u;   // edge 0 stands in for a missing one
            x[2] = erow(c.eag_h, e0); x[3] = erow(c.eag_d, e0);
            x[4] = erow(c.eag_h, e1); x[5] = erow(c.eag_d, e1);
        };
        auto comp = [&](int b, const Rec& r, const u64* x, const u64* nh, const u64* nd, u64 ph, u64 pd, int sweep,
                        u64& vh, u64& vd) {
            if (r.meta & REC_ENTRY) { vh = 0; vd = 0; return; }
            const int cnt = (int)(r.meta & REC_COUNT);
            u64 mh = 0, md = 0;
            for (int j = 0; j < cnt; ++j) {
                int p; uint32_t e;
                nbr_f(r, j, p, e);
                if (e & 0x80000000u) continue;   // loop entry: nothing stays pending
                u64 gh, gd, sh, sd;
                if (j < 2) { gh = x[2 + 2 * j]; gd = x[3 + 2 * j]; sh = nh[j]; sd = nd[j]; }
                else {
                    gh = erow(c.eag_h, e); gd = erow(c.eag_d, e);
                    extra(S, b, p, sweep, 0ull, ph, pd, sh, sd);
                }
                mh |= gh | sh;
                md |= gd | sd;
            }
            u64 uh, ud, sth, std_;
            use_wr(b, r, x[0], x[1], uh, ud, sth, std_);
            vh = mh & ~sth & vm;
            vd = md & ~std_ & vm;
        };
        run_phase(S, 0ull, pre, comp);
        return;
    }

    // -------------------------------------------------------- delayed placement (forward, LFP)
    // LATER_s(e) = EAG_s(e) | LATERout_s(p); L'_s(e) = LATER_s(e) & ~LE(e)
    // N'_s(e) = BOTH(e) | (LATER_s(e) & LE(e)), BOTH(e) = FV_H(e) & FV_D(e)
    // LATERin_s(q) = AND_e (L'_s | N'_s) & OR_e L'_s; LATERout_s(q) = LATERin_s(q) & ~USE'_s(q) & ~WR_s(q)
    // materialised on every sweep: INS_ENTRY_s(q) = LATERin_s(q) & USE'_s(q),
    //   INS_EDGE_s(e=p->q) = LATER_s(e) & (LE(e) | ~LATERin_s(q))
    if constexpr (PH == PH_LATER) {
        if (!(c.placement & 1)) {
            const Rows S = rows_of(c.later_h, c.later_d, 0);
            // x0 = R, x1 = W, x2..x4 / x5..x7 = EAG_H, EAG_D, BOTH of the two inline in-edges
            auto pre = [&](int b, const Rec& r, u64* x) {
                x[0] = row(c.R, b); x[1] = row(c.W, b);
                const int cnt = (int)(r.meta & REC_COUNT);
                const uint32_t e0 = cnt > 0 ? r.e0 : 0u, e1 = cnt > 1 ? r.e1 : 0u;
                x[2] = erow(c.eag_h, e0); x[3] = erow(c.eag_d, e0); x[4] = erow(c.both, e0);
                x[5] = erow(c.eag_h, e1); x[6] = erow(c.eag_d, e1); x[7] = erow(c.both, e1);
            };
            auto comp = [&](int b, const Rec& r, const u64* x, const u64* nh, const u64* nd, u64 ph, u64 pd,
                            int sweep, u64& vh, u64& vd) {
                u64 uh, ud, sth, std_;
                use_wr(b, r, x[0], x[1], uh, ud, sth, std_);
                if (r.meta & REC_ENTRY) {
                    vh = 0; vd = 0;
                    G(c.ie_h)[(size_t)b * wd + wo] = 0;
                    G(c.ie_d)[(size_t)b * wd + wo] = 0;
                    return;
                }
                const int cnt = (int)(r.meta & REC_COUNT);
                u64 allh = ~0ull, alld = ~0ull, anyh = 0, anyd = 0;
                u64 lat_h[2] = {0, 0}, lat_d[2] = {0, 0};
                auto edge = [&](int j, int p, uint32_t e, u64& gh, u64& gd, u64& bo, u64& sh, u64& sd) {
                    if (j < 2) { gh = x[2 + 3 * j]; gd = x[3 + 3 * j]; bo = x[4 + 3 * j]; sh = nh[j]; sd = nd[j]; }
                    else {
                        gh = erow(c.eag_h, e); gd = erow(c.eag_d, e); bo = erow(c.both, e);
                        extra(S, b, p, sweep, 0ull, ph, pd, sh, sd);
                    }
                };
                for (int j = 0; j < cnt; ++j) {
                    int p; uint32_t e;
                    nbr_f(r, j, p, e);
                    u64 gh, gd, bo, sh, sd;
                    edge(j, p, e, gh, gd, bo, sh, sd);
                    const u64 le = (e & 0x80000000u) ? ~0ull : 0ull;
                    const u64 lh = gh | sh, ld = gd | sd;
                    const u64 lph = lh & ~le, lpd = ld & ~le;
                    allh &= lph | bo | (lh & le);
                    alld &= lpd | bo | (ld & le);
                    anyh |= lph;
                    anyd |= lpd;
                    if (j < 2) { lat_h[j] = lh; lat_d[j] = ld; }
                }
                const u64 inh = allh & anyh & vm, ind = alld & anyd & vm;
                vh = inh & ~sth;
                vd = ind & ~std_;
                G(c.ie_h)[(size_t)b * wd + wo] = inh & uh;
                G(c.ie_d)[(size_t)b * wd + wo] = ind & ud;
                for (int j = 0; j < cnt; ++j) {
                    int p; uint32_t e;
                    nbr_f(r, j, p, e);
                    u64 lh, ld;
                    if (j < 2) { lh = lat_h[j]; ld = lat_d[j]; }
                    else {
                        u64 gh, gd, bo, sh, sd;
                        edge(j, p, e, gh, gd, bo, sh, sd);
                        lh = gh | sh; ld = gd | sd;
                    }
                    const u64 le = (e & 0x80000000u) ? ~0ull : 0ull;
                    const size_t eid = e & 0x7FFFFFFFu;
                    G(c.ig_h)[eid * wd + wo] = lh & (le | ~inh) & vm;
                    G(c.ig_d)[eid * wd + wo] = ld & (le | ~ind) & vm;
                }
            };
            run_phase(S, 0ull, pre, comp);
        } else if (dat) {
            // eager placement only: every EAG is materialised on its edge
            for (int b = 0; b < nb; ++b) {
                G(c.ie_h)[(size_t)b * wd + wo] = 0;
                G(c.ie_d)[(size_t)b * wd + wo] = 0;
            }
            for (int e = 0; e < c.ne; ++e) {
                G(c.ig_h)[(size_t)e * wd + wo] = G(c.eag_h)[(size_t)e * wd + wo];
                G(c.ig_d)[(size_t)e * wd + wo] = G(c.eag_d)[(size_t)e * wd + wo];
            }
        }
        return;
    }

    // ------------------------------------------------------------ validity after placement (forward, must)
    // AVFin_s(q) = INS_ENTRY_s(q) | AND_e (AVFout_s(p) | INS_EDGE_s(e)); the state reuses the
    // eager-validity rows.
    if constexpr (PH == PH_AVF) {
        const Rows S = rows_of(c.aveout_h, c.aveout_d, 2);
        const u64 init = ~0ull & vm;
        // x0/x1 = INS_ENTRY, x2 = W, x3..x6 = INS_EDGE_H/D of the two inline in-edges
        auto pre = [&](int b, const Rec& r, u64* x) {
            x[0] = row(c.ie_h, b); x[1] = row(c.ie_d, b); x[2] = row(c.W, b);
            const int cnt = (int)(r.meta & REC_COUNT);
            const uint32_t e0 = cnt > 0 ? r.e0 : 0u, e1 = cnt > 1 ? r.e1 : 0u;
            x[3] = erow(c.ig_h, e0); x[4] = erow(c.ig_d, e0);
            x[5] = erow(c.ig_h, e1); x[6] = erow(c.ig_d, e1);
        };
        auto comp = [&](int b, const Rec& r, const u64* x, const u64* nh, const u64* nd, u64 ph, u64 pd, int sweep,
                        u64& vh, u64& vd) {
            u64 ih, id;
            if (r.meta & REC_ENTRY) { ih = vec(c.ev_h); id = vec(c.ev_d); }
            else {
                const int cnt = (int)(r.meta & REC_COUNT);
                u64 mh = ~0ull, md = ~0ull;
                for (int j = 0; j < cnt; ++j) {
                    int p; uint32_t e;
                    nbr_f(r, j, p, e);
                    u64 gh, gd, sh, sd;
                    if (j < 2) { gh = x[3 + 2 * j]; gd = x[4 + 2 * j]; sh = nh[j]; sd = nd[j]; }
                    else {
                        gh = erow(c.ig_h, e); gd = erow(c.ig_d, e);
                        extra(S, b, p, sweep, init, ph, pd, sh, sd);
                    }
                    mh &= sh | gh;
                    md &= sd | gd;
                }
                ih = x[0] | mh;
                id = x[1] | md;
            }
            ih &= vm; id &= vm;
            if (c.avf_h) { G(c.avf_h)[(size_t)b * wd + wo] = ih; G(c.avf_d)[(size_t)b * wd + wo] = id; }
            valid_out(b, r, ih, id, x[2], vh, vd);
        };
        if (!run_phase(S, init, pre, comp)) return;

        // Per-variable map kind (Table II), from the final placement in one pass:
        // map(to) = a copy into the device on p->q with no DEVICE block before p, or before q
        // when no predecessor has one; map(from) = a copy into the host on p->q or before q
        // when no DEVICE block follows q; alloc = used only on the device.
        if (c.var_kind && dat) {
            u64 to = 0, fr = 0, dv = 0;
            for (int b = 0; b < nb; ++b) {
                const Rec r = ldrec(c.rec_f, b);
                const int cnt = (int)(r.meta & REC_COUNT);
                const u64 not_before = ((FLG[(size_t)nb + b] >> 1) & 1) - 1;   // all ones: no DEVICE block follows b
                if (!(r.meta & REC_ENTRY)) {
                    u64 none_after = ~0ull;                                        // no predecessor after a DEVICE block
                    for (int j = 0; j < cnt; ++j) {
                        int p; uint32_t e;
                        nbr_f(r, j, p, e);
                        const u64 p_clear = 0ull - ((FLG[(size_t)2 * nb + p] >> 1) & 1);   // all ones: p not after DEVICE
                        to |= erow(c.ig_d, e) & p_clear;
                        fr |= erow(c.ig_h, e) & not_before;
                        none_after &= p_clear;
                    }
                    to |= row(c.ie_d, b) & none_after;
                    fr |= row(c.ie_h, b) & not_before;
                }
                if ((r.meta & REC_DEV) && !(r.meta & REC_EXIT)) dv |= row(c.R, b) | row(c.W, b);
            }
            const int base = w * 64;
            for (int i = 0; i < 64 && base + i < c.nv; ++i) {
                const uint32_t t1 = (uint32_t)((to >> i) & 1), f1 = (uint32_t)((fr >> i) & 1);
                const uint32_t d1 = (uint32_t)((dv >> i) & 1);
                G(c.var_kind)[base + i] = (uint8_t)(t1 | (f1 << 1) | ((d1 && !t1 && !f1) ? 4u : 0u));
            }
        }
    }
}

// Edge-parallel steps between the walks (no iteration): lanes over words,
// one wavefront per (tile, block) chunk of 64 source blocks.
//   after AVE : EAG_s(e=p->q) = NU_s(q) & ~AVEout_s(p);  VE_s(e) = AVEout_s(p) | NU_s(q)
//               (VE is kept in the INS_EDGE rows until the delayed placement overwrites them)
//   after MAYP: BOTH(e) = FV_H(e) & FV_D(e), FV_x(e) = VE_x(e) & ~((EAG_x(e) | MAYPout_x(p)) & ~LE(e))
template <int STEP>
__device__ __forceinline__ void edge_step(const DevCfg& c, int s0, int nw, int b0)
{
    const int lane = threadIdx.x;
    if (lane >= nw) return;
    const int wd = c.wd;
    const size_t wo = (size_t)(s0 + lane);
    const CAS int32_t* SP = K(c.succ_ptr);
    const CAS int32_t* SI = K(c.succ_idx);
    const CAS uint8_t* KD = K(c.kind);
    const int b1 = min(b0 + 64, c.nb);
#pragma unroll 4
    for (int p = b0; p < b1; ++p) {
        const int a = SP[p], z = SP[p + 1];
        if (a == z) continue;
        const u64 aoh = G(c.aveout_h)[(size_t)p * wd + wo], aod = G(c.aveout_d)[(size_t)p * wd + wo];
        u64 mph = 0, mpd = 0;
        if constexpr (STEP == 1) { mph = G(c.mayp_h)[(size_t)p * wd + wo]; mpd = G(c.mayp_d)[(size_t)p * wd + wo]; }
        for (int e = a; e < z; ++e) {
            const size_t ei = (size_t)e * wd + wo;
            if constexpr (STEP == 0) {
                const int q = SI[e];
                const u64 nuh = G(c.nu_h)[(size_t)q * wd + wo], nud = G(c.nu_d)[(size_t)q * wd + wo];
                G(c.eag_h)[ei] = nuh & ~aoh;
                G(c.eag_d)[ei] = nud & ~aod;
                G(c.ig_h)[ei] = aoh | nuh;
                G(c.ig_d)[ei] = aod | nud;
            } else {
                const u64 nle = KD[e] == 2 ? 0ull : ~0ull;
                const u64 fvh = G(c.ig_h)[ei] & ~((G(c.eag_h)[ei] | mph) & nle);
                const u64 fvd = G(c.ig_d)[ei] & ~((G(c.eag_d)[ei] | mpd) & nle);
                G(c.both)[ei] = fvh & fvd;
            }
        }
    }
}

template <int PH>
__device__ __forceinline__ void phase_kernel(const DevCfg* __restrict__ cfgs, const Tile* __restrict__ tiles, int n_tiles,
                                             int32_t* __restrict__ counter, int ring_words)
{
    extern __shared__ __align__(16) u64 ring[];
    for (;;) {
        int t = 0;
        if (threadIdx.x == 0) t = atomicAdd(&counter[PH], 1);
        t = __builtin_amdgcn_readfirstlane(__shfl(t, 0, 64));
        if (t >= n_tiles) break;
        const Tile tl = tiles[t];
        const DevCfg c = cfgs[tl.cfg];
        if (G(c.info)[INFO_STATUS] != 0) continue;
        solve_phase<PH>(c, tl.s0, tl.nw, tl.fslot, ring, ring_words);
    }
}

// Work items of the edge steps: (tile, first block of a 64-block chunk),
// claimed through counter slots 5 and 6.
template <int STEP>
__device__ __forceinline__ void edge_kernel(const DevCfg* __restrict__ cfgs, const Tile* __restrict__ tiles,
                                            const EdgeItem* __restrict__ items, int n_items, int32_t* __restrict__ counter)
{
    for (;;) {
        int it = 0;
        if (threadIdx.x == 0) it = atomicAdd(&counter[5 + STEP], 1);
        it = __builtin_amdgcn_readfirstlane(__shfl(it, 0, 64));
        if (it >= n_items) break;
        const EdgeItem item = items[it];
        const Tile tl = tiles[item.tile];
        const DevCfg c = cfgs[tl.cfg];
        if (G(c.info)[INFO_STATUS] != 0 || tl.nw == 0) continue;
        if (STEP == 1 && (c.placement & 1)) continue;   // the eager placement needs no pending-copy facts
        edge_step<STEP>(c, tl.s0, tl.nw, item.b0);
    }
}

// One persistent kernel per phase; the phases of all tiles run in this order.
#define OMPD_PHASE_KERNEL(name, ph)                                                                          \
    extern "C" __global__ void __launch_bounds__(64) name(const DevCfg* __restrict__ cfgs,                  \
                                                           const Tile* __restrict__ tiles, int n_tiles,     \
                                                           int32_t* __restrict__ counter, int ring_words)   \
    {                                                                                                        \
        phase_kernel<ph>(cfgs, tiles, n_tiles, counter, ring_words);                                         \
    }
OMPD_PHASE_KERNEL(ompd_k_nu, PH_NU)
OMPD_PHASE_KERNEL(ompd_k_ave, PH_AVE)
OMPD_PHASE_KERNEL(ompd_k_mayp, PH_MAYP)
OMPD_PHASE_KERNEL(ompd_k_later, PH_LATER)
OMPD_PHASE_KERNEL(ompd_k_avf, PH_AVF)

extern "C" __global__ void __launch_bounds__(64)
ompd_k_edge0(const DevCfg* __restrict__ cfgs, const Tile* __restrict__ tiles, const EdgeItem* __restrict__ items,
             int n_items, int32_t* __restrict__ counter)
{
    edge_kernel<0>(cfgs, tiles, items, n_items, counter);
}
extern "C" __global__ void __launch_bounds__(64)
ompd_k_edge1(const DevCfg* __restrict__ cfgs, const Tile* __restrict__ tiles, const EdgeItem* __restrict__ items,
             int n_items, int32_t* __restrict__ counter)
{
    edge_kernel<1>(cfgs, tiles, items, n_items, counter);
}

}  // namespace ompd
