// HIP kernels (gfx950) for the OMPDart data-flow solve.
//
// ompd_k_prep (one 256-thread workgroup per CFG): ingest and normalise --
//   validates the CSR and the boundary rules, builds the predecessor CSR
//   (with the successor-edge id of every predecessor link) and writes one
//   32-byte record per block for each direction (flags, first two
//   neighbours with their edge ids, CSR start of the rest, call index),
//   and for each direction a 32-byte step entry per position of the walk
//   (where the states of the first two neighbours are found for the
//   launch's ring size, the far neighbour and how many steps back its state
//   was computed, the block and its first two edge ids).
//
// Phase kernels (persistent, two wavefronts per tile): a tile is one CFG
//   and a run of up to 15 64-bit words of its variables.  One kernel per
//   iterated problem of the method, in this order:
//     ompd_k_nu     next use (backward may)
//     ompd_k_ave    validity with eager copies (forward must) and the
//                   reachability facts behind the map/update labels
//     ompd_k_mayp   pending copies (forward may)
//     ompd_k_later  delayed placement (forward AND/OR)
//     ompd_k_avf    validity after placement (forward must)
// Pass kernels (one wavefront per 64-block chunk of a tile, no iteration)
//   write what follows from a fixed point: ompd_k_post_ave (AVEin, eager
//   copies per edge), ompd_k_post_mayp (valid in both spaces per edge),
//   ompd_k_post_later (the copies themselves), ompd_k_post_avf (AVFin and
//   the map-kind masks); ompd_k_varkind turns the masks into the
//   per-variable map kind (Table II).
//
// All arithmetic is integer AND / OR / ANDN; variables never interact, so
// any split of the variable axis is exact.
#include <hip/hip_runtime.h>

#include "ompd_device.h"

#define OMPD_E_INVAL_ (-1)
#define OMPD_E_DEVICE_ (-3)
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

// Step flags (the x word of a step entry and of a step descriptor).  Bits 0-1 / 2-3: where the
// state of neighbour 0 / 1 is found: 0 nowhere (missing), 1 the block computed last, 2 the ring,
// 3 the far input.
constexpr uint32_t DF_SLOW = 1u << 4;   // ENTRY, EXIT, a call, no or more than two neighbours, two far ones
constexpr uint32_t DF_DEV = 1u << 5;    // a DEVICE block
constexpr uint32_t DF_LE0 = 1u << 6;    // edge of neighbour 0 is a loop entry (forward phases)
constexpr uint32_t DF_LE1 = 1u << 7;    // edge of neighbour 1 is a loop entry
constexpr uint32_t SF_FAR = 1u << 8;    // one of the first two neighbours is far (step entries only)
constexpr uint32_t SF_BACK = 1u << 9;   // ... and not visited yet in the sweep
constexpr uint32_t SF_ONE = 1u << 10;   // at most one neighbour: no rows of a second edge are read
constexpr uint32_t DF_MASK = 0xFFu;     // the bits a step descriptor carries from the step entry
// bits the helper adds to a step descriptor, so that the transfer functions select with masks
// (one scalar bit-field extract each) instead of compares
constexpr int DD_LAST0 = 8, DD_LAST1 = 9;   // neighbour j is the block computed last (registers)
constexpr int DD_P0 = 10, DD_P1 = 11;       // neighbour j exists
constexpr int DD_A0 = 12, DD_A1 = 13;       // ... and its edge does not enter a loop
constexpr int DD_DEV = 5;                   // the bit of DF_DEV
static_assert(DF_DEV == 1u << DD_DEV && DF_MASK < 1u << DD_LAST0, "descriptor bits");
// all ones if bit `bit` of the wave-uniform word fl is set, else zero
__device__ __forceinline__ uint32_t fmask(uint32_t fl, int bit) { return (uint32_t)((int32_t)(fl << (31 - bit)) >> 31); }
// Does an edge of kind k stop the delay?  Loop entries do, unless the placement is pure lazy.
__device__ __forceinline__ bool is_le(const DevCfg& c, uint8_t k) { return k == 2 && !(c.placement & PL_LAZY); }
// A step entry (two int4, one per walk position): x flags; y the ring distances of neighbours
// 0 and 1 (bits 0-7, 8-15; flag code 2 only); z the far neighbour; w how many steps before the
// current one its state was computed (this sweep's or, when SF_BACK, the previous sweep's); then
// the block, the edge ids of neighbours 0 and 1 (0 when missing) and a word of the re-check list
// (entry k's holds the k-th block with a neighbour read before its own visit, -1 past the list).
// The step entry of the block b at walk position i, from its record r0 / r1 (ring of rs slots);
// pos: each block's position in the forward walk (NULL: its id).
__device__ __forceinline__ void make_step(const int4& r0, const int4& r1, int b, bool bwd, int nb, int rs,
                                          const int32_t* pos, int4& t0, int4& t1)
{
    const int pb = pos ? pos[b] : b;
    const uint32_t meta = (uint32_t)r0.x, e0 = (uint32_t)r0.w, e1 = (uint32_t)r1.x;
    const int cnt = (int)(meta & REC_COUNT);
    uint32_t fl = (cnt > 2 || cnt == 0 || (meta & (REC_ENTRY | REC_EXIT | REC_CALL))) ? DF_SLOW : 0u;
    fl |= (meta & REC_DEV) ? DF_DEV : 0u;
    fl |= (e0 & 0x80000000u) ? DF_LE0 : 0u;
    fl |= ((e1 & 0x80000000u) && cnt > 1) ? DF_LE1 : 0u;
    fl |= cnt <= 1 ? SF_ONE : 0u;
    int dd = 0, fp = 0, fo = 0;
    bool far = false;
    for (int j = 0; j < 2 && j < cnt; ++j) {
        const int p = j == 0 ? r0.y : r0.z;
        const int pp = pos ? pos[p] : p;
        const int d = bwd ? pp - pb : pb - pp;   // 1: the block just before in the walk
        uint32_t k;
        if (d == 1) k = 1;
        else if (d >= 2 && d <= rs) { k = 2; dd |= d << (8 * j); }
        else if (!far) {
            k = 3;
            far = true;
            fp = p;
            fo = d > 0 ? d : d + nb;
            fl |= SF_FAR | (d > 0 ? 0u : SF_BACK);
        }
        else { k = 0; fl |= DF_SLOW; }
        fl |= k << (2 * j);
    }
    t0 = make_int4((int)fl, dd, fp, fo);
    t1 = make_int4(b, cnt > 0 ? (int)(e0 & 0x7FFFFFFFu) : 0, cnt > 1 ? (int)(e1 & 0x7FFFFFFFu) : 0, -1);
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
ompd_k_prep(const DevCfg* __restrict__ cfgs, int n_cfgs, int32_t* __restrict__ solve_counter, int ring_slots)
{
    __shared__ int s_err;
    __shared__ int32_t s_scan[16];
    const int ci = blockIdx.x;
    if (ci == 0 && threadIdx.x < N_COUNTERS) solve_counter[threadIdx.x] = 0;   // work counters of the solve kernels
    if (ci >= n_cfgs) return;
    const DevCfg c = cfgs[ci];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nb = c.nb, ne = c.ne, wd = c.wd;
    if (tid == 0) s_err = 0;
    for (int i = tid; i < INFO_WORDS; i += nt) c.info[i] = 0;
    if (c.var_kind)
        for (int i = tid; i < 4 * wd; i += nt) c.vk_acc[i] = 0;
    for (int w = tid; w < wd; w += nt) c.fp[w] = 0;
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
            if (!(c.placement & PL_SUMMARY) && ((eh | ed) & m) != m) err = 1;   // a summary evaluation may leave gaps
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

    // firstprivate variables: marked scalars that no DEVICE block writes (the OR of the device
    // blocks' writes gathers in c.fp first)
    if (c.scalar && wd > 0) {
        for (size_t i = tid; i < (size_t)nb * wd; i += nt) {
            const int b = (int)(i / wd), w = (int)(i % wd);
            if (c.space[b]) {
                const uint64_t x = c.W[i];
                if (x) atomicOr((unsigned long long*)&c.fp[w], (unsigned long long)x);
            }
        }
        __syncthreads();
        const uint64_t last = (c.nv & 63) ? ((1ull << (c.nv & 63)) - 1ull) : ~0ull;
        for (int w = tid; w < wd; w += nt) {
            // the atomics above ran in L2: read their result there, past this CU's cache
            const uint64_t dw = __hip_atomic_load(&c.fp[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            c.fp[w] = c.scalar[w] & ~dw & (w == wd - 1 ? last : ~0ull);
        }
        __syncthreads();
    }
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
        r0.w = (int)((uint32_t)e0 | ((cnt > 0 && is_le(c, c.kind[e0])) ? 0x80000000u : 0u));
        r1.x = (int)((uint32_t)e1 | ((cnt > 1 && is_le(c, c.kind[e1])) ? 0x80000000u : 0u));
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
    __syncthreads();
    // Walk order (walk schedule): the caller's ids when every edge other than BACK goes from a
    // lower to a higher id (the source order a front end emits; the sweeps then reach the fixed
    // point in loop depth + 1), else the order of the peel below, in which every such edge goes
    // forward too;
    // then lorder[i] is the block at forward walk position i and loff[b] the position of block b.
    // Levels (level schedule): peel the graph from ENTRY over the edges other than BACK; the
    // blocks of a round form a level.  Blocks left over (a cycle closed by an edge not marked
    // BACK, or unreachable ones, which the validity phase rejects) get a level each, in id order.
    const bool lv = c.sched == SCHED_LEVEL;
    __shared__ int s_unord;
    if (tid == 0) s_unord = 0;
    __syncthreads();
    if (!lv) {
        int un = 0;
        for (int b = tid; b < nb; b += nt)
            for (int e = c.succ_ptr[b]; e < c.succ_ptr[b + 1]; ++e)
                if (c.kind[e] != 1 && c.succ_idx[e] <= b) un = 1;
        if (un) atomicOr(&s_unord, 1);
        __syncthreads();
    }
    const bool unord = s_unord != 0;
    if (lv || unord) {
        __shared__ int s_tail;
        int32_t* deg = c.tmp;
        for (int b = tid; b < nb; b += nt) {
            int k = 0;
            for (int j = pp[b]; j < pp[b + 1]; ++j) k += c.kind[c.pred_eid[j]] != 1;
            deg[b] = k;
        }
        if (tid == 0) { c.lorder[0] = c.entry; s_tail = 1; }
        __syncthreads();
        int fa = 0, fb = 1, nl = 0;
        while (fa < fb) {
            if (tid == 0 && lv) c.loff[nl] = fa;
            for (int i = fa + tid; i < fb; i += nt) {
                const int b = c.lorder[i];
                for (int e = c.succ_ptr[b]; e < c.succ_ptr[b + 1]; ++e) {
                    if (c.kind[e] == 1) continue;
                    const int q = c.succ_idx[e];
                    if (atomicSub(&deg[q], 1) == 1) c.lorder[atomicAdd(&s_tail, 1)] = q;
                }
            }
            __syncthreads();
            fa = fb;
            fb = s_tail;
            ++nl;
            __syncthreads();
        }
        if (fb < nb) {
            // leftovers: blocks never placed, one level each
            __shared__ int s_n;
            for (int i = tid; i < fb; i += nt) deg[c.lorder[i]] = -1;
            __syncthreads();
            if (tid == 0) {
                int n = fb;
                for (int b = 0; b < nb; ++b)
                    if (deg[b] != -1) {
                        c.lorder[n] = b;
                        if (lv) c.loff[nl] = n;
                        ++nl;
                        ++n;
                    }
                s_n = nl;
            }
            __syncthreads();
            nl = s_n;
        }
        if (tid == 0) {
            if (lv) c.loff[nl] = nb;
            c.info[INFO_LEVELS] = lv ? nl : 0;
        }
        __syncthreads();
        if (!lv)
            for (int i = tid; i < nb; i += nt) c.loff[c.lorder[i]] = i;
        __syncthreads();
    }
    if (tid == 0) c.info[INFO_ORDER] = lv || !unord;
    int4* SF = reinterpret_cast<int4*>(c.step_f);
    int4* SB = reinterpret_cast<int4*>(c.step_b);
    if (lv) {
        // Re-check lists of the level schedule (what the walk's step entries carry, for levels):
        // the blocks that read a neighbour whose level is not below their own (a BACK edge into
        // them, or a self loop), that is a predecessor of a forward phase or a successor of a
        // backward one.  Each block's level goes to the spare word of its records first.  The
        // forward list fills c.tmp from the front, the backward one from the back (entry nb
        // first), each ended by -1; if the two do not fit in its nb + 1 words, c.tmp[0] = -2 and
        // the level kernels confirm with a sweep instead.
        const int nlv = c.info[INFO_LEVELS];
        for (int l = 0; l < nlv; ++l)
            for (int k = c.loff[l] + tid; k < c.loff[l + 1]; k += nt) {
                const int b = c.lorder[k];
                reinterpret_cast<int32_t*>(RF + 2 * b + 1)[3] = l;
                reinterpret_cast<int32_t*>(RB + 2 * b + 1)[3] = l;
            }
        __syncthreads();
        auto lev = [&](int b) -> int { return reinterpret_cast<const int32_t*>(RF + 2 * b + 1)[3]; };
        auto back_in = [&](int b, int dir) -> bool {
            const int lb = lev(b);
            if (!dir) {
                for (int j = pp[b]; j < pp[b + 1]; ++j)
                    if (lev(c.pred_idx[j]) >= lb) return true;
            }
            else {
                for (int e = c.succ_ptr[b]; e < c.succ_ptr[b + 1]; ++e)
                    if (lev(c.succ_idx[e]) <= lb) return true;
            }
            return false;
        };
        __shared__ int s_lw[2][4];
        const int wv = tid >> 6;
        int cnt2[2] = {0, 0};
        for (int pass = 0; pass < 2; ++pass) {   // 0: count, 1: write
            if (pass == 1 && cnt2[0] + cnt2[1] >= nb) {
                if (tid == 0) c.tmp[0] = -2;
                break;
            }
            int base[2] = {0, 0};
            for (int b0 = 0; b0 < nb; b0 += nt) {
                const int b = b0 + tid;
                const bool f = b < nb && back_in(b, 0), g = b < nb && back_in(b, 1);
                const uint64_t mf = __ballot(f), mg = __ballot(g);
                if ((tid & 63) == 0) { s_lw[0][wv] = __popcll(mf); s_lw[1][wv] = __popcll(mg); }
                __syncthreads();
                const uint64_t below = (1ull << (tid & 63)) - 1ull;
                int af = base[0], ag = base[1];
                for (int k = 0; k < wv; ++k) { af += s_lw[0][k]; ag += s_lw[1][k]; }
                af += __popcll(mf & below);
                ag += __popcll(mg & below);
                if (pass == 1) {
                    if (f) c.tmp[af] = b;
                    if (g) c.tmp[nb - ag] = b;
                }
                for (int k = 0; k < (nt >> 6); ++k) { base[0] += s_lw[0][k]; base[1] += s_lw[1][k]; }
                __syncthreads();
            }
            if (pass == 0) { cnt2[0] = base[0]; cnt2[1] = base[1]; }
            else if (tid == 0) { c.tmp[base[0]] = -1; c.tmp[nb - base[1]] = -1; }
        }
        __syncthreads();
        // level schedule (no walk steps): the records in level order, the block in the last word,
        // so that a level's positions lead to their records in one load
        for (int k = tid; k < nb; k += nt) {
            const int b = c.lorder[k];
            int4 t1 = RF[2 * b + 1];
            t1.w = b;
            SF[2 * k] = RF[2 * b];
            SF[2 * k + 1] = t1;
            t1 = RB[2 * b + 1];
            t1.w = b;
            SB[2 * k] = RB[2 * b];
            SB[2 * k + 1] = t1;
        }
        return;
    }
    // step entries in walk order: forward position i is block i (or lorder[i]), backward position i
    // the block at forward position nb - 1 - i
    const int32_t* pos = unord ? c.loff : nullptr;
    for (int i = tid; i < nb; i += nt) {
        int4 t0, t1;
        const int bf = pos ? c.lorder[i] : i;
        make_step(RF[2 * bf], RF[2 * bf + 1], bf, false, nb, ring_slots, pos, t0, t1);
        SF[2 * i] = t0;
        SF[2 * i + 1] = t1;
        const int bb = pos ? c.lorder[nb - 1 - i] : nb - 1 - i;
        make_step(RB[2 * bb], RB[2 * bb + 1], bb, true, nb, ring_slots, pos, t0, t1);
        SB[2 * i] = t0;
        SB[2 * i + 1] = t1;
    }
    __syncthreads();
    // Re-check lists, in walk order: the blocks a sweep computes from a neighbour it has not
    // visited yet in that sweep (the neighbour's walk position is not before the block's own: a
    // BACK edge into it, or a self loop), that is a predecessor of a forward phase or a successor
    // of a backward one.  Only through them can the next sweep see states other than this
    // sweep's.  Entry k's last word takes the k-th such block (make_step left -1 in every one).
    __shared__ int s_wave[4];
    const int wv = tid >> 6;
    for (int dir = 0; dir < 2; ++dir) {
        int4* S = dir ? SB : SF;
        int base = 0;
        for (int i0 = 0; i0 < nb; i0 += nt) {
            const int i = i0 + tid;
            int b = -1;
            bool back = false;
            if (i < nb) {
                b = dir ? (pos ? c.lorder[nb - 1 - i] : nb - 1 - i) : (pos ? c.lorder[i] : i);
                const int pb = pos ? pos[b] : b;
                if (!dir) {
                    for (int j = pp[b]; j < pp[b + 1] && !back; ++j) {
                        const int q = c.pred_idx[j];
                        back = (pos ? pos[q] : q) >= pb;
                    }
                }
                else {
                    for (int e = c.succ_ptr[b]; e < c.succ_ptr[b + 1] && !back; ++e) {
                        const int q = c.succ_idx[e];
                        back = (pos ? pos[q] : q) <= pb;
                    }
                }
            }
            const uint64_t m = __ballot(back);
            if ((tid & 63) == 0) s_wave[wv] = __popcll(m);
            __syncthreads();
            int at = base;
            for (int k = 0; k < wv; ++k) at += s_wave[k];
            at += __popcll(m & ((1ull << (tid & 63)) - 1ull));
            if (back) reinterpret_cast<int32_t*>(S + 2 * at + 1)[3] = b;
            for (int k = 0; k < (nt >> 6); ++k) base += s_wave[k];
            __syncthreads();
        }
    }
}

// --------------------------------------------------------------------------
// solve
// --------------------------------------------------------------------------
// One workgroup of two wavefronts solves one tile: a CFG and a run of up to
// TILE_WORDS (15) consecutive 64-bit words of its variable axis; lanes 0 to
// 2 LANES - 1 (32) of each wavefront take part.  Lanes l and l + LANES own the
// low and high halves of word s0 + l of every row; in the two phases that
// compute the CFG's reachability facts,
// lane nw (the flag lane) carries them as a pseudo-variable word whose inputs
// are synthesised so that the same equations compute them:
//   next use, host channel, bit 0 : the block reaches EXIT
//   next use, device channel, bit 1: a DEVICE block is reachable from here
//   eager validity, host channel, bit 0: the block is NOT reached from ENTRY
//   eager validity, host channel, bit 1: no DEVICE block reaches the block
// Lanes past the tile (below LANES, and their high partners) shadow word s0 (same inputs, same
// results), so the walk has no lane divergence and everything about a step
// except its data is wave-uniform.  Narrow tiles keep the LDS of a workgroup
// small (25-40 KiB with the default ring), so that several tiles are resident
// per CU: most CFGs have few words, and a step costs the same instructions
// whatever the tile's width.
//
// A phase is a sequence of Gauss-Seidel sweeps in block-id order (reverse
// order for the backward phase).  The compute wavefront walks the blocks and
// touches global memory only on rare paths: the value of the block just
// computed stays in registers, the last RS steps sit in an LDS ring, and the
// helper wavefront keeps, up to IR steps ahead, each step's descriptor and
// inputs (including the state of its first other neighbour) ready in LDS,
// planned from the step entries the ingest kernel wrote; the helper also
// copies the compute wavefront's results to the state rows.
// The two meet through counters in LDS.
// Every phase is monotone on a finite lattice, so any visiting order reaches
// the same fixed point, and each block's value only moves one way between
// sweeps: a sweep changed nothing exactly when the popcount of the state is
// unchanged.  After a sweep that changed something, re-evaluating the blocks
// that read a neighbour not yet visited in the sweep tells whether the next
// sweep would change anything (see `settled`), which saves the confirming
// sweep.  Outputs derived from the state are written by edge-parallel passes
// after the phase (no iteration).
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

// Record b of a record array, b per lane.
__device__ __forceinline__ Rec ldrec_v(const int32_t* base, int b)
{
    typedef int v4i __attribute__((ext_vector_type(4)));
    const GAS v4i* q = reinterpret_cast<const GAS v4i*>(G(base)) + 2 * (size_t)b;
    const v4i x = q[0], y = q[1];
    Rec r;
    r.meta = (uint32_t)x.x; r.n0 = x.y; r.n1 = x.z; r.e0 = (uint32_t)x.w;
    r.e1 = (uint32_t)y.x; r.ovf = y.y; r.ci = y.z; r.pad = y.w;
    return r;
}

template <class T>
__device__ __forceinline__ T tsel(T a1, T l, T t00, T t01, T t10, T t11)
{
    return (~a1 & ~l & t00) | (~a1 & l & t01) | (a1 & ~l & t10) | (a1 & l & t11);
}


// A state row written by the other wavefront of the workgroup in this kernel:
// read past the (non-coherent) first-level cache.
__device__ __forceinline__ u64 ld_fresh(const GAS u64* p)
{
    return __hip_atomic_load(const_cast<GAS u64*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t ld_half(const GAS u64* p, bool hi)
{
    return __hip_atomic_load(const_cast<GAS uint32_t*>(reinterpret_cast<const GAS uint32_t*>(p)) + (hi ? 1 : 0),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A value loaded on a rarely taken path, made ready before the paths join: the
// compiler then waits for the load on that path only, instead of at the join,
// where the wait would also drain the loads issued ahead on the common path.
template <class T>
__device__ __forceinline__ T settle(T x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Copy of one 64-bit word per owning lane from global memory into LDS without
// registers, by 2 LANES lanes: lane l < LANES copies the low half of its word
// `src` to dst[l], lane LANES + l (hi, the same src) the high half to
// dst[LANES + l]; dst is wave-uniform.  Completion is counted by vmcnt.
constexpr unsigned CPOL_SC1 = 16;   // read past the first-level cache
template <unsigned CPOL>
__device__ __forceinline__ void dma_word(const GAS u64* src, bool hi, uint32_t* dst)
{
    const GAS uint32_t* s32 = reinterpret_cast<const GAS uint32_t*>(src) + (hi ? 1 : 0);
    __builtin_amdgcn_global_load_lds(s32, (__attribute__((address_space(3))) void*)dst, 4, 0, CPOL);
}
// The same from a row whose start `row` is wave-uniform, the lane's half at byte `off` of it
// (scalar base plus a 32-bit lane offset: no per-lane address arithmetic), to the LDS address
// `dst` (wave-uniform, kept in scalar registers).
#define LDS3 __attribute__((address_space(3)))
template <unsigned CPOL>
__device__ __forceinline__ void dma_row(const GAS u64* row, uint32_t off, LDS3 char* dst)
{
    const GAS uint32_t* s32 = reinterpret_cast<const GAS uint32_t*>(reinterpret_cast<const GAS char*>(row) + off);
    __builtin_amdgcn_global_load_lds(s32, (LDS3 void*)dst, 4, 0, CPOL);
}

// Coordination of the two wavefronts of a tile (LDS).
struct Ctl {
    int tile;        // the tile of this round
    int skip;        // its CFG already failed
    int produced;    // steps whose state is in the ring (compute wavefront)
    int consumed;    // steps the helper has read from the ring
    int flushed;     // steps whose state-row stores have completed
    int done;        // the compute wavefront has finished the phase
    int abort;       // a wait ran out: both wavefronts stop
    int in_ready;    // steps whose inputs and descriptors are in LDS (helper)
};
constexpr int CTL_WORDS = CTL_BYTES / 8;   // u64 words reserved for Ctl at the start of the LDS
static_assert(sizeof(Ctl) <= CTL_BYTES, "coordination words");

__device__ __forceinline__ int lds_get(int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ __forceinline__ void lds_put(int* p, int v)
{
    if ((threadIdx.x & 63) == 0) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// LDS accesses before this point complete before LDS writes after it (LDS only: pending
// global loads are not waited for)
__device__ __forceinline__ void lds_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local"); }
// LDS reads after this point are not moved before the counter read that precedes it
__device__ __forceinline__ void lds_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local"); }

// The device's constant-rate wall clock (ticks at the rate the host queries as
// hipDeviceAttributeWallClockRate).
__device__ __forceinline__ uint64_t wall_ticks() { return __builtin_amdgcn_s_memrealtime(); }

// Wait until *p >= target, for at most `limit` wall-clock ticks; false if the wait ran out (then
// `abort` is set and `seen` / `waited` say what it saw) or the other side gave up first.
__device__ __forceinline__ bool wait_for(int* p, int target, int* abort, int32_t limit, int& seen, int64_t& waited)
{
    const uint64_t t0 = wall_ticks();
    for (;;) {
        seen = __builtin_amdgcn_readfirstlane(lds_get(p));
        if (seen >= target) { lds_acquire(); return true; }
        if (__builtin_amdgcn_readfirstlane(lds_get(abort))) { waited = -1; return false; }
        waited = (int64_t)(wall_ticks() - t0);
        if (waited > (int64_t)limit) break;
        __builtin_amdgcn_s_sleep(1);
    }
    lds_put(abort, 1);
    return false;
}

// First wait of a CFG's solve that gave up: what it waited for (one lane writes).
__device__ __forceinline__ void post_mortem(int32_t* info, int ph, int tile, int what, int seen, int target,
                                            int64_t ticks)
{
    if ((threadIdx.x & 63) != 0) return;
    if (atomicCAS(&info[INFO_PM_PHASE], 0, ph + 1) != 0) return;
    info[INFO_PM_TILE] = tile;
    info[INFO_PM_WHAT] = what;
    info[INFO_PM_SEEN] = seen;
    info[INFO_PM_TARGET] = target;
    info[INFO_PM_TICKS] = (int32_t)(ticks > 0x7FFFFFFF ? 0x7FFFFFFF : ticks);
}

// State rows of the iterated vector of one phase, per lane: data lanes
// address [nb][wd] rows at their word, the flag lane its own [nb] column.
struct Rows {
    GAS u64* h;
    GAS u64* d;
    int str;
    // the low (hi = false) or high half of the word
    __device__ __forceinline__ uint32_t ldh32(int b, bool hi) const { return ld_half(h + (size_t)b * str, hi); }
    __device__ __forceinline__ uint32_t ldd32(int b, bool hi) const { return ld_half(d + (size_t)b * str, hi); }
    // store the low (hi = false) or high halves of the words
    __device__ __forceinline__ void st32(int b, bool hi, uint32_t x, uint32_t y) const
    {
        reinterpret_cast<GAS uint32_t*>(h + (size_t)b * str)[hi ? 1 : 0] = x;
        reinterpret_cast<GAS uint32_t*>(d + (size_t)b * str)[hi ? 1 : 0] = y;
    }
};

// IDORD: the walk follows the block ids (position = id); else the ingest kernel's order, with the
// block of each planned step kept in LDS and positions in loff (two instantiations, so that the
// common case carries nothing extra).
template <int PH, bool IDORD>
__device__ __forceinline__ void solve_phase(const DevCfg& c, int s0, int nw, int fslot, u64* lds, int RS)
{
    constexpr bool with_flags = PH == PH_NU || PH == PH_AVE;   // phases with the flag lane
    constexpr bool BWD = PH == PH_NU || PH == PH_LIVE;
    constexpr int NX = PH == PH_NU ? 2 : PH == PH_AVE ? 4 : PH == PH_MAYP ? 6 : 8;
    // the first input that is a row of the second edge (NX: the phase reads no edge rows)
    constexpr int NX1 = PH == PH_MAYP ? 4 : PH == PH_LATER ? 5 : PH == PH_AVF || PH == PH_LIVE ? 6 : NX;
    constexpr int NI = NX + 2;        // inputs of a step: the phase's own and the first far neighbour (h, d)
    constexpr int IR = in_ring(PH);   // steps whose inputs the helper keeps ready
    // Lanes 0 .. LANES - 1 of both wavefronts own the tile's words, lanes LANES .. 2 LANES - 1
    // (`hi`) the same words again: both wavefronts work on half-words, lane ln holding the low
    // 32 bits of word s0 + ln and lane ln + LANES the high 32 bits, so that a bitwise operation
    // is one instruction and a word's LDS access, copy or store one 32-lane access.
    const int lane = threadIdx.x & 63;
    const int ln = lane & (LANES - 1);
    const bool hi = lane >= LANES;
    const int l32 = lane & (2 * LANES - 1);   // the lane's half-word in the split LDS layout
    typedef uint32_t hw;                      // a half-word
    // a constant of the flag lane (bits 0-1: the low half)
    auto lo = [&](uint32_t v) -> hw { return hi ? 0u : v; };
    const bool helper = threadIdx.x >= 64;
    const int nb = c.nb, wd = c.wd;
    // a tile without variables (nw = 0) has only flag lanes (they compute the same facts)
    const bool dat = ln < nw, flg = with_flags && (ln == nw || nw == 0), act = dat || flg;
    const int w = s0 + (dat ? ln : 0);
    Ctl* ctl = reinterpret_cast<Ctl*>(lds);
    // Every row's LANES words in LDS are stored split: LANES low halves, then LANES high
    // halves (WORD_BYTES), which is lane l32's half-word at index l32; a state (h, d) is two
    // such rows (STATE_BYTES).
    char* lds8 = reinterpret_cast<char*>(lds);
    // the same as a wave-uniform 32-bit LDS address (scalar registers)
    const uint32_t lds3 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(size_t)(LDS3 char*)lds8);
    static_assert(BLK_RING >= 64 + 32, "block ring: result ring plus input ring");
    int* blkr = reinterpret_cast<int*>(lds8 + CTL_BYTES);                 // blocks of the last planned steps
    constexpr int RING_OFF = LDS_FIXED;                                   // RS states: the last results
    const int IN_OFF = RING_OFF + RS * STATE_BYTES;                       // IR steps of NI input words
    const int DESC_OFF = IN_OFF + IR * NI * WORD_BYTES;                   // IR step descriptors
    const int IDENT_OFF = DESC_OFF + IR * 16;                             // one state of identity words
    int4* dring = reinterpret_cast<int4*>(lds8 + DESC_OFF);
    // valid-variable mask of the lane's word (shadow lanes share word s0's; the flag lane uses bits 0-1)
    const u64 vm64 = flg ? 3ull : ((w == wd - 1 && (c.nv & 63)) ? ((1ull << (c.nv & 63)) - 1ull) : ~0ull);
    const hw vm = (hw)(hi ? vm64 >> 32 : vm64);   // its half
    // the firstprivate variables of the lane's word (a kernel's read of one is a host use, and the
    // device copy is not valid after that kernel); none for the flag lane
    const hw fph = (flg || !wd) ? 0u : ld_half(G(c.fp) + (size_t)w, hi);
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
    // the lane's half of a word
    auto half = [&](const GAS u64* p) -> hw { return reinterpret_cast<const GAS uint32_t*>(p)[hi ? 1 : 0]; };
    auto row = [&](const u64* a, int b) -> hw { return half(arr(a) + (size_t)b * wd + wo); };
    // start of the row at byte offset ob (wave-uniform) and the byte of the lane's half-word
    // within a row
    auto rowu = [&](const u64* a, u64 ob) -> const GAS u64* {
        return reinterpret_cast<const GAS u64*>(reinterpret_cast<const GAS char*>(arr(a)) + ob);
    };
    const uint32_t hoff = (uint32_t)wo * 8u + (hi ? 4u : 0u);
    // (both only at compute time, on rare paths: ENTRY, EXIT, call blocks)
    auto vec = [&](const u64* a) -> hw { return settle(half(arr(a) + wo)); };
    auto sum = [&](int ci, int r) -> hw { return settle(half(arr(c.sums) + ((size_t)ci * SUM_ROWS + r) * wd + wo)); };
    auto rows_of = [&](u64* h, u64* d, int fl) -> Rows {
        Rows r;
        if (flg) { r.h = FLG + (size_t)fl * nb; r.d = FLG + (size_t)(fl + 1) * nb; r.str = 1; }
        else { r.h = G(h) + wo; r.d = G(d) + wo; r.str = wd; }
        return r;
    };
    // the lane's half of the word at LDS byte offset `at` (split layout)
    auto c_get = [&](int at) -> hw { return reinterpret_cast<const uint32_t*>(lds8 + at)[l32]; };
    auto c_put = [&](int at, hw v) { reinterpret_cast<uint32_t*>(lds8 + at)[l32] = v; };
    auto ring_at = [&](int g) -> int { return RING_OFF + (g & (RS - 1)) * STATE_BYTES; };   // state of step g
    auto cslot_h = [&](int g) -> hw { return c_get(ring_at(g)); };
    auto cslot_d = [&](int g) -> hw { return c_get(ring_at(g) + WORD_BYTES); };
    // input k of step g: LANES low halves, then LANES high halves
    uint32_t* iring32 = reinterpret_cast<uint32_t*>(lds8 + IN_OFF);
    auto in32 = [&](int g, int k) -> uint32_t* { return iring32 + ((size_t)(g & (IR - 1)) * NI + k) * (2 * LANES); };
    auto cin = [&](int g, int k) -> hw { return in32(g, k)[l32]; };

    // neighbour j of a record (j >= 2 from the CSR); edge id with LOOP_ENTRY in bit 31
    auto nbr_f = [&](const Rec& r, int j, int& p, uint32_t& e) {
        if (j == 0) { p = r.n0; e = r.e0; return; }
        if (j == 1) { p = r.n1; e = r.e1; return; }
        p = PI[r.ovf + j];
        int ee = PE[r.ovf + j];
        e = (uint32_t)ee | (is_le(c, KD[ee]) ? 0x80000000u : 0u);
    };
    auto nbr_b = [&](const Rec& r, int j) -> int {
        if (j == 0) return r.n0;
        if (j == 1) return r.n1;
        return SI[r.ovf + j];
    };
    // distance of neighbour p from block b in walk order (1 = the block just before)
    auto dist = [&](int b, int p) -> int {
        int pb = b, pp = p;
        if constexpr (!IDORD) { pb = K(c.loff)[b]; pp = K(c.loff)[p]; }
        return BWD ? (pp - pb) : (pb - pp);
    };
    auto blk = [&](int i) -> int { return BWD ? nb - 1 - i : i; };   // (IDORD)
    // At compute time a neighbour at distance 1 is in registers and one at 2..RS in the ring;
    // the first other one ("far": not yet visited in this sweep, or more than RS steps back)
    // comes with the step's inputs.
    // ---------------------------------------------------------------- helper wavefront
    // Each round: plans the steps up to IR ahead of the compute wavefront (one step per lane;
    // each step's descriptor and, when it is not in the rows, its far
    // neighbour's state go to LDS); stores the results the compute wavefront has put in the ring
    // since the last round; copies the other inputs from global memory straight into LDS; waits
    // for all of it; then publishes the inputs and how far the ring may be reused and the rows
    // read.
    // The far neighbour of step s was last computed at step u (this sweep, or the previous one
    // when it is not yet visited): from the rows when u was stored in an earlier round, from the
    // ring when it is computed but not stored yet (its slot is not released before this round
    // ends), the initial value in the first sweep.  Steps whose u is not computed yet wait.
    // step u of the far neighbour's state for step st with entry word x / w (-1: the initial value)
    auto far_step = [&](uint32_t x, int w, int st) -> int {
        return ((x & SF_BACK) && st < nb) ? -1 : st - w;
    };
    auto helper_loop = [&](const Rows& S, u64 init64, auto&& pre) {
        const hw init = (hw)(hi ? init64 >> 32 : init64);
        int gf = 0, fi = 0;   // next step to store and its walk position within the sweep
        int pf = 0, pi = 0;   // next step whose inputs are loaded and its index within the sweep
        uint64_t idle_since = 0;   // wall clock when the helper last found nothing to do (0: busy)
        // Lane j plans step pf + j (walk position pi + j): its step entry is loaded by the lane
        // after the previous round, so that the load is in flight while the helper waits.
        typedef int v4i __attribute__((ext_vector_type(4)));
        const GAS v4i* STV = reinterpret_cast<const GAS v4i*>(G(BWD ? c.step_b : c.step_f));
        v4i ev, xv;   // words 0-3 and 4-7 of the lane's entry
        auto load_entries = [&]() {
            int l = pi + lane;
            while (l >= nb) l -= nb;
            ev = STV[2 * l];
            xv = STV[2 * l + 1];
        };
        load_entries();
        for (;;) {
            const int prod = __builtin_amdgcn_readfirstlane(lds_get(&ctl->produced));
            lds_acquire();
            const int fend = prod < gf + 32 ? prod : gf + 32;
            const int pend = prod < pf ? prod + IR : pf + IR;   // input slots free
            const int gf0 = gf;
            // plan, one step per lane: descriptors, and far values that do not come from the rows
            // (LDS writes only); steps stop at the first one whose far state is not computed yet
            const int st = pf + lane;
            const uint32_t fl = (uint32_t)ev.x;
            const int u = far_step(fl, ev.w, st);
            const bool cand = st < pend;
            const u64 stopm = __ballot(cand && (fl & SF_FAR) && u >= prod);
            const int n = stopm ? (int)__builtin_ctzll(stopm) : pend - pf;
            if (lane < n) {
                const int far_at = IN_OFF + ((st & (IR - 1)) * NI + NX) * WORD_BYTES;
                const uint32_t k0 = fl & 3u, k1 = (fl >> 2) & 3u;
                const int loc0 = k0 == 2 ? ring_at(st - (ev.y & 0xFF)) : k0 == 3 ? far_at : IDENT_OFF;
                const int loc1 = k1 == 2 ? ring_at(st - ((ev.y >> 8) & 0xFF)) : k1 == 3 ? far_at : IDENT_OFF;
                uint32_t dd = fl & DF_MASK;
                dd |= (k0 == 1 ? 1u << DD_LAST0 : 0u) | (k1 == 1 ? 1u << DD_LAST1 : 0u);
                dd |= (k0 ? 1u << DD_P0 : 0u) | (k1 ? 1u << DD_P1 : 0u);
                dd |= (k0 && !(fl & DF_LE0) ? 1u << DD_A0 : 0u) | (k1 && !(fl & DF_LE1) ? 1u << DD_A1 : 0u);
                dring[st & (IR - 1)] = make_int4((int)dd, loc0, loc1, IDORD ? 0 : xv.x);
                if constexpr (!IDORD) blkr[st & (BLK_RING - 1)] = xv.x;
            }
            // far states from the ring (computed, not stored yet) or the initial value
            for (u64 cm = __ballot(lane < n && (fl & SF_FAR) && (u < 0 || u >= gf0)); cm; cm &= cm - 1) {
                const int j = (int)__builtin_ctzll(cm);
                const int uj = __builtin_amdgcn_readlane(u, j);
                const hw h = uj < 0 ? init : cslot_h(uj), d = uj < 0 ? init : cslot_d(uj);
                uint32_t* qq = in32(pf + j, NX) + l32;
                qq[0] = h;
                qq[2 * LANES] = d;
            }
            // nothing to store and nothing that can be loaded yet (the prefetch may also be waiting
            // for a step the compute wavefront will never reach, after its last sweep)
            if (fend == gf && n == 0) {
                if (__builtin_amdgcn_readfirstlane(lds_get(&ctl->done)) &&
                    __builtin_amdgcn_readfirstlane(lds_get(&ctl->produced)) == gf)
                    return;
                if (__builtin_amdgcn_readfirstlane(lds_get(&ctl->abort))) return;
                // the compute wavefront always ends with `done` or `abort`; this bound (no step
                // produced for c.wait_ticks) only keeps the kernel finite
                const uint64_t now = wall_ticks();
                if (!idle_since) idle_since = now;
                else if ((int64_t)(now - idle_since) > (int64_t)c.wait_ticks) {
                    lds_put(&ctl->abort, 1);
                    post_mortem(c.info, PH, fslot, WAIT_PRODUCED, prod, gf + 1, (int64_t)(now - idle_since));
                    return;
                }
                // a compute step takes thousands of cycles: poll less once idle, leaving the
                // issue slots to the other wavefronts of the SIMD
                __builtin_amdgcn_s_sleep(8);
                continue;
            }
            idle_since = 0;
            // results of steps gf .. fend - 1 to the rows, eight ring reads in flight at a time
            while (gf < fend) {
                hw h[8], d[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) { h[t] = cslot_h(gf + t); d[t] = cslot_d(gf + t); }
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    if (gf < fend) {
                        // the block of the step: its walk position, else as planned
                        int b;
                        if constexpr (IDORD) b = blk(fi);
                        else b = __builtin_amdgcn_readfirstlane(blkr[gf & (BLK_RING - 1)]);
                        if (act) S.st32(b, hi, h[t], d[t]);
                        fi = fi + 1 == nb ? 0 : fi + 1;
                        ++gf;
                    }
                }
            }
            // the other inputs: copies from global memory straight into the input slots (no LDS read
            // follows them before the wait); far rows past the first-level cache (the helper stored them)
            // per step, worked out by its plan lane: the LDS address of its input slots, whether a
            // block with one neighbour skips the second edge's rows, whether the far state comes
            // from the rows
            const uint32_t slotv = lds3 + IN_OFF + (uint32_t)((st & (IR - 1)) * NI) * WORD_BYTES;
            const u64 onem = __ballot(fl & SF_ONE);
            const u64 rowm = __ballot((fl & SF_FAR) && u >= 0 && u < gf0);
            // and the byte offsets of its block's row and of its first two edges' rows
            const u64 rowb = (u64)wd * 8u;
            const u64 obv = (uint32_t)xv.x * rowb, oe0v = (uint32_t)xv.y * rowb, oe1v = (uint32_t)xv.z * rowb;
            auto at = [&](u64 v, int j) -> u64 {
                return (u64)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, j) |
                       ((u64)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), j) << 32);
            };
            for (int j = 0; j < n; ++j) {
                const int sj = pf + j;
                const GAS u64* a[NX];
                pre(at(obv, j), at(oe0v, j), at(oe1v, j), a);
                const uint32_t slot = (uint32_t)__builtin_amdgcn_readlane((int)slotv, j);
                // (a block with one neighbour never reads the second edge's slots)
                const int nx = ((onem >> j) & 1) ? NX1 : NX;
#pragma unroll
                for (int k = 0; k < NX; ++k)
                    if (k < nx) dma_row<0>(a[k], hoff, (LDS3 char*)(size_t)(slot + k * WORD_BYTES));
                if ((rowm >> j) & 1) {
                    const int p = __builtin_amdgcn_readlane(ev.z, j);
                    dma_word<CPOL_SC1>(S.h + (size_t)p * S.str, hi, in32(sj, NX));
                    dma_word<CPOL_SC1>(S.d + (size_t)p * S.str, hi, in32(sj, NX + 1));
                }
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            lds_release();
            lds_put(&ctl->consumed, gf);
            lds_put(&ctl->flushed, gf);
            pf += n;
            pi += n;
            while (pi >= nb) pi -= nb;
            lds_put(&ctl->in_ready, pf);
            if (n) load_entries();
        }
    };

    // ---------------------------------------------------------------- compute wavefront
    int gbase = 0;          // global step index of the current sweep's first step
    int cons = 0, flsh = 0, inr = 0;   // last seen helper progress
    bool ok = true;
    // wait (bounded) until the helper's counter *p exceeds g; `seen` caches its last value
    auto need = [&](int* p, int& seen, int g) {
        if (seen > g) return;
        seen = __builtin_amdgcn_readfirstlane(lds_get(p));
        if (seen > g) { lds_acquire(); return; }
        int last = 0;
        int64_t waited = 0;
        if (!wait_for(p, g + 1, &ctl->abort, c.wait_ticks, last, waited)) {
            ok = false;
            if (waited >= 0)
                post_mortem(c.info, PH, fslot,
                            p == &ctl->in_ready ? WAIT_IN_READY : p == &ctl->consumed ? WAIT_CONSUMED : WAIT_FLUSHED,
                            last, g + 1, waited);
        }
        seen = g + 1;
    };
    // neighbour p at distance d of the block of step g, from the rows: the previous sweep's (or
    // the initial value in sweep 0) for a block not yet visited, this sweep's for one visited
    // more than RS steps ago
    auto far_val = [&](const Rows& S, int p, int d, int g, int sweep, hw init, hw& h, hw& dd) {
        if (d <= 0 && sweep == 0) { h = init; dd = init; return; }
        if (d > 0) need(&ctl->flushed, flsh, g - d);
        h = settle(S.ldh32(p, hi));
        dd = settle(S.ldd32(p, hi));
    };

    // One sweep.  fast(x, nh, nd, fl, vh, vd) computes the new state of an ordinary block (not
    // ENTRY, EXIT or a call, at most two neighbours, at most one of them far) from its inputs x,
    // its step flags and its first two neighbours' states (`ident` for a missing one);
    // comp(b, r, x, nh, nd, ph, pd, sweep, g, vh, vd) computes any block.
    // The walk is pipelined: while step g computes, the reads of step g + 1's inputs and of the
    // states of its neighbours other than the block computed last (a ring slot or the far
    // input) are in flight, and so is the read of step g + 3's descriptor; step g + 2's
    // descriptor, read during step g - 1, is decoded after step g.  LDS completes a wavefront's
    // accesses in order, so waiting for older reads leaves the newer ones in flight; the
    // counters are read before the next step's reads are issued, since a wait for a counter
    // also waits for every LDS access before it.
    auto desc = [&](int g, uint32_t& fl, int& l0, int& l1) {
        const int4 dn = dring[g & (IR - 1)];
        fl = (uint32_t)__builtin_amdgcn_readfirstlane(dn.x);
        l0 = __builtin_amdgcn_readfirstlane(dn.y);
        l1 = __builtin_amdgcn_readfirstlane(dn.z);
    };
    // inputs of step g and the states at its neighbours' locations (no branch: a missing
    // neighbour and the block computed last point at the identity state)
    auto fetch = [&](int g, int l0, int l1, hw* x, hw* nh, hw* nd) {
#pragma unroll
        for (int k = 0; k < NX; ++k) x[k] = cin(g, k);
        nh[0] = c_get(l0); nd[0] = c_get(l0 + WORD_BYTES);
        nh[1] = c_get(l1); nd[1] = c_get(l1 + WORD_BYTES);
    };
    auto walk = [&](const Rows& S, hw init, int sweep, uint32_t& pc, auto&& fast, auto&& comp) {
        hw ph = init, pd = init;   // state of the block computed last
        uint32_t fl0, fl1 = 0;      // flags of steps g and g + 1
        int a0, b0, a1 = IDENT_OFF, b1 = IDENT_OFF;
        int4 dq2 = make_int4(0, IDENT_OFF, IDENT_OFF, 0);   // descriptor of step g + 2, not decoded
        // two sets of step inputs, used in turn (the loop below runs two steps per round)
        hw xa[NX], nha[2], nda[2], xb[NX], nhb[2], ndb[2];
        need(&ctl->in_ready, inr, gbase);
        desc(gbase, fl0, a0, b0);
        fetch(gbase, a0, b0, xa, nha, nda);
        if (nb > 1) {
            need(&ctl->in_ready, inr, gbase + 1);
            desc(gbase + 1, fl1, a1, b1);
        }
        if (nb > 2) {
            need(&ctl->in_ready, inr, gbase + 2);
            dq2 = dring[(gbase + 2) & (IR - 1)];
        }
        // step gbase + i with its inputs in (x, nh, nd); the next step's go to (y, ny, nz)
        auto step = [&](int i, const hw* x, const hw* nh, const hw* nd, hw* y, hw* ny, hw* nz) {
            const int g = gbase + i;
            const uint32_t fl = fl0;
            // the ring slot of step g was last used by step g - RS: the helper must have read it
            need(&ctl->consumed, cons, g - RS);
            int4 dq3 = make_int4(0, IDENT_OFF, IDENT_OFF, 0);
            if (i + 3 < nb) {
                need(&ctl->in_ready, inr, g + 3);
                dq3 = dring[(g + 3) & (IR - 1)];
            }
            if (i + 1 < nb) fetch(g + 1, a1, b1, y, ny, nz);
            hw vh_[2], vd_[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const hw last = fmask(fl, DD_LAST0 + j);
                vh_[j] = (ph & last) | (nh[j] & ~last);
                vd_[j] = (pd & last) | (nd[j] & ~last);
            }
            hw vh, vd;
            if (!(fl & DF_SLOW)) fast(x, vh_, vd_, fl, vh, vd);
            else {
                // any block: neighbour values by the general rule, then the full transfer
                const int b = IDORD ? blk(i) : __builtin_amdgcn_readfirstlane(dring[g & (IR - 1)].w);
                const Rec r = ldrec(REC, b);
                const int cnt = (int)(r.meta & REC_COUNT);
                bool far_used = false;
                for (int j = 0; j < 2; ++j) {
                    vh_[j] = 0; vd_[j] = 0;
                    if (j >= cnt) continue;
                    const int p = j == 0 ? r.n0 : r.n1, d = dist(b, p);
                    if (d == 1) { vh_[j] = ph; vd_[j] = pd; }
                    else if (d >= 2 && d <= RS) { vh_[j] = cslot_h(g - d); vd_[j] = cslot_d(g - d); }
                    else if (!far_used) { vh_[j] = cin(g, NX); vd_[j] = cin(g, NX + 1); far_used = true; }
                    else far_val(S, p, d, g, sweep, init, vh_[j], vd_[j]);
                }
                comp(b, r, x, vh_, vd_, ph, pd, sweep, g, vh, vd);
            }
            pc += (uint32_t)(__popc(vh) + __popc(vd));
            c_put(ring_at(g), vh);
            c_put(ring_at(g) + WORD_BYTES, vd);
            // the state goes before the counter (program order; LDS keeps it)
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            lds_put(&ctl->produced, g + 1);
            ph = vh; pd = vd;
            fl0 = fl1;
            fl1 = (uint32_t)__builtin_amdgcn_readfirstlane(dq2.x);
            a1 = __builtin_amdgcn_readfirstlane(dq2.y);
            b1 = __builtin_amdgcn_readfirstlane(dq2.z);
            dq2 = dq3;
        };
        for (int i = 0; i < nb; i += 2) {
            step(i, xa, nha, nda, xb, nhb, ndb);
            if (i + 1 >= nb) break;
            step(i + 1, xb, nhb, ndb, xa, nha, nda);
        }
    };
    bool recheck = false;   // the transfer functions run for the re-check: every state from the rows
    // a neighbour beyond the first two, at compute time (g = the current step)
    auto extra = [&](const Rows& S, int b, int p, int sweep, int g, hw init, hw ph, hw pd, hw& h, hw& d) {
        if (recheck) { h = settle(S.ldh32(p, hi)); d = settle(S.ldd32(p, hi)); return; }
        const int dd = dist(b, p);
        if (dd == 1) { h = ph; d = pd; }
        else if (dd >= 2 && dd <= RS) { h = cslot_h(g - dd); d = cslot_d(g - dd); }
        else far_val(S, p, dd, g, sweep, init, h, d);
    };
    // After a sweep whose states are all in the rows: would the next sweep change nothing?  It
    // reads the same states as this one except where a block reads a neighbour it has not yet
    // visited in the sweep (that neighbour's previous-sweep state); so if every block of the
    // re-check list, evaluated again from the states this sweep left, keeps its state, then by
    // induction along the walk the next sweep repeats this one and the states are the fixed
    // point.  Stops at the first block that would change.
    auto settled = [&](const Rows& S, auto&& pre, auto&& comp) -> bool {
        const GAS int32_t* L = reinterpret_cast<const GAS int32_t*>(G(BWD ? c.step_b : c.step_f)) + 7;
        const u64 rowb = (u64)wd * 8u;
        // a listed block with what its evaluation reads: its record, the phase's input rows, its
        // first two neighbours' states and its own (the next block's loads are issued before
        // the current one is evaluated)
        struct Item { int b; Rec r; hw x[NX], nh[2], nd[2], oh, od; };
        // (rv: the records of the current entries, one per lane)
        auto load = [&](int b, const Rec& rv, int k, Item& t) {
            t.b = b;
            t.r.meta = (uint32_t)__builtin_amdgcn_readlane((int)rv.meta, k);
            t.r.n0 = __builtin_amdgcn_readlane(rv.n0, k);
            t.r.n1 = __builtin_amdgcn_readlane(rv.n1, k);
            t.r.e0 = (uint32_t)__builtin_amdgcn_readlane((int)rv.e0, k);
            t.r.e1 = (uint32_t)__builtin_amdgcn_readlane((int)rv.e1, k);
            t.r.ovf = __builtin_amdgcn_readlane(rv.ovf, k);
            t.r.ci = __builtin_amdgcn_readlane(rv.ci, k);
            t.r.pad = 0;
            const int cnt = (int)(t.r.meta & REC_COUNT);
            const GAS u64* a[NX];
            pre((u64)(uint32_t)b * rowb, cnt > 0 ? (u64)(t.r.e0 & 0x7FFFFFFFu) * rowb : 0ull,
                cnt > 1 ? (u64)(t.r.e1 & 0x7FFFFFFFu) * rowb : 0ull, a);
#pragma unroll
            for (int k2 = 0; k2 < NX; ++k2)   // (a block with one neighbour has no second edge)
                t.x[k2] = (k2 < NX1 || cnt > 1)
                              ? reinterpret_cast<const GAS uint32_t*>(reinterpret_cast<const GAS char*>(a[k2]) + hoff)[0]
                              : 0u;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int p = j ? t.r.n1 : t.r.n0;
                t.nh[j] = j < cnt ? S.ldh32(p, hi) : 0u;
                t.nd[j] = j < cnt ? S.ldd32(p, hi) : 0u;
            }
            t.oh = S.ldh32(b, hi);
            t.od = S.ldd32(b, hi);
        };
        bool same = true;
        recheck = true;
        // (2 LANES entries at a time: the walk runs on lanes 0 .. 2 LANES - 1 only)
        for (int j0 = 0; j0 < nb && same; j0 += 2 * LANES) {
            const int lb = j0 + l32 < nb ? L[8 * (size_t)(j0 + l32)] : -1;
            // (the list is a prefix of the entries)
            const int n = __popcll(__ballot(lb >= 0) & ((1ull << (2 * LANES)) - 1ull));
            if (n == 0) break;
            const Rec rv = ldrec_v(REC, lb >= 0 ? lb : 0);
            // two items used in turn (two blocks per round, so nothing is copied between them and
            // the next block's loads stay in flight while the current one is evaluated)
            auto changes = [&](const Item& t) -> bool {
                hw vh, vd;
                comp(t.b, t.r, t.x, t.nh, t.nd, 0u, 0u, 1, 0, vh, vd);
                return __ballot(act && (vh != t.oh || vd != t.od)) != 0ull;
            };
            Item ia, ib;
            load(__builtin_amdgcn_readlane(lb, 0), rv, 0, ia);
            for (int k = 0; k < n; k += 2) {
                if (k + 1 < n) load(__builtin_amdgcn_readlane(lb, k + 1), rv, k + 1, ib);
                if (changes(ia)) { same = false; break; }
                if (k + 1 >= n) break;
                if (k + 2 < n) load(__builtin_amdgcn_readlane(lb, k + 2), rv, k + 2, ia);
                if (changes(ib)) { same = false; break; }
            }
            if (n < 2 * LANES) break;
        }
        recheck = false;
        return same;
    };
    // Run a phase: the compute wavefront sweeps, the helper feeds and stores; false on an error.
    // (init64: the initial state of the lane's word; ident64: the state of a missing neighbour)
    auto run_phase = [&](const Rows& S, u64 init64, u64 ident64, auto&& pre, auto&& fast, auto&& comp) -> bool {
        if (helper) {
            helper_loop(S, init64, pre);
            return true;
        }
        const hw init = (hw)(hi ? init64 >> 32 : init64), ident = (hw)ident64;
        c_put(IDENT_OFF, ident);
        c_put(IDENT_OFF + WORD_BYTES, ident);
        int sweeps = 0;
        uint32_t last = (uint32_t)nb * 2u * (uint32_t)__popc(init);
        bool good = true;
        for (;;) {
            uint32_t pc = 0;
            walk(S, init, sweeps, pc, fast, comp);
            gbase += nb;
            ++sweeps;
            // the next sweep reads this sweep's rows for blocks it has not visited yet
            need(&ctl->flushed, flsh, gbase - 1);
            if (!ok) break;
            const bool ch = act && pc != last;
            last = pc;
            if (__ballot(ch) == 0ull) break;
            if (settled(S, pre, comp)) break;
            if (sweeps >= cap) {
                if (lane == 0) set_status(c.info, OMPD_E_NOCONVERGE_);
                good = false;
                break;
            }
        }
        lds_put(&ctl->done, 1);
        if (!ok) {
            if (lane == 0) set_status(c.info, OMPD_E_DEVICE_);
            return false;
        }
        if (lane == 0) atomicMax(&c.info[INFO_SWEEPS + PH], sweeps);
        return good;
    };
    // NUout of a call block: OR over its successors' next use (final)
    auto nu_after = [&](int b, hw& lh, hw& ld) {
        const Rec rb = ldrec(c.rec_b, b);
        const int cnt = (int)(rb.meta & REC_COUNT);
        lh = 0; ld = 0;
        for (int j = 0; j < cnt; ++j) {
            int q = nbr_b(rb, j);
            lh |= settle(row(c.nu_h, q));
            ld |= settle(row(c.nu_d, q));
        }
    };
    // validity transfer of block b (a call applies the callee's exit-validity
    // tables to the validity after the block's own accesses and the next use after the call)
    auto valid_out = [&](int b, const Rec& r, hw ih, hw id, hw wr, hw rr, hw& oh, hw& od) {
        const bool dev = r.meta & REC_DEV;
        hw ah = dev ? (ih & ~wr) : (ih | wr);
        hw ad = dev ? ((id | wr) & ~(rr & fph)) : (id & ~wr);
        if (r.meta & REC_CALL) {
            hw lh, ld;
            nu_after(b, lh, ld);
            const int ci = r.ci;   // the flag lane passes through (identity tables)
            const hw th = tsel(ah, lh, sum(ci, SUM_TH + 0), sum(ci, SUM_TH + 1), sum(ci, SUM_TH + 2), sum(ci, SUM_TH + 3));
            const hw td = tsel(ad, ld, sum(ci, SUM_TD + 0), sum(ci, SUM_TD + 1), sum(ci, SUM_TD + 2), sum(ci, SUM_TD + 3));
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
        // x0 = R, x1 = W (flag lane: R = 2, W = 2 at DEVICE blocks, substituted when computed)
        auto pre = [&](u64 ob, u64, u64, const GAS u64** x) {
            x[0] = rowu(c.R, ob);
            x[1] = rowu(c.W, ob);
        };
        auto comp = [&](int b, const Rec& r, const hw* x, const hw* nh, const hw* nd, hw ph, hw pd, int sweep,
                        int g, hw& vh, hw& vd) {
            if (r.meta & REC_EXIT) {
                const hw lh = vec(c.lx_h), ld = vec(c.lx_d);
                vh = flg ? lo(1) : lh;
                vd = flg ? 0u : ld;
                return;
            }
            const int cnt = (int)(r.meta & REC_COUNT);
            hw oh = nh[0] | nh[1], od = nd[0] | nd[1];
            for (int j = 2; j < cnt; ++j) {
                hw h, d;
                extra(S, b, nbr_b(r, j), sweep, g, 0u, ph, pd, h, d);
                oh |= h; od |= d;
            }
            const bool dev = r.meta & REC_DEV;
            const hw rr = flg ? lo(2) : x[0], ww = flg ? (dev ? lo(2) : 0u) : x[1];
            if (r.meta & REC_CALL) {
                const int ci = r.ci;   // the flag lane passes through (NU0 = 0, NU1 = all ones)
                const hw ch = sum(ci, SUM_NU0_H) | (sum(ci, SUM_NU1_H) & oh);
                const hw cd = sum(ci, SUM_NU0_D) | (sum(ci, SUM_NU1_D) & od);
                oh = flg ? oh : ch;
                od = flg ? od : cd;
            }
            vh = (dev ? (rr & fph) : rr) | (~ww & oh);
            vd = (dev ? (rr & ~fph) : 0u) | (~ww & od);
        };
        auto fast = [&](const hw* x, const hw* nh, const hw* nd, uint32_t fl, hw& vh, hw& vd) {
            const hw dev = fmask(fl, DD_DEV);
            const hw rr = flg ? lo(2) : x[0], ww = flg ? (lo(2) & dev) : x[1];
            const hw oh = nh[0] | nh[1], od = nd[0] | nd[1];
            vh = (rr & (~dev | fph)) | (~ww & oh);
            vd = (rr & dev & ~fph) | (~ww & od);
        };
        run_phase(S, 0ull, 0ull, pre, fast, comp);
        return;
    }

    // ------------------------------------------------------------ validity with eager copies (forward, must)
    // AVEout_s(q) = transfer of AVEin_s(q) = NUin_s(q) | AND over preds AVEout_s(p); AVEin(ENTRY) = boundary.
    if constexpr (PH == PH_AVE) {
        const Rows S = rows_of(c.aveout_h, c.aveout_d, 2);
        const hw init = vm;
        // x0/x1 = NU (flag lane: 0), x2 = W (flag lane: 2 at DEVICE blocks), substituted when computed,
        // x3 = R (the firstprivate reads of a kernel)
        auto pre = [&](u64 ob, u64, u64, const GAS u64** x) {
            x[0] = rowu(c.nu_h, ob);
            x[1] = rowu(c.nu_d, ob);
            x[2] = rowu(c.W, ob);
            x[3] = rowu(c.R, ob);
        };
        auto comp = [&](int b, const Rec& r, const hw* x, const hw* nh, const hw* nd, hw ph, hw pd, int sweep,
                        int g, hw& vh, hw& vd) {
            hw ih, id;
            if (r.meta & REC_ENTRY) {
                const hw eh = vec(c.ev_h), ed = vec(c.ev_d);
                ih = flg ? lo(2) : eh;
                id = flg ? 0u : ed;
            } else {
                const int cnt = (int)(r.meta & REC_COUNT);
                // meet over the predecessors (all ones over none: a block no edge enters)
                hw mh = cnt == 0 ? ~0u : cnt > 1 ? (nh[0] & nh[1]) : nh[0];
                hw md = cnt == 0 ? ~0u : cnt > 1 ? (nd[0] & nd[1]) : nd[0];
                for (int j = 2; j < cnt; ++j) {
                    int p; uint32_t e;
                    nbr_f(r, j, p, e);
                    hw h, d;
                    extra(S, b, p, sweep, g, init, ph, pd, h, d);
                    mh &= h; md &= d;
                }
                ih = (flg ? 0u : x[0]) | mh;
                id = (flg ? 0u : x[1]) | md;
            }
            valid_out(b, r, ih & vm, id & vm, flg ? ((r.meta & REC_DEV) ? lo(2) : 0u) : x[2], x[3], vh, vd);
        };
        auto fast = [&](const hw* x, const hw* nh, const hw* nd, uint32_t fl, hw& vh, hw& vd) {
            const hw dev = fmask(fl, DD_DEV);
            const hw ih = ((flg ? 0u : x[0]) | (nh[0] & nh[1])) & vm, id = ((flg ? 0u : x[1]) | (nd[0] & nd[1])) & vm;
            const hw wr = flg ? (lo(2) & dev) : x[2];
            vh = ((ih & ~wr & dev) | ((ih | wr) & ~dev)) & vm;
            vd = (((id | wr) & dev & ~(x[3] & fph)) | (id & ~wr & ~dev)) & vm;
        };
        if (!run_phase(S, vm64, ~0ull, pre, fast, comp)) return;
        if (helper) return;
        // reachability: every block reached from ENTRY and reaching EXIT
        bool bad = false;
        for (int b = l32; b < nb; b += 2 * LANES) {
            const u64 fnu = ld_fresh(FLG + b), fave = ld_fresh(FLG + (size_t)2 * nb + b);
            const u64 fnud = ld_fresh(FLG + (size_t)nb + b);
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
    auto use_wr = [&](int b, const Rec& r, hw rr, hw ww, hw& uh, hw& ud, hw& sh, hw& sd) {
        const bool dev = r.meta & REC_DEV;
        if (r.meta & REC_EXIT) { uh = vec(c.lx_h); ud = vec(c.lx_d); sh = uh; sd = ud; return; }
        uh = dev ? (rr & fph) : rr;
        ud = dev ? (rr & ~fph) : 0u;
        if (r.meta & REC_CALL) {
            const int ci = r.ci;
            hw mw = sum(ci, SUM_MAYW_H) | sum(ci, SUM_MAYW_D);
            uh |= sum(ci, SUM_MAYR_H) | mw;
            ud |= sum(ci, SUM_MAYR_D) | mw;
        }
        sh = uh | (dev ? 0u : ww);
        sd = ud | (dev ? ww : 0u);
    };
    auto erow = [&](const u64* a, uint32_t e) -> hw { return half(G(a) + (size_t)(e & 0x7FFFFFFFu) * wd + wo); };
    auto erowu = [&](const u64* a, u64 oe) -> const GAS u64* {
        return reinterpret_cast<const GAS u64*>(reinterpret_cast<const GAS char*>(G(a)) + oe);
    };

    // -------------------------------------------------------- pending copies (forward, may)
    // MAYP_s(e) = (EAG_s(e) | MAYPout_s(p)) & ~LE(e), EAG_s(e=p->q) = NU_s(q) & ~AVEout_s(p);
    // MAYPout_s(q) = OR_e MAYP_s(e) & ~USE'_s(q) & ~WR_s(q)
    if constexpr (PH == PH_MAYP) {
        if (c.placement & PL_EAGER) return;
        const Rows S = rows_of(c.mayp_h, c.mayp_d, 0);
        // x0 = R, x1 = W, x2..x5 = EAG_H/D of the two inline in-edges
        // (the second edge's rows are not loaded for a block with one neighbour)
        auto pre = [&](u64 ob, u64 oe0, u64 oe1, const GAS u64** x) {
            x[0] = rowu(c.R, ob); x[1] = rowu(c.W, ob);
            x[2] = erowu(c.eag_h, oe0); x[3] = erowu(c.eag_d, oe0);
            x[4] = erowu(c.eag_h, oe1); x[5] = erowu(c.eag_d, oe1);
        };
        auto comp = [&](int b, const Rec& r, const hw* x, const hw* nh, const hw* nd, hw ph, hw pd, int sweep,
                        int g, hw& vh, hw& vd) {
            if (r.meta & REC_ENTRY) { vh = 0; vd = 0; return; }
            const int cnt = (int)(r.meta & REC_COUNT);
            hw mh = 0, md = 0;
            for (int j = 0; j < cnt; ++j) {
                int p; uint32_t e;
                nbr_f(r, j, p, e);
                if (e & 0x80000000u) continue;   // loop entry: nothing stays pending
                hw gh, gd, sh, sd;
                if (j < 2) {   // (selects, not indexing: the arrays stay in registers)
                    gh = j ? x[4] : x[2]; gd = j ? x[5] : x[3]; sh = j ? nh[1] : nh[0]; sd = j ? nd[1] : nd[0];
                }
                else {
                    gh = settle(erow(c.eag_h, e)); gd = settle(erow(c.eag_d, e));
                    extra(S, b, p, sweep, g, 0u, ph, pd, sh, sd);
                }
                mh |= gh | sh;
                md |= gd | sd;
            }
            hw uh, ud, sth, std_;
            use_wr(b, r, x[0], x[1], uh, ud, sth, std_);
            vh = mh & ~sth & vm;
            vd = md & ~std_ & vm;
        };
        // (the stop masks of an ordinary block: its own accesses)
        auto fast = [&](const hw* x, const hw* nh, const hw* nd, uint32_t fl, hw& vh, hw& vd) {
            const hw dev = fmask(fl, DD_DEV), t0 = fmask(fl, DD_A0), t1 = fmask(fl, DD_A1);
            const hw mh = ((x[2] | nh[0]) & t0) | ((x[4] | nh[1]) & t1);
            const hw md = ((x[3] | nd[0]) & t0) | ((x[5] | nd[1]) & t1);
            const hw sth = ((x[0] | x[1]) & ~dev) | (x[0] & fph & dev), std_ = ((x[0] & ~fph) | x[1]) & dev;
            vh = mh & ~sth & vm;
            vd = md & ~std_ & vm;
        };
        run_phase(S, 0ull, 0ull, pre, fast, comp);
        return;
    }

    // -------------------------------------------------------- delayed placement (forward, LFP)
    // LATER_s(e) = EAG_s(e) | LATERout_s(p); L'_s(e) = LATER_s(e) & ~LE(e)
    // N'_s(e) = BOTH(e) | (LATER_s(e) & LE(e)), BOTH(e) = FV_H(e) & FV_D(e)
    // LATERin_s(q) = AND_e (L'_s | N'_s) & OR_e L'_s; LATERout_s(q) = LATERin_s(q) & ~USE'_s(q) & ~WR_s(q)
    // (the copies themselves are materialised after the phase)
    if constexpr (PH == PH_LATER) {
        if (c.placement & PL_EAGER) return;
        const Rows S = rows_of(c.later_h, c.later_d, 0);
        // x0 = R, x1 = W, x2..x4 / x5..x7 = EAG_H, EAG_D, BOTH of the two inline in-edges
        auto pre = [&](u64 ob, u64 oe0, u64 oe1, const GAS u64** x) {
            x[0] = rowu(c.R, ob); x[1] = rowu(c.W, ob);
            x[2] = erowu(c.eag_h, oe0); x[3] = erowu(c.eag_d, oe0); x[4] = erowu(c.both, oe0);
            x[5] = erowu(c.eag_h, oe1); x[6] = erowu(c.eag_d, oe1); x[7] = erowu(c.both, oe1);
        };
        auto comp = [&](int b, const Rec& r, const hw* x, const hw* nh, const hw* nd, hw ph, hw pd, int sweep,
                        int g, hw& vh, hw& vd) {
            if (r.meta & REC_ENTRY) { vh = 0; vd = 0; return; }
            hw uh, ud, sth, std_;
            use_wr(b, r, x[0], x[1], uh, ud, sth, std_);
            const int cnt = (int)(r.meta & REC_COUNT);
            hw allh = ~0u, alld = ~0u, anyh = 0, anyd = 0;
            for (int j = 0; j < cnt; ++j) {
                int p; uint32_t e;
                nbr_f(r, j, p, e);
                hw gh, gd, bo, sh, sd;
                if (j < 2) {
                    gh = j ? x[5] : x[2]; gd = j ? x[6] : x[3]; bo = j ? x[7] : x[4];
                    sh = j ? nh[1] : nh[0]; sd = j ? nd[1] : nd[0];
                }
                else {
                    gh = settle(erow(c.eag_h, e)); gd = settle(erow(c.eag_d, e)); bo = settle(erow(c.both, e));
                    extra(S, b, p, sweep, g, 0u, ph, pd, sh, sd);
                }
                const hw le = (e & 0x80000000u) ? ~0u : 0u;
                const hw lh = gh | sh, ld = gd | sd;
                const hw lph = lh & ~le, lpd = ld & ~le;
                allh &= lph | bo | (lh & le);
                alld &= lpd | bo | (ld & le);
                anyh |= lph;
                anyd |= lpd;
            }
            vh = allh & anyh & vm & ~sth;
            vd = alld & anyd & vm & ~std_;
        };
        // (per edge, (L & ~LE) | N' = L | BOTH whatever LE is; only the OR term skips loop entries)
        auto fast = [&](const hw* x, const hw* nh, const hw* nd, uint32_t fl, hw& vh, hw& vd) {
            const hw dev = fmask(fl, DD_DEV), a0 = fmask(fl, DD_A0);
            const hw sth = ((x[0] | x[1]) & ~dev) | (x[0] & fph & dev), std_ = ((x[0] & ~fph) | x[1]) & dev;
            const hw l0h = x[2] | nh[0], l0d = x[3] | nd[0];
            if ((fl & (3u << DD_P0)) == (1u << DD_P0)) {
                // one predecessor: its term is both the AND and (unless the edge enters a loop) the OR
                vh = l0h & a0 & vm & ~sth;
                vd = l0d & a0 & vm & ~std_;
                return;
            }
            const hw p0 = fmask(fl, DD_P0), p1 = fmask(fl, DD_P1), a1 = fmask(fl, DD_A1);
            const hw l1h = x[5] | nh[1], l1d = x[6] | nd[1];
            const hw allh = (l0h | x[4] | ~p0) & (l1h | x[7] | ~p1);
            const hw alld = (l0d | x[4] | ~p0) & (l1d | x[7] | ~p1);
            const hw anyh = (l0h & a0) | (l1h & a1), anyd = (l0d & a0) | (l1d & a1);
            vh = allh & anyh & vm & ~sth;
            vd = alld & anyd & vm & ~std_;
        };
        run_phase(S, 0ull, 0ull, pre, fast, comp);
        return;
    }

    // ------------------------------------------------------------ loop-entry refinement (backward, may)
    // Is the value in space s at b's entry read before a write or a copy into s replaces it:
    // A_s(b) = READ_s(b) | (LO_s(b) & ~KILL_s(b)), LI_s(b) = (A_s(b) & ~INS_ENTRY_s(b)) | INS_ENTRY_o(b),
    // LO_s(b) = OR over out-edges e = b->t of (LI_s(t) & ~INS_EDGE_s(e)) | INS_EDGE_o(e)  (a copy reads
    // its source); READ at EXIT: the liveness after it, at a call: everything; KILL: a write in s,
    // and a kernel's firstprivate read for the device copy.  The state uses the pending-copy rows.
    if constexpr (PH == PH_LIVE) {
        if (!refines(c.placement)) return;
        const Rows S = rows_of(c.mayp_h, c.mayp_d, 0);
        // x0 = R, x1 = W, x2/x3 = INS_ENTRY_H/D, x4..x7 = INS_EDGE_H/D of the first two out-edges
        auto pre = [&](u64 ob, u64 oe0, u64 oe1, const GAS u64** x) {
            x[0] = rowu(c.R, ob); x[1] = rowu(c.W, ob); x[2] = rowu(c.ie_h, ob); x[3] = rowu(c.ie_d, ob);
            x[4] = erowu(c.ig_h, oe0); x[5] = erowu(c.ig_d, oe0);
            x[6] = erowu(c.ig_h, oe1); x[7] = erowu(c.ig_d, oe1);
        };
        auto comp = [&](int b, const Rec& r, const hw* x, const hw* nh, const hw* nd, hw ph, hw pd, int sweep,
                        int g, hw& vh, hw& vd) {
            const int cnt = (int)(r.meta & REC_COUNT);
            hw oh = 0, od = 0;
            for (int j = 0; j < cnt; ++j) {
                hw sh, sd, gh, gd;
                if (j < 2) {
                    sh = j ? nh[1] : nh[0]; sd = j ? nd[1] : nd[0]; gh = j ? x[6] : x[4]; gd = j ? x[7] : x[5];
                }
                else {
                    const uint32_t e = (uint32_t)(r.ovf + j);
                    gh = settle(erow(c.ig_h, e)); gd = settle(erow(c.ig_d, e));
                    extra(S, b, nbr_b(r, j), sweep, g, 0u, ph, pd, sh, sd);
                }
                oh |= (sh & ~gh) | gd;
                od |= (sd & ~gd) | gh;
            }
            const bool dev = r.meta & REC_DEV;
            hw rh, rd, kh = 0u, kd = 0u;
            if (r.meta & REC_EXIT) { rh = vec(c.lx_h); rd = vec(c.lx_d); }
            else if (r.meta & REC_CALL) { rh = ~0u; rd = ~0u; }
            else {
                const hw rr = x[0], ww = x[1];
                rh = dev ? (rr & fph) : rr;
                rd = dev ? (rr & ~fph) : 0u;
                kh = dev ? 0u : ww;
                kd = dev ? (ww | (rr & fph)) : 0u;
            }
            const hw ah = rh | (oh & ~kh), ad = rd | (od & ~kd);
            vh = ((ah & ~x[2]) | x[3]) & vm;
            vd = ((ad & ~x[3]) | x[2]) & vm;
        };
        // (a missing second out-edge's rows are not loaded: masked by its presence bit)
        auto fast = [&](const hw* x, const hw* nh, const hw* nd, uint32_t fl, hw& vh, hw& vd) {
            const hw dev = fmask(fl, DD_DEV), p0 = fmask(fl, DD_P0), p1 = fmask(fl, DD_P1);
            const hw oh = (((nh[0] & ~x[4]) | x[5]) & p0) | (((nh[1] & ~x[6]) | x[7]) & p1);
            const hw od = (((nd[0] & ~x[5]) | x[4]) & p0) | (((nd[1] & ~x[7]) | x[6]) & p1);
            const hw rr = x[0], ww = x[1];
            const hw rh = rr & (~dev | fph), rd = rr & dev & ~fph;
            const hw kh = ww & ~dev, kd = (ww | (rr & fph)) & dev;
            const hw ah = rh | (oh & ~kh), ad = rd | (od & ~kd);
            vh = ((ah & ~x[2]) | x[3]) & vm;
            vd = ((ad & ~x[3]) | x[2]) & vm;
        };
        run_phase(S, 0ull, 0ull, pre, fast, comp);
        return;
    }

    // ------------------------------------------------------------ validity after placement (forward, must)
    // AVFout_s(q) = transfer of AVFin_s(q) = INS_ENTRY_s(q) | AND_e (AVFout_s(p) | INS_EDGE_s(e));
    // the state reuses the eager-validity rows.
    if constexpr (PH == PH_AVF) {
        const Rows S = rows_of(c.aveout_h, c.aveout_d, 2);
        const hw init = vm;
        // x0/x1 = INS_ENTRY, x2 = W, x3 = R, x4..x7 = INS_EDGE_H/D of the two inline in-edges
        auto pre = [&](u64 ob, u64 oe0, u64 oe1, const GAS u64** x) {
            x[0] = rowu(c.ie_h, ob); x[1] = rowu(c.ie_d, ob); x[2] = rowu(c.W, ob); x[3] = rowu(c.R, ob);
            x[4] = erowu(c.ig_h, oe0); x[5] = erowu(c.ig_d, oe0);
            x[6] = erowu(c.ig_h, oe1); x[7] = erowu(c.ig_d, oe1);
        };
        auto comp = [&](int b, const Rec& r, const hw* x, const hw* nh, const hw* nd, hw ph, hw pd, int sweep,
                        int g, hw& vh, hw& vd) {
            hw ih, id;
            if (r.meta & REC_ENTRY) { ih = vec(c.ev_h); id = vec(c.ev_d); }
            else {
                const int cnt = (int)(r.meta & REC_COUNT);
                hw mh = ~0u, md = ~0u;
                for (int j = 0; j < cnt; ++j) {
                    int p; uint32_t e;
                    nbr_f(r, j, p, e);
                    hw gh, gd, sh, sd;
                    if (j < 2) {
                        gh = j ? x[6] : x[4]; gd = j ? x[7] : x[5]; sh = j ? nh[1] : nh[0]; sd = j ? nd[1] : nd[0];
                    }
                    else {
                        gh = settle(erow(c.ig_h, e)); gd = settle(erow(c.ig_d, e));
                        extra(S, b, p, sweep, g, init, ph, pd, sh, sd);
                    }
                    mh &= sh | gh;
                    md &= sd | gd;
                }
                ih = x[0] | mh;
                id = x[1] | md;
            }
            valid_out(b, r, ih & vm, id & vm, x[2], x[3], vh, vd);
        };
        auto fast = [&](const hw* x, const hw* nh, const hw* nd, uint32_t fl, hw& vh, hw& vd) {
            const hw dev = fmask(fl, DD_DEV), p0 = fmask(fl, DD_P0), p1 = fmask(fl, DD_P1);
            const hw mh = (nh[0] | x[4] | ~p0) & (nh[1] | x[6] | ~p1);
            const hw md = (nd[0] | x[5] | ~p0) & (nd[1] | x[7] | ~p1);
            const hw ih = (x[0] | mh) & vm, id = (x[1] | md) & vm, wr = x[2];
            vh = ((ih & ~wr & dev) | ((ih | wr) & ~dev)) & vm;
            vd = (((id | wr) & dev & ~(x[3] & fph)) | (id & ~wr & ~dev)) & vm;
        };
        run_phase(S, vm64, ~0ull, pre, fast, comp);
    }
}

// ---------------------------------------------------------------------------
// Level schedule: the same phases with the blocks of a level in parallel.
// The ingest kernel sorts a CFG's blocks into levels (a block's level is one
// more than the highest level of its predecessors over edges other than
// BACK, found by peeling the graph from ENTRY); no edge other than BACK joins
// two blocks of one level, so a sweep visits the levels in order (backward:
// in reverse) and all blocks of a level at once, each against its
// neighbours' latest states: Gauss-Seidel across levels, Jacobi within one.
// A level tile is one 32-bit column of a CFG (half of a 64-bit word: 32
// variables) or its flag column; one workgroup holds the column's state of
// every block in LDS (8 bytes per block: host and device halves), so a
// level costs LDS reads of the neighbours, the blocks' inputs from global
// memory and a barrier.  At the end of a phase the state goes to the same
// rows the walk writes, so the passes and later phases read the same arrays
// whatever schedule produced them.
// One wavefront per level tile: a level of a few dozen blocks keeps one wavefront busy, and a
// barrier inside a single wavefront costs no cross-wave synchronisation (a wider level takes
// several passes of the wavefront).
constexpr int LV_THREADS = LEVEL_THREADS;

template <int PH>
__device__ __forceinline__ void level_phase(const DevCfg& c, int hc, uint32_t* SH, uint32_t* SD)
{
    constexpr bool with_flags = PH == PH_NU || PH == PH_AVE;
    constexpr bool BWD = PH == PH_NU || PH == PH_LIVE;
    const bool flg = hc < 0;
    if (flg && !with_flags) return;
    if ((PH == PH_MAYP || PH == PH_LATER) && (c.placement & PL_EAGER)) return;
    if (PH == PH_LIVE && !refines(c.placement)) return;
    const int nb = c.nb, wd = c.wd, tid = threadIdx.x;
    const int w = flg ? 0 : hc >> 1;
    const bool hi = !flg && (hc & 1);
    const u64 vm64 = (w == wd - 1 && (c.nv & 63)) ? ((1ull << (c.nv & 63)) - 1ull) : ~0ull;
    const uint32_t vm = flg ? 3u : (uint32_t)(hi ? vm64 >> 32 : vm64);
    typedef uint32_t hw;
    const size_t wo = (size_t)w;
    // the column's half of row b of a block vector / of edge e of an edge vector
    auto in = [&](const u64* a, int b) -> hw {
        return reinterpret_cast<const GAS uint32_t*>(G(a) + (size_t)b * wd + wo)[hi ? 1 : 0];
    };
    auto vec = [&](const u64* a) -> hw { return reinterpret_cast<const GAS uint32_t*>(G(a) + wo)[hi ? 1 : 0]; };
    auto sum = [&](int ci, int r) -> hw { return in(c.sums, ci * SUM_ROWS + r); };
    // the column's firstprivate variables (none for the flag column)
    const hw fph = (flg || !wd) ? 0u : reinterpret_cast<const GAS uint32_t*>(G(c.fp) + wo)[hi ? 1 : 0];
    const int32_t* REC = BWD ? c.rec_b : c.rec_f;
    const int* LO = c.lorder;
    const int* LF = c.loff;
    const int nlev = G(c.info)[INFO_LEVELS];
    GAS u64* FLG = G(c.flg);   // the flag columns of tile slot 0
    // neighbour j of a record (j >= 2 from the CSR); edge id with LOOP_ENTRY in bit 31
    auto nbr = [&](const Rec& r, int j, int& p, uint32_t& e) {
        if (j == 0) { p = r.n0; e = r.e0; return; }
        if (j == 1) { p = r.n1; e = r.e1; return; }
        if (BWD) { p = G(c.succ_idx)[r.ovf + j]; e = (uint32_t)(r.ovf + j); return; }
        p = G(c.pred_idx)[r.ovf + j];
        const int ee = G(c.pred_eid)[r.ovf + j];
        e = (uint32_t)ee | (is_le(c, G(c.kind)[ee]) ? 0x80000000u : 0u);
    };
    auto eid = [&](uint32_t e) -> int { return (int)(e & 0x7FFFFFFFu); };
    // next use after a call block (OR over its successors; final when validity runs)
    auto nu_after = [&](int b, hw& lh, hw& ld) {
        lh = 0; ld = 0;
        for (int e = G(c.succ_ptr)[b]; e < G(c.succ_ptr)[b + 1]; ++e) {
            const int q = G(c.succ_idx)[e];
            lh |= in(c.nu_h, q);
            ld |= in(c.nu_d, q);
        }
    };
    auto valid_out = [&](int b, const Rec& r, hw ih, hw id, hw wr, hw rr, hw& oh, hw& od) {
        const bool dev = r.meta & REC_DEV;
        hw ah = dev ? (ih & ~wr) : (ih | wr);
        hw ad = dev ? ((id | wr) & ~(rr & fph)) : (id & ~wr);
        if ((r.meta & REC_CALL) && !flg) {
            hw lh, ld;
            nu_after(b, lh, ld);
            const int ci = r.ci;
            ah = tsel(ah, lh, sum(ci, SUM_TH + 0), sum(ci, SUM_TH + 1), sum(ci, SUM_TH + 2), sum(ci, SUM_TH + 3));
            ad = tsel(ad, ld, sum(ci, SUM_TD + 0), sum(ci, SUM_TD + 1), sum(ci, SUM_TD + 2), sum(ci, SUM_TD + 3));
        }
        oh = ah & vm;
        od = ad & vm;
    };
    auto stop = [&](int b, const Rec& r, hw rr, hw ww, hw& sh, hw& sd) {
        if (r.meta & REC_EXIT) { sh = vec(c.lx_h); sd = vec(c.lx_d); return; }
        const bool dev = r.meta & REC_DEV;
        hw uh = dev ? (rr & fph) : rr, ud = dev ? (rr & ~fph) : 0u;
        if (r.meta & REC_CALL) {
            const int ci = r.ci;
            const hw mw = sum(ci, SUM_MAYW_H) | sum(ci, SUM_MAYW_D);
            uh |= sum(ci, SUM_MAYR_H) | mw;
            ud |= sum(ci, SUM_MAYR_D) | mw;
        }
        sh = uh | (dev ? 0u : ww);
        sd = ud | (dev ? ww : 0u);
    };
    // the new state of block b from its neighbours' states in LDS
    auto transfer = [&](int b, hw& vh, hw& vd) {
        const Rec r = ldrec_v(REC, b);
        const int cnt = (int)(r.meta & REC_COUNT);
        const bool dev = r.meta & REC_DEV;
        if constexpr (PH == PH_NU) {
            if (r.meta & REC_EXIT) { vh = flg ? 1u : vec(c.lx_h); vd = flg ? 0u : vec(c.lx_d); return; }
            hw oh = 0, od = 0;
            for (int j = 0; j < cnt; ++j) {
                int q; uint32_t e;
                nbr(r, j, q, e);
                oh |= SH[q];
                od |= SD[q];
            }
            const hw rr = flg ? 2u : in(c.R, b), ww = flg ? (dev ? 2u : 0u) : in(c.W, b);
            if ((r.meta & REC_CALL) && !flg) {
                oh = sum(r.ci, SUM_NU0_H) | (sum(r.ci, SUM_NU1_H) & oh);
                od = sum(r.ci, SUM_NU0_D) | (sum(r.ci, SUM_NU1_D) & od);
            }
            vh = (dev ? (rr & fph) : rr) | (~ww & oh);
            vd = (dev ? (rr & ~fph) : 0u) | (~ww & od);
        } else if constexpr (PH == PH_AVE) {
            hw ih, id;
            if (r.meta & REC_ENTRY) { ih = flg ? 2u : vec(c.ev_h); id = flg ? 0u : vec(c.ev_d); }
            else {
                hw mh = ~0u, md = ~0u;
                for (int j = 0; j < cnt; ++j) {
                    int p; uint32_t e;
                    nbr(r, j, p, e);
                    mh &= SH[p];
                    md &= SD[p];
                }
                ih = (flg ? 0u : in(c.nu_h, b)) | mh;
                id = (flg ? 0u : in(c.nu_d, b)) | md;
            }
            valid_out(b, r, ih & vm, id & vm, flg ? (dev ? 2u : 0u) : in(c.W, b), flg ? 0u : in(c.R, b), vh, vd);
        } else if constexpr (PH == PH_MAYP) {
            if (r.meta & REC_ENTRY) { vh = 0; vd = 0; return; }
            hw mh = 0, md = 0;
            for (int j = 0; j < cnt; ++j) {
                int p; uint32_t e;
                nbr(r, j, p, e);
                if (e & 0x80000000u) continue;   // loop entry: nothing stays pending
                mh |= in(c.eag_h, eid(e)) | SH[p];
                md |= in(c.eag_d, eid(e)) | SD[p];
            }
            hw sth, std_;
            stop(b, r, in(c.R, b), in(c.W, b), sth, std_);
            vh = mh & ~sth & vm;
            vd = md & ~std_ & vm;
        } else if constexpr (PH == PH_LATER) {
            if (r.meta & REC_ENTRY) { vh = 0; vd = 0; return; }
            hw allh = ~0u, alld = ~0u, anyh = 0, anyd = 0;
            for (int j = 0; j < cnt; ++j) {
                int p; uint32_t e;
                nbr(r, j, p, e);
                const hw le = (e & 0x80000000u) ? ~0u : 0u;
                const hw lh = in(c.eag_h, eid(e)) | SH[p], ld = in(c.eag_d, eid(e)) | SD[p];
                const hw bo = in(c.both, eid(e));
                allh &= lh | bo;
                alld &= ld | bo;
                anyh |= lh & ~le;
                anyd |= ld & ~le;
            }
            hw sth, std_;
            stop(b, r, in(c.R, b), in(c.W, b), sth, std_);
            vh = allh & anyh & vm & ~sth;
            vd = alld & anyd & vm & ~std_;
        } else if constexpr (PH == PH_LIVE) {
            hw oh = 0, od = 0;
            for (int j = 0; j < cnt; ++j) {
                int q; uint32_t e;
                nbr(r, j, q, e);
                const hw gh = in(c.ig_h, eid(e)), gd = in(c.ig_d, eid(e));
                oh |= (SH[q] & ~gh) | gd;
                od |= (SD[q] & ~gd) | gh;
            }
            hw rh, rd, kh = 0u, kd = 0u;
            if (r.meta & REC_EXIT) { rh = vec(c.lx_h); rd = vec(c.lx_d); }
            else if (r.meta & REC_CALL) { rh = ~0u; rd = ~0u; }
            else {
                const hw rr = in(c.R, b), ww = in(c.W, b);
                rh = dev ? (rr & fph) : rr;
                rd = dev ? (rr & ~fph) : 0u;
                kh = dev ? 0u : ww;
                kd = dev ? (ww | (rr & fph)) : 0u;
            }
            const hw ih = in(c.ie_h, b), id = in(c.ie_d, b);
            const hw ah = rh | (oh & ~kh), ad = rd | (od & ~kd);
            vh = ((ah & ~ih) | id) & vm;
            vd = ((ad & ~id) | ih) & vm;
        } else {   // PH_AVF
            hw ih, id;
            if (r.meta & REC_ENTRY) { ih = vec(c.ev_h); id = vec(c.ev_d); }
            else {
                hw mh = ~0u, md = ~0u;
                for (int j = 0; j < cnt; ++j) {
                    int p; uint32_t e;
                    nbr(r, j, p, e);
                    mh &= SH[p] | in(c.ig_h, eid(e));
                    md &= SD[p] | in(c.ig_d, eid(e));
                }
                ih = in(c.ie_h, b) | mh;
                id = in(c.ie_d, b) | md;
            }
            valid_out(b, r, ih & vm, id & vm, in(c.W, b), in(c.R, b), vh, vd);
        }
    };
    // The common block (not ENTRY, EXIT or a call) in two halves: its global inputs (rows of the
    // block and of its first two edges, constant within the phase) into X, and the new state from
    // X and its neighbours' states in LDS (further neighbours' edge rows loaded there).
    constexpr int NXL = PH == PH_NU ? 2 : PH == PH_AVE ? 4 : PH == PH_MAYP ? 6 : 8;
    // (the flag column reads a word of its own flag rows instead, which always exist, and uses
    // constants: no branch, so that the loads of a round go out together)
    const GAS uint32_t* safe = reinterpret_cast<const GAS uint32_t*>(FLG);
    auto at = [&](const u64* a, int i) -> hw {
        const GAS uint32_t* p = reinterpret_cast<const GAS uint32_t*>(G(a) + (size_t)i * wd + wo) + (hi ? 1 : 0);
        return *(flg ? safe : p);
    };
    auto is_fast = [&](uint32_t meta) { return !(meta & (REC_ENTRY | REC_EXIT | REC_CALL)); };
    // Neighbours 2 .. cnt-1 of a block with more than two, folded into the accumulators by
    // `fold(state h, state d, edge row h, edge row d, third edge row, loop entry)`: eight at a
    // time, first their CSR entries, then their states and edge rows, every slot loaded (past
    // the last neighbour the last one again: each phase's meet is idempotent).
    auto extra = [&](const int4& r0, const int4& r1, auto&& fold) {
        const int cnt = (int)((uint32_t)r0.x & REC_COUNT), ovf = r1.y;
        for (int j0 = 2; j0 < cnt; j0 += 8) {
            int pj[8], ej[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int jj = ovf + (j0 + t < cnt ? j0 + t : cnt - 1);
                if constexpr (BWD) { pj[t] = G(c.succ_idx)[jj]; ej[t] = jj; }
                else { pj[t] = G(c.pred_idx)[jj]; ej[t] = G(c.pred_eid)[jj]; }
            }
            hw g0[8], g1[8], g2[8];
            bool le[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                le[t] = false;
                g0[t] = g1[t] = g2[t] = 0u;
                if constexpr (PH == PH_MAYP || PH == PH_LATER) {
                    le[t] = is_le(c, G(c.kind)[ej[t]]);
                    g0[t] = at(c.eag_h, ej[t]);
                    g1[t] = at(c.eag_d, ej[t]);
                    if constexpr (PH == PH_LATER) g2[t] = at(c.both, ej[t]);
                }
                if constexpr (PH == PH_LIVE || PH == PH_AVF) {
                    g0[t] = at(c.ig_h, ej[t]);
                    g1[t] = at(c.ig_d, ej[t]);
                }
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) fold(SH[pj[t]], SD[pj[t]], g0[t], g1[t], g2[t], le[t]);
        }
    };
    auto gather = [&](const int4& r0, const int4& r1, hw* X) {
        // every load is issued whatever the block, at a clamped index (a missing edge reads
        // edge 0), so that a round issues the same loads every time
        const int b = r1.w;
        const int cnt = (int)((uint32_t)r0.x & REC_COUNT);
        int e0 = r0.w & 0x7FFFFFFF, e1 = r1.x & 0x7FFFFFFF;
        if (cnt < 1 || e0 >= c.ne) e0 = 0;
        if (cnt < 2 || e1 >= c.ne) e1 = e0;
        if constexpr (PH == PH_NU) { X[0] = at(c.R, b); X[1] = at(c.W, b); }
        if constexpr (PH == PH_AVE) { X[0] = at(c.nu_h, b); X[1] = at(c.nu_d, b); X[2] = at(c.W, b); X[3] = at(c.R, b); }
        if constexpr (PH == PH_MAYP || PH == PH_LATER) {
            X[0] = at(c.eag_h, e0); X[1] = at(c.eag_d, e0); X[2] = at(c.eag_h, e1); X[3] = at(c.eag_d, e1);
        }
        if constexpr (PH == PH_MAYP) { X[4] = at(c.R, b); X[5] = at(c.W, b); }
        if constexpr (PH == PH_LATER) { X[4] = at(c.both, e0); X[5] = at(c.both, e1); X[6] = at(c.R, b); X[7] = at(c.W, b); }
        if constexpr (PH == PH_LIVE || PH == PH_AVF) {
            X[0] = at(c.ig_h, e0); X[1] = at(c.ig_d, e0); X[2] = at(c.ig_h, e1); X[3] = at(c.ig_d, e1);
        }
        if constexpr (PH == PH_LIVE) { X[4] = at(c.R, b); X[5] = at(c.W, b); X[6] = at(c.ie_h, b); X[7] = at(c.ie_d, b); }
        if constexpr (PH == PH_AVF) { X[4] = at(c.ie_h, b); X[5] = at(c.ie_d, b); X[6] = at(c.W, b); X[7] = at(c.R, b); }
    };
    auto apply = [&](const int4& r0, const int4& r1, const hw* X, hw& vh, hw& vd) {
        const uint32_t meta = (uint32_t)r0.x;
        const int cnt = (int)(meta & REC_COUNT);
        const bool dev = meta & REC_DEV;
        const int nbr0 = r0.y, nbr1 = r0.z;
        const bool le0 = (uint32_t)r0.w & 0x80000000u, le1 = (uint32_t)r1.x & 0x80000000u;
        if constexpr (PH == PH_NU) {
            hw oh = 0, od = 0;
            if (cnt > 0) { oh |= SH[nbr0]; od |= SD[nbr0]; }
            if (cnt > 1) { oh |= SH[nbr1]; od |= SD[nbr1]; }
            if (cnt > 2) extra(r0, r1, [&](hw sh, hw sd, hw, hw, hw, bool) { oh |= sh; od |= sd; });
            const hw rr = flg ? 2u : X[0], ww = flg ? (dev ? 2u : 0u) : X[1];
            vh = (dev ? (rr & fph) : rr) | (~ww & oh);
            vd = (dev ? (rr & ~fph) : 0u) | (~ww & od);
        } else if constexpr (PH == PH_AVE) {
            hw mh = ~0u, md = ~0u;
            if (cnt > 0) { mh &= SH[nbr0]; md &= SD[nbr0]; }
            if (cnt > 1) { mh &= SH[nbr1]; md &= SD[nbr1]; }
            if (cnt > 2) extra(r0, r1, [&](hw sh, hw sd, hw, hw, hw, bool) { mh &= sh; md &= sd; });
            const hw ih = ((flg ? 0u : X[0]) | mh) & vm, id = ((flg ? 0u : X[1]) | md) & vm;
            const hw wr = flg ? (dev ? 2u : 0u) : X[2], rr = flg ? 0u : X[3];
            const hw ah = dev ? (ih & ~wr) : (ih | wr);
            const hw ad = dev ? ((id | wr) & ~(rr & fph)) : (id & ~wr);
            vh = ah & vm;
            vd = ad & vm;
        } else if constexpr (PH == PH_MAYP || PH == PH_LATER) {
            const hw rr = X[PH == PH_MAYP ? 4 : 6], ww = X[PH == PH_MAYP ? 5 : 7];
            const hw sth = (dev ? (rr & fph) : rr) | (dev ? 0u : ww);
            const hw std_ = (dev ? (rr & ~fph) : 0u) | (dev ? ww : 0u);
            if constexpr (PH == PH_MAYP) {
                hw mh = 0, md = 0;
                if (cnt > 0 && !le0) { mh |= X[0] | SH[nbr0]; md |= X[1] | SD[nbr0]; }
                if (cnt > 1 && !le1) { mh |= X[2] | SH[nbr1]; md |= X[3] | SD[nbr1]; }
                if (cnt > 2)
                    extra(r0, r1, [&](hw sh, hw sd, hw gh, hw gd, hw, bool l) {
                        if (!l) { mh |= gh | sh; md |= gd | sd; }
                    });
                vh = mh & ~sth & vm;
                vd = md & ~std_ & vm;
            } else {
                hw allh = ~0u, alld = ~0u, anyh = 0, anyd = 0;
                if (cnt > 0) {
                    const hw lh = X[0] | SH[nbr0], ld = X[1] | SD[nbr0];
                    allh &= lh | X[4];
                    alld &= ld | X[4];
                    if (!le0) { anyh |= lh; anyd |= ld; }
                }
                if (cnt > 1) {
                    const hw lh = X[2] | SH[nbr1], ld = X[3] | SD[nbr1];
                    allh &= lh | X[5];
                    alld &= ld | X[5];
                    if (!le1) { anyh |= lh; anyd |= ld; }
                }
                if (cnt > 2)
                    extra(r0, r1, [&](hw sh, hw sd, hw gh, hw gd, hw bo, bool l) {
                        const hw lh = gh | sh, ld = gd | sd;
                        allh &= lh | bo;
                        alld &= ld | bo;
                        if (!l) { anyh |= lh; anyd |= ld; }
                    });
                vh = allh & anyh & vm & ~sth;
                vd = alld & anyd & vm & ~std_;
            }
        } else if constexpr (PH == PH_LIVE) {
            hw oh = 0, od = 0;
            if (cnt > 0) { oh |= (SH[nbr0] & ~X[0]) | X[1]; od |= (SD[nbr0] & ~X[1]) | X[0]; }
            if (cnt > 1) { oh |= (SH[nbr1] & ~X[2]) | X[3]; od |= (SD[nbr1] & ~X[3]) | X[2]; }
            if (cnt > 2)
                extra(r0, r1, [&](hw sh, hw sd, hw gh, hw gd, hw, bool) {
                    oh |= (sh & ~gh) | gd;
                    od |= (sd & ~gd) | gh;
                });
            const hw rr = X[4], ww = X[5];
            const hw rh = dev ? (rr & fph) : rr, rd = dev ? (rr & ~fph) : 0u;
            const hw kh = dev ? 0u : ww, kd = dev ? (ww | (rr & fph)) : 0u;
            const hw ih = X[6], id = X[7];
            const hw ah = rh | (oh & ~kh), ad = rd | (od & ~kd);
            vh = ((ah & ~ih) | id) & vm;
            vd = ((ad & ~id) | ih) & vm;
        } else {   // PH_AVF
            hw mh = ~0u, md = ~0u;
            if (cnt > 0) { mh &= SH[nbr0] | X[0]; md &= SD[nbr0] | X[1]; }
            if (cnt > 1) { mh &= SH[nbr1] | X[2]; md &= SD[nbr1] | X[3]; }
            if (cnt > 2) extra(r0, r1, [&](hw sh, hw sd, hw gh, hw gd, hw, bool) { mh &= sh | gh; md &= sd | gd; });
            const hw ih = (X[4] | mh) & vm, id = (X[5] | md) & vm, wr = X[6], rr = X[7];
            const hw ah = dev ? (ih & ~wr) : (ih | wr);
            const hw ad = dev ? ((id | wr) & ~(rr & fph)) : (id & ~wr);
            vh = ah & vm;
            vd = ad & vm;
        }
    };
    // After a sweep that changed something: would the next one change nothing?  Only blocks
    // that read a neighbour whose level is not below their own can see other states in the
    // next sweep than in this one; the ingest kernel lists them in c.tmp (forward phases from
    // the front, backward ones from the back, -1 ends a list, c.tmp[0] = -2: no lists).  If
    // none of them, evaluated against the states in LDS, changes, then level by level the next
    // sweep repeats this one and the states are the fixed point.
    auto settled = [&]() -> bool {
        const GAS int32_t* LST = G(c.tmp);
        if (LST[0] == -2) return false;
        bool diff = false;
        for (int j0 = 0;; j0 += LV_THREADS) {
            const int idx = BWD ? nb - (j0 + tid) : j0 + tid;
            const int b = (idx >= 0 && idx <= nb) ? LST[idx] : -1;
            const u64 endm = __ballot(b < 0);
            const int t = endm ? (int)__builtin_ctzll(endm) : LV_THREADS;
            if (tid < t) {
                hw vh, vd;
                transfer(b, vh, vd);
                if (vh != SH[b] || vd != SD[b]) diff = true;
            }
            if (__syncthreads_or(diff) || t < LV_THREADS) break;
        }
        return !__syncthreads_or(diff);
    };
    const hw init = (PH == PH_AVE || PH == PH_AVF) ? vm : 0u;
    for (int b = tid; b < nb; b += LV_THREADS) { SH[b] = init; SD[b] = init; }
    __syncthreads();
    const int cap = c.sweep_cap > 0 ? c.sweep_cap : 2 * nb + 2;
    int sweeps = 0;
    bool good = true;
    // Super-steps of S levels: the loads of S levels go out in three rounds (their bounds, then
    // the records of the thread's positions in them, in level order with the block in the last
    // word, then the rows of those blocks and their first two edges), every load issued whatever
    // the level (indices clamped), so that each round is one latency for S levels; then the S
    // levels are computed one after another.  Lane tid takes position LF[lv] + tid of each
    // level (and every LV_THREADS-th one after it, with direct loads, as do calls, ENTRY and
    // EXIT).
    constexpr int S = 8;
    const int4* LR = reinterpret_cast<const int4*>(BWD ? c.step_b : c.step_f);
    int2 bq[S];
    int4 r0q[S], r1q[S];
    hw xq[S][NXL];
    int chg = 0;
    for (;;) {
        for (int li0 = 0; li0 < nlev; li0 += S) {
            const int ns = nlev - li0 < S ? nlev - li0 : S;
#pragma unroll
            for (int v = 0; v < S; ++v) {
                const int li = li0 + v < nlev ? li0 + v : nlev - 1;
                const int lv = BWD ? nlev - 1 - li : li;
                bq[v].x = G(LF)[lv];
                bq[v].y = G(LF)[lv + 1];
            }
#pragma unroll
            for (int v = 0; v < S; ++v) {
                typedef int v4i __attribute__((ext_vector_type(4)));
                int k = bq[v].x + tid;
                if (k >= nb) k = nb - 1;
                const GAS v4i* p = reinterpret_cast<const GAS v4i*>(G(LR)) + 2 * (size_t)k;
                const v4i x = p[0], y = p[1];
                r0q[v] = make_int4(x.x, x.y, x.z, x.w);
                r1q[v] = make_int4(y.x, y.y, y.z, y.w);
            }
#pragma unroll
            for (int v = 0; v < S; ++v) gather(r0q[v], r1q[v], xq[v]);
#pragma unroll
            for (int v = 0; v < S; ++v) {
                if (v < ns) {
                    const int2 q = bq[v];
                    if (q.x + tid < q.y) {
                        const int4 r0 = r0q[v], r1 = r1q[v];
                        const int b = r1.w;
                        hw vh, vd;
                        if (is_fast((uint32_t)r0.x)) apply(r0, r1, xq[v], vh, vd);
                        else transfer(b, vh, vd);
                        if (vh != SH[b] || vd != SD[b]) {
                            SH[b] = vh;
                            SD[b] = vd;
                            chg = 1;
                        }
                    }
                    // positions past the first LV_THREADS of a wide level
                    for (int k = q.x + tid + LV_THREADS; k < q.y; k += LV_THREADS) {
                        const int bb = LO[k];
                        hw vh, vd;
                        transfer(bb, vh, vd);
                        if (vh != SH[bb] || vd != SD[bb]) {
                            SH[bb] = vh;
                            SD[bb] = vd;
                            chg = 1;
                        }
                    }
                    // the level's LDS writes before the next level's reads (no wait for the
                    // loads: none is in flight here)
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
                    __builtin_amdgcn_s_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
                }
            }
        }
        ++sweeps;
        if (!__syncthreads_or(chg)) break;
        if (settled()) break;
        if (sweeps >= cap) {
            if (tid == 0) set_status(c.info, OMPD_E_NOCONVERGE_);
            good = false;
            break;
        }
        chg = 0;
    }
    if (tid == 0) atomicMax(&c.info[INFO_SWEEPS + PH], sweeps);
    // the state to the rows of the phase (flag column: tile slot 0's columns)
    if (flg) {
        const int fl = PH == PH_NU ? 0 : 2;
        for (int b = tid; b < nb; b += LV_THREADS) {
            FLG[(size_t)fl * nb + b] = SH[b];
            FLG[(size_t)(fl + 1) * nb + b] = SD[b];
        }
    } else {
        // (the refinement keeps its state in the pending-copy rows, free after the placement)
        u64* h = PH == PH_NU ? c.nu_h : PH == PH_MAYP || PH == PH_LIVE ? c.mayp_h : PH == PH_LATER ? c.later_h : c.aveout_h;
        u64* d = PH == PH_NU ? c.nu_d : PH == PH_MAYP || PH == PH_LIVE ? c.mayp_d : PH == PH_LATER ? c.later_d : c.aveout_d;
        for (int b = tid; b < nb; b += LV_THREADS) {
            reinterpret_cast<GAS uint32_t*>(G(h) + (size_t)b * wd + wo)[hi ? 1 : 0] = SH[b];
            reinterpret_cast<GAS uint32_t*>(G(d) + (size_t)b * wd + wo)[hi ? 1 : 0] = SD[b];
        }
    }
    if constexpr (PH == PH_AVE) {
        if (!flg || !good) return;
        // reachability: every block reached from ENTRY and reaching EXIT; the label facts
        int bad = 0;
        for (int b = tid; b < nb; b += LV_THREADS) {
            const u64 fnu = FLG[b], fnud = FLG[(size_t)nb + b];
            const hw fave = SH[b];
            if (!(fnu & 1) || (fave & 1)) bad = 1;
            if (c.after_dev) G(c.after_dev)[b] = (uint8_t)(((fave >> 1) & 1) ^ 1);
            if (c.before_dev) G(c.before_dev)[b] = (uint8_t)((fnud >> 1) & 1);
        }
        if (__syncthreads_or(bad) && tid == 0) set_status(c.info, OMPD_E_INVAL_);
    }
}

// One persistent kernel per phase over the level tiles (one workgroup of LV_THREADS per tile,
// the column's state in dynamic LDS).  A tile (cfg, s0, nw, fslot): s0 = the 32-bit column
// (word s0 / 2, its high half when s0 is odd) or -1 for the flag column.
template <int PH>
__device__ __forceinline__ void level_kernel(const DevCfg* __restrict__ cfgs, const Tile* __restrict__ tiles,
                                             int n_tiles, int32_t* __restrict__ counter)
{
    extern __shared__ __align__(16) u64 lds[];
    __shared__ int s_tile, s_skip;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&counter[16 + PH], 1);
        __syncthreads();
        const int t = s_tile;
        __syncthreads();
        if (t >= n_tiles) break;
        const Tile tl = tiles[t];
        const DevCfg c = cfgs[tl.cfg];
        if (threadIdx.x == 0) s_skip = G(c.info)[INFO_STATUS] != 0;
        __syncthreads();
        if (!s_skip) {
            uint32_t* SH = reinterpret_cast<uint32_t*>(lds);
            level_phase<PH>(c, tl.s0, SH, SH + c.nb);
        }
        __syncthreads();
    }
}
#define OMPD_LEVEL_KERNEL(name, ph)                                                                          \
    extern "C" __global__ void __launch_bounds__(LV_THREADS) name(const DevCfg* __restrict__ cfgs,          \
                                                                   const Tile* __restrict__ tiles,           \
                                                                   int n_tiles, int32_t* __restrict__ counter) \
    {                                                                                                        \
        level_kernel<ph>(cfgs, tiles, n_tiles, counter);                                                     \
    }
OMPD_LEVEL_KERNEL(ompd_k_lv_nu, PH_NU)
OMPD_LEVEL_KERNEL(ompd_k_lv_ave, PH_AVE)
OMPD_LEVEL_KERNEL(ompd_k_lv_mayp, PH_MAYP)
OMPD_LEVEL_KERNEL(ompd_k_lv_later, PH_LATER)
OMPD_LEVEL_KERNEL(ompd_k_lv_avf, PH_AVF)
OMPD_LEVEL_KERNEL(ompd_k_lv_live, PH_LIVE)

// ---------------------------------------------------------------------------
// Edge-parallel passes (no iteration): one wavefront per (tile, 64-block
// chunk) item; the item's nw words are spread over the lanes 64 / nw times
// (lane = block slot * nw + word), so that a narrow item keeps that many
// blocks in flight instead of walking its chunk one block at a time.
//   PASS_AVE  : AVEin_s(b) (output); per out-edge e = b->q:
//               EAG_s(e) = NU_s(q) & ~AVEout_s(b), VE_s(e) = AVEout_s(b) | NU_s(q)
//               (VE is kept in the INS_EDGE rows until the placement overwrites them)
//   PASS_MAYP : per out-edge: BOTH(e) = FV_H(e) & FV_D(e),
//               FV_x(e) = VE_x(e) & ~((EAG_x(e) | MAYPout_x(b)) & ~LE(e))
//   PASS_LATER: LATERin_s(q) and the copies INS_ENTRY_s(q) = LATERin_s(q) & USE'_s(q),
//               INS_EDGE_s(e = p->q) = LATER_s(e) & (LE(e) | ~LATERin_s(q)); eager placement:
//               INS_ENTRY = 0, INS_EDGE = EAG
//   PASS_AVF  : AVFin_s(q) (output) and the per-variable map kind accumulators (Table II):
//               map(to) = a copy into the device on p->q with no DEVICE block before p, or
//               before q when no predecessor has one; map(from) = a copy into the host on
//               p->q or before q when no DEVICE block follows q; alloc = used only on the device
//   PASS_LIVE : the loop-entry refinement: INS_EDGE_s(e = p->q) &= LI_s(q) on loop-entry edges
//               (a copy whose value no read uses is dropped)
enum { PASS_AVE = 0, PASS_MAYP = 1, PASS_LATER = 2, PASS_AVF = 3, PASS_LIVE = 4 };
// work counter of a pass kernel
constexpr int pass_counter(int pass) { return pass == PASS_LIVE ? 14 : 8 + pass; }

template <int PASS>
__device__ __forceinline__ void edge_pass(const DevCfg& c, int s0, int nw, int fslot, int b0)
{
    const int lane = threadIdx.x & 63;
    if (nw <= 0) return;
    const int bpw = nw >= 64 ? 1 : 64 / nw;     // blocks in flight per wavefront
    const int sub = lane / nw;                  // the lane's block slot
    if (sub >= bpw) return;
    const int nb = c.nb, wd = c.wd;
    const int w = s0 + (lane - sub * nw);
    const size_t wo = (size_t)w;
    const u64 vm = (w == wd - 1 && (c.nv & 63)) ? ((1ull << (c.nv & 63)) - 1ull) : ~0ull;
    // CSR indices differ between the lanes' blocks: vector loads
    const GAS int32_t* SP = G(c.succ_ptr);
    const GAS int32_t* SI = G(c.succ_idx);
    const GAS int32_t* PP = G(c.pred_ptr);
    const GAS int32_t* PI = G(c.pred_idx);
    const GAS int32_t* PE = G(c.pred_eid);
    const GAS uint8_t* KD = G(c.kind);
    const GAS u64* FLG = G(c.flg) + (size_t)fslot * 4 * nb;
    auto row = [&](const u64* a, int b) -> u64 { return G(a)[(size_t)b * wd + wo]; };
    auto erow = [&](const u64* a, int e) -> u64 { return G(a)[(size_t)e * wd + wo]; };
    auto put = [&](u64* a, size_t r, u64 v) { G(a)[r * wd + wo] = v; };
    const int b1 = min(b0 + 64, nb);
    if constexpr (PASS == PASS_AVE || PASS == PASS_MAYP) {
        for (int b = b0 + sub; b < b1; b += bpw) {
            const u64 aoh = row(c.aveout_h, b), aod = row(c.aveout_d, b);
            if constexpr (PASS == PASS_AVE) {
                u64 ih, id;
                if (b == c.entry) { ih = G(c.ev_h)[wo]; id = G(c.ev_d)[wo]; }
                else {
                    u64 mh = ~0ull, md = ~0ull;
                    for (int k = PP[b]; k < PP[b + 1]; ++k) {
                        const int p = PI[k];
                        mh &= row(c.aveout_h, p);
                        md &= row(c.aveout_d, p);
                    }
                    ih = row(c.nu_h, b) | mh;
                    id = row(c.nu_d, b) | md;
                }
                put(c.ave_h, b, ih & vm);
                put(c.ave_d, b, id & vm);
                for (int e = SP[b]; e < SP[b + 1]; ++e) {
                    const int q = SI[e];
                    const u64 nuh = row(c.nu_h, q), nud = row(c.nu_d, q);
                    put(c.eag_h, e, nuh & ~aoh);
                    put(c.eag_d, e, nud & ~aod);
                    put(c.ig_h, e, aoh | nuh);
                    put(c.ig_d, e, aod | nud);
                }
            } else {
                const u64 mph = row(c.mayp_h, b), mpd = row(c.mayp_d, b);
                for (int e = SP[b]; e < SP[b + 1]; ++e) {
                    const u64 nle = is_le(c, KD[e]) ? 0ull : ~0ull;
                    const u64 fvh = erow(c.ig_h, e) & ~((erow(c.eag_h, e) | mph) & nle);
                    const u64 fvd = erow(c.ig_d, e) & ~((erow(c.eag_d, e) | mpd) & nle);
                    put(c.both, e, fvh & fvd);
                }
            }
        }
    }
    if constexpr (PASS == PASS_LATER) {
        const bool eager = c.placement & PL_EAGER;
        for (int q = b0 + sub; q < b1; q += bpw) {
            const int a = PP[q], z = PP[q + 1];
            if (eager || q == c.entry) {
                put(c.ie_h, q, 0);
                put(c.ie_d, q, 0);
                for (int k = a; k < z; ++k) {
                    const int e = PE[k];
                    put(c.ig_h, e, eager ? erow(c.eag_h, e) : 0ull);
                    put(c.ig_d, e, eager ? erow(c.eag_d, e) : 0ull);
                }
                continue;
            }
            u64 allh = ~0ull, alld = ~0ull, anyh = 0, anyd = 0;
            for (int k = a; k < z; ++k) {
                const int p = PI[k], e = PE[k];
                const u64 le = is_le(c, KD[e]) ? ~0ull : 0ull;
                const u64 lh = erow(c.eag_h, e) | row(c.later_h, p), ld = erow(c.eag_d, e) | row(c.later_d, p);
                const u64 bo = erow(c.both, e);
                const u64 lph = lh & ~le, lpd = ld & ~le;
                allh &= lph | bo | (lh & le);
                alld &= lpd | bo | (ld & le);
                anyh |= lph;
                anyd |= lpd;
            }
            const u64 inh = allh & anyh & vm, ind = alld & anyd & vm;
            // USE'_s(q)
            const bool dev = c.space[q] != 0;
            u64 uh, ud;
            if (q == c.exit) { uh = G(c.lx_h)[wo]; ud = G(c.lx_d)[wo]; }
            else {
                const u64 rr = row(c.R, q), fp = G(c.fp)[wo];
                uh = dev ? (rr & fp) : rr;
                ud = dev ? (rr & ~fp) : 0ull;
                const int ci = c.call ? c.call[q] : -1;
                if (ci >= 0) {
                    const GAS u64* sm = G(c.sums) + (size_t)ci * SUM_ROWS * wd + wo;
                    const u64 mw = sm[SUM_MAYW_H * wd] | sm[SUM_MAYW_D * wd];
                    uh |= sm[SUM_MAYR_H * wd] | mw;
                    ud |= sm[SUM_MAYR_D * wd] | mw;
                }
            }
            put(c.ie_h, q, inh & uh);
            put(c.ie_d, q, ind & ud);
            for (int k = a; k < z; ++k) {
                const int p = PI[k], e = PE[k];
                const u64 le = is_le(c, KD[e]) ? ~0ull : 0ull;
                const u64 lh = erow(c.eag_h, e) | row(c.later_h, p), ld = erow(c.eag_d, e) | row(c.later_d, p);
                put(c.ig_h, e, lh & (le | ~inh) & vm);
                put(c.ig_d, e, ld & (le | ~ind) & vm);
            }
        }
    }
    if constexpr (PASS == PASS_LIVE) {
        for (int q = b0 + sub; q < b1; q += bpw) {
            const u64 lh = row(c.mayp_h, q), ld = row(c.mayp_d, q);
            for (int k = PP[q]; k < PP[q + 1]; ++k) {
                const int e = PE[k];
                if (!is_le(c, KD[e])) continue;
                put(c.ig_h, e, erow(c.ig_h, e) & lh);
                put(c.ig_d, e, erow(c.ig_d, e) & ld);
            }
        }
    }
    if constexpr (PASS == PASS_AVF) {
        u64 to = 0, fr = 0, dv = 0, fr_read = 0;
        const u64 fp = G(c.fp)[wo];
        for (int q = b0 + sub; q < b1; q += bpw) {
            const int a = PP[q], z = PP[q + 1];
            const u64 ieh = row(c.ie_h, q), ied = row(c.ie_d, q);
            const u64 not_before = ((FLG[(size_t)nb + q] >> 1) & 1) - 1;   // all ones: no DEVICE block follows q
            u64 ih, id;
            if (q == c.entry) { ih = G(c.ev_h)[wo]; id = G(c.ev_d)[wo]; }
            else {
                u64 mh = ~0ull, md = ~0ull, none_after = ~0ull;
                for (int k = a; k < z; ++k) {
                    const int p = PI[k], e = PE[k];
                    const u64 gh = erow(c.ig_h, e), gd = erow(c.ig_d, e);
                    mh &= row(c.aveout_h, p) | gh;
                    md &= row(c.aveout_d, p) | gd;
                    const u64 p_clear = 0ull - ((FLG[(size_t)2 * nb + p] >> 1) & 1);   // all ones: p not after DEVICE
                    to |= gd & p_clear;
                    fr |= gh & not_before;
                    none_after &= p_clear;
                }
                ih = ieh | mh;
                id = ied | md;
                to |= ied & none_after;
                fr |= ieh & not_before;
            }
            if (c.space[q] && q != c.exit) {
                const u64 rr = row(c.R, q);
                dv |= (rr & ~fp) | row(c.W, q);
                fr_read |= rr & fp;
                if (c.fpc) put(c.fpc, q, rr & fp);
            } else if (c.fpc) put(c.fpc, q, 0);
            if (c.avf_h) { put(c.avf_h, q, ih & vm); put(c.avf_d, q, id & vm); }
        }
        if (c.var_kind) {
            GAS u64* acc = G(c.vk_acc);
            if (to) atomicOr((unsigned long long*)&acc[wo], (unsigned long long)to);
            if (fr) atomicOr((unsigned long long*)&acc[wd + wo], (unsigned long long)fr);
            if (dv) atomicOr((unsigned long long*)&acc[2 * wd + wo], (unsigned long long)dv);
            if (fr_read) atomicOr((unsigned long long*)&acc[3 * wd + wo], (unsigned long long)fr_read);
        }
    }
}

// One phase of one tile by the whole workgroup (both wavefronts); a CFG that already failed is skipped.
template <int PH>
__device__ __forceinline__ void tile_phase(const DevCfg& c, const Tile& tl, u64* lds, int ring_slots)
{
    Ctl* ctl = reinterpret_cast<Ctl*>(lds);
    if (threadIdx.x == 0) {
        // one read of the CFG's status for both wavefronts (another tile may fail meanwhile)
        ctl->skip = G(c.info)[INFO_STATUS] != 0;
        ctl->produced = 0; ctl->consumed = 0; ctl->flushed = 0; ctl->done = 0; ctl->abort = 0;
        ctl->in_ready = 0;
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(ctl->skip)) {
        __syncthreads();
        return;
    }
    // a CFG on the level schedule is solved by the level kernels; lanes past 2 LANES hold no word
    // (the walk order the ingest kernel chose: the block ids, or its own)
    if (c.sched != SCHED_LEVEL && (threadIdx.x & 63) < 2 * LANES) {
        if (__builtin_amdgcn_readfirstlane(G(c.info)[INFO_ORDER]))
            solve_phase<PH, true>(c, tl.s0, tl.nw, tl.fslot, lds, ring_slots);
        else
            solve_phase<PH, false>(c, tl.s0, tl.nw, tl.fslot, lds, ring_slots);
    }
    __syncthreads();
}

template <int PH>
__device__ __forceinline__ void phase_kernel(const DevCfg* __restrict__ cfgs, const Tile* __restrict__ tiles, int n_tiles,
                                             int32_t* __restrict__ counter, int ring_slots)
{
    extern __shared__ __align__(16) u64 lds[];
    Ctl* ctl = reinterpret_cast<Ctl*>(lds);
    // tiles come longest first; those of the longest CFGs bound the launch, so their wavefronts
    // take the SIMD's issue slots first
    const int nb_max = n_tiles > 0 ? cfgs[tiles[0].cfg].nb : 0;
    for (;;) {
        if (threadIdx.x == 0) ctl->tile = atomicAdd(&counter[PH], 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(ctl->tile);
        __syncthreads();
        if (t >= n_tiles) break;
        const Tile tl = tiles[t];
        const DevCfg c = cfgs[tl.cfg];
        if (2 * c.nb >= nb_max) __builtin_amdgcn_s_setprio(3);
        else __builtin_amdgcn_s_setprio(0);
        tile_phase<PH>(c, tl, lds, ring_slots);
    }
}

// One persistent kernel per phase (two wavefronts per tile); the phases of all tiles run in this order.
#define OMPD_PHASE_KERNEL(name, ph)                                                                          \
    extern "C" __global__ void __launch_bounds__(128) name(const DevCfg* __restrict__ cfgs,                 \
                                                            const Tile* __restrict__ tiles, int n_tiles,    \
                                                            int32_t* __restrict__ counter, int ring_slots)  \
    {                                                                                                        \
        phase_kernel<ph>(cfgs, tiles, n_tiles, counter, ring_slots);                                         \
    }
OMPD_PHASE_KERNEL(ompd_k_nu, PH_NU)
OMPD_PHASE_KERNEL(ompd_k_ave, PH_AVE)
OMPD_PHASE_KERNEL(ompd_k_mayp, PH_MAYP)
OMPD_PHASE_KERNEL(ompd_k_later, PH_LATER)
OMPD_PHASE_KERNEL(ompd_k_avf, PH_AVF)
OMPD_PHASE_KERNEL(ompd_k_live, PH_LIVE)

// Edge-parallel passes over (tile, chunk) items, claimed through counter slots 8..11 and 14.
template <int PASS>
__device__ __forceinline__ void pass_kernel(const DevCfg* __restrict__ cfgs, const Tile* __restrict__ tiles,
                                            const EdgeItem* __restrict__ items, int n_items, int32_t* __restrict__ counter)
{
    for (;;) {
        int it = 0;
        if (threadIdx.x == 0) it = atomicAdd(&counter[pass_counter(PASS)], 1);
        it = __builtin_amdgcn_readfirstlane(__shfl(it, 0, 64));
        if (it >= n_items) break;
        const EdgeItem item = items[it];
        const DevCfg c = cfgs[item.cfg];
        if (G(c.info)[INFO_STATUS] != 0 || item.nw == 0) continue;
        if ((PASS == PASS_MAYP) && (c.placement & PL_EAGER)) continue;   // the eager placement needs no pending copies
        if ((PASS == PASS_LIVE) && !refines(c.placement)) continue;
        // every solve tile's flag lane computes the same reachability facts: tile 0's columns
        edge_pass<PASS>(c, item.s0, item.nw, 0, item.b0);
    }
}
#define OMPD_PASS_KERNEL(name, pass)                                                                         \
    extern "C" __global__ void __launch_bounds__(64) name(const DevCfg* __restrict__ cfgs,                  \
                                                           const Tile* __restrict__ tiles,                  \
                                                           const EdgeItem* __restrict__ items, int n_items, \
                                                           int32_t* __restrict__ counter)                   \
    {                                                                                                        \
        pass_kernel<pass>(cfgs, tiles, items, n_items, counter);                                             \
    }
OMPD_PASS_KERNEL(ompd_k_post_ave, PASS_AVE)
OMPD_PASS_KERNEL(ompd_k_post_mayp, PASS_MAYP)
OMPD_PASS_KERNEL(ompd_k_post_later, PASS_LATER)
OMPD_PASS_KERNEL(ompd_k_post_avf, PASS_AVF)
OMPD_PASS_KERNEL(ompd_k_post_live, PASS_LIVE)

// The map kinds of one tile's variables from its masks; wavefront k takes words s0 + k, s0 + k + waves, ...
__device__ __forceinline__ void tile_varkind(const DevCfg& c, const Tile& tl, int first, int step)
{
    const GAS u64* acc = G(c.vk_acc);
    const int i = threadIdx.x & 63;
    for (int w = tl.s0 + first; w < tl.s0 + tl.nw; w += step) {
        const int v = w * 64 + i;
        if (v >= c.nv) break;
        const u64 t = ld_fresh(acc + w), f = ld_fresh(acc + c.wd + w), d = ld_fresh(acc + 2 * c.wd + w);
        const u64 fr = ld_fresh(acc + 3 * c.wd + w);
        const uint32_t t1 = (uint32_t)((t >> i) & 1), f1 = (uint32_t)((f >> i) & 1), d1 = (uint32_t)((d >> i) & 1);
        const uint32_t p1 = (uint32_t)((fr >> i) & 1);
        G(c.var_kind)[v] = (uint8_t)(t1 | (f1 << 1) | ((d1 && !t1 && !f1) ? 4u : 0u) | (p1 << 3));
    }
}

// Map kinds from the masks: one wavefront per tile (claimed through counter
// slot 12), one lane per variable of each of the tile's words.
extern "C" __global__ void __launch_bounds__(64) ompd_k_varkind(const DevCfg* __restrict__ cfgs,
                                                                 const Tile* __restrict__ tiles, int n_tiles,
                                                                 int32_t* __restrict__ counter)
{
    for (;;) {
        int t = 0;
        if (threadIdx.x == 0) t = atomicAdd(&counter[12], 1);
        t = __builtin_amdgcn_readfirstlane(__shfl(t, 0, 64));
        if (t >= n_tiles) break;
        const Tile tl = tiles[t];
        const DevCfg c = cfgs[tl.cfg];
        if (!c.var_kind || tl.nw == 0 || G(c.info)[INFO_STATUS] != 0) continue;
        tile_varkind(c, tl, 0, 1);
    }
}

// A pass over one tile by the whole workgroup: wavefront k takes the 64-block chunks k, k + 2, ...
// (after an acquire, so that the state rows the helper wavefront stored are read fresh).
template <int PASS>
__device__ __forceinline__ void tile_pass(const DevCfg& c, const Tile& tl)
{
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const bool skip = G(c.info)[INFO_STATUS] != 0 || tl.nw == 0 || (PASS == PASS_MAYP && (c.placement & PL_EAGER)) ||
                      (PASS == PASS_LIVE && !refines(c.placement));
    if (!skip)
        for (int b0 = 64 * (int)(threadIdx.x >> 6); b0 < c.nb; b0 += 128) edge_pass<PASS>(c, tl.s0, tl.nw, tl.fslot, b0);
    __syncthreads();
}

// The whole solve of each tile in one persistent kernel: a workgroup takes a tile (longest first,
// claimed through counter slot 13) and runs every phase and pass on it, so tiles never wait for
// each other between phases.
extern "C" __global__ void __launch_bounds__(128) ompd_k_solve(const DevCfg* __restrict__ cfgs,
                                                                const Tile* __restrict__ tiles, int n_tiles,
                                                                int32_t* __restrict__ counter, int ring_slots)
{
    extern __shared__ __align__(16) u64 lds[];
    Ctl* ctl = reinterpret_cast<Ctl*>(lds);
    for (;;) {
        if (threadIdx.x == 0) ctl->tile = atomicAdd(&counter[13], 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(ctl->tile);
        __syncthreads();
        if (t >= n_tiles) break;
        const Tile tl = tiles[t];
        const DevCfg c = cfgs[tl.cfg];
        tile_phase<PH_NU>(c, tl, lds, ring_slots);
        tile_phase<PH_AVE>(c, tl, lds, ring_slots);
        tile_pass<PASS_AVE>(c, tl);
        tile_phase<PH_MAYP>(c, tl, lds, ring_slots);
        tile_pass<PASS_MAYP>(c, tl);
        tile_phase<PH_LATER>(c, tl, lds, ring_slots);
        tile_pass<PASS_LATER>(c, tl);
        if (refines(c.placement)) {
            tile_phase<PH_LIVE>(c, tl, lds, ring_slots);
            tile_pass<PASS_LIVE>(c, tl);
        }
        tile_phase<PH_AVF>(c, tl, lds, ring_slots);
        tile_pass<PASS_AVF>(c, tl);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (c.var_kind && tl.nw > 0 && G(c.info)[INFO_STATUS] == 0) tile_varkind(c, tl, (int)(threadIdx.x >> 6), 2);
        __syncthreads();
    }
}

}  // namespace ompd
