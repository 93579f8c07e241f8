// Whole-program (interprocedural) solve of libompd: per-procedure summaries
// bottom-up over the call graph's strongly connected components, call-string
// contexts top-down, and the host-read demands and exit-validity caps that
// feed back until they settle.  Every CFG solve is a batched device solve
// (ompd_plan_*); the small kernels below build the call tables, gather the
// summary rows, form the may-sets, and meet the callers' contributions into
// the callee contexts.  The host only orders the work (components, levels,
// rounds) and tests for convergence.
//
// Summaries (per procedure P, over the globals; section "Interprocedural
// Analysis": the side effects of a call on global variables, per space):
//   NU0_s, NU1_s : next use in s at P's entry when the globals are dead /
//                  live in s after P returns,
//   T_s[e][l]    : validity in s at P's exit (eager copies) when the globals
//                  are valid in both / neither space at entry (e) and live /
//                  dead after the return (l),
//   MAYR_s, MAYW_s: may be read / written in s by P or anything it calls.
// Each problem is gen/kill per bit, so the four boundary evaluations define
// the transfer exactly.  Inside a recursive component the next-use rows
// iterate from 0, then the validity tables from all ones, then the may-sets
// from 0.  External callees need every global on the host, may read and
// write all of them there and leave the device copies stale.
//
// Contexts (procedure, last two call sites): each call gives the callee
// context it leads to the caller's next use after the call (exit liveness)
// and the validity after the call block's own accesses under eager copies
// (entry validity).  Liveness meets by OR and only grows with liveness;
// eager validity meets by AND and only shrinks with validity; so the exit
// liveness of all contexts is one least fixed point and, given it, the entry
// validity one greatest fixed point, each solved here in rounds of batched
// context solves.  A global then valid in neither space that the context
// reads before writing it is demanded as a host read at the call site
// leading to the context (a host read at the call block), unless a calling
// context lacks it too.  Each call is capped by the validity at EXIT, under
// the final placement, of the callee context it leads to (from the previous
// outer round).  Outer rounds repeat until the demands and caps no longer
// change.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ompd.h"
#include "ompd_device.h"
#include "ompd_internal.h"

using namespace ompd;

#define GAS __attribute__((address_space(1)))

namespace {

__device__ __forceinline__ uint64_t word_mask(int nbits, int w)
{
    const int lo = 64 * w;
    if (nbits >= lo + 64) return ~0ull;
    if (nbits <= lo) return 0ull;
    return (1ull << (nbits - lo)) - 1ull;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// Arguments of one call site: caller variable bound to each, and for an external callee whether
// it is a pointer to const.  A procedure's shared variables are the globals [0, G) and then its
// pointer parameters [G, G + n_params); parameter t of the callee is the site's argument t.
struct Args {
    const int32_t* var;
    const uint8_t* cst;
    int32_t n;
};

__device__ __forceinline__ bool bit_of(const uint64_t* row, int v) { return (row[v >> 6] >> (v & 63)) & 1ull; }

// Call table of one call site in the caller's variable layout: the callee's
// summary rows on the globals (an external callee's fixed rows), the cap of
// the callee context on the validity tables, identity for the caller's
// other variables (NU1 = 1, T[e][l] = e); then each argument's column (the
// callee's parameter row, or an external argument's fixed one: read on the
// host, written there unless const, the device copy stale unless const) on
// the bound caller variable, replacing the identity on its first binding and
// otherwise combined with what reaches it already (a global, an earlier
// argument): may and next-use rows by OR, validity tables by AND.
struct CallTabItem {
    uint64_t* dst;        // [16][wd]
    const uint64_t* src;  // [16][sw] callee rows, or NULL for an external callee
    const uint64_t* cap;  // [2][sw] host / device caps, or NULL
    const uint64_t* cmask;   // [gw] const globals (an external callee neither writes nor stales them)
    Args a;
    int32_t wd, gw, sw, G, nv;
};

__device__ __forceinline__ bool ext_row(int r, bool cst)
{
    if (r == SUM_MAYR_H || r == SUM_NU0_H || r == SUM_NU1_H || r == SUM_NU1_D) return true;
    if (r == SUM_MAYW_H) return !cst;
    if (r >= SUM_TH && r < SUM_TH + 4) return true;
    if (r == SUM_TD + 2 || r == SUM_TD + 3) return cst;
    return false;
}

__global__ void __launch_bounds__(256) k_calltab(const CallTabItem* __restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const CallTabItem I = items[it];
        for (int x = threadIdx.x; x < SUM_ROWS * I.wd; x += blockDim.x) {
            const int r = x / I.wd, w = x % I.wd;
            const uint64_t gm = word_mask(I.G, w), lm = word_mask(I.nv, w) & ~gm;
            const bool trow = r >= SUM_TH;
            uint64_t v = 0;
            if (w < I.gw) {
                if (I.src) v = I.src[r * I.sw + w];
                else {
                    const bool one = r == SUM_MAYR_H || r == SUM_NU0_H || r == SUM_NU1_H || r == SUM_NU1_D ||
                                     (r >= SUM_TH && r < SUM_TH + 4);
                    v = one ? ~0ull : 0ull;
                    if (r == SUM_MAYW_H) v = ~I.cmask[w];
                    if (r == SUM_TD + 2 || r == SUM_TD + 3) v = I.cmask[w];   // a const device copy is kept
                }
                v &= gm;
                if (I.cap) {
                    if (r >= SUM_TH && r < SUM_TH + 4) v &= I.cap[w];
                    if (r >= SUM_TD && r < SUM_TD + 4) v &= I.cap[I.sw + w];
                }
            }
            if (r == SUM_NU1_H || r == SUM_NU1_D || r == SUM_TH + 2 || r == SUM_TH + 3 || r == SUM_TD + 2 ||
                r == SUM_TD + 3)
                v |= lm;
            for (int t = 0; t < I.a.n; ++t) {
                const int xv = I.a.var[t];
                if ((xv >> 6) != w) continue;
                bool col;
                if (I.src) {
                    const int y = I.G + t;
                    col = bit_of(I.src + r * I.sw, y);
                    if (I.cap && trow) col = col && bit_of(I.cap + (r < SUM_TD ? 0 : I.sw), y);
                } else {
                    col = ext_row(r, I.a.cst[t] != 0);
                }
                bool seen = xv < I.G;
                for (int u = 0; u < t && !seen; ++u) seen = I.a.var[u] == xv;
                const uint64_t bt = 1ull << (xv & 63);
                if (!seen) v = col ? (v | bt) : (v & ~bt);
                else if (!trow) { if (col) v |= bt; }
                else if (!col) v &= ~bt;
            }
            I.dst[r * I.wd + w] = v;
        }
    }
}

// Summary rows of a procedure from one boundary evaluation (e, l): the next
// use at its entry (e = 0 only) and the validity at its exit.
struct SumItem {
    uint64_t* S;          // [16][sw] rows of the procedure
    const uint64_t *nu_h, *nu_d, *ave_h, *ave_d;
    int32_t entry, exit, wd, sw, sh, eps, ell, rows;   // sh: shared variables; rows: bit 0 next use, bit 1 tables
    int32_t* changed;
};

__global__ void __launch_bounds__(64) k_sumgather(const SumItem* __restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const SumItem I = items[it];
        for (int w = threadIdx.x; w < I.sw; w += blockDim.x) {
            const uint64_t gm = word_mask(I.sh, w);
            const bool in = w < I.wd;
            bool ch = false;
            auto put = [&](int r, uint64_t v) {
                v &= gm;
                if (I.S[r * I.sw + w] != v) { I.S[r * I.sw + w] = v; ch = true; }
            };
            if ((I.rows & 1) && I.eps == 0) {
                const int base = I.ell ? SUM_NU1_H : SUM_NU0_H;
                put(base, in ? I.nu_h[(size_t)I.entry * I.wd + w] : 0ull);
                put(base + 1, in ? I.nu_d[(size_t)I.entry * I.wd + w] : 0ull);
            }
            if (I.rows & 2) {
                put(SUM_TH + 2 * I.eps + I.ell, in ? I.ave_h[(size_t)I.exit * I.wd + w] : 0ull);
                put(SUM_TD + 2 * I.eps + I.ell, in ? I.ave_d[(size_t)I.exit * I.wd + w] : 0ull);
            }
            if (ch) atomicOr(I.changed, 1);
        }
    }
}

// May-read / may-write rows of a procedure over its shared variables: its
// own host / device blocks (reads including the demanded ones and the calls
// made inside kernels) and every host call's callee, through the bindings (a
// callee's parameter row lands on the bound caller variable when that is one
// of the caller's shared variables); an external callee reads every global
// and its arguments on the host and writes them there (not the const ones).
struct MayItem {
    uint64_t* S;
    const uint64_t *R, *W;
    const uint8_t* space;
    const int32_t* callees;   // [n_sites], -1 = external
    const int32_t* sites;     // [n_sites] call-site ids
    const int32_t* ap;        // [n_calls + 1] into av / ac
    const int32_t* av;
    const uint8_t* ac;
    const uint64_t* Sall;     // rows of every procedure
    const uint64_t* cmask;    // [gw] const globals
    int32_t nb, wd, gw, sw, G, sh, n_sites;
    int32_t* changed;
};

__global__ void __launch_bounds__(64) k_may(const MayItem* __restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const MayItem I = items[it];
        for (int w = threadIdx.x; w < I.sw; w += blockDim.x) {
            const uint64_t gm = word_mask(I.G, w), sm = word_mask(I.sh, w);
            uint64_t m[4] = {0, 0, 0, 0};
            if (w < I.wd)
                for (int b = 0; b < I.nb; ++b) {
                    const int d = I.space[b] ? 1 : 0;
                    m[d] |= I.R[(size_t)b * I.wd + w];
                    m[2 + d] |= I.W[(size_t)b * I.wd + w];
                }
            for (int k = 0; k < I.n_sites; ++k) {
                const int q = I.callees[k], j = I.sites[k];
                const int a0 = I.ap[j], na = I.ap[j + 1] - a0;
                if (q < 0) {
                    m[SUM_MAYR_H] |= gm;
                    m[SUM_MAYW_H] |= w < I.gw ? (~I.cmask[w] & gm) : 0ull;
                } else if (w < I.gw)
                    for (int r = 0; r < 4; ++r) m[r] |= I.Sall[((size_t)q * SUM_ROWS + r) * I.sw + w] & gm;
                for (int t = 0; t < na; ++t) {
                    const int x = I.av[a0 + t];
                    if ((x >> 6) != w || x >= I.sh) continue;
                    const uint64_t bt = 1ull << (x & 63);
                    if (q < 0) {
                        m[SUM_MAYR_H] |= bt;
                        if (!I.ac[a0 + t]) m[SUM_MAYW_H] |= bt;
                    } else
                        for (int r = 0; r < 4; ++r)
                            if (bit_of(I.Sall + ((size_t)q * SUM_ROWS + r) * I.sw, I.G + t)) m[r] |= bt;
                }
            }
            bool ch = false;
            for (int r = 0; r < 4; ++r) {
                const uint64_t v = m[r] & sm;
                if (I.S[r * I.sw + w] != v) { I.S[r * I.sw + w] = v; ch = true; }
            }
            if (ch) atomicOr(I.changed, 1);
        }
    }
}

// Host reads demanded at call blocks: Rd = R with the demand rows ORed in.
// A demand is in the call site's layout: bit v < G the global v, bit G + t
// the caller variable bound to argument t.
struct DemandItem {
    uint64_t* Rd;
    const uint64_t* R;
    const uint64_t* demand;   // [sw]
    Args a;
    int32_t block, wd, gw, G;
};

__global__ void __launch_bounds__(64) k_demand(const DemandItem* __restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const DemandItem I = items[it];
        for (int w = threadIdx.x; w < I.wd; w += blockDim.x) {
            uint64_t v = I.R[(size_t)I.block * I.wd + w];
            if (w < I.gw) v |= I.demand[w] & word_mask(I.G, w);
            for (int t = 0; t < I.a.n; ++t) {
                const int x = I.a.var[t];
                if ((x >> 6) == w && bit_of(I.demand, I.G + t)) v |= 1ull << (x & 63);
            }
            I.Rd[(size_t)I.block * I.wd + w] = v;
        }
    }
}

// A call made inside a kernel: the call block (a DEVICE block) reads every variable the callee
// may read or write, in either space, and writes every one it may write, through the bindings
// (the globals, and the caller variable bound to each parameter); an external callee reads
// every global and its arguments and writes them (not the const ones).  ORed into the caller's
// rows (the may sets only grow, so repeating it is harmless).
struct DevCallItem {
    uint64_t *Rd, *W;
    const uint64_t* S;       // [16][sw] callee rows, or NULL for an external callee
    const uint64_t* cmask;   // [gw]
    Args a;
    int32_t block, wd, gw, sw, G;
};

__global__ void __launch_bounds__(64) k_devcall(const DevCallItem* __restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const DevCallItem I = items[it];
        for (int w = threadIdx.x; w < I.wd; w += blockDim.x) {
            const uint64_t gm = word_mask(I.G, w);
            uint64_t rd = 0, wr = 0;
            if (w < I.gw) {
                if (I.S) {
                    wr = I.S[SUM_MAYW_H * I.sw + w] | I.S[SUM_MAYW_D * I.sw + w];
                    rd = I.S[SUM_MAYR_H * I.sw + w] | I.S[SUM_MAYR_D * I.sw + w] | wr;
                } else {
                    rd = ~0ull;
                    wr = ~I.cmask[w];
                }
                rd &= gm;
                wr &= gm;
            }
            for (int t = 0; t < I.a.n; ++t) {
                const int x = I.a.var[t];
                if ((x >> 6) != w) continue;
                const uint64_t bt = 1ull << (x & 63);
                bool r, wt;
                if (I.S) {
                    const int y = I.G + t;
                    wt = bit_of(I.S + SUM_MAYW_H * I.sw, y) || bit_of(I.S + SUM_MAYW_D * I.sw, y);
                    r = wt || bit_of(I.S + SUM_MAYR_H * I.sw, y) || bit_of(I.S + SUM_MAYR_D * I.sw, y);
                } else {
                    r = true;
                    wt = !I.a.cst[t];
                }
                if (r) rd |= bt;
                if (wt) wr |= bt;
            }
            I.Rd[(size_t)I.block * I.wd + w] |= rd;
            I.W[(size_t)I.block * I.wd + w] |= wr;
        }
    }
}

// Contribution of one solved call to the callee context it leads to, in the
// callee's shared layout (the globals, then each parameter from the caller
// variable bound to it): in the liveness system the caller's next use after
// the call (the OR of next use over the call block's successors), in the
// validity system the validity after the call block's own accesses under
// eager copies.  One slot per call edge of the context graph keeps the latest
// contribution.
struct ContribItem {
    const uint64_t *a_h, *a_d;   // liveness: next use (H, D); validity: eager validity (H, D)
    const uint64_t* W;
    const int32_t *succ_ptr, *succ_idx;
    uint64_t* out;               // [2][sw] slot of the call edge
    Args a;
    int32_t c, wd, gw, sw, G, live;
};

__global__ void __launch_bounds__(64) k_contrib(const ContribItem* __restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const ContribItem I = items[it];
        // the caller's word wc of the two rows
        auto word = [&](int wc, uint64_t& h, uint64_t& d) {
            h = 0;
            d = 0;
            if (I.live) {
                for (int e = I.succ_ptr[I.c]; e < I.succ_ptr[I.c + 1]; ++e) {
                    const size_t t = (size_t)I.succ_idx[e] * I.wd + wc;
                    h |= I.a_h[t];
                    d |= I.a_d[t];
                }
            } else {
                const size_t cw = (size_t)I.c * I.wd + wc;
                const uint64_t wr = I.W[cw];
                h = I.a_h[cw] | wr;
                d = I.a_d[cw] & ~wr;
            }
        };
        for (int w = threadIdx.x; w < I.sw; w += blockDim.x) {
            uint64_t h = 0, d = 0;
            if (w < I.gw) {
                word(w, h, d);
                const uint64_t gm = word_mask(I.G, w);
                h &= gm;
                d &= gm;
            }
            for (int t = 0; t < I.a.n; ++t) {
                const int y = I.G + t;
                if ((y >> 6) != w) continue;
                const int x = I.a.var[t];
                uint64_t xh, xd;
                word(x >> 6, xh, xd);
                const uint64_t bt = 1ull << (y & 63);
                if ((xh >> (x & 63)) & 1ull) h |= bt;
                if ((xd >> (x & 63)) & 1ull) d |= bt;
            }
            I.out[w] = h;
            I.out[I.sw + w] = d;
        }
    }
}

// Meet of the latest contributions of every call edge into a context:
// liveness by OR (exit liveness; the callee's other locals are dead after
// it), validity by AND (entry validity; the callee's other locals are valid
// on the host at its entry).  The boundary is rewritten, and the context
// marked, when the meet differs from it.
struct MeetItem {
    uint64_t* bnd;               // [4][wd] of the context
    const uint64_t* contrib;     // [n_call_edges][2][sw]
    const int32_t* in_edges;     // call edges into the context
    int32_t* changed;
    int32_t n_in, wd, sw, sh, nv, live;
};

__global__ void __launch_bounds__(64) k_meet(const MeetItem* __restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const MeetItem I = items[it];
        bool ch = false;
        for (int w = threadIdx.x; w < I.wd; w += blockDim.x) {
            const uint64_t gm = word_mask(I.sh, w), lm = word_mask(I.nv, w) & ~gm;
            uint64_t h = I.live ? 0ull : ~0ull, d = h;
            if (w < I.sw) {
                for (int k = 0; k < I.n_in; ++k) {
                    const uint64_t* c = I.contrib + (size_t)I.in_edges[k] * 2 * I.sw;
                    if (I.live) { h |= c[w]; d |= c[I.sw + w]; }
                    else { h &= c[w]; d &= c[I.sw + w]; }
                }
            }
            const int base = I.live ? 2 : 0;
            if (I.live) { h &= gm; d &= gm; }
            else { h = (h & gm) | lm; d &= gm; }
            uint64_t* bh = I.bnd + (size_t)base * I.wd + w;
            uint64_t* bd = I.bnd + (size_t)(base + 1) * I.wd + w;
            if (*bh != h || *bd != d) { *bh = h; *bd = d; ch = true; }
        }
        if (ch) atomicOr(I.changed, 1);
    }
}

// Shared variables a context leaves valid in neither space at its entry and
// reads there before writing them (next use at ENTRY, either space).
struct GapItem {
    uint64_t* gap;               // [sw] of the context
    const uint64_t *bnd, *nu_h, *nu_d;
    int32_t* any;
    int32_t entry, wd, sw, sh;
};

__global__ void __launch_bounds__(64) k_gap(const GapItem* __restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const GapItem I = items[it];
        for (int w = threadIdx.x; w < I.sw; w += blockDim.x) {
            uint64_t v = 0;
            if (w < I.wd) {
                const size_t ew = (size_t)I.entry * I.wd + w;
                const uint64_t need = I.nu_h[ew] | I.nu_d[ew];
                v = word_mask(I.sh, w) & ~(I.bnd[w] | I.bnd[I.wd + w]) & need;
            }
            I.gap[w] = v;
            if (v) atomicOr(I.any, 1);
        }
    }
}

// Host-read demand at the call site leading to a context (the site's
// layout, which is the context's shared layout): its gaps that no calling
// context lacks at its own entry (a caller's gap on the variable bound to a
// parameter counts for that parameter), or every gap, when `all`.
struct OwnItem {
    const uint64_t* gaps;        // [n_contexts][sw]
    const int32_t* callers;      // calling context of each call edge into this one
    uint64_t* demand;            // [sw] of the leading call site
    int32_t* any;
    Args a;
    int32_t x, n_callers, gw, sw, G, sh_caller, all;
};

__global__ void __launch_bounds__(64) k_own(const OwnItem* __restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const OwnItem I = items[it];
        for (int w = threadIdx.x; w < I.sw; w += blockDim.x) {
            uint64_t inherited = 0;
            if (!I.all)
                for (int k = 0; k < I.n_callers; ++k) {
                    const uint64_t* cg = I.gaps + (size_t)I.callers[k] * I.sw;
                    if (w < I.gw) inherited |= cg[w] & word_mask(I.G, w);
                    for (int t = 0; t < I.a.n; ++t) {
                        const int y = I.G + t, x = I.a.var[t];
                        if ((y >> 6) == w && x < I.sh_caller && bit_of(cg, x)) inherited |= 1ull << (y & 63);
                    }
                }
            const uint64_t own = I.gaps[(size_t)I.x * I.sw + w] & ~inherited;
            if (own) {
                atomicOr((unsigned long long*)&I.demand[w], (unsigned long long)own);
                atomicOr(I.any, 1);
            }
        }
    }
}

// Plain word copy (initial context boundaries).
struct CopyItem {
    uint64_t* dst;
    const uint64_t* src;
    int32_t n;
};

__global__ void __launch_bounds__(64) k_copy(const CopyItem* __restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const CopyItem I = items[it];
        for (int w = threadIdx.x; w < I.n; w += blockDim.x) I.dst[w] = I.src[w];
    }
}

// Validity at EXIT under the final placement of a context, on its shared
// variables (its callers' cap).
struct CapItem {
    uint64_t* cap;            // [2][sw]
    const uint64_t *avf_h, *avf_d;
    int32_t exit, wd, sw, sh;
};

__global__ void __launch_bounds__(64) k_cap(const CapItem* __restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const CapItem I = items[it];
        for (int w = threadIdx.x; w < I.sw; w += blockDim.x) {
            const uint64_t gm = word_mask(I.sh, w);
            const bool in = w < I.wd;
            I.cap[w] = in ? I.avf_h[(size_t)I.exit * I.wd + w] & gm : 0ull;
            I.cap[I.sw + w] = in ? I.avf_d[(size_t)I.exit * I.wd + w] & gm : 0ull;
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
#define CK(x)                                                                                   \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess)                                                                   \
            return ompd_fail(OMPD_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_));    \
    } while (0)

static inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Structure {
    int n = 0, G = 0, gw = 0, nc = 0;
    int sw = 0;                            // words of the widest shared layout (globals + parameters)
    std::vector<int> wd, nb, ne;
    std::vector<int> sh;                   // per procedure: globals + its pointer parameters
    std::vector<int32_t> ap;               // [nc + 1] arguments of each call site in arg_var
    std::vector<std::vector<int>> sites;   // per procedure: its host call sites in order
    std::vector<std::vector<int>> dsites;  // per procedure: its calls made inside kernels
    std::vector<int> site_k;               // call site -> index among its caller's sites
    // contexts
    std::vector<int> cproc, cs0, cs1;
    std::vector<std::vector<int>> child;   // per context: per site k, the callee context or -1
    std::vector<std::vector<int>> comps;   // strongly connected components, callees first
    std::vector<int> comp_level;           // per component
};

int check_program(const ompd_program* P, Structure& st)
{
    char buf[200];
    auto bad = [&](const char* why, int i) {
        snprintf(buf, sizeof buf, "program: %s (%d)", why, i);
        return ompd_fail(OMPD_E_INVAL, buf);
    };
    if (!P || P->n_procs <= 0 || !P->procs || P->n_globals < 0 || P->n_calls < 0 || P->n_roots <= 0 || !P->roots)
        return bad("bad sizes or missing arrays", 0);
    if (P->n_calls > 0 && (!P->call_proc || !P->call_block || !P->callee)) return bad("call arrays missing", 0);
    st.n = P->n_procs;
    st.G = P->n_globals;
    st.gw = (st.G + 63) / 64;
    st.nc = P->n_calls;
    st.wd.resize(st.n);
    st.nb.resize(st.n);
    st.ne.resize(st.n);
    st.sites.assign(st.n, {});
    st.dsites.assign(st.n, {});
    for (int i = 0; i < st.n; ++i) {
        const ompd_cfg& g = P->procs[i];
        if (g.n_vars < st.G) return bad("procedure has fewer variables than globals", i);
        if (g.call_summary || g.summaries || g.n_summaries) return bad("procedure carries call summaries", i);
        if (g.n_blocks < 2 || g.entry < 0 || g.exit < 0 || g.entry >= g.n_blocks || g.exit >= g.n_blocks)
            return bad("bad procedure shape", i);
        st.wd[i] = (g.n_vars + 63) / 64;
        st.nb[i] = g.n_blocks;
        st.ne[i] = g.n_edges;
    }
    // pointer parameters and the arguments bound to them
    st.sh.assign(st.n, st.G);
    int maxnp = 0;
    for (int i = 0; i < st.n; ++i) {
        const int np = P->n_params ? P->n_params[i] : 0;
        if (np < 0 || np > P->procs[i].n_vars - st.G) return bad("bad parameter count", i);
        st.sh[i] = st.G + np;
        maxnp = std::max(maxnp, np);
    }
    st.sw = (st.G + maxnp + 63) / 64;
    st.ap.assign(st.nc + 1, 0);
    if (P->arg_ptr) {
        if (P->arg_ptr[0] != 0) return bad("arg_ptr[0] is not 0", 0);
        for (int j = 0; j < st.nc; ++j) {
            if (P->arg_ptr[j + 1] < P->arg_ptr[j]) return bad("arg_ptr decreases", j);
            st.ap[j + 1] = P->arg_ptr[j + 1];
        }
        if (st.ap[st.nc] > 0 && !P->arg_var) return bad("arg_var missing", 0);
    }
    for (int j = 0; j < st.nc; ++j) {
        const int p = P->call_proc[j], q = P->callee[j], a0 = st.ap[j], na = st.ap[j + 1] - a0;
        if (p < 0 || p >= st.n || q < -1 || q >= st.n) return bad("call site out of range", j);
        if (q >= 0 && na != st.sh[q] - st.G) return bad("argument count differs from the callee's parameters", j);
        const bool host_body = q >= 0 && !(P->call_space && P->call_space[j]);
        for (int t = 0; t < na; ++t) {
            const int x = P->arg_var[a0 + t];
            if (x < 0 || x >= P->procs[p].n_vars) return bad("argument is not a caller variable", j);
            if (host_body) {
                if (x < st.G) return bad("a host call binds a global to a parameter", j);
                for (int u = 0; u < t; ++u)
                    if (P->arg_var[a0 + u] == x) return bad("a host call binds one variable twice", j);
            }
        }
    }
    st.site_k.assign(st.nc, -1);
    std::map<std::pair<int, int>, int> seen;
    for (int j = 0; j < st.nc; ++j) {
        const int p = P->call_proc[j], b = P->call_block[j], q = P->callee[j];
        if (p < 0 || p >= st.n || q < -1 || q >= st.n) return bad("call site out of range", j);
        const ompd_cfg& g = P->procs[p];
        const int dev = P->call_space ? P->call_space[j] : 0;
        if (dev != 0 && dev != 1) return bad("call space is neither host nor device", j);
        if (b < 0 || b >= g.n_blocks || b == g.entry || b == g.exit || g.space[b] != dev)
            return bad("call block is not a block of its procedure in the call's space", j);
        if (seen.count({p, b})) return bad("two calls in one block", j);
        seen[{p, b}] = j;
        if (dev) { st.dsites[p].push_back(j); continue; }
        st.site_k[j] = (int)st.sites[p].size();
        st.sites[p].push_back(j);
    }
    if (P->const_globals && st.G > 0) {
        // nothing writes a const global
        for (int i = 0; i < st.n; ++i) {
            const ompd_cfg& g = P->procs[i];
            if (!g.write_bits) continue;
            for (int b = 0; b < g.n_blocks; ++b)
                for (int w = 0; w < st.gw; ++w) {
                    const int lo = 64 * w;
                    const uint64_t gm = st.G >= lo + 64 ? ~0ull : (1ull << (st.G - lo)) - 1ull;
                    if (g.write_bits[(size_t)b * st.wd[i] + w] & P->const_globals[w] & gm)
                        return bad("a procedure writes a const global", i);
                }
        }
    }
    for (int k = 0; k < P->n_roots; ++k)
        if (P->roots[k] < 0 || P->roots[k] >= st.n) return bad("root out of range", k);
    // contexts, breadth first from the roots
    std::map<std::tuple<int, int, int>, int> idx;
    std::deque<int> work;
    auto add = [&](int q, int s0, int s1) -> int {
        auto key = std::make_tuple(q, s0, s1);
        auto itr = idx.find(key);
        if (itr != idx.end()) return itr->second;
        const int id = (int)st.cproc.size();
        idx[key] = id;
        st.cproc.push_back(q);
        st.cs0.push_back(s0);
        st.cs1.push_back(s1);
        st.child.emplace_back();
        work.push_back(id);
        return id;
    };
    for (int k = 0; k < P->n_roots; ++k) add(P->roots[k], -1, -1);
    while (!work.empty()) {
        const int x = work.front();
        work.pop_front();
        const int p = st.cproc[x];
        std::vector<int> ch(st.sites[p].size(), -1);
        for (size_t k = 0; k < st.sites[p].size(); ++k) {
            const int j = st.sites[p][k], q = P->callee[j];
            if (q >= 0) ch[k] = add(q, st.cs1[x], j);
        }
        st.child[x] = ch;
    }
    // strongly connected components (iterative Tarjan), callees first
    std::vector<std::vector<int>> succ(st.n);
    for (int j = 0; j < st.nc; ++j)
        if (P->callee[j] >= 0) succ[P->call_proc[j]].push_back(P->callee[j]);
    std::vector<int> index(st.n, -1), low(st.n, 0), comp_of(st.n, -1);
    std::vector<char> on(st.n, 0);
    std::vector<int> stk;
    int counter = 0;
    for (int root = 0; root < st.n; ++root) {
        if (index[root] >= 0) continue;
        std::vector<std::pair<int, size_t>> call{{root, 0}};
        while (!call.empty()) {
            auto& fr = call.back();
            const int v = fr.first;
            if (fr.second == 0 && index[v] < 0) {
                index[v] = low[v] = counter++;
                stk.push_back(v);
                on[v] = 1;
            }
            bool pushed = false;
            while (fr.second < succ[v].size()) {
                const int u = succ[v][fr.second++];
                if (index[u] < 0) { call.push_back({u, 0}); pushed = true; break; }
                if (on[u]) low[v] = std::min(low[v], index[u]);
            }
            if (pushed) continue;
            if (low[v] == index[v]) {
                std::vector<int> comp;
                for (;;) {
                    const int u = stk.back();
                    stk.pop_back();
                    on[u] = 0;
                    comp_of[u] = (int)st.comps.size();
                    comp.push_back(u);
                    if (u == v) break;
                }
                st.comps.push_back(comp);
            }
            call.pop_back();
            if (!call.empty()) low[call.back().first] = std::min(low[call.back().first], low[v]);
        }
    }
    st.comp_level.assign(st.comps.size(), 0);
    for (size_t ci = 0; ci < st.comps.size(); ++ci)   // callees' components come first
        for (int v : st.comps[ci])
            for (int u : succ[v])
                if (comp_of[u] != (int)ci) st.comp_level[ci] = std::max(st.comp_level[ci], st.comp_level[comp_of[u]] + 1);
    return OMPD_OK;
}

// Device copy of the program and the state of the solve.
struct Prog {
    ompd_ctx* ctx = nullptr;
    const ompd_program* P = nullptr;
    Structure st;
    hipStream_t s = nullptr;
    uint32_t flags = 0;
    int64_t solves = 0;
    char* arena = nullptr;
    // per procedure (device pointers into the arena)
    std::vector<int32_t*> sp, si, call;
    std::vector<uint8_t*> kind, space;
    std::vector<uint64_t*> R, Rd, W, sbnd;   // sbnd: [4 evaluations][4][wd] summary boundaries
    std::vector<int32_t*> callees;           // [n_sites]
    std::vector<uint64_t*> ptab;             // [n_sites][16][wd] call tables of the summary evaluations
    uint64_t* S = nullptr;                   // [n][16][sw]
    int32_t *d_ap = nullptr, *d_av = nullptr;  // call-site argument offsets and bound caller variables
    uint8_t* d_ac = nullptr;                 // pointer-to-const flags of the arguments
    std::vector<int32_t*> sitej;             // per procedure: its host call-site ids
    uint64_t* cmask = nullptr;               // [gw] const globals
    uint64_t* demand = nullptr;              // [nc][sw]   (accumulated; call-site layout)
    uint64_t* demand_new = nullptr;          // [nc][sw]   (this outer round)
    uint64_t* caps = nullptr;                // [nctx][2][sw]
    int32_t* flag = nullptr;                 // scratch flags
    // per context
    std::vector<uint64_t*> bnd, ctab;
    // context graph: call edges (caller context, site), numbered caller by caller
    int n_edges = 0;
    std::vector<std::vector<int>> eid;       // per context: per site k, its call edge or -1
    std::vector<int> in_ptr;                 // [nctx+1] into in_edges / callers
    int32_t* in_edges = nullptr;             // call edges into each context
    int32_t* callers = nullptr;              // the calling context of each of those edges
    uint64_t* contrib = nullptr;             // [n_edges][2][sw] latest contribution per edge
    uint64_t* gaps = nullptr;                // [nctx][sw]
    uint64_t* bnd0 = nullptr;                // initial boundaries, contexts back to back
    std::vector<size_t> bnd0_off;
    std::vector<uint64_t*> o_nu_h, o_nu_d, o_ave_h, o_ave_d, o_avf_h, o_avf_d, o_ie_h, o_ie_d, o_ig_h, o_ig_d;
    std::vector<uint8_t*> o_vk, o_ad, o_bd;
    std::vector<char*> ctx_end;              // end of each context's arena region (bnd .. outputs)
    std::vector<int32_t> sweeps;             // [nctx][6]
    // summary evaluation outputs (per procedure, 4 evaluations, nu/ave H/D)
    std::vector<uint64_t*> e_out;            // [4][4][nb][wd]
    char* arena_items = nullptr;             // staging of kernel work items
    std::vector<char> cap_valid;             // per context: a cap from the previous outer round exists
    ~Prog() { if (arena) (void)hipFree(arena); }
};

template <typename T>
int upload_items(const std::vector<T>& v, void (*k)(const T*, int), int threads, hipStream_t s, char* scratch)
{
    if (v.empty()) return OMPD_OK;
    CK(hipMemcpyAsync(scratch, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
    const int grid = (int)std::min<size_t>(v.size(), 4096);
    hipLaunchKernelGGL(k, dim3(grid), dim3(threads), 0, s, (const T*)scratch, (int)v.size());
    CK(hipGetLastError());
    CK(hipStreamSynchronize(s));
    return OMPD_OK;
}

// Solve a batch of CFGs given by device-pointer descriptors.
int run_batch(Prog& G, std::vector<ompd_cfg>& cfgs, std::vector<ompd_result>& res, uint32_t flags)
{
    if (cfgs.empty()) return OMPD_OK;
    PlanConfig pc;
    pc.use_graph = false;   // one-shot plans: capturing a graph would not be replayed
    ompd_plan* plan = nullptr;
    int rc = ompd_plan_build(G.ctx, cfgs.data(), res.data(), (int32_t)cfgs.size(), flags | OMPD_F_DEVICE_PTRS | G.flags,
                             pc, &plan);
    if (rc) return rc;
    rc = ompd_plan_run_locked(plan, G.s);
    if (rc == OMPD_OK) rc = ompd_plan_collect(plan, nullptr);
    for (size_t i = 0; i < cfgs.size(); ++i) memcpy(res[i].sweeps, plan->res[i].sweeps, sizeof res[i].sweeps);
    ompd_plan_destroy(plan);
    G.solves += (int64_t)cfgs.size();
    return rc;
}

int read_flag(Prog& G, int32_t* dflag, int& out)
{
    CK(hipMemcpyAsync(&out, dflag, 4, hipMemcpyDeviceToHost, G.s));
    CK(hipStreamSynchronize(G.s));
    return OMPD_OK;
}

int zero_flag(Prog& G, int32_t* dflag)
{
    CK(hipMemsetAsync(dflag, 0, 4, G.s));
    return OMPD_OK;
}

int setup(Prog& G)
{
    const Structure& st = G.st;
    const ompd_program* P = G.P;
    const int n = st.n, gw = st.gw, sw = st.sw, nctx = (int)st.cproc.size();
    // arena layout
    size_t total = 0;
    auto take = [&](size_t bytes) { size_t x = total; total += a256(std::max<size_t>(bytes, 8)); return x; };
    struct PO { size_t sp, si, kind, space, R, Rd, W, call, sbnd, callees, sitej, ptab, eout; };
    std::vector<PO> po(n);
    for (int i = 0; i < n; ++i) {
        const size_t nb = st.nb[i], ne = st.ne[i], wd = st.wd[i], ns = st.sites[i].size();
        po[i].sp = take(4 * (nb + 1));
        po[i].si = take(4 * ne);
        po[i].kind = take(ne);
        po[i].space = take(nb);
        po[i].R = take(8 * nb * wd);
        po[i].Rd = take(8 * nb * wd);
        po[i].W = take(8 * nb * wd);
        po[i].call = take(4 * nb);
        po[i].sbnd = take(8 * 16 * wd);
        po[i].callees = take(4 * ns);
        po[i].sitej = take(4 * ns);
        po[i].ptab = take(8 * ns * SUM_ROWS * wd);
        po[i].eout = take(8 * 16 * nb * wd);
    }
    const size_t oS = take(8 * (size_t)n * SUM_ROWS * sw);
    const size_t oCm = take(8 * (size_t)std::max(gw, 1));
    const size_t oD = take(8 * (size_t)std::max(st.nc, 1) * sw);
    const size_t oDn = take(8 * (size_t)std::max(st.nc, 1) * sw);
    const size_t oC = take(8 * (size_t)nctx * 2 * sw);
    const size_t nargs = (size_t)st.ap[st.nc];
    const size_t oAp = take(4 * ((size_t)st.nc + 1));
    const size_t oAv = take(4 * std::max<size_t>(nargs, 1));
    const size_t oAc = take(std::max<size_t>(nargs, 1));
    const size_t oF = take(4 * (size_t)(nctx + 16));
    // call edges of the context graph and, per context, the edges into it
    G.eid.assign(nctx, {});
    G.n_edges = 0;
    std::vector<int> indeg(nctx + 1, 0);
    for (int x = 0; x < nctx; ++x) {
        G.eid[x].assign(st.child[x].size(), -1);
        for (size_t k = 0; k < st.child[x].size(); ++k)
            if (st.child[x][k] >= 0) { G.eid[x][k] = G.n_edges++; ++indeg[st.child[x][k]]; }
    }
    G.in_ptr.assign(nctx + 1, 0);
    for (int x = 0; x < nctx; ++x) G.in_ptr[x + 1] = G.in_ptr[x] + indeg[x];
    std::vector<int32_t> h_in(std::max(G.n_edges, 1)), h_callers(std::max(G.n_edges, 1));
    {
        std::vector<int> fill(G.in_ptr.begin(), G.in_ptr.end() - 1);
        for (int x = 0; x < nctx; ++x)
            for (size_t k = 0; k < st.child[x].size(); ++k) {
                const int cx = st.child[x][k];
                if (cx < 0) continue;
                h_in[fill[cx]] = G.eid[x][k];
                h_callers[fill[cx]++] = x;
            }
    }
    const size_t oCb = take(8 * (size_t)std::max(G.n_edges, 1) * 2 * sw);
    const size_t oIn = take(4 * h_in.size());
    const size_t oCl = take(4 * h_callers.size());
    const size_t oGap = take(8 * (size_t)nctx * sw);
    G.bnd0_off.assign(nctx + 1, 0);
    for (int x = 0; x < nctx; ++x) G.bnd0_off[x + 1] = G.bnd0_off[x] + 4 * (size_t)st.wd[st.cproc[x]];
    const size_t oB0 = take(8 * G.bnd0_off[nctx]);
    struct CO { size_t bnd, ctab, out; };
    std::vector<CO> co(nctx);
    for (int x = 0; x < nctx; ++x) {
        const int p = st.cproc[x];
        const size_t nb = st.nb[p], ne = st.ne[p], wd = st.wd[p], ns = st.sites[p].size();
        co[x].bnd = take(8 * 4 * wd);
        co[x].ctab = take(8 * ns * SUM_ROWS * wd);
        co[x].out = take(8 * (8 * nb * wd + 2 * ne * wd) + (size_t)P->procs[p].n_vars + 2 * nb + 64);
    }
    const size_t oItems = take(64ull << 20);   // staging of kernel work items
    hipError_t e = hipMalloc(&G.arena, total);
    if (e != hipSuccess) return ompd_fail(OMPD_E_NOMEM, std::string("program arena: ") + hipGetErrorString(e));
    char* A = G.arena;
    G.sp.resize(n); G.si.resize(n); G.kind.resize(n); G.space.resize(n); G.R.resize(n); G.Rd.resize(n);
    G.W.resize(n); G.call.resize(n); G.sbnd.resize(n); G.callees.resize(n); G.ptab.resize(n); G.e_out.resize(n);
    G.sitej.resize(n);
    std::vector<uint64_t> hb;
    for (int i = 0; i < n; ++i) {
        const ompd_cfg& g = P->procs[i];
        const size_t nb = st.nb[i], ne = st.ne[i], wd = st.wd[i], ns = st.sites[i].size();
        G.sp[i] = (int32_t*)(A + po[i].sp); G.si[i] = (int32_t*)(A + po[i].si);
        G.kind[i] = (uint8_t*)(A + po[i].kind); G.space[i] = (uint8_t*)(A + po[i].space);
        G.R[i] = (uint64_t*)(A + po[i].R); G.Rd[i] = (uint64_t*)(A + po[i].Rd); G.W[i] = (uint64_t*)(A + po[i].W);
        G.call[i] = (int32_t*)(A + po[i].call); G.sbnd[i] = (uint64_t*)(A + po[i].sbnd);
        G.callees[i] = (int32_t*)(A + po[i].callees); G.ptab[i] = (uint64_t*)(A + po[i].ptab);
        G.sitej[i] = (int32_t*)(A + po[i].sitej);
        G.e_out[i] = (uint64_t*)(A + po[i].eout);
        CK(hipMemcpyAsync(G.sp[i], g.succ_ptr, 4 * (nb + 1), hipMemcpyHostToDevice, G.s));
        if (ne) {
            CK(hipMemcpyAsync(G.si[i], g.succ_idx, 4 * ne, hipMemcpyHostToDevice, G.s));
            CK(hipMemcpyAsync(G.kind[i], g.edge_kind, ne, hipMemcpyHostToDevice, G.s));
        }
        CK(hipMemcpyAsync(G.space[i], g.space, nb, hipMemcpyHostToDevice, G.s));
        if (wd) {
            CK(hipMemcpyAsync(G.R[i], g.read_bits, 8 * nb * wd, hipMemcpyHostToDevice, G.s));
            CK(hipMemcpyAsync(G.Rd[i], g.read_bits, 8 * nb * wd, hipMemcpyHostToDevice, G.s));
            CK(hipMemcpyAsync(G.W[i], g.write_bits, 8 * nb * wd, hipMemcpyHostToDevice, G.s));
        }
        std::vector<int32_t> call(nb, -1), cal(std::max<size_t>(ns, 1), -1), sj(std::max<size_t>(ns, 1), 0);
        for (size_t k = 0; k < ns; ++k) {
            call[P->call_block[st.sites[i][k]]] = (int32_t)k;
            cal[k] = P->callee[st.sites[i][k]];
            sj[k] = st.sites[i][k];
        }
        CK(hipMemcpyAsync(G.call[i], call.data(), 4 * nb, hipMemcpyHostToDevice, G.s));
        CK(hipMemcpyAsync(G.callees[i], cal.data(), 4 * cal.size(), hipMemcpyHostToDevice, G.s));
        CK(hipMemcpyAsync(G.sitej[i], sj.data(), 4 * sj.size(), hipMemcpyHostToDevice, G.s));
        // summary boundaries, evaluation 2e+l: entry valid (e ? shared : none) on both spaces
        // plus the other locals on the host; the shared variables (globals and parameters) live
        // after exit in both spaces iff l
        hb.assign(16 * wd, 0);
        for (int ev = 0; ev < 4; ++ev) {
            const int eps = ev >> 1, ell = ev & 1;
            for (size_t w = 0; w < wd; ++w) {
                const int lo = 64 * (int)w;
                auto mask = [&](int bits) -> uint64_t {
                    if (bits >= lo + 64) return ~0ull;
                    if (bits <= lo) return 0ull;
                    return (1ull << (bits - lo)) - 1ull;
                };
                const uint64_t gm = mask(st.sh[i]), lm = mask(g.n_vars) & ~gm;
                hb[(ev * 4 + 0) * wd + w] = (eps ? gm : 0) | lm;
                hb[(ev * 4 + 1) * wd + w] = eps ? gm : 0;
                hb[(ev * 4 + 2) * wd + w] = ell ? gm : 0;
                hb[(ev * 4 + 3) * wd + w] = ell ? gm : 0;
            }
        }
        if (wd) CK(hipMemcpyAsync(G.sbnd[i], hb.data(), 8 * 16 * wd, hipMemcpyHostToDevice, G.s));
        CK(hipStreamSynchronize(G.s));   // host vectors are reused
    }
    G.S = (uint64_t*)(A + oS);
    G.cmask = (uint64_t*)(A + oCm);
    G.d_ap = (int32_t*)(A + oAp);
    G.d_av = (int32_t*)(A + oAv);
    G.d_ac = (uint8_t*)(A + oAc);
    {
        std::vector<int32_t> av(std::max<size_t>(nargs, 1), 0);
        std::vector<uint8_t> ac(std::max<size_t>(nargs, 1), 0);
        for (size_t t = 0; t < nargs; ++t) {
            av[t] = P->arg_var[t];
            ac[t] = P->arg_const ? (P->arg_const[t] ? 1 : 0) : 0;
        }
        CK(hipMemcpyAsync(G.d_ap, st.ap.data(), 4 * st.ap.size(), hipMemcpyHostToDevice, G.s));
        CK(hipMemcpyAsync(G.d_av, av.data(), 4 * av.size(), hipMemcpyHostToDevice, G.s));
        CK(hipMemcpyAsync(G.d_ac, ac.data(), ac.size(), hipMemcpyHostToDevice, G.s));
        CK(hipStreamSynchronize(G.s));
    }
    {
        std::vector<uint64_t> cm(std::max(gw, 1), 0);
        if (P->const_globals)
            for (int w = 0; w < gw; ++w) cm[w] = P->const_globals[w];
        CK(hipMemcpyAsync(G.cmask, cm.data(), 8 * cm.size(), hipMemcpyHostToDevice, G.s));
        CK(hipStreamSynchronize(G.s));
    }
    G.demand = (uint64_t*)(A + oD);
    G.demand_new = (uint64_t*)(A + oDn);
    G.caps = (uint64_t*)(A + oC);
    G.flag = (int32_t*)(A + oF);
    CK(hipMemsetAsync(G.demand, 0, 8 * (size_t)std::max(st.nc, 1) * sw, G.s));
    G.contrib = (uint64_t*)(A + oCb);
    G.in_edges = (int32_t*)(A + oIn);
    G.callers = (int32_t*)(A + oCl);
    G.gaps = (uint64_t*)(A + oGap);
    G.bnd0 = (uint64_t*)(A + oB0);
    CK(hipMemcpyAsync(G.in_edges, h_in.data(), 4 * h_in.size(), hipMemcpyHostToDevice, G.s));
    CK(hipMemcpyAsync(G.callers, h_callers.data(), 4 * h_callers.size(), hipMemcpyHostToDevice, G.s));
    // initial boundaries: a root context its procedure's own (defaults: valid and live on the
    // host only); any other context valid everywhere on its shared variables (the top of the
    // validity meet), its other locals valid on the host, nothing live after its exit
    {
        std::vector<uint64_t> b0(std::max<size_t>(G.bnd0_off[nctx], 1), 0);
        for (int x = 0; x < nctx; ++x) {
            const int p = st.cproc[x];
            const ompd_cfg& g = P->procs[p];
            const size_t wd = st.wd[p];
            uint64_t* b = b0.data() + G.bnd0_off[x];
            for (size_t w = 0; w < wd; ++w) {
                const int lo = 64 * (int)w;
                auto mask = [&](int bits) -> uint64_t {
                    if (bits >= lo + 64) return ~0ull;
                    if (bits <= lo) return 0ull;
                    return (1ull << (bits - lo)) - 1ull;
                };
                const uint64_t vm = mask(g.n_vars), gm = mask(st.sh[p]);
                if (st.cs1[x] < 0) {
                    b[w] = g.entry_valid_host ? g.entry_valid_host[w] : vm;
                    b[wd + w] = g.entry_valid_dev ? g.entry_valid_dev[w] : 0;
                    b[2 * wd + w] = g.exit_live_host ? g.exit_live_host[w] : vm;
                    b[3 * wd + w] = g.exit_live_dev ? g.exit_live_dev[w] : 0;
                } else {
                    b[w] = vm;
                    b[wd + w] = gm;
                }
            }
        }
        CK(hipMemcpyAsync(G.bnd0, b0.data(), 8 * b0.size(), hipMemcpyHostToDevice, G.s));
        CK(hipStreamSynchronize(G.s));
    }
    G.bnd.resize(nctx); G.ctab.resize(nctx);
    for (auto* v : {&G.o_nu_h, &G.o_nu_d, &G.o_ave_h, &G.o_ave_d, &G.o_avf_h, &G.o_avf_d, &G.o_ie_h, &G.o_ie_d,
                    &G.o_ig_h, &G.o_ig_d})
        v->resize(nctx);
    G.o_vk.resize(nctx); G.o_ad.resize(nctx); G.o_bd.resize(nctx); G.ctx_end.resize(nctx);
    G.sweeps.assign((size_t)nctx * 6, 0);
    for (int x = 0; x < nctx; ++x) {
        const int p = st.cproc[x];
        const size_t nb = st.nb[p], ne = st.ne[p], wd = st.wd[p];
        G.bnd[x] = (uint64_t*)(A + co[x].bnd);
        G.ctab[x] = (uint64_t*)(A + co[x].ctab);
        uint64_t* o = (uint64_t*)(A + co[x].out);
        const size_t bv = nb * wd, evv = ne * wd;
        G.o_nu_h[x] = o; G.o_nu_d[x] = o + bv; G.o_ave_h[x] = o + 2 * bv; G.o_ave_d[x] = o + 3 * bv;
        G.o_avf_h[x] = o + 4 * bv; G.o_avf_d[x] = o + 5 * bv; G.o_ie_h[x] = o + 6 * bv; G.o_ie_d[x] = o + 7 * bv;
        G.o_ig_h[x] = o + 8 * bv; G.o_ig_d[x] = o + 8 * bv + evv;
        uint8_t* b8 = (uint8_t*)(o + 8 * bv + 2 * evv);
        G.o_vk[x] = b8; G.o_ad[x] = b8 + P->procs[p].n_vars; G.o_bd[x] = b8 + P->procs[p].n_vars + nb;
        G.ctx_end[x] = (char*)(b8 + P->procs[p].n_vars + 2 * nb);
    }
    G.arena_items = A + oItems;
    return OMPD_OK;
}

Args site_args(const Prog& G, int j)
{
    Args a;
    a.var = G.d_av + G.st.ap[j];
    a.cst = G.d_ac + G.st.ap[j];
    a.n = G.st.ap[j + 1] - G.st.ap[j];
    return a;
}

// Call tables of procedure p for the summary evaluations (no caps) or of
// context x (caps of the callee contexts when they exist).
void calltab_items(Prog& G, int p, int x, std::vector<CallTabItem>& out)
{
    const Structure& st = G.st;
    const size_t wd = st.wd[p];
    for (size_t k = 0; k < st.sites[p].size(); ++k) {
        const int j = st.sites[p][k], q = G.P->callee[j];
        CallTabItem I;
        I.dst = (x < 0 ? G.ptab[p] : G.ctab[x]) + k * SUM_ROWS * wd;
        I.src = q < 0 ? nullptr : G.S + (size_t)q * SUM_ROWS * st.sw;
        I.cap = nullptr;
        if (x >= 0 && q >= 0) {
            const int cx = st.child[x][k];
            if (cx >= 0 && G.cap_valid[cx]) I.cap = G.caps + (size_t)cx * 2 * st.sw;
        }
        I.cmask = G.cmask;
        I.a = site_args(G, j);
        I.wd = (int32_t)wd; I.gw = st.gw; I.sw = st.sw; I.G = st.G; I.nv = G.P->procs[p].n_vars;
        out.push_back(I);
    }
}

ompd_cfg dev_cfg(Prog& G, int p)
{
    const ompd_cfg& g = G.P->procs[p];
    ompd_cfg d;
    memset(&d, 0, sizeof d);
    d.n_blocks = g.n_blocks; d.n_edges = g.n_edges; d.n_vars = g.n_vars; d.entry = g.entry; d.exit = g.exit;
    d.succ_ptr = G.sp[p]; d.succ_idx = G.si[p]; d.edge_kind = G.kind[p]; d.space = G.space[p];
    d.read_bits = G.Rd[p]; d.write_bits = G.W[p];
    if (!G.st.sites[p].empty()) {
        d.call_summary = G.call[p];
        d.n_summaries = (int32_t)G.st.sites[p].size();
    }
    return d;
}

// Evaluate the summaries of a set of procedures (4 boundary solves each) and
// gather the rows selected by `rows` (bit 0 next use, bit 1 validity tables).
int evaluate(Prog& G, const std::vector<int>& procs, int rows, int& changed)
{
    const Structure& st = G.st;
    changed = 0;
    if (procs.empty()) return OMPD_OK;
    std::vector<CallTabItem> ct;
    for (int p : procs) calltab_items(G, p, -1, ct);
    int rc = upload_items(ct, k_calltab, 256, G.s, G.arena_items);
    if (rc) return rc;
    std::vector<ompd_cfg> cfgs;
    std::vector<ompd_result> res;
    for (int p : procs) {
        const size_t wd = st.wd[p], bv = (size_t)st.nb[p] * wd;
        for (int ev = 0; ev < 4; ++ev) {
            ompd_cfg d = dev_cfg(G, p);
            if (d.call_summary) d.summaries = G.ptab[p];
            d.entry_valid_host = G.sbnd[p] + (ev * 4 + 0) * wd;
            d.entry_valid_dev = G.sbnd[p] + (ev * 4 + 1) * wd;
            d.exit_live_host = G.sbnd[p] + (ev * 4 + 2) * wd;
            d.exit_live_dev = G.sbnd[p] + (ev * 4 + 3) * wd;
            ompd_result r;
            memset(&r, 0, sizeof r);
            uint64_t* o = G.e_out[p] + (size_t)ev * 4 * bv;
            r.nu_host = o; r.nu_dev = o + bv; r.ave_host = o + 2 * bv; r.ave_dev = o + 3 * bv;
            cfgs.push_back(d);
            res.push_back(r);
        }
    }
    rc = run_batch(G, cfgs, res, OMPD_F_SUMMARY);
    if (rc) return rc;
    std::vector<SumItem> si;
    for (int p : procs) {
        const size_t wd = st.wd[p], bv = (size_t)st.nb[p] * wd;
        for (int ev = 0; ev < 4; ++ev) {
            SumItem I;
            const uint64_t* o = G.e_out[p] + (size_t)ev * 4 * bv;
            I.S = G.S + (size_t)p * SUM_ROWS * st.sw;
            I.nu_h = o; I.nu_d = o + bv; I.ave_h = o + 2 * bv; I.ave_d = o + 3 * bv;
            I.entry = G.P->procs[p].entry; I.exit = G.P->procs[p].exit;
            I.wd = (int32_t)wd; I.sw = st.sw; I.sh = st.sh[p]; I.eps = ev >> 1; I.ell = ev & 1; I.rows = rows;
            I.changed = G.flag;
            si.push_back(I);
        }
    }
    rc = zero_flag(G, G.flag);
    if (rc) return rc;
    rc = upload_items(si, k_sumgather, 64, G.s, G.arena_items);
    if (rc) return rc;
    return read_flag(G, G.flag, changed);
}

int may_rows(Prog& G, const std::vector<int>& procs, int& changed)
{
    const Structure& st = G.st;
    std::vector<MayItem> mi;
    for (int p : procs) {
        MayItem I;
        I.S = G.S + (size_t)p * SUM_ROWS * st.sw;
        I.R = G.Rd[p]; I.W = G.W[p]; I.space = G.space[p];
        I.callees = G.callees[p]; I.sites = G.sitej[p]; I.ap = G.d_ap; I.av = G.d_av; I.ac = G.d_ac;
        I.Sall = G.S; I.cmask = G.cmask;
        I.nb = st.nb[p]; I.wd = st.wd[p]; I.gw = st.gw; I.sw = st.sw; I.G = st.G; I.sh = st.sh[p];
        I.n_sites = (int32_t)st.sites[p].size();
        I.changed = G.flag;
        mi.push_back(I);
    }
    int rc = zero_flag(G, G.flag);
    if (rc) return rc;
    rc = upload_items(mi, k_may, 64, G.s, G.arena_items);
    if (rc) return rc;
    return read_flag(G, G.flag, changed);
}

// The rows of the calls made inside kernels of a set of procedures, from their callees' current
// may sets.
int device_calls(Prog& G, const std::vector<int>& procs)
{
    const Structure& st = G.st;
    std::vector<DevCallItem> it;
    for (int p : procs)
        for (int j : st.dsites[p]) {
            const int q = G.P->callee[j];
            DevCallItem I;
            I.Rd = G.Rd[p]; I.W = G.W[p];
            I.S = q < 0 ? nullptr : G.S + (size_t)q * SUM_ROWS * st.sw;
            I.cmask = G.cmask;
            I.a = site_args(G, j);
            I.block = G.P->call_block[j]; I.wd = st.wd[p]; I.gw = st.gw; I.sw = st.sw; I.G = st.G;
            it.push_back(I);
        }
    return upload_items(it, k_devcall, 64, G.s, G.arena_items);
}

// Bottom-up: components by level; a non-recursive procedure is evaluated
// once, a recursive component iterates its may-sets from 0, then its
// next-use rows from 0, then its validity tables from all ones.
int summarize(Prog& G)
{
    const Structure& st = G.st;
    CK(hipMemsetAsync(G.S, 0, 8 * (size_t)st.n * SUM_ROWS * st.sw, G.s));
    int max_level = 0;
    for (int l : st.comp_level) max_level = std::max(max_level, l);
    for (int level = 0; level <= max_level; ++level) {
        std::vector<int> single, recur_procs;
        std::vector<const std::vector<int>*> recur;
        for (size_t ci = 0; ci < st.comps.size(); ++ci) {
            if (st.comp_level[ci] != level) continue;
            const std::vector<int>& comp = st.comps[ci];
            bool self = false;
            if (comp.size() == 1)
                for (int j : st.sites[comp[0]]) self |= G.P->callee[j] == comp[0];
                for (int j : st.dsites[comp[0]]) self |= G.P->callee[j] == comp[0];
            if (comp.size() == 1 && !self) single.push_back(comp[0]);
            else {
                recur.push_back(&comp);
                recur_procs.insert(recur_procs.end(), comp.begin(), comp.end());
            }
        }
        int ch = 0;
        // calls made inside kernels read their callees' may sets (final below this level)
        int rc = device_calls(G, single);
        if (rc) return rc;
        rc = evaluate(G, single, 3, ch);
        if (rc) return rc;
        rc = may_rows(G, single, ch);
        if (rc) return rc;
        if (recur_procs.empty()) continue;
        // recursive components: validity tables start at all ones over the shared variables
        std::vector<uint64_t> rows(8 * (size_t)st.sw * recur_procs.size());
        for (size_t i = 0; i < recur_procs.size(); ++i) {
            const int sh = st.sh[recur_procs[i]];
            uint64_t* row = rows.data() + 8 * (size_t)st.sw * i;
            for (int w = 0; w < st.sw; ++w) {
                const int lo = 64 * w;
                const uint64_t gm = sh >= lo + 64 ? ~0ull : (sh <= lo ? 0ull : (1ull << (sh - lo)) - 1ull);
                for (int k = 0; k < 8; ++k) row[(size_t)k * st.sw + w] = gm;
            }
            CK(hipMemcpyAsync(G.S + ((size_t)recur_procs[i] * SUM_ROWS + SUM_TH) * st.sw, row, 8 * 8 * (size_t)st.sw,
                              hipMemcpyHostToDevice, G.s));
        }
        CK(hipStreamSynchronize(G.s));
        // may sets first (calls made inside kernels feed them into the callers' rows), then next
        // use from 0, then validity tables from all ones
        do {
            rc = device_calls(G, recur_procs);
            if (rc) return rc;
            rc = may_rows(G, recur_procs, ch);
            if (rc) return rc;
        } while (ch);
        for (int rows : {1, 2}) {
            do {
                rc = evaluate(G, recur_procs, rows, ch);
                if (rc) return rc;
            } while (ch);
        }
    }
    return OMPD_OK;
}

// Solve a set of contexts with their current boundaries and call tables
// (summary mode: a non-root context may leave a global valid nowhere).
int solve_contexts(Prog& G, const std::vector<int>& xs)
{
    const Structure& st = G.st;
    std::vector<CallTabItem> ct;
    for (int x : xs) calltab_items(G, st.cproc[x], x, ct);
    int rc = upload_items(ct, k_calltab, 256, G.s, G.arena_items);
    if (rc) return rc;
    std::vector<ompd_cfg> cfgs;
    std::vector<ompd_result> res;
    for (int x : xs) {
        const int p = st.cproc[x];
        const size_t wd = st.wd[p];
        ompd_cfg d = dev_cfg(G, p);
        if (d.call_summary) d.summaries = G.ctab[x];
        d.entry_valid_host = G.bnd[x]; d.entry_valid_dev = G.bnd[x] + wd;
        d.exit_live_host = G.bnd[x] + 2 * wd; d.exit_live_dev = G.bnd[x] + 3 * wd;
        ompd_result r;
        memset(&r, 0, sizeof r);
        r.nu_host = G.o_nu_h[x]; r.nu_dev = G.o_nu_d[x]; r.ave_host = G.o_ave_h[x]; r.ave_dev = G.o_ave_d[x];
        r.avf_host = G.o_avf_h[x]; r.avf_dev = G.o_avf_d[x];
        r.ins_entry_to_host = G.o_ie_h[x]; r.ins_entry_to_dev = G.o_ie_d[x];
        r.ins_edge_to_host = G.o_ig_h[x]; r.ins_edge_to_dev = G.o_ig_d[x];
        r.var_kind = G.o_vk[x]; r.after_dev = G.o_ad[x]; r.before_dev = G.o_bd[x];
        cfgs.push_back(d);
        res.push_back(r);
    }
    rc = run_batch(G, cfgs, res, OMPD_F_SUMMARY);
    if (rc) return rc;
    for (size_t i = 0; i < xs.size(); ++i) memcpy(&G.sweeps[(size_t)xs[i] * 6], res[i].sweeps, sizeof res[i].sweeps);
    return OMPD_OK;
}

// One monotone boundary system over the context graph, solved by rounds:
// every context whose boundary changed is solved, each of its calls writes
// its contribution to its edge slot, and every context reached recomputes the
// meet over all edges into it.  live = 1: exit liveness (least fixed point,
// contributions only grow); live = 0: entry validity (greatest fixed point,
// contributions only shrink).  Each system has one fixed point, so the order
// of the solves does not matter.  Every context is solved in the first round,
// so every edge slot holds a contribution before any meet reads it.
int boundary_system(Prog& G, int live)
{
    const Structure& st = G.st;
    const ompd_program* P = G.P;
    const int nctx = (int)st.cproc.size(), sw = st.sw;
    std::vector<int> dirty(nctx);
    for (int x = 0; x < nctx; ++x) dirty[x] = x;
    std::vector<char> is_t(nctx, 0);
    std::vector<int32_t> hc(nctx);
    while (!dirty.empty()) {
        int rc = solve_contexts(G, dirty);
        if (rc) return rc;
        std::vector<int> touched;
        std::vector<ContribItem> cb;
        for (int x : dirty) {
            const int p = st.cproc[x];
            for (size_t k = 0; k < st.sites[p].size(); ++k) {
                const int cx = st.child[x][k];
                if (cx < 0) continue;
                if (!is_t[cx]) { is_t[cx] = 1; touched.push_back(cx); }
                ContribItem I;
                I.a_h = live ? G.o_nu_h[x] : G.o_ave_h[x];
                I.a_d = live ? G.o_nu_d[x] : G.o_ave_d[x];
                I.W = G.W[p]; I.succ_ptr = G.sp[p]; I.succ_idx = G.si[p];
                I.out = G.contrib + (size_t)G.eid[x][k] * 2 * sw;
                I.a = site_args(G, st.sites[p][k]);
                I.c = P->call_block[st.sites[p][k]]; I.wd = st.wd[p]; I.gw = st.gw; I.sw = sw; I.G = st.G;
                I.live = live;
                cb.push_back(I);
            }
        }
        rc = upload_items(cb, k_contrib, 64, G.s, G.arena_items);
        if (rc) return rc;
        int32_t* chg = G.flag + 16;
        CK(hipMemsetAsync(chg, 0, 4 * (size_t)nctx, G.s));
        std::vector<MeetItem> mi;
        for (int cx : touched) {
            is_t[cx] = 0;
            const int q = st.cproc[cx];
            MeetItem I;
            I.bnd = G.bnd[cx]; I.contrib = G.contrib; I.in_edges = G.in_edges + G.in_ptr[cx];
            I.changed = chg + cx; I.n_in = G.in_ptr[cx + 1] - G.in_ptr[cx];
            I.wd = st.wd[q]; I.sw = sw; I.sh = st.sh[q]; I.nv = P->procs[q].n_vars; I.live = live;
            mi.push_back(I);
        }
        rc = upload_items(mi, k_meet, 64, G.s, G.arena_items);
        if (rc) return rc;
        CK(hipMemcpyAsync(hc.data(), chg, 4 * (size_t)nctx, hipMemcpyDeviceToHost, G.s));
        CK(hipStreamSynchronize(G.s));
        dirty.clear();
        for (int cx : touched)
            if (hc[cx]) dirty.push_back(cx);
        std::sort(dirty.begin(), dirty.end());
    }
    return OMPD_OK;
}

// Contexts of one outer round: fresh initial boundaries, the exit-liveness
// system, then the entry-validity system with that liveness (its last solve
// of every context is the context's final solution), then the host-read
// demands of the globals the contexts leave valid nowhere but read before
// writing them: each at the call site leading to the context, unless a
// calling context lacks that global at its own entry; when that leaves no
// demand at all (a cycle of recursive contexts), every gap is demanded.
int contexts(Prog& G)
{
    const Structure& st = G.st;
    const ompd_program* P = G.P;
    const int nctx = (int)st.cproc.size(), sw = st.sw;
    CK(hipMemsetAsync(G.demand_new, 0, 8 * (size_t)std::max(st.nc, 1) * sw, G.s));
    std::vector<CopyItem> cp;
    for (int x = 0; x < nctx; ++x) {
        CopyItem I;
        I.dst = G.bnd[x]; I.src = G.bnd0 + G.bnd0_off[x]; I.n = (int32_t)(G.bnd0_off[x + 1] - G.bnd0_off[x]);
        cp.push_back(I);
    }
    int rc = upload_items(cp, k_copy, 64, G.s, G.arena_items);
    if (rc) return rc;
    rc = boundary_system(G, 1);
    if (rc) return rc;
    rc = boundary_system(G, 0);
    if (rc) return rc;
    if (!sw) return OMPD_OK;
    CK(hipMemsetAsync(G.gaps, 0, 8 * (size_t)nctx * sw, G.s));
    int32_t* any = G.flag;
    CK(hipMemsetAsync(any, 0, 8, G.s));
    std::vector<GapItem> gi;
    std::vector<OwnItem> oi;
    for (int x = 0; x < nctx; ++x) {
        if (st.cs1[x] < 0) continue;
        const int p = st.cproc[x];
        GapItem I;
        I.gap = G.gaps + (size_t)x * sw; I.bnd = G.bnd[x]; I.nu_h = G.o_nu_h[x]; I.nu_d = G.o_nu_d[x];
        I.any = any; I.entry = P->procs[p].entry; I.wd = st.wd[p]; I.sw = sw; I.sh = st.sh[p];
        gi.push_back(I);
        const int j = st.cs1[x];
        OwnItem O;
        O.gaps = G.gaps; O.callers = G.callers + G.in_ptr[x]; O.demand = G.demand_new + (size_t)j * sw;
        O.any = any + 1; O.a = site_args(G, j); O.x = x; O.n_callers = G.in_ptr[x + 1] - G.in_ptr[x];
        O.gw = st.gw; O.sw = sw; O.G = st.G; O.sh_caller = st.sh[P->call_proc[j]]; O.all = 0;
        oi.push_back(O);
    }
    rc = upload_items(gi, k_gap, 64, G.s, G.arena_items);
    if (rc) return rc;
    int32_t flags[2];
    CK(hipMemcpyAsync(flags, any, 8, hipMemcpyDeviceToHost, G.s));
    CK(hipStreamSynchronize(G.s));
    if (!flags[0]) return OMPD_OK;
    rc = upload_items(oi, k_own, 64, G.s, G.arena_items);
    if (rc) return rc;
    CK(hipMemcpyAsync(flags, any, 8, hipMemcpyDeviceToHost, G.s));
    CK(hipStreamSynchronize(G.s));
    if (flags[1]) return OMPD_OK;
    for (auto& O : oi) O.all = 1;
    return upload_items(oi, k_own, 64, G.s, G.arena_items);
}

}  // namespace

extern "C" int ompd_program_contexts(ompd_ctx* ctx, const ompd_program* prog, int32_t* n_contexts, int32_t* ctx_proc,
                                     int32_t* ctx_site0, int32_t* ctx_site1, int32_t capacity)
{
    if (!ctx || !n_contexts) return ompd_fail(OMPD_E_INVAL, "ctx / n_contexts is NULL");
    Structure st;
    int rc = check_program(prog, st);
    if (rc) return rc;
    const int n = (int)st.cproc.size();
    *n_contexts = n;
    for (int x = 0; x < n && x < capacity; ++x) {
        if (ctx_proc) ctx_proc[x] = st.cproc[x];
        if (ctx_site0) ctx_site0[x] = st.cs0[x];
        if (ctx_site1) ctx_site1[x] = st.cs1[x];
    }
    return OMPD_OK;
}

extern "C" int ompd_analyze_program(ompd_ctx* ctx, const ompd_program* prog, ompd_program_result* out, uint32_t flags)
{
    if (!ctx || !out) return ompd_fail(OMPD_E_INVAL, "ctx / out is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    Prog G;
    G.ctx = ctx;
    G.P = prog;
    G.flags = flags & (0xFFFF0000u | OMPD_F_SCHED_LEVEL | OMPD_F_SCHED_WALK);
    int rc = check_program(prog, G.st);
    if (rc) return rc;
    CK(hipSetDevice(ctx->device));
    CK(hipStreamCreateWithFlags(&G.s, hipStreamNonBlocking));
    struct StreamGuard { hipStream_t s; ~StreamGuard() { (void)hipStreamDestroy(s); } } sg{G.s};
    rc = setup(G);
    if (rc) return rc;
    const Structure& st = G.st;
    const int nctx = (int)st.cproc.size(), sw = st.sw;   // rows over the shared layout
    G.cap_valid.assign(nctx, 0);
    std::vector<uint64_t> dem((size_t)std::max(st.nc, 1) * sw, 0), dnew(dem.size()), capv((size_t)nctx * 2 * sw),
        capn(capv.size());
    int rounds = 0;
    bool settled = false;
    while (rounds < 64) {
        ++rounds;
        rc = summarize(G);
        if (rc) return rc;
        rc = contexts(G);
        if (rc) return rc;
        // new caps: validity at EXIT of every non-root context
        std::vector<CapItem> ci;
        for (int x = 0; x < nctx; ++x) {
            if (st.cs1[x] < 0) continue;
            const int p = st.cproc[x];
            CapItem I;
            I.cap = G.caps + (size_t)x * 2 * sw;
            I.avf_h = G.o_avf_h[x]; I.avf_d = G.o_avf_d[x];
            I.exit = prog->procs[p].exit; I.wd = st.wd[p]; I.sw = sw; I.sh = st.sh[p];
            ci.push_back(I);
        }
        // previous caps, for the comparison
        if (sw) CK(hipMemcpyAsync(capv.data(), G.caps, 8 * capv.size(), hipMemcpyDeviceToHost, G.s));
        CK(hipStreamSynchronize(G.s));
        rc = upload_items(ci, k_cap, 64, G.s, G.arena_items);
        if (rc) return rc;
        if (sw) CK(hipMemcpyAsync(capn.data(), G.caps, 8 * capn.size(), hipMemcpyDeviceToHost, G.s));
        if (st.nc && sw) CK(hipMemcpyAsync(dnew.data(), G.demand_new, 8 * (size_t)st.nc * sw, hipMemcpyDeviceToHost, G.s));
        CK(hipStreamSynchronize(G.s));
        bool grew = false;
        for (int x = 0; x < nctx; ++x) {
            if (st.cs1[x] < 0) continue;
            bool same = G.cap_valid[x];
            for (int w = 0; w < 2 * sw && same; ++w) same = capv[(size_t)x * 2 * sw + w] == capn[(size_t)x * 2 * sw + w];
            if (!same) grew = true;
            G.cap_valid[x] = 1;
        }
        for (size_t k = 0; k < (size_t)st.nc * sw; ++k) {
            const uint64_t v = dem[k] | dnew[k];
            if (v != dem[k]) { dem[k] = v; grew = true; }
        }
        if (!grew) { settled = true; break; }
        // apply the demands: reads at the call blocks
        if (st.nc && sw) CK(hipMemcpyAsync(G.demand, dem.data(), 8 * (size_t)st.nc * sw, hipMemcpyHostToDevice, G.s));
        // (only a host call to a procedure leads to a context, so only such a site has a demand;
        // its bit n_globals + t is argument t, t < the callee's parameters)
        std::vector<DemandItem> di;
        for (int j = 0; j < st.nc; ++j) {
            if (st.site_k[j] < 0 || prog->callee[j] < 0) continue;
            const int p = prog->call_proc[j];
            DemandItem I;
            I.Rd = G.Rd[p]; I.R = G.R[p]; I.demand = G.demand + (size_t)j * sw;
            I.a = site_args(G, j);
            I.block = prog->call_block[j]; I.wd = st.wd[p]; I.gw = st.gw; I.G = st.G;
            di.push_back(I);
        }
        rc = upload_items(di, k_demand, 64, G.s, G.arena_items);
        if (rc) return rc;
    }
    out->rounds = rounds;
    out->solves = G.solves;
    if (!settled) return ompd_fail(OMPD_E_NOCONVERGE, "program: demands and caps did not settle in 64 rounds");
    // results to the host
    if (out->summaries && sw)
        CK(hipMemcpyAsync(out->summaries, G.S, 8 * (size_t)st.n * SUM_ROWS * sw, hipMemcpyDeviceToHost, G.s));
    if (out->demands && st.nc && sw)
        memcpy(out->demands, dem.data(), 8 * (size_t)st.nc * sw);
    // Per-context results: each context's region of the arena (boundaries, tables, outputs) is
    // contiguous and the regions follow each other, so runs of contexts go to a pinned staging
    // buffer in one copy and are scattered to the caller's arrays on the host (thousands of
    // small copies to pageable memory would cost more than the solve).
    std::vector<size_t> boffs(nctx);
    {
        size_t boff = 0;
        for (int x = 0; x < nctx; ++x) { boffs[x] = boff; boff += 4 * (size_t)st.wd[st.cproc[x]]; }
    }
    auto scatter = [&](int x, const char* base, const char* src) {
        // base: device address that src (a host copy of the same bytes) stands for
        const int p = st.cproc[x];
        const size_t nb = st.nb[p], ne = st.ne[p], wd = st.wd[p], bv = nb * wd, ev = ne * wd;
        auto at = [&](const void* dev) { return src + ((const char*)dev - base); };
        if (out->boundaries && wd) memcpy(out->boundaries + boffs[x], at(G.bnd[x]), 8 * 4 * wd);
        if (!out->per_context) return;
        ompd_result& r = out->per_context[x];
        auto cp = [&](void* dst, const void* dev, size_t bytes) { if (dst && bytes) memcpy(dst, at(dev), bytes); };
        cp(r.nu_host, G.o_nu_h[x], 8 * bv); cp(r.nu_dev, G.o_nu_d[x], 8 * bv);
        cp(r.ave_host, G.o_ave_h[x], 8 * bv); cp(r.ave_dev, G.o_ave_d[x], 8 * bv);
        cp(r.avf_host, G.o_avf_h[x], 8 * bv); cp(r.avf_dev, G.o_avf_d[x], 8 * bv);
        cp(r.ins_entry_to_host, G.o_ie_h[x], 8 * bv); cp(r.ins_entry_to_dev, G.o_ie_d[x], 8 * bv);
        cp(r.ins_edge_to_host, G.o_ig_h[x], 8 * ev); cp(r.ins_edge_to_dev, G.o_ig_d[x], 8 * ev);
        cp(r.var_kind, G.o_vk[x], (size_t)prog->procs[p].n_vars);
        cp(r.after_dev, G.o_ad[x], nb); cp(r.before_dev, G.o_bd[x], nb);
        if (r.fp_clause && bv) memset(r.fp_clause, 0, 8 * bv);   // procedures' scalar marks are not used
        memcpy(r.sweeps, &G.sweeps[(size_t)x * 6], sizeof r.sweeps);
    };
    const size_t STAGE = (size_t)64 << 20;
    char* stage = nullptr;
    if (hipHostMalloc((void**)&stage, STAGE, hipHostMallocDefault) != hipSuccess)
        return ompd_fail(OMPD_E_NOMEM, "program: pinned staging buffer");
    struct StageGuard { char* p; ~StageGuard() { (void)hipHostFree(p); } } stg{stage};
    CK(hipStreamSynchronize(G.s));
    std::vector<char> big;   // a context larger than the staging buffer (not in the shapes this targets)
    for (int x = 0; x < nctx;) {
        const char* base = (const char*)G.bnd[x];
        int y = x;
        while (y < nctx && (size_t)(G.ctx_end[y] - base) <= STAGE) ++y;
        if (y == x) {
            big.resize((size_t)(G.ctx_end[x] - base));
            CK(hipMemcpy(big.data(), base, big.size(), hipMemcpyDeviceToHost));
            scatter(x, base, big.data());
            ++x;
            continue;
        }
        CK(hipMemcpyAsync(stage, base, (size_t)(G.ctx_end[y - 1] - base), hipMemcpyDeviceToHost, G.s));
        CK(hipStreamSynchronize(G.s));
        for (int c = x; c < y; ++c) scatter(c, base, stage);
        x = y;
    }
    CK(hipStreamSynchronize(G.s));
    return OMPD_OK;
}
