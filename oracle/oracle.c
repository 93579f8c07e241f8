/*
 * ORACLE — test infrastructure only.
 *
 * A plain, single-threaded CPU worklist solver for the data-flow problems of
 * OMPDart (Marzen, Dutta, Jannesari, "Static Generation of Efficient OpenMP
 * Offload Data Mappings", SC24).  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the GPU library never links
 * or calls it, and the two share no source, header or helper.
 *
 * The paper describes its analysis operationally (a forward traversal that
 * tracks, per variable, whether the host and the device copy are valid; RAW
 * dependencies across memory spaces; loop-aware placement of map/update
 * constructs; region-exit liveness).  This file computes the exact fixed
 * points of one equational reading of that description, phase by phase, in
 * the order the paper's traversal implies:
 *
 *   NU   next use per memory space      backward, may (OR),  least f.p.
 *        (region-exit liveness, paper section "Data-Flow Analysis", last
 *        paragraph; liveness definition in the background section)
 *   AVE  validity per memory space      forward, must (AND), greatest f.p.
 *        (valid = last written in that space; a host write makes the device
 *        copy stale and vice versa; a read of stale data is a true RAW
 *        dependency — "Data-Flow Analysis")
 *   EAG  eager copy on an edge: needed next and not valid at the source
 *   MAYP copies that may still be pending after an edge   forward, may
 *   LATER delayed placement: a copy owed on a path slides down the CFG until
 *        a read needs it, never into a loop and never across a join where
 *        another path holds fresh data only in the target space (the loop
 *        rule of "Data-Flow Analysis" and the outermost-loop placement of the
 *        array-access section / Algorithm 1)
 *   AVF  validity after the final placement   forward, must
 *   labels map(to/from/tofrom/alloc) versus target update (Table II), from
 *        reachability of device blocks (one target data region per function)
 *
 * Two variants of the placement, selected by the caller:
 *   pure lazy  the delay without the loop rule: loop-entry edges are
 *        ordinary edges for MAYP and LATER, so a copy may slide into a loop
 *        and be made on every trip (the placement the loop rule of
 *        "Data-Flow Analysis" avoids; for comparison).  The join rule still
 *        holds, so a copy enters a loop only where every trip around it
 *        leaves both copies valid again.
 *   loop-entry refinement  Algorithm 1 puts the update that a loop's
 *        writes make necessary after the loop nest.  The delay stops at
 *        loop entries, so a copy owed before a loop stays on its entry edge
 *        even when every path through the loop copies again before reading.
 *        LIVE (backward, may) finds whether the value a copy leaves is read
 *        before a write or another copy into the same space replaces it; a
 *        copy on a loop-entry edge whose value is never read is dropped.
 *
 * firstprivate (section "Data-Flow Analysis", the firstprivate paragraph,
 * and Table II): a read-only scalar may reach a kernel as a firstprivate
 * argument initialised from the host copy instead of being mapped.  The
 * caller marks scalar variables; a marked variable that no DEVICE block
 * writes is firstprivate.  A DEVICE block's read of it then needs the HOST
 * copy valid at the kernel launch (a host use, not a device use), and at the
 * end of that kernel the device copy is no longer valid; the kernel carries
 * a firstprivate clause for it.
 *
 * Interprocedural call blocks (section "Interprocedural Analysis") are
 * modelled by exact per-global summaries of the callee passed in by the
 * caller of this function: next use at the callee entry for exit-liveness 0
 * and 1, validity at the callee exit for the four (entry-valid, exit-live)
 * combinations, and flow-insensitive may-read / may-write bits.
 *
 * Bit layout: variable v is bit (v & 63) of word (v >> 6); block vectors are
 * [block][word], edge vectors are [edge][word] in successor-CSR order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

#define KIND_NORMAL 0
#define KIND_BACK 1
#define KIND_LOOP_ENTRY 2

/* summary table rows, each a [wd] word vector (identity for locals) */
enum {
    SUM_MAYR_H = 0, SUM_MAYR_D, SUM_MAYW_H, SUM_MAYW_D,
    SUM_NU0_H, SUM_NU0_D, SUM_NU1_H, SUM_NU1_D,
    SUM_TH_00, SUM_TH_01, SUM_TH_10, SUM_TH_11,   /* T_H[entry valid][exit live] */
    SUM_TD_00, SUM_TD_01, SUM_TD_10, SUM_TD_11,
    SUM_ROWS
};

typedef struct {
    int nb, ne, nv, wd, entry, exit;
    const int32_t* sp;  const int32_t* si;   /* successor CSR */
    int32_t* pp; int32_t* pi; int32_t* pe;   /* predecessor CSR: pred block, succ-edge id */
    const uint8_t* kind; const uint8_t* space;
    const uint64_t* R; const uint64_t* W;
    const uint64_t* ev[2]; const uint64_t* lx[2];
    const int32_t* call; const uint64_t* sums;
    uint64_t lastmask;
    uint64_t* fp;          /* [wd] firstprivate variables (all zero when no scalar is marked) */
    int summary_mode;
    int lazy;              /* pure lazy: loop-entry edges do not stop the delay */
    int32_t* rpo;  /* reverse post-order from ENTRY */
} G;

static inline size_t ix(const G* g, int b, int w) { return (size_t)b * (size_t)g->wd + (size_t)w; }

static inline uint64_t vmask(const G* g, int w) { return (w == g->wd - 1) ? g->lastmask : ~0ull; }

static const uint64_t* sumrow(const G* g, int b, int row)
{
    return g->sums + ((size_t)g->call[b] * SUM_ROWS + (size_t)row) * (size_t)g->wd;
}

static inline int is_call(const G* g, int b) { return g->call && g->call[b] >= 0; }

/* USE_s(b) = R_b when b lies in space s; at EXIT it is the caller-supplied
 * liveness after the region (region-exit liveness).  A DEVICE block's read
 * of a firstprivate variable is a use of the HOST copy (the kernel is
 * launched with the host value). */
static inline uint64_t use_s(const G* g, int s, int b, int w)
{
    if (b == g->exit) return g->lx[s][w];
    uint64_t r = g->R[ix(g, b, w)];
    if (g->space[b] == 1) return s == 1 ? (r & ~g->fp[w]) : (r & g->fp[w]);
    return s == 0 ? r : 0ull;
}

/* WR_s(b) = W_b when b lies in space s. */
static inline uint64_t wr_s(const G* g, int s, int b, int w)
{
    return ((int)g->space[b] == s) ? g->W[ix(g, b, w)] : 0ull;
}

/* USE' : a call block whose callee may touch the variable stops a pending
 * copy exactly like a read (owed copies never cross an opaque call). */
static inline uint64_t use_stop(const G* g, int s, int b, int w)
{
    uint64_t u = use_s(g, s, b, w);
    if (is_call(g, b))
        u |= sumrow(g, b, s == 0 ? SUM_MAYR_H : SUM_MAYR_D)[w] |
             sumrow(g, b, SUM_MAYW_H)[w] | sumrow(g, b, SUM_MAYW_D)[w];
    return u;
}

/* FIFO worklist with membership flags */
typedef struct { int32_t* q; uint8_t* in; int head, n, cap; } WL;
static int wl_init(WL* l, int cap)
{
    l->q = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    l->in = (uint8_t*)calloc((size_t)cap, 1);
    l->head = 0; l->n = 0; l->cap = cap;
    return (l->q && l->in) ? 0 : -1;
}
static void wl_free(WL* l) { free(l->q); free(l->in); }
static void wl_push(WL* l, int b)
{
    if (l->in[b]) return;
    l->in[b] = 1;
    l->q[(l->head + l->n) % l->cap] = b;
    l->n++;
}
static int wl_pop(WL* l)
{
    int b = l->q[l->head];
    l->head = (l->head + 1) % l->cap;
    l->n--;
    l->in[b] = 0;
    return b;
}

/* ------------------------------------------------------------------ */
/* validation and normalisation                                        */
/* ------------------------------------------------------------------ */
static int validate_and_prepare(G* g)
{
    int nb = g->nb, ne = g->ne;
    if (nb < 2 || ne < 0 || g->nv < 0) return OR_EINVAL;
    if (g->entry < 0 || g->entry >= nb || g->exit < 0 || g->exit >= nb || g->entry == g->exit) return OR_EINVAL;
    if (g->sp[0] != 0 || g->sp[nb] != ne) return OR_EINVAL;
    for (int b = 0; b < nb; ++b) if (g->sp[b + 1] < g->sp[b]) return OR_EINVAL;
    for (int e = 0; e < ne; ++e) {
        if (g->si[e] < 0 || g->si[e] >= nb) return OR_EINVAL;
        if (g->kind[e] > KIND_LOOP_ENTRY) return OR_EINVAL;
    }
    for (int b = 0; b < nb; ++b) if (g->space[b] > 1) return OR_EINVAL;
    if (g->space[g->entry] != 0 || g->space[g->exit] != 0) return OR_EINVAL;
    if (g->sp[g->exit + 1] != g->sp[g->exit]) return OR_EINVAL;          /* EXIT has no successors */
    for (int e = 0; e < ne; ++e) {
        if (g->si[e] == g->entry) return OR_EINVAL;                       /* ENTRY has no predecessors */
        if (g->si[e] == g->exit && g->kind[e] != KIND_NORMAL) return OR_EINVAL;
    }
    for (int e = g->sp[g->entry]; e < g->sp[g->entry + 1]; ++e)
        if (g->kind[e] == KIND_BACK) return OR_EINVAL;
    for (int w = 0; w < g->wd; ++w) {
        if (g->R[ix(g, g->entry, w)] | g->W[ix(g, g->entry, w)] |
            g->R[ix(g, g->exit, w)] | g->W[ix(g, g->exit, w)]) return OR_EINVAL;
        uint64_t pad = ~vmask(g, w);
        if ((g->ev[0][w] | g->ev[1][w] | g->lx[0][w] | g->lx[1][w]) & pad) return OR_EINVAL;
        if (!g->summary_mode && ((g->ev[0][w] | g->ev[1][w]) & vmask(g, w)) != vmask(g, w)) return OR_EINVAL;
    }
    for (int b = 0; b < nb; ++b)
        for (int w = 0; w < g->wd; ++w)
            if ((g->R[ix(g, b, w)] | g->W[ix(g, b, w)]) & ~vmask(g, w)) return OR_EINVAL;
    if (g->call) {
        for (int b = 0; b < nb; ++b)
            if (g->call[b] >= 0 && (g->space[b] != 0 || b == g->entry || b == g->exit)) return OR_EINVAL;
    }

    /* predecessor CSR (pred block + id of the successor-CSR edge) */
    g->pp = (int32_t*)calloc((size_t)nb + 1, sizeof(int32_t));
    g->pi = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
    g->pe = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
    g->rpo = (int32_t*)malloc(sizeof(int32_t) * (size_t)nb);
    if (!g->pp || !g->pi || !g->pe || !g->rpo) return OR_ENOMEM;
    for (int e = 0; e < ne; ++e) g->pp[g->si[e] + 1]++;
    for (int b = 0; b < nb; ++b) g->pp[b + 1] += g->pp[b];
    int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)nb);
    if (!fill) return OR_ENOMEM;
    memcpy(fill, g->pp, sizeof(int32_t) * (size_t)nb);
    for (int b = 0; b < nb; ++b)
        for (int e = g->sp[b]; e < g->sp[b + 1]; ++e) {
            int q = g->si[e];
            g->pi[fill[q]] = b; g->pe[fill[q]] = e; fill[q]++;
        }
    free(fill);

    /* DFS from ENTRY (children in CSR order) -> reverse post-order */
    int32_t* stk = (int32_t*)malloc(sizeof(int32_t) * (size_t)nb);
    int32_t* it = (int32_t*)malloc(sizeof(int32_t) * (size_t)nb);
    uint8_t* seen = (uint8_t*)calloc((size_t)nb, 1);
    if (!stk || !it || !seen) return OR_ENOMEM;
    int top = 0, npost = 0;
    stk[top++] = g->entry; seen[g->entry] = 1; it[g->entry] = g->sp[g->entry];
    while (top > 0) {
        int b = stk[top - 1];
        if (it[b] < g->sp[b + 1]) {
            int q = g->si[it[b]++];
            if (!seen[q]) { seen[q] = 1; it[q] = g->sp[q]; stk[top++] = q; }
        } else {
            g->rpo[nb - 1 - npost] = b; npost++; top--;
        }
    }
    int ok = (npost == nb);                 /* every block reachable from ENTRY */
    if (ok) {                               /* every block reaches EXIT */
        memset(seen, 0, (size_t)nb);
        top = 0; stk[top++] = g->exit; seen[g->exit] = 1;
        int cnt = 1;
        while (top > 0) {
            int q = stk[--top];
            for (int k = g->pp[q]; k < g->pp[q + 1]; ++k) {
                int p = g->pi[k];
                if (!seen[p]) { seen[p] = 1; stk[top++] = p; cnt++; }
            }
        }
        ok = (cnt == nb);
    }
    free(stk); free(it); free(seen);
    return ok ? OR_OK : OR_EINVAL;
}

/* ------------------------------------------------------------------ */
/* NU: next use per space (backward, may, least fixed point)            */
/*   NUin_s(b)  = USE_s(b) | (NUout_s(b) & ~W_b)                        */
/*   NUout_s(b) = OR over successors q of NUin_s(q)                      */
/* a write in either space ends the next use (the reader would see the  */
/* new value); reads in a block precede its writes.                     */
/* call block: NUin = USE | (~W & (NU0 | (NU1 & NUout)))                */
/* ------------------------------------------------------------------ */
static int64_t phase_nu(const G* g, uint64_t* nu_h, uint64_t* nu_d)
{
    uint64_t* nu[2] = { nu_h, nu_d };
    memset(nu_h, 0, sizeof(uint64_t) * (size_t)g->nb * (size_t)g->wd);
    memset(nu_d, 0, sizeof(uint64_t) * (size_t)g->nb * (size_t)g->wd);
    WL l; if (wl_init(&l, g->nb)) return -1;
    for (int i = g->nb - 1; i >= 0; --i) wl_push(&l, g->rpo[i]);
    int64_t visits = 0;
    while (l.n > 0) {
        int b = wl_pop(&l);
        visits++;
        int changed = 0;
        for (int s = 0; s < 2; ++s)
            for (int w = 0; w < g->wd; ++w) {
                uint64_t out = 0;
                for (int e = g->sp[b]; e < g->sp[b + 1]; ++e) out |= nu[s][ix(g, g->si[e], w)];
                uint64_t v;
                if (is_call(g, b)) {
                    uint64_t nu0 = sumrow(g, b, s == 0 ? SUM_NU0_H : SUM_NU0_D)[w];
                    uint64_t nu1 = sumrow(g, b, s == 0 ? SUM_NU1_H : SUM_NU1_D)[w];
                    v = use_s(g, s, b, w) | (~g->W[ix(g, b, w)] & (nu0 | (nu1 & out)));
                } else {
                    v = use_s(g, s, b, w) | (out & ~g->W[ix(g, b, w)]);
                }
                v &= vmask(g, w);
                if (v != nu[s][ix(g, b, w)]) { nu[s][ix(g, b, w)] = v; changed = 1; }
            }
        if (changed)
            for (int k = g->pp[b]; k < g->pp[b + 1]; ++k) wl_push(&l, g->pi[k]);
    }
    wl_free(&l);
    return visits;
}

/* Validity transfer of one block (shared by AVE and AVF):
 *   block in space s:        out_s = in_s | W   (written here: valid here)
 *   block in the other space: out_s = in_s & ~W (written there: stale here)
 *   DEVICE block, device copy: also & ~(R & FP) (firstprivate: not valid after the kernel)
 * call block: A1 = the above; out_s = T_s[A1][NUout_s]. */
static uint64_t valid_out(const G* g, int s, int b, int w, uint64_t in_s, const uint64_t* nu_s)
{
    uint64_t Wb = g->W[ix(g, b, w)];
    uint64_t a1 = ((int)g->space[b] == s) ? (in_s | Wb) : (in_s & ~Wb);
    /* after a kernel that reads a firstprivate variable its device copy is no longer valid */
    if (s == 1 && g->space[b] == 1) a1 &= ~(g->R[ix(g, b, w)] & g->fp[w]);
    if (!is_call(g, b)) return a1;
    uint64_t l = 0;
    for (int e = g->sp[b]; e < g->sp[b + 1]; ++e) l |= nu_s[ix(g, g->si[e], w)];
    int base = (s == 0) ? SUM_TH_00 : SUM_TD_00;
    uint64_t t00 = sumrow(g, b, base + 0)[w], t01 = sumrow(g, b, base + 1)[w];
    uint64_t t10 = sumrow(g, b, base + 2)[w], t11 = sumrow(g, b, base + 3)[w];
    return (~a1 & ~l & t00) | (~a1 & l & t01) | (a1 & ~l & t10) | (a1 & l & t11);
}

/* ------------------------------------------------------------------ */
/* AVE: validity with eager copies (forward, must, greatest f.p.)       */
/*   AVEin_s(ENTRY) = ENTRY_VALID_s                                     */
/*   AVEin_s(q)     = NUin_s(q) | AND over preds p of AVEout_s(p)        */
/* the NU term is the effect of an eager copy on every in-edge where s  */
/* is needed next.                                                      */
/* ------------------------------------------------------------------ */
static int64_t phase_ave(const G* g, const uint64_t* nu_h, const uint64_t* nu_d,
                         uint64_t* in_h, uint64_t* in_d, uint64_t* out_h, uint64_t* out_d)
{
    const uint64_t* nu[2] = { nu_h, nu_d };
    uint64_t* in[2] = { in_h, in_d };
    uint64_t* out[2] = { out_h, out_d };
    size_t n = (size_t)g->nb * (size_t)g->wd;
    for (size_t i = 0; i < n; ++i) { out_h[i] = ~0ull; out_d[i] = ~0ull; in_h[i] = ~0ull; in_d[i] = ~0ull; }
    WL l; if (wl_init(&l, g->nb)) return -1;
    for (int i = 0; i < g->nb; ++i) wl_push(&l, g->rpo[i]);
    int64_t visits = 0;
    while (l.n > 0) {
        int q = wl_pop(&l);
        visits++;
        int changed = 0;
        for (int s = 0; s < 2; ++s)
            for (int w = 0; w < g->wd; ++w) {
                uint64_t vin;
                if (q == g->entry) vin = g->ev[s][w];
                else {
                    uint64_t meet = ~0ull;
                    for (int k = g->pp[q]; k < g->pp[q + 1]; ++k) meet &= out[s][ix(g, g->pi[k], w)];
                    vin = nu[s][ix(g, q, w)] | meet;
                }
                vin &= vmask(g, w);
                uint64_t vout = valid_out(g, s, q, w, vin, nu[s]) & vmask(g, w);
                in[s][ix(g, q, w)] = vin;
                if (vout != out[s][ix(g, q, w)]) { out[s][ix(g, q, w)] = vout; changed = 1; }
            }
        if (changed)
            for (int e = g->sp[q]; e < g->sp[q + 1]; ++e) wl_push(&l, g->si[e]);
    }
    wl_free(&l);
    return visits;
}

/* EAG_s(e = p->q) = NUin_s(q) & ~AVEout_s(p): the eager copy right after
 * the producer, wherever s is needed next and not surely valid. */
static inline uint64_t eag(const G* g, const uint64_t* nu_s, const uint64_t* aveout_s, int p, int q, int w)
{
    return nu_s[ix(g, q, w)] & ~aveout_s[ix(g, p, w)];
}

static inline uint64_t le_mask(const G* g, int e)
{
    return (!g->lazy && g->kind[e] == KIND_LOOP_ENTRY) ? ~0ull : 0ull;
}

/* ------------------------------------------------------------------ */
/* MAYP: copies that may be pending (forward, may, least f.p.)          */
/*   MAYP_s(e=p->q) = (EAG_s(e) | MAYPout_s(p)) & ~LE(e)                */
/*   MAYPin_s(q)    = OR over in-edges of MAYP_s(e)                      */
/*   MAYPout_s(q)   = MAYPin_s(q) & ~USE'_s(q) & ~WR_s(q)                */
/* ------------------------------------------------------------------ */
static int64_t phase_mayp(const G* g, const uint64_t* nu[2], const uint64_t* aveout[2], uint64_t* mout[2])
{
    size_t n = (size_t)g->nb * (size_t)g->wd;
    memset(mout[0], 0, sizeof(uint64_t) * n);
    memset(mout[1], 0, sizeof(uint64_t) * n);
    WL l; if (wl_init(&l, g->nb)) return -1;
    for (int i = 0; i < g->nb; ++i) wl_push(&l, g->rpo[i]);
    int64_t visits = 0;
    while (l.n > 0) {
        int q = wl_pop(&l);
        visits++;
        if (q == g->entry) continue;   /* MAYPout(ENTRY) = 0 */
        int changed = 0;
        for (int s = 0; s < 2; ++s)
            for (int w = 0; w < g->wd; ++w) {
                uint64_t min = 0;
                for (int k = g->pp[q]; k < g->pp[q + 1]; ++k) {
                    int p = g->pi[k], e = g->pe[k];
                    min |= (eag(g, nu[s], aveout[s], p, q, w) | mout[s][ix(g, p, w)]) & ~le_mask(g, e);
                }
                uint64_t v = min & ~use_stop(g, s, q, w) & ~wr_s(g, s, q, w) & vmask(g, w);
                if (v != mout[s][ix(g, q, w)]) { mout[s][ix(g, q, w)] = v; changed = 1; }
            }
        if (changed)
            for (int e = g->sp[q]; e < g->sp[q + 1]; ++e) wl_push(&l, g->si[e]);
    }
    wl_free(&l);
    return visits;
}

/* FV_x(e=p->q) = (AVEout_x(p) | EAG_x(e)) & ~MAYP_x(e): x surely valid
 * after edge e under the final placement. */
static inline uint64_t fv(const G* g, int x, const uint64_t* nu[2], const uint64_t* aveout[2],
                          uint64_t* const mout[2], int p, int q, int e, int w)
{
    uint64_t ea = eag(g, nu[x], aveout[x], p, q, w);
    uint64_t mayp_e = (ea | mout[x][ix(g, p, w)]) & ~le_mask(g, e);
    return (aveout[x][ix(g, p, w)] | ea) & ~mayp_e;
}

/* ------------------------------------------------------------------ */
/* LATER: delayed placement (forward, least f.p., monotone AND/OR)      */
/*   LATER_s(e)   = EAG_s(e) | LATERout_s(p)        copy owed on e       */
/*   L'_s(e)      = LATER_s(e) & ~LE(e)             may keep moving down */
/*   N'_s(e)      = (FV_s(e) & FV_o(e)) | (LATER_s(e) & LE(e))  neutral   */
/*   LATERin_s(q) = AND_e (L'_s(e) | N'_s(e))  &  OR_e L'_s(e)          */
/*   LATERout_s(q)= LATERin_s(q) & ~USE'_s(q) & ~WR_s(q)                */
/* ------------------------------------------------------------------ */
static int64_t phase_later(const G* g, const uint64_t* nu[2], const uint64_t* aveout[2],
                           uint64_t* const mout[2], uint64_t* lin[2], uint64_t* lout[2])
{
    size_t n = (size_t)g->nb * (size_t)g->wd;
    for (int s = 0; s < 2; ++s) { memset(lin[s], 0, sizeof(uint64_t) * n); memset(lout[s], 0, sizeof(uint64_t) * n); }
    WL l; if (wl_init(&l, g->nb)) return -1;
    for (int i = 0; i < g->nb; ++i) wl_push(&l, g->rpo[i]);
    int64_t visits = 0;
    while (l.n > 0) {
        int q = wl_pop(&l);
        visits++;
        if (q == g->entry) continue;   /* LATERin(ENTRY) = 0 */
        int changed = 0;
        for (int s = 0; s < 2; ++s) {
            int o = 1 - s;
            for (int w = 0; w < g->wd; ++w) {
                uint64_t all = ~0ull, any = 0;
                for (int k = g->pp[q]; k < g->pp[q + 1]; ++k) {
                    int p = g->pi[k], e = g->pe[k];
                    uint64_t later_e = eag(g, nu[s], aveout[s], p, q, w) | lout[s][ix(g, p, w)];
                    uint64_t lp = later_e & ~le_mask(g, e);
                    uint64_t np = (fv(g, s, nu, aveout, mout, p, q, e, w) & fv(g, o, nu, aveout, mout, p, q, e, w)) |
                                  (later_e & le_mask(g, e));
                    all &= (lp | np);
                    any |= lp;
                }
                uint64_t vin = all & any & vmask(g, w);
                uint64_t vout = vin & ~use_stop(g, s, q, w) & ~wr_s(g, s, q, w);
                lin[s][ix(g, q, w)] = vin;
                if (vout != lout[s][ix(g, q, w)]) { lout[s][ix(g, q, w)] = vout; changed = 1; }
            }
        }
        if (changed)
            for (int e = g->sp[q]; e < g->sp[q + 1]; ++e) wl_push(&l, g->si[e]);
    }
    wl_free(&l);
    return visits;
}

/* ------------------------------------------------------------------ */
/* LIVE: is the value in space s read before it is replaced             */
/*   (backward, may, least f.p.; o = the other space)                   */
/*   READ_s(q): a read of the s copy: USE_s(q); a call block reads both */
/*              copies of every variable (its callee may)               */
/*   KILL_s(q): WR_s(q), and at a DEVICE block the device copy of a     */
/*              firstprivate variable it reads (no longer valid after)  */
/*   A_s(q)   = READ_s(q) | (LO_s(q) & ~KILL_s(q))   after entry copies */
/*   LI_s(q)  = (A_s(q) & ~IE_s(q)) | IE_o(q)                           */
/*              a copy into s replaces the s value, a copy into o reads */
/*              it (every copy that stays reads its source, so a copy   */
/*              counts as a read whether or not its own value is read)  */
/*   LO_s(q)  = OR over edges e = q->t of (LI_s(t) & ~IG_s(e)) | IG_o(e) */
/* ------------------------------------------------------------------ */
static int64_t phase_live(const G* g, uint64_t* const ie[2], uint64_t* const ig[2], uint64_t* li[2])
{
    size_t n = (size_t)g->nb * (size_t)g->wd;
    memset(li[0], 0, sizeof(uint64_t) * n);
    memset(li[1], 0, sizeof(uint64_t) * n);
    WL l; if (wl_init(&l, g->nb)) return -1;
    for (int i = g->nb - 1; i >= 0; --i) wl_push(&l, g->rpo[i]);
    int64_t visits = 0;
    while (l.n > 0) {
        int q = wl_pop(&l);
        visits++;
        int changed = 0;
        for (int s = 0; s < 2; ++s) {
            int o = 1 - s;
            for (int w = 0; w < g->wd; ++w) {
                uint64_t lo = 0;
                for (int e = g->sp[q]; e < g->sp[q + 1]; ++e)
                    lo |= (li[s][ix(g, g->si[e], w)] & ~ig[s][(size_t)e * g->wd + w]) | ig[o][(size_t)e * g->wd + w];
                uint64_t rd = is_call(g, q) ? ~0ull : use_s(g, s, q, w);
                uint64_t kill = wr_s(g, s, q, w);
                if (s == 1 && g->space[q] == 1) kill |= g->R[ix(g, q, w)] & g->fp[w];
                uint64_t a = rd | (lo & ~kill);
                uint64_t v = ((a & ~ie[s][ix(g, q, w)]) | ie[o][ix(g, q, w)]) & vmask(g, w);
                if (v != li[s][ix(g, q, w)]) { li[s][ix(g, q, w)] = v; changed = 1; }
            }
        }
        if (changed)
            for (int k = g->pp[q]; k < g->pp[q + 1]; ++k) wl_push(&l, g->pi[k]);
    }
    wl_free(&l);
    return visits;
}

/* ------------------------------------------------------------------ */
/* AVF: validity after the final placement (forward, must, greatest)    */
/*   AVFin_s(q) = INS_ENTRY_s(q) | AND_e (AVFout_s(p) | INS_EDGE_s(e))  */
/* ------------------------------------------------------------------ */
static int64_t phase_avf(const G* g, const uint64_t* nu[2], uint64_t* const ins_entry[2], uint64_t* const ins_edge[2],
                         uint64_t* in[2], uint64_t* out[2])
{
    size_t n = (size_t)g->nb * (size_t)g->wd;
    for (int s = 0; s < 2; ++s)
        for (size_t i = 0; i < n; ++i) { in[s][i] = ~0ull; out[s][i] = ~0ull; }
    WL l; if (wl_init(&l, g->nb)) return -1;
    for (int i = 0; i < g->nb; ++i) wl_push(&l, g->rpo[i]);
    int64_t visits = 0;
    while (l.n > 0) {
        int q = wl_pop(&l);
        visits++;
        int changed = 0;
        for (int s = 0; s < 2; ++s)
            for (int w = 0; w < g->wd; ++w) {
                uint64_t vin;
                if (q == g->entry) vin = g->ev[s][w];
                else {
                    uint64_t meet = ~0ull;
                    for (int k = g->pp[q]; k < g->pp[q + 1]; ++k) {
                        int p = g->pi[k], e = g->pe[k];
                        meet &= out[s][ix(g, p, w)] | ins_edge[s][(size_t)e * g->wd + w];
                    }
                    vin = ins_entry[s][ix(g, q, w)] | meet;
                }
                vin &= vmask(g, w);
                uint64_t vout = valid_out(g, s, q, w, vin, nu[s]) & vmask(g, w);
                in[s][ix(g, q, w)] = vin;
                if (vout != out[s][ix(g, q, w)]) { out[s][ix(g, q, w)] = vout; changed = 1; }
            }
        if (changed)
            for (int e = g->sp[q]; e < g->sp[q + 1]; ++e) wl_push(&l, g->si[e]);
    }
    wl_free(&l);
    return visits;
}

/* ------------------------------------------------------------------ */
/* public entry point                                                  */
/* ------------------------------------------------------------------ */
/*
 * oracle_solve — solve one CFG.
 *   n_blocks includes the access-free HOST blocks ENTRY and EXIT.
 *   ev_h/ev_d  : validity of each variable in host/device memory at ENTRY [wd]
 *   lx_h/lx_d  : next use after EXIT (liveness after the region)        [wd]
 *   call       : [n_blocks] summary index for call blocks, -1 otherwise (NULL = no calls)
 *   sums       : [n_summaries][SUM_ROWS][wd]
 *   scalar     : [wd] variables the front end marks as scalars (NULL = none); those that
 *                no DEVICE block writes are firstprivate
 *   placement  : bit 0: 0 = delayed placement (LATER), 1 = eager placement only;
 *                bit 1: pure lazy: the delay ignores loop entries (with bit 0 clear);
 *                bit 2: loop-entry refinement of the delayed placement (LIVE);
 *                bit 8: evaluate a procedure summary — the boundary may leave a
 *                variable valid in neither space (a summary's entry-validity
 *                argument ranges over all of {0,1} per space)
 * Outputs (caller-owned; every pointer required):
 *   nu_*[nb*wd] NUin, ave_*[nb*wd] AVEin, avf_*[nb*wd] AVFin,
 *   ins_entry_*[nb*wd] copy into that space just before block b,
 *   ins_edge_*[ne*wd] copy into that space on edge e,
 *   var_kind[nv] (1 MAP_TO | 2 MAP_FROM | 4 MAP_ALLOC | 8 FIRSTPRIVATE), after_dev[nb], before_dev[nb],
 *   fp_clause[nb*wd] the firstprivate clause of each DEVICE block (the firstprivate variables it reads),
 *   visits[6] worklist pops per phase (NU, AVE, MAYP, LATER, AVF, labels).
 * Returns 0, -1 (malformed input) or -2 (out of host memory).
 */
int oracle_solve(int32_t nb, int32_t ne, int32_t nv, int32_t entry, int32_t exit_,
                 const int32_t* succ_ptr, const int32_t* succ_idx, const uint8_t* kind, const uint8_t* space,
                 const uint64_t* R, const uint64_t* W,
                 const uint64_t* ev_h, const uint64_t* ev_d, const uint64_t* lx_h, const uint64_t* lx_d,
                 const int32_t* call, const uint64_t* sums, int32_t placement,
                 const uint64_t* scalar,
                 uint64_t* nu_h, uint64_t* nu_d, uint64_t* ave_h, uint64_t* ave_d,
                 uint64_t* avf_h, uint64_t* avf_d,
                 uint64_t* ins_entry_h, uint64_t* ins_entry_d, uint64_t* ins_edge_h, uint64_t* ins_edge_d,
                 uint8_t* var_kind, uint8_t* after_dev, uint8_t* before_dev, uint64_t* fp_clause, int64_t* visits)
{
    G g;
    memset(&g, 0, sizeof(g));
    g.nb = nb; g.ne = ne; g.nv = nv; g.wd = (nv + 63) / 64; g.entry = entry; g.exit = exit_;
    g.sp = succ_ptr; g.si = succ_idx; g.kind = kind; g.space = space; g.R = R; g.W = W;
    g.ev[0] = ev_h; g.ev[1] = ev_d; g.lx[0] = lx_h; g.lx[1] = lx_d;
    g.call = call; g.sums = sums;
    g.lastmask = (nv % 64) ? ((1ull << (nv % 64)) - 1ull) : ~0ull;
    g.summary_mode = (placement >> 8) & 1;
    g.lazy = !(placement & 1) && ((placement >> 1) & 1);
    const int refine = !(placement & 1) && !g.lazy && ((placement >> 2) & 1);
    placement &= 1;
    g.fp = (uint64_t*)calloc((size_t)(g.wd > 0 ? g.wd : 1), sizeof(uint64_t));
    if (!g.fp) return OR_ENOMEM;
    int rc = validate_and_prepare(&g);
    if (rc != OR_OK) { free(g.pp); free(g.pi); free(g.pe); free(g.rpo); free(g.fp); return rc; }
    /* firstprivate: marked scalars that no DEVICE block writes */
    if (scalar) {
        for (int w = 0; w < g.wd; ++w) {
            uint64_t dev_w = 0;
            for (int b = 0; b < nb; ++b) if (space[b] == 1) dev_w |= W[ix(&g, b, w)];
            g.fp[w] = scalar[w] & ~dev_w & vmask(&g, w);
        }
    }

    size_t n = (size_t)nb * (size_t)g.wd;
    size_t nedge = (size_t)ne * (size_t)g.wd;
    uint64_t* aveout_h = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t* aveout_d = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t* mout_h = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t* mout_d = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t* lin_h = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t* lin_d = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t* lout_h = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t* lout_d = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t* avfout_h = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t* avfout_d = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    if (!aveout_h || !aveout_d || !mout_h || !mout_d || !lin_h || !lin_d || !lout_h || !lout_d || !avfout_h || !avfout_d) {
        rc = OR_ENOMEM; goto done;
    }
    for (int i = 0; i < 6; ++i) visits[i] = 0;

    visits[0] = phase_nu(&g, nu_h, nu_d);
    visits[1] = phase_ave(&g, nu_h, nu_d, ave_h, ave_d, aveout_h, aveout_d);
    {
        const uint64_t* nu[2] = { nu_h, nu_d };
        const uint64_t* aveout[2] = { aveout_h, aveout_d };
        uint64_t* mout[2] = { mout_h, mout_d };
        uint64_t* lin[2] = { lin_h, lin_d };
        uint64_t* lout[2] = { lout_h, lout_d };
        uint64_t* ie[2] = { ins_entry_h, ins_entry_d };
        uint64_t* ig[2] = { ins_edge_h, ins_edge_d };
        if (placement == 0) {
            visits[2] = phase_mayp(&g, nu, aveout, mout);
            visits[3] = phase_later(&g, nu, aveout, mout, lin, lout);
            /* materialise:
             *   INS_EDGE_s(e=p->q) = LATER_s(e) & (LE(e) | ~LATERin_s(q))
             *   INS_ENTRY_s(q)     = LATERin_s(q) & USE'_s(q)            */
            for (int s = 0; s < 2; ++s) {
                for (int q = 0; q < nb; ++q)
                    for (int w = 0; w < g.wd; ++w)
                        ie[s][ix(&g, q, w)] = lin[s][ix(&g, q, w)] & use_stop(&g, s, q, w) & vmask(&g, w);
                for (int p = 0; p < nb; ++p)
                    for (int e = succ_ptr[p]; e < succ_ptr[p + 1]; ++e) {
                        int q = succ_idx[e];
                        for (int w = 0; w < g.wd; ++w) {
                            uint64_t later_e = eag(&g, nu[s], aveout[s], p, q, w) | lout[s][ix(&g, p, w)];
                            ig[s][(size_t)e * g.wd + w] =
                                later_e & (le_mask(&g, e) | ~lin[s][ix(&g, q, w)]) & vmask(&g, w);
                        }
                    }
            }
        } else {
            /* eager placement only: every EAG is materialised on its edge */
            for (int s = 0; s < 2; ++s) {
                memset(ie[s], 0, sizeof(uint64_t) * n);
                for (int p = 0; p < nb; ++p)
                    for (int e = succ_ptr[p]; e < succ_ptr[p + 1]; ++e)
                        for (int w = 0; w < g.wd; ++w)
                            ig[s][(size_t)e * g.wd + w] = eag(&g, nu[s], aveout[s], p, succ_idx[e], w) & vmask(&g, w);
            }
        }
        if (refine) {
            /* drop the copies on loop-entry edges whose value no read uses (the AVF
             * buffers serve as LIVE's state: AVF overwrites them next) */
            uint64_t* li[2] = { avf_h, avf_d };
            if (phase_live(&g, ie, ig, li) < 0) { rc = OR_ENOMEM; goto done; }
            for (int e = 0; e < ne; ++e) {
                if (kind[e] != KIND_LOOP_ENTRY) continue;
                int t = succ_idx[e];
                for (int s = 0; s < 2; ++s)
                    for (int w = 0; w < g.wd; ++w) ig[s][(size_t)e * g.wd + w] &= li[s][ix(&g, t, w)];
            }
        }
        uint64_t* ain[2] = { avf_h, avf_d };
        uint64_t* aout[2] = { avfout_h, avfout_d };
        visits[4] = phase_avf(&g, nu, ie, ig, ain, aout);
    }

    /* labels (Table II): one target data region per function.
     * AFTER_DEV(b): some DEVICE block reaches b (b included)
     * BEFORE_DEV(b): b reaches some DEVICE block (b included)
     * copy into D on p->q is map(to) iff !AFTER_DEV(p); before q iff no
     * predecessor is AFTER_DEV; otherwise target update to.
     * copy into H on p->q or before q is map(from) iff !BEFORE_DEV(q);
     * otherwise target update from. */
    {
        int32_t* stk = (int32_t*)malloc(sizeof(int32_t) * (size_t)nb);
        if (!stk) { rc = OR_ENOMEM; goto done; }
        int top = 0;
        memset(after_dev, 0, (size_t)nb);
        memset(before_dev, 0, (size_t)nb);
        for (int b = 0; b < nb; ++b) if (space[b] == 1) { after_dev[b] = 1; stk[top++] = b; }
        while (top > 0) {
            int b = stk[--top];
            for (int e = succ_ptr[b]; e < succ_ptr[b + 1]; ++e) {
                int q = succ_idx[e];
                if (!after_dev[q]) { after_dev[q] = 1; stk[top++] = q; }
            }
        }
        for (int b = 0; b < nb; ++b) if (space[b] == 1) { before_dev[b] = 1; stk[top++] = b; }
        while (top > 0) {
            int q = stk[--top];
            for (int k = g.pp[q]; k < g.pp[q + 1]; ++k) {
                int p = g.pi[k];
                if (!before_dev[p]) { before_dev[p] = 1; stk[top++] = p; }
            }
        }
        free(stk);
        /* firstprivate clauses: a kernel reading a firstprivate variable */
        for (int b = 0; b < nb; ++b)
            for (int w = 0; w < g.wd; ++w)
                fp_clause[ix(&g, b, w)] = space[b] == 1 ? (R[ix(&g, b, w)] & g.fp[w]) : 0ull;
        memset(var_kind, 0, (size_t)(nv > 0 ? nv : 0));
        for (int v = 0; v < nv; ++v) {
            int w = v >> 6;
            uint64_t bit = 1ull << (v & 63);
            int to = 0, from = 0, dev_access = 0, fp_read = 0;
            for (int q = 0; q < nb; ++q) {
                int pred_after = 0;
                for (int k = g.pp[q]; k < g.pp[q + 1]; ++k) pred_after |= after_dev[g.pi[k]];
                if ((ins_entry_d[ix(&g, q, w)] & bit) && !pred_after) to = 1;
                if ((ins_entry_h[ix(&g, q, w)] & bit) && !before_dev[q]) from = 1;
                if (space[q] == 1 && (((R[ix(&g, q, w)] & ~g.fp[w]) | W[ix(&g, q, w)]) & bit)) dev_access = 1;
                if (space[q] == 1 && (R[ix(&g, q, w)] & g.fp[w] & bit)) fp_read = 1;
                for (int e = succ_ptr[q]; e < succ_ptr[q + 1]; ++e) {
                    int t = succ_idx[e];
                    if ((ins_edge_d[(size_t)e * g.wd + w] & bit) && !after_dev[q]) to = 1;
                    if ((ins_edge_h[(size_t)e * g.wd + w] & bit) && !before_dev[t]) from = 1;
                }
            }
            var_kind[v] = (uint8_t)((to ? 1 : 0) | (from ? 2 : 0) | ((dev_access && !to && !from) ? 4 : 0) |
                                    (fp_read ? 8 : 0));
        }
        visits[5] = nb;
    }
    (void)nedge;
done:
    free(aveout_h); free(aveout_d); free(mout_h); free(mout_d);
    free(lin_h); free(lin_d); free(lout_h); free(lout_d); free(avfout_h); free(avfout_d);
    free(g.pp); free(g.pi); free(g.pe); free(g.rpo); free(g.fp);
    return rc;
}
