/*
 * Seeded synthetic workloads for the OMPDart data-flow solve.
 *
 * This module only PRODUCES inputs: structured control-flow graphs whose
 * blocks are tagged host or device, per-block read/write bitmaps, call
 * graphs and call sites.  It contains none of the analysis arithmetic; the
 * oracle and the GPU solver both consume what it writes.
 *
 * Random streams:
 *   SplitMix64 (Steele, Lea, Flood 2014) mixes seeds;
 *   xoshiro256** (Blackman and Vigna 2018) is the stream generator.
 * Both are written here from their published definitions.
 *
 * CFG model (the AST-CFG of the paper's approach section, statement nodes
 * only): a random structured program is grown from one statement by
 * repeatedly expanding a uniformly chosen leaf statement into a sequence,
 * an if, an if/else, a while loop or a do-while loop, until exactly
 * n_user blocks exist.  Blocks are numbered in source (pre-order) order,
 * ENTRY = 0, user blocks 1..n_user, EXIT = n_user + 1.  Edges into a loop
 * header from outside the loop are LOOP_ENTRY, edges from inside the loop
 * back to its header are BACK, all others NORMAL.  Whole statement
 * subtrees (loops first) become offload kernels until the requested
 * fraction of blocks is DEVICE.  A fraction of loops receives one extra
 * NORMAL edge from the statement just before the loop into a non-header
 * block of the loop body, which makes that loop irreducible.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ------------------------------------------------------------------ */
/* random streams                                                      */
/* ------------------------------------------------------------------ */
uint64_t synth_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct { uint64_t s[4]; } xo_t;

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static void xo_seed(xo_t* g, uint64_t seed)
{
    uint64_t st = seed;
    for (int i = 0; i < 4; ++i) {
        st += 0x9E3779B97F4A7C15ull;
        uint64_t z = st;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        g->s[i] = z ^ (z >> 31);
    }
}

static inline uint64_t xo_next(xo_t* g)
{
    uint64_t* s = g->s;
    const uint64_t out = rotl64(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return out;
}

static inline double xo_unif(xo_t* g) { return (double)(xo_next(g) >> 11) * 0x1.0p-53; }

static inline uint64_t xo_below(xo_t* g, uint64_t n)
{
    return (uint64_t)(((__uint128_t)xo_next(g) * (__uint128_t)n) >> 64);
}

/* Word of 64 independent Bernoulli(thr/65536) bits: binary-expansion
 * method, least significant digit first (OR for a 1 digit, AND for 0). */
static inline uint64_t xo_bernoulli_word(xo_t* g, uint32_t thr16)
{
    if (thr16 == 0) return 0;
    if (thr16 >= 65536u) return ~0ull;
    uint64_t x = 0;
    for (int i = 0; i < 16; ++i) {
        uint64_t r = xo_next(g);
        x = ((thr16 >> i) & 1u) ? (x | r) : (x & r);
    }
    return x;
}

int64_t synth_log_uniform_int(uint64_t seed, int64_t lo, int64_t hi)
{
    xo_t g;
    xo_seed(&g, seed);
    double u = xo_unif(&g);
    double v = exp(log((double)lo) + u * (log((double)hi) - log((double)lo)));
    int64_t r = (int64_t)llround(v);
    if (r < lo) r = lo;
    if (r > hi) r = hi;
    return r;
}

/* ------------------------------------------------------------------ */
/* structured program (AST of statements)                              */
/* ------------------------------------------------------------------ */
enum { N_LEAF = 0, N_SEQ, N_IF, N_IFELSE, N_WHILE, N_DOWHILE };

typedef struct {
    int type;
    int parent;
    int first, next;      /* first child, next sibling */
    int loop_depth;       /* loops strictly enclosing this node */
    int blk, blk2;        /* own blocks: leaf / cond / header / head, and do-while cond */
    int lo, hi;           /* pre-order block range of the subtree */
    int prev_sib;         /* previous sibling (for irreducible entries) */
} node_t;

typedef struct {
    node_t* nd;
    int n_nodes, cap_nodes;
    int* leaves; int* leaf_pos;  /* expandable leaves */
    int n_leaves;
    int n_blocks_user;           /* blocks created so far */
} ast_t;

static int ast_new(ast_t* a, int type, int parent, int depth)
{
    if (a->n_nodes == a->cap_nodes) {
        a->cap_nodes = a->cap_nodes ? 2 * a->cap_nodes : 64;
        a->nd = (node_t*)realloc(a->nd, sizeof(node_t) * (size_t)a->cap_nodes);
        a->leaf_pos = (int*)realloc(a->leaf_pos, sizeof(int) * (size_t)a->cap_nodes);
    }
    int id = a->n_nodes++;
    node_t* n = &a->nd[id];
    memset(n, 0, sizeof(*n));
    n->type = type; n->parent = parent; n->first = -1; n->next = -1;
    n->loop_depth = depth; n->blk = -1; n->blk2 = -1; n->prev_sib = -1;
    a->leaf_pos[id] = -1;
    return id;
}

static void leaf_add(ast_t* a, int id) { a->leaf_pos[id] = a->n_leaves; a->leaves[a->n_leaves++] = id; }
static void leaf_del(ast_t* a, int id)
{
    int p = a->leaf_pos[id];
    int last = a->leaves[--a->n_leaves];
    a->leaves[p] = last; a->leaf_pos[last] = p; a->leaf_pos[id] = -1;
}

static void append_child(ast_t* a, int parent, int child)
{
    node_t* P = &a->nd[parent];
    if (P->first < 0) { P->first = child; return; }
    int c = P->first;
    while (a->nd[c].next >= 0) c = a->nd[c].next;
    a->nd[c].next = child;
}

/* Grow a program with exactly n_user blocks. */
static void ast_grow(ast_t* a, xo_t* g, int n_user, int max_depth)
{
    a->leaves = (int*)malloc(sizeof(int) * (size_t)(2 * n_user + 8));
    int root = ast_new(a, N_SEQ, -1, 0);
    int l0 = ast_new(a, N_LEAF, root, 0);
    append_child(a, root, l0);
    leaf_add(a, l0);
    a->n_blocks_user = 1;
    /* statement kinds: seq 0.40, if 0.20, if/else 0.15, loop 0.25 (30 % do-while) */
    while (a->n_blocks_user < n_user) {
        int remaining = n_user - a->n_blocks_user;
        int L = a->leaves[xo_below(g, (uint64_t)a->n_leaves)];
        int depth = a->nd[L].loop_depth;
        double u = xo_unif(g);
        int kind;
        if (u < 0.40) kind = N_SEQ;
        else if (u < 0.60) kind = N_IF;
        else if (u < 0.75) kind = N_IFELSE;
        else kind = (xo_unif(g) < 0.30) ? N_DOWHILE : N_WHILE;
        if ((kind == N_WHILE || kind == N_DOWHILE) && depth >= max_depth) kind = N_SEQ;
        if ((kind == N_IFELSE || kind == N_DOWHILE) && remaining < 2) kind = N_SEQ;
        if (kind == N_SEQ) {
            int par = a->nd[L].parent;
            if (par >= 0 && a->nd[par].type == N_SEQ) {
                int M = ast_new(a, N_LEAF, par, a->nd[par].loop_depth);
                /* insert M right after L */
                a->nd[M].next = a->nd[L].next;
                a->nd[L].next = M;
                leaf_add(a, M);
            } else {
                /* wrap L in a new sequence inside its parent */
                int S = ast_new(a, N_SEQ, par, depth);
                /* replace L by S in parent's child list */
                node_t* P = &a->nd[par];
                if (P->first == L) { P->first = S; }
                else {
                    int c = P->first;
                    while (a->nd[c].next != L) c = a->nd[c].next;
                    a->nd[c].next = S;
                }
                a->nd[S].next = a->nd[L].next;
                a->nd[L].next = -1;
                a->nd[L].parent = S;
                a->nd[S].first = L;
                int M = ast_new(a, N_LEAF, S, depth);
                a->nd[L].next = M;
                leaf_add(a, M);
            }
            a->n_blocks_user += 1;
        } else if (kind == N_IF) {
            leaf_del(a, L);
            a->nd[L].type = N_IF;
            int T = ast_new(a, N_LEAF, L, depth);
            a->nd[L].first = T;
            leaf_add(a, T);
            a->n_blocks_user += 1;
        } else if (kind == N_IFELSE) {
            leaf_del(a, L);
            a->nd[L].type = N_IFELSE;
            int T = ast_new(a, N_LEAF, L, depth);
            int E = ast_new(a, N_LEAF, L, depth);
            a->nd[L].first = T; a->nd[T].next = E;
            leaf_add(a, T); leaf_add(a, E);
            a->n_blocks_user += 2;
        } else if (kind == N_WHILE) {
            leaf_del(a, L);
            a->nd[L].type = N_WHILE;
            int B = ast_new(a, N_LEAF, L, depth + 1);
            a->nd[L].first = B;
            leaf_add(a, B);
            a->n_blocks_user += 1;
        } else { /* do-while: fixed head statement, body leaf, condition */
            leaf_del(a, L);
            a->nd[L].type = N_DOWHILE;
            int B = ast_new(a, N_LEAF, L, depth + 1);
            a->nd[L].first = B;
            leaf_add(a, B);
            a->n_blocks_user += 2;
        }
    }
}

/* pre-order block numbering; user blocks start at 1 */
static int ast_number(ast_t* a, int id, int next_blk)
{
    node_t* n = &a->nd[id];
    n->lo = next_blk;
    switch (n->type) {
    case N_LEAF: n->blk = next_blk++; break;
    case N_SEQ: {
        int prev = -1;
        for (int c = n->first; c >= 0; c = a->nd[c].next) {
            a->nd[c].prev_sib = prev;
            next_blk = ast_number(a, c, next_blk);
            prev = c;
        }
        break;
    }
    case N_IF: case N_IFELSE: case N_WHILE:
        n->blk = next_blk++;
        for (int c = n->first; c >= 0; c = a->nd[c].next) next_blk = ast_number(a, c, next_blk);
        break;
    case N_DOWHILE:
        n->blk = next_blk++;
        for (int c = n->first; c >= 0; c = a->nd[c].next) next_blk = ast_number(a, c, next_blk);
        n->blk2 = next_blk++;
        break;
    }
    n->hi = next_blk - 1;
    return next_blk;
}

static int entry_blk(const ast_t* a, int id)
{
    const node_t* n = &a->nd[id];
    if (n->type == N_SEQ) return entry_blk(a, n->first);
    return n->blk;
}

typedef struct { int32_t* src; int32_t* dst; int n, cap; } edges_t;
static void add_edge(edges_t* e, int s, int d)
{
    if (e->n == e->cap) {
        e->cap = e->cap ? 2 * e->cap : 256;
        e->src = (int32_t*)realloc(e->src, sizeof(int32_t) * (size_t)e->cap);
        e->dst = (int32_t*)realloc(e->dst, sizeof(int32_t) * (size_t)e->cap);
    }
    e->src[e->n] = s; e->dst[e->n] = d; e->n++;
}

static void ast_edges(const ast_t* a, int id, int cont, edges_t* e)
{
    const node_t* n = &a->nd[id];
    switch (n->type) {
    case N_LEAF: add_edge(e, n->blk, cont); break;
    case N_SEQ:
        for (int c = n->first; c >= 0; c = a->nd[c].next) {
            int nx = a->nd[c].next;
            ast_edges(a, c, nx >= 0 ? entry_blk(a, nx) : cont, e);
        }
        break;
    case N_IF: {
        int t = n->first;
        add_edge(e, n->blk, entry_blk(a, t));
        add_edge(e, n->blk, cont);
        ast_edges(a, t, cont, e);
        break;
    }
    case N_IFELSE: {
        int t = n->first, f = a->nd[t].next;
        add_edge(e, n->blk, entry_blk(a, t));
        add_edge(e, n->blk, entry_blk(a, f));
        ast_edges(a, t, cont, e);
        ast_edges(a, f, cont, e);
        break;
    }
    case N_WHILE: {
        int b = n->first;
        add_edge(e, n->blk, entry_blk(a, b));
        add_edge(e, n->blk, cont);
        ast_edges(a, b, n->blk, e);
        break;
    }
    case N_DOWHILE: {
        int b = n->first;
        add_edge(e, n->blk, entry_blk(a, b));
        ast_edges(a, b, n->blk2, e);
        add_edge(e, n->blk2, n->blk);
        add_edge(e, n->blk2, cont);
        break;
    }
    }
}

/* Fenwick tree over block ids for "any device block in range" queries */
static void fw_add(int* t, int n, int i, int v) { for (++i; i <= n; i += i & -i) t[i] += v; }
static int fw_sum(const int* t, int i) { int s = 0; for (++i; i > 0; i -= i & -i) s += t[i]; return s; }

/* ------------------------------------------------------------------ */
/* public: one CFG                                                     */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t n_user;          /* user blocks (ENTRY/EXIT not counted) */
    int32_t n_vars;
    int32_t max_loop_depth;
    int32_t n_call_sites;    /* host leaf blocks marked as call sites (program generator) */
    double  device_frac;
    double  irr_loop_frac;
    uint32_t thr_read;       /* Bernoulli thresholds in 1/65536 */
    uint32_t thr_write;
} synth_params;

typedef struct {
    int n_blocks, n_edges;
    int32_t* succ_ptr; int32_t* succ_idx; uint8_t* kind; uint8_t* space;
    int32_t* loop_depth;     /* per block */
    int32_t* call_blocks;    /* [n_call_sites] */
    int n_calls;
} cfg_tmp_t;

static void cfg_tmp_free(cfg_tmp_t* c)
{
    free(c->succ_ptr); free(c->succ_idx); free(c->kind); free(c->space);
    free(c->loop_depth); free(c->call_blocks);
    memset(c, 0, sizeof(*c));
}

/* Builds the structure (not the access bits). Returns 0 or -1. */
static int build_structure(uint64_t seed, const synth_params* p, cfg_tmp_t* out)
{
    memset(out, 0, sizeof(*out));
    if (p->n_user < 1 || p->max_loop_depth < 0) return -1;
    xo_t g;
    xo_seed(&g, seed);
    ast_t a; memset(&a, 0, sizeof(a));
    ast_grow(&a, &g, p->n_user, p->max_loop_depth);
    int nb = p->n_user + 2;
    ast_number(&a, 0, 1);
    edges_t e; memset(&e, 0, sizeof(e));
    add_edge(&e, 0, entry_blk(&a, 0));
    ast_edges(&a, 0, nb - 1, &e);

    /* per-block loop depth and loop header ranges */
    int32_t* ldepth = (int32_t*)calloc((size_t)nb, sizeof(int32_t));
    int* hdr_lo = (int*)malloc(sizeof(int) * (size_t)nb);   /* header block -> loop range */
    int* hdr_hi = (int*)malloc(sizeof(int) * (size_t)nb);
    for (int b = 0; b < nb; ++b) { hdr_lo[b] = -1; hdr_hi[b] = -1; }
    int n_loops = 0;
    for (int i = 0; i < a.n_nodes; ++i) {
        node_t* n = &a.nd[i];
        if (n->type == N_WHILE || n->type == N_DOWHILE) {
            hdr_lo[n->blk] = n->lo; hdr_hi[n->blk] = n->hi; n_loops++;
            for (int b = n->lo; b <= n->hi; ++b) ldepth[b]++;
        }
    }

    /* irreducible entries */
    int n_irr = (int)llround(p->irr_loop_frac * (double)n_loops);
    if (n_irr > 0) {
        int* cand = (int*)malloc(sizeof(int) * (size_t)a.n_nodes);
        int nc = 0;
        for (int i = 0; i < a.n_nodes; ++i) {
            node_t* n = &a.nd[i];
            if ((n->type == N_WHILE || n->type == N_DOWHILE) && n->hi > n->lo &&
                n->prev_sib >= 0 && a.nd[n->prev_sib].type == N_LEAF)
                cand[nc++] = i;
        }
        for (int k = 0; k < n_irr && nc > 0; ++k) {
            int j = (int)xo_below(&g, (uint64_t)nc);
            int li = cand[j]; cand[j] = cand[--nc];
            node_t* n = &a.nd[li];
            int u = a.nd[n->prev_sib].blk;
            int tgt = n->lo + 1 + (int)xo_below(&g, (uint64_t)(n->hi - n->lo));
            add_edge(&e, u, tgt);
        }
        free(cand);
    }

    /* CSR by source, preserving insertion order */
    int ne = e.n;
    int32_t* ptr = (int32_t*)calloc((size_t)nb + 1, sizeof(int32_t));
    for (int i = 0; i < ne; ++i) ptr[e.src[i] + 1]++;
    for (int b = 0; b < nb; ++b) ptr[b + 1] += ptr[b];
    int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)nb);
    memcpy(fill, ptr, sizeof(int32_t) * (size_t)nb);
    int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
    uint8_t* kind = (uint8_t*)malloc((size_t)(ne > 0 ? ne : 1));
    for (int i = 0; i < ne; ++i) {
        int s = e.src[i], d = e.dst[i];
        int pos = fill[s]++;
        idx[pos] = d;
        uint8_t k = 0;
        if (hdr_lo[d] >= 0) k = (s >= hdr_lo[d] && s <= hdr_hi[d]) ? 1 : 2;
        kind[pos] = k;
    }
    free(fill);

    /* offload kernels: whole statement subtrees, loops first */
    uint8_t* space = (uint8_t*)calloc((size_t)nb, 1);
    int target = (int)llround(p->device_frac * (double)p->n_user);
    if (target > 0) {
        int* order = (int*)malloc(sizeof(int) * (size_t)a.n_nodes);
        int no = 0;
        for (int i = 1; i < a.n_nodes; ++i)
            if (a.nd[i].type == N_WHILE || a.nd[i].type == N_DOWHILE) order[no++] = i;
        int n_first = no;
        for (int i = 1; i < a.n_nodes; ++i)
            if (!(a.nd[i].type == N_WHILE || a.nd[i].type == N_DOWHILE)) order[no++] = i;
        for (int i = n_first - 1; i > 0; --i) { int j = (int)xo_below(&g, (uint64_t)i + 1); int t = order[i]; order[i] = order[j]; order[j] = t; }
        for (int i = no - 1; i > n_first; --i) { int j = n_first + (int)xo_below(&g, (uint64_t)(i - n_first) + 1); int t = order[i]; order[i] = order[j]; order[j] = t; }
        int* fw = (int*)calloc((size_t)nb + 1, sizeof(int));
        int remaining = target;
        for (int k = 0; k < no && remaining > 0; ++k) {
            node_t* n = &a.nd[order[k]];
            int size = n->hi - n->lo + 1;
            if (size > remaining) continue;
            if (fw_sum(fw, n->hi) - fw_sum(fw, n->lo - 1) != 0) continue;
            for (int b = n->lo; b <= n->hi; ++b) { space[b] = 1; fw_add(fw, nb, b, 1); }
            remaining -= size;
        }
        free(fw); free(order);
    }

    /* call sites: distinct host leaf statements */
    int32_t* calls = NULL;
    int n_calls = 0;
    if (p->n_call_sites > 0) {
        int* cand = (int*)malloc(sizeof(int) * (size_t)a.n_nodes);
        int nc = 0;
        for (int i = 0; i < a.n_nodes; ++i)
            if (a.nd[i].type == N_LEAF && space[a.nd[i].blk] == 0) cand[nc++] = a.nd[i].blk;
        calls = (int32_t*)malloc(sizeof(int32_t) * (size_t)p->n_call_sites);
        for (int k = 0; k < p->n_call_sites && nc > 0; ++k) {
            int j = (int)xo_below(&g, (uint64_t)nc);
            calls[n_calls++] = cand[j]; cand[j] = cand[--nc];
        }
        free(cand);
    }

    free(hdr_lo); free(hdr_hi);
    free(e.src); free(e.dst);
    free(a.nd); free(a.leaves); free(a.leaf_pos);
    out->n_blocks = nb; out->n_edges = ne;
    out->succ_ptr = ptr; out->succ_idx = idx; out->kind = kind; out->space = space;
    out->loop_depth = ldepth; out->call_blocks = calls; out->n_calls = n_calls;
    return 0;
}

/* Number of edges of the CFG that synth_cfg_fill will produce. */
int64_t synth_cfg_edges(uint64_t seed, const synth_params* p)
{
    cfg_tmp_t c;
    if (build_structure(seed, p, &c) != 0) return -1;
    int64_t ne = c.n_edges;
    cfg_tmp_free(&c);
    return ne;
}

/* Fills one CFG.  Arrays are caller-owned and sized n_blocks+1 (succ_ptr),
 * n_edges (succ_idx, edge_kind), n_blocks (space, loop_depth),
 * n_blocks*ceil(n_vars/64) (R, W), n_call_sites (call_blocks).
 * Optional arrays may be NULL.  Returns the number of call sites placed,
 * or -1 on bad parameters. */
int synth_cfg_fill(uint64_t seed, const synth_params* p,
                   int32_t* succ_ptr, int32_t* succ_idx, uint8_t* edge_kind, uint8_t* space,
                   uint64_t* R, uint64_t* W, int32_t* loop_depth, int32_t* call_blocks)
{
    cfg_tmp_t c;
    if (build_structure(seed, p, &c) != 0) return -1;
    int nb = c.n_blocks, ne = c.n_edges;
    if (succ_ptr) memcpy(succ_ptr, c.succ_ptr, sizeof(int32_t) * (size_t)(nb + 1));
    if (succ_idx) memcpy(succ_idx, c.succ_idx, sizeof(int32_t) * (size_t)ne);
    if (edge_kind) memcpy(edge_kind, c.kind, (size_t)ne);
    if (space) memcpy(space, c.space, (size_t)nb);
    if (loop_depth) memcpy(loop_depth, c.loop_depth, sizeof(int32_t) * (size_t)nb);
    if (call_blocks && c.n_calls) memcpy(call_blocks, c.call_blocks, sizeof(int32_t) * (size_t)c.n_calls);
    int n_calls = c.n_calls;
    cfg_tmp_free(&c);
    if (R || W) {
        int wd = (p->n_vars + 63) / 64;
        uint64_t lastmask = (p->n_vars % 64) ? ((1ull << (p->n_vars % 64)) - 1ull) : ~0ull;
        xo_t g;
        xo_seed(&g, synth_splitmix64(seed ^ 0xACCE55B175ull));
        for (int b = 0; b < nb; ++b) {
            for (int w = 0; w < wd; ++w) {
                uint64_t r = 0, x = 0;
                if (b != 0 && b != nb - 1) {
                    r = xo_bernoulli_word(&g, p->thr_read);
                    x = xo_bernoulli_word(&g, p->thr_write);
                    if (w == wd - 1) { r &= lastmask; x &= lastmask; }
                }
                if (R) R[(size_t)b * wd + w] = r;
                if (W) W[(size_t)b * wd + w] = x;
            }
        }
    }
    return n_calls;
}
