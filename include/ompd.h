/*
 * ompd.h — C ABI of the MI355X (gfx950) solver for the OMPDart data-flow
 * problems (Marzen, Dutta, Jannesari, "Static Generation of Efficient OpenMP
 * Offload Data Mappings", SC24).
 *
 * The library takes control-flow graphs whose basic blocks are tagged host
 * or device (offload kernels, Table I) with per-block read/write bitmaps
 * (the memory-access classification of the approach section) and returns,
 * per variable, the fixed points of
 *   - next use per memory space      (region-exit liveness, section
 *                                     "Data-Flow Analysis", last paragraph)
 *   - validity per memory space      (valid = last written there; a write in
 *                                     one space makes the other copy stale;
 *                                     a stale read is a RAW dependency)
 *   - the placement of copies        (map(to/from) and target update, with
 *                                     the loop rule: no copy enters a loop,
 *                                     copies needed inside a loop go on its
 *                                     entry edge; Table II)
 *   - validity after the placement, and the map/update labels of one target
 *     data region per function (Table II),
 * and, for whole programs, exact per-procedure summaries with call-string
 * contexts (section "Interprocedural Analysis").
 *
 * Conventions (every entry point):
 *   Return value: OMPD_OK (0) or a negative OMPD_E_* code.  On error,
 *   ompd_last_error(ctx) gives a message owned by ctx, valid until the next
 *   call on ctx from the same thread.
 *   Bit layout: variable v is bit (v & 63) of 64-bit word (v >> 6).  A block
 *   vector is n_blocks rows of ceil(n_vars/64) words, row-major
 *   [block][word]; an edge vector is n_edges rows in successor-CSR edge
 *   order.  Padding bits above n_vars must be zero on input and are
 *   returned as zero.
 *   Pointers are host pointers unless OMPD_F_DEVICE_PTRS is set, in which
 *   case every pointer in ompd_cfg / ompd_result is a device pointer on the
 *   context's GPU and `stream` (a hipStream_t, NULL = default stream) is
 *   the caller's stream.  Host inputs are copied before the call returns;
 *   device inputs must stay valid until the work completes.
 *   The caller owns every input and output buffer.
 *   Thread safety: calls on one context are serialised by an internal lock.
 */
#ifndef OMPD_H
#define OMPD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define OMPD_OK 0
#define OMPD_E_INVAL (-1)          /* malformed CFG or argument (see S1 rules below)      */
#define OMPD_E_NOMEM (-2)          /* device memory / admission budget exceeded            */
#define OMPD_E_DEVICE (-3)         /* HIP runtime error                                    */
#define OMPD_E_NOCONVERGE (-4)     /* sweep cap reached (only below the proven bound)      */
#define OMPD_E_BUSY (-5)           /* serving queue full: poll and retry                   */
#define OMPD_E_UNKNOWN_TICKET (-6) /* ticket never issued or already collected             */
#define OMPD_E_TIMEOUT (-7)        /* ompd_wait timed out                                  */

/* ---- enums ----------------------------------------------------------- */
enum { OMPD_HOST = 0, OMPD_DEVICE = 1 };                                  /* block space */
enum { OMPD_EDGE_NORMAL = 0, OMPD_EDGE_BACK = 1, OMPD_EDGE_LOOP_ENTRY = 2 };  /* edge kind */
enum { OMPD_MAP_TO = 1, OMPD_MAP_FROM = 2, OMPD_MAP_ALLOC = 4, OMPD_FIRSTPRIVATE = 8 };   /* var_kind bits */

/* ---- flags ----------------------------------------------------------- */
#define OMPD_F_DEVICE_PTRS (1u << 0)      /* all pointers are device pointers               */
#define OMPD_F_PLACEMENT_EAGER (1u << 1)  /* materialise every eager copy (no delay)         */
#define OMPD_F_SUMMARY (1u << 2)          /* procedure-summary evaluation: the entry boundary may
                                             leave variables valid in neither space            */
#define OMPD_F_TILE_KERNEL (1u << 3)      /* one persistent kernel runs every phase of a tile
                                             (same results) instead of one kernel per phase */
/* Schedule of the sweeps (results do not depend on it).  WALK: one block
 * after another in block order, the states of recent blocks kept in LDS
 * (best when a CFG has few blocks per level).  LEVEL: the blocks of a level
 * (blocks that no chain of edges other than BACK edges orders) in parallel,
 * a level at a time (best when levels are wide).  Neither flag: the library
 * picks per CFG from its shape. */
#define OMPD_F_SCHED_LEVEL (1u << 4)
#define OMPD_F_SCHED_WALK (1u << 5)
/* Placement variants (section "Data-Flow Analysis", the loop rule, and
 * Algorithm 1).  The default placement makes each copy right after the
 * producer and then delays it towards the read that needs it, never into a
 * loop and never across a join where another path holds fresh data in one
 * space only.  PLACEMENT_LAZY: the delay ignores loop entries (copies may
 * land inside loops; for comparison).  PLACEMENT_REFINE: the loop-entry
 * refinement: a copy the delay left on a loop-entry edge is dropped when no
 * read uses its value (every path re-copies or overwrites it first), which
 * gives the single update after a writing loop that Algorithm 1 places;
 * one more backward fixed point and one pass.  EAGER takes precedence over
 * both, LAZY over REFINE. */
#define OMPD_F_PLACEMENT_LAZY (1u << 6)
#define OMPD_F_PLACEMENT_REFINE (1u << 7)
#define OMPD_F_SWEEP_CAP(n) ((((uint32_t)(n)) & 0xFFFFu) << 16) /* cap sweeps per phase */
/* Ring of recently solved blocks per solve workgroup, for the one-shot entry
 * points (what ompd_plan_configure sets for a plan): n = 8, 16, 32 or 64
 * blocks (other values round down to one of these; 0 = default, 64).  Results
 * do not depend on it. */
#define OMPD_F_RING_SLOTS(n) ((uint32_t)((n) >= 64 ? 4 : (n) >= 32 ? 3 : (n) >= 16 ? 2 : (n) >= 8 ? 1 : 0) << 8)

/* ---- one procedure ----------------------------------------------------
 * A CFG of basic blocks (the CFG half of the paper's AST-CFG, Figure 2).
 * n_blocks includes an access-free HOST block `entry` with no predecessors
 * and an access-free HOST block `exit` with no successors.  Every block must
 * be reachable from entry and reach exit.  Edge kinds come from the AST
 * loops (For/While/Do): LOOP_ENTRY marks an edge into a loop header from
 * outside the loop, BACK an edge from inside the loop to its header.  Edges
 * into exit must be NORMAL and no edge out of entry may be BACK.
 * Reads of a block precede its writes; a write is a whole-variable write.
 * Block ids define the sweep order: numbering blocks in source order makes
 * the fixed points converge in few sweeps; any numbering gives the same
 * result.
 * Boundaries (NULL = default):
 *   entry_valid_host [wd] variables valid in host memory at entry   (default all)
 *   entry_valid_dev  [wd] variables valid in device memory at entry (default none)
 *   exit_live_host   [wd] variables read on the host after exit      (default all)
 *   exit_live_dev    [wd] variables read on the device after exit    (default none)
 * entry_valid_host | entry_valid_dev must cover every variable.
 * Call blocks (interprocedural use): call_summary[b] >= 0 names row
 * call_summary[b] of `summaries` (layout [n_summaries][16][wd], rows
 * MAYR_H MAYR_D MAYW_H MAYW_D NU0_H NU0_D NU1_H NU1_D T_H00 T_H01 T_H10
 * T_H11 T_D00 T_D01 T_D10 T_D11, identity for variables the callee cannot
 * see); call blocks must be HOST.  call_summary NULL = no calls.
 * firstprivate (section "Data-Flow Analysis", the firstprivate paragraph,
 * and Table II): scalar [wd] marks the variables the front end knows to be
 * scalars (NULL = none).  A marked variable that no DEVICE block writes is
 * firstprivate: a kernel that reads it receives the host value at launch
 * (its read needs the HOST copy valid, not the device copy), after that
 * kernel the device copy is not valid, and the kernel carries a
 * firstprivate clause for it (fp_clause).  ompd_analyze_program ignores the
 * marks of its procedures (their fp_clause outputs are all zero).          */
typedef struct {
    int32_t n_blocks, n_edges, n_vars;
    int32_t entry, exit;
    const int32_t* succ_ptr;          /* [n_blocks+1] */
    const int32_t* succ_idx;          /* [n_edges]    */
    const uint8_t* edge_kind;         /* [n_edges]    */
    const uint8_t* space;             /* [n_blocks]   */
    const uint64_t* read_bits;        /* [n_blocks*wd] */
    const uint64_t* write_bits;       /* [n_blocks*wd] */
    const uint64_t* entry_valid_host; /* [wd] or NULL */
    const uint64_t* entry_valid_dev;  /* [wd] or NULL */
    const uint64_t* exit_live_host;   /* [wd] or NULL */
    const uint64_t* exit_live_dev;    /* [wd] or NULL */
    const int32_t* call_summary;      /* [n_blocks] or NULL */
    const uint64_t* summaries;        /* [n_summaries*16*wd] or NULL */
    int32_t n_summaries;
    int32_t reserved;
    const uint64_t* scalar;           /* [wd] or NULL */
} ompd_cfg;

/* Outputs; any pointer may be NULL (not requested).
 *   nu_*          [n_blocks*wd] next use in that space at block entry
 *   ave_*         [n_blocks*wd] validity at block entry assuming eager copies
 *   avf_*         [n_blocks*wd] validity at block entry after the placement
 *   ins_entry_to_dev / _to_host [n_blocks*wd] copy into that space just before block b
 *   ins_edge_to_dev  / _to_host [n_edges*wd]  copy into that space on edge e
 *   var_kind      [n_vars]   OMPD_MAP_TO | OMPD_MAP_FROM (both = tofrom), or OMPD_MAP_ALLOC
 *                 (a device access that no map clause covers); | OMPD_FIRSTPRIVATE
 *                 when a kernel reads it as firstprivate
 *   fp_clause     [n_blocks*wd] the firstprivate clause of each DEVICE block (the
 *                 firstprivate variables it reads; zero elsewhere)
 *   after_dev     [n_blocks] 1 iff some DEVICE block reaches b (b included)
 *   before_dev    [n_blocks] 1 iff b reaches some DEVICE block (b included)
 * Labels: a copy into the device on edge p->q is map(to) iff !after_dev[p],
 * before block q iff no predecessor of q is after_dev; otherwise it is
 * target update to.  A copy into the host on p->q or before q is map(from)
 * iff !before_dev[q]; otherwise target update from.
 *   sweeps[6]     sweeps used per phase (next use, validity, pending,
 *                 delay, final validity, loop-entry refinement); host
 *                 memory, filled after completion; informational.         */
typedef struct {
    uint64_t *nu_host, *nu_dev;
    uint64_t *ave_host, *ave_dev;
    uint64_t *avf_host, *avf_dev;
    uint64_t *ins_entry_to_dev, *ins_entry_to_host;
    uint64_t *ins_edge_to_dev, *ins_edge_to_host;
    uint8_t* var_kind;
    uint8_t* after_dev;
    uint8_t* before_dev;
    uint64_t* fp_clause;
    int32_t sweeps[6];
} ompd_result;

typedef struct ompd_ctx ompd_ctx;
typedef struct ompd_plan ompd_plan;
typedef uint64_t ompd_ticket;

/* Create a context on HIP device `device_ordinal`.  device_mem_budget_bytes
 * bounds what the serving path admits (0 = 64 GiB).  Returns OMPD_E_DEVICE
 * if the device cannot be used. */
int ompd_ctx_create(ompd_ctx** out, int device_ordinal, uint64_t device_mem_budget_bytes);
void ompd_ctx_destroy(ompd_ctx* ctx);
const char* ompd_last_error(const ompd_ctx* ctx);
/* Device facts the solver plans with: compute units, LDS bytes a workgroup
 * of the solve kernel may use, and device memory.  Any pointer may be NULL. */
int ompd_device_info(ompd_ctx* ctx, int32_t* n_cu, int32_t* lds_bytes, int64_t* mem_bytes);
/* Bound of a wait inside the solve kernels.  The two wavefronts of a solve
 * workgroup (one computes the steps of the walk, the other feeds it inputs
 * and stores its results) wait for each other; a wait that sees no progress
 * for `ns` nanoseconds of the device's wall clock gives up, both wavefronts
 * stop, the CFG's status becomes OMPD_E_DEVICE, and ompd_last_error names
 * the phase, the tile and the counter that did not move (a bug in the
 * library, never a property of the input: a legitimate wait lasts one step
 * of the other wavefront, microseconds).  Applies to plans built and
 * requests launched after the call.  ns = 0 restores the default (2 s); ns
 * < 0 is OMPD_E_INVAL.  A tiny bound makes every wait give up at once (every
 * kernel still exits normally), which is how the give-up path is tested. */
int ompd_set_wait_limit(ompd_ctx* ctx, int64_t ns);

/* Solve one CFG; synchronous (returns when the results are in `res`).
 * Errors: OMPD_E_INVAL for a malformed CFG, OMPD_E_NOCONVERGE if a sweep
 * cap below the proven bound (2*n_blocks+2) stops a phase. */
int ompd_analyze_cfg(ompd_ctx* ctx, const ompd_cfg* cfg, ompd_result* res, uint32_t flags, void* stream);

/* Solve n CFGs in one persistent launch; synchronous.  Per-CFG errors are
 * reported as the first failing CFG's code; results of valid CFGs are
 * written regardless. */
int ompd_analyze_batch(ompd_ctx* ctx, const ompd_cfg* cfgs, ompd_result* res, int32_t n,
                       uint32_t flags, void* stream);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, tight serving loops, harnesses that forbid allocation): the
 * same solve as ompd_analyze_batch with OMPD_F_DEVICE_PTRS, with every byte
 * of solver scratch and launch tables taken from a static device array of
 * OMPD_NOALLOC_SCRATCH_MIB MiB that the library holds on each device it
 * runs on (from the first context on that device until the process ends).
 * The caller passes inputs and outputs as device pointers (flags must
 * include OMPD_F_DEVICE_PTRS) and `stream` (NULL = default stream); the call
 * is synchronous, allocates no device memory and returns OMPD_E_NOMEM,
 * touching nothing, when the batch needs more scratch than the array holds
 * (roughly ten words of scratch per block and word of each CFG, so tens of
 * MiB for a 16,384-block x 2,048-variable procedure).  Every call on one
 * device shares that device's array, which keeps the last call's contents
 * (each call rewrites what it reads, so nothing carries over): calls that
 * overlap on one GPU would race, so the library serialises them, across all
 * contexts of the process, for the whole call.  Results, errors and sweeps
 * are those of ompd_analyze_batch. */
#define OMPD_NOALLOC_SCRATCH_MIB 256
int ompd_analyze_batch_noalloc(ompd_ctx* ctx, const ompd_cfg* cfgs, ompd_result* res, int32_t n,
                               uint32_t flags, void* stream);

/* Resident batch: ompd_plan_create records the CFGs (device pointers only:
 * OMPD_F_DEVICE_PTRS is required), allocates scratch and chooses tiles;
 * ompd_plan_run enqueues one complete solve (ingest kernels, all phases,
 * labels) on `stream` without synchronising, replaying a captured HIP
 * graph; ompd_plan_status synchronises and returns OMPD_OK or the first
 * per-CFG error (per_cfg may be NULL or [n]).  The plan keeps pointers to
 * the caller's buffers, which must stay valid while it exists. */
int ompd_plan_create(ompd_ctx* ctx, const ompd_cfg* cfgs, ompd_result* res, int32_t n, uint32_t flags,
                     ompd_plan** out);
int ompd_plan_run(ompd_plan* plan, void* stream);
int ompd_plan_status(ompd_plan* plan, int32_t* per_cfg);
/* Autotuner: first the schedule of each size bucket (below), each bucket's
 * CFGs timed alone under the walk and the level schedule; then each
 * candidate launch configuration (LDS ring bytes per solve workgroup,
 * workgroups per CU) on the whole plan; every candidate is timed `trials`
 * times on `stream` and the fastest kept.  Results are bit-identical for
 * every candidate.  best_ms (the whole plan with the choice) may be NULL. */
int ompd_plan_autotune(ompd_plan* plan, void* stream, int32_t trials, float* best_ms);
/* Schedule per size bucket (what the autotuner chooses first, then the
 * launch configuration with that schedule): bucket k holds the CFGs with
 * fewer than 256, 1,024, 4,096, 16,384 blocks, or more (k = 0..4); per_bucket[k]
 * is -1 (the library's rule), 0 (walk) or 1 (level); CFGs whose schedule the
 * plan's flags name, and CFGs too large for the level schedule, keep theirs.
 * The autotuner times each bucket alone under both schedules.  Results are
 * bit-identical for every choice.  ompd_plan_describe reports the choice. */
#define OMPD_SCHED_BUCKETS 5
int ompd_plan_set_schedule(ompd_plan* plan, const int32_t* per_bucket);
/* Set the launch configuration by hand (what the autotuner chooses among):
 * LDS bytes per solve workgroup for the ring of recently solved blocks
 * (256 bytes per block; 0 = default, 16 KiB; rounded down to a power of
 * two of blocks within [8, 64] and to what the device's LDS holds) and
 * solve workgroups per CU (0 = as many as fit). */
int ompd_plan_configure(ompd_plan* plan, int64_t lds_bytes, int32_t wg_per_cu);
/* Profiling: with enable != 0, ompd_plan_run launches the kernels directly
 * (no graph) and records a HIP event after each on the caller's stream;
 * ompd_plan_kernel_ms then gives the duration (ms) of each kernel of the
 * last run, in launch order: ingest, next use, validity, validity pass
 * (AVEin, eager copies), pending copies, pending pass (valid in both
 * spaces), delayed placement, placement pass (the copies), loop-entry
 * refinement and its pass (0 ms unless a CFG asks for it), final
 * validity, final pass (AVFin, map-kind masks), map kinds (*n_kernels =
 * 13), or ingest and the per-tile kernel (*n_kernels = 2) after
 * ompd_plan_split_kernels(plan, 0).  At most `capacity` are written.
 * OMPD_E_INVAL if profiling is off. */
int ompd_plan_profile(ompd_plan* plan, int32_t enable);
/* Launch layout; results are identical either way.  By default (split !=
 * 0) one kernel per phase and per pass runs over all tiles; with split ==
 * 0 one persistent kernel runs every phase and pass of a tile, tile after
 * tile.  OMPD_E_INVAL for a NULL plan. */
int ompd_plan_split_kernels(ompd_plan* plan, int32_t split);
int ompd_plan_kernel_ms(ompd_plan* plan, float* ms, int32_t capacity, int32_t* n_kernels);
/* Describe the plan's current configuration as a NUL-terminated string. */
int ompd_plan_describe(ompd_plan* plan, char* buf, int32_t len);
/* Duration (ms) of the last ompd_plan_run measured with HIP events on its
 * stream: total, and the solve kernel alone. */
int ompd_plan_last_ms(ompd_plan* plan, float* total_ms, float* solve_ms);
void ompd_plan_destroy(ompd_plan* plan);

/* Serving: continuous batching.  submit copies the host CFG to the device
 * if it fits the context's device-memory budget and a slot is free
 * (otherwise OMPD_E_BUSY: poll/wait on earlier tickets and retry), and
 * returns at once; a background thread groups admitted requests into steps
 * that run concurrently on several streams (while one runs, the next waits
 * for 32 pending requests or 20 ms, whichever comes first, so that steps are
 * large).  `res` (host pointers) must
 * stay valid until poll reports done.  poll: *done = 0 pending, 1 done,
 * negative = that request's error code; a done ticket is released by the
 * poll that reports it.  wait blocks until done or timeout_ns (< 0 = no
 * limit). */
int ompd_submit(ompd_ctx* ctx, const ompd_cfg* cfg, ompd_result* res, uint32_t flags, ompd_ticket* out);
int ompd_poll(ompd_ctx* ctx, ompd_ticket t, int* done);
/* As ompd_poll; when done, *done_ns (may be NULL) is the completion time on
 * the host's monotonic clock (CLOCK_MONOTONIC, nanoseconds). */
int ompd_poll_ex(ompd_ctx* ctx, ompd_ticket t, int* done, int64_t* done_ns);
int ompd_wait(ompd_ctx* ctx, ompd_ticket t, int64_t timeout_ns, int* done);
/* Serving counters: admitted, completed, in flight, bytes in use. */
int ompd_serving_stats(ompd_ctx* ctx, int64_t* admitted, int64_t* completed, int64_t* in_flight,
                       int64_t* bytes_in_use);

/* ---- whole programs (section "Interprocedural Analysis") ---------------
 * The side effects of a call on the globals are summarised per procedure
 * and applied at its call sites, repeated over the call graph until nothing
 * changes; external functions are treated pessimistically.
 * procs[i] (host pointers) are the procedures; their call_summary,
 * summaries and n_summaries fields must be NULL / 0 (the library fills
 * them), and their boundary fields are used for roots only.  Variables
 * [0, n_globals) are the globals of every procedure (n_vars >= n_globals;
 * the rest are its locals).  Call site j is block call_block[j] of
 * procedure call_proc[j] (a HOST block, at most one call per block) and
 * calls procedure callee[j], or an external function if callee[j] = -1: it
 * needs every global current on the host, may read and write every global
 * there, and leaves the device copies stale.  A context is a procedure with
 * the last two call sites of a call string that reaches it from a root;
 * roots are contexts with an empty string.
 * call_space [n_calls] (NULL = all 0): 1 for a call made inside a kernel (a
 * device function; its block must be a DEVICE block).  It runs on the
 * device: the call block reads every global the callee may read or write,
 * in either space, and writes every global it may write (an external
 * callee: every global), and it leads to no context (a device function
 * carries no mapping directives).
 * const_globals [gw] (NULL = none): globals that are never written (the
 * paper's rule for data behind a pointer to const, per global): a
 * procedure that writes one is rejected (OMPD_E_INVAL), and an external
 * callee neither writes them nor leaves their device copy stale.
 * n_params [n_procs] (NULL = all 0): procedure i's first n_params[i] locals,
 * variables [n_globals, n_globals + n_params[i]), are pointer parameters (the
 * data at the address a caller passes; section "Interprocedural Analysis").
 * A procedure's shared variables are the globals and then its parameters;
 * its summary covers them.  arg_ptr [n_calls + 1] (NULL = no arguments,
 * arg_ptr[0] = 0, non-decreasing) and arg_var [arg_ptr[n_calls]]: call site
 * j binds argument t (parameter t of the callee) to caller variable
 * arg_var[arg_ptr[j] + t]; a call to a procedure passes exactly its
 * n_params.  Each procedure is solved name by name, so a host call to a
 * procedure (not to an external function) must bind distinct locals of the
 * caller, none a global (OMPD_E_INVAL otherwise); a call made inside a
 * kernel and an external call may bind any caller variables.  An external
 * callee reads its arguments on the host and writes them there, except
 * those with arg_const [arg_ptr[n_calls]] (NULL = none) set: pointers to
 * const, never written.                                                    */
typedef struct {
    int32_t n_procs, n_globals;
    const ompd_cfg* procs;            /* [n_procs] */
    int32_t n_calls;
    const int32_t* call_proc;         /* [n_calls] */
    const int32_t* call_block;        /* [n_calls] */
    const int32_t* callee;            /* [n_calls] */
    int32_t n_roots;
    const int32_t* roots;             /* [n_roots] */
    const uint8_t* call_space;        /* [n_calls] or NULL */
    const uint64_t* const_globals;    /* [gw] or NULL */
    const int32_t* n_params;          /* [n_procs] or NULL */
    const int32_t* arg_ptr;           /* [n_calls + 1] or NULL */
    const int32_t* arg_var;           /* [arg_ptr[n_calls]] */
    const uint8_t* arg_const;         /* [arg_ptr[n_calls]] or NULL */
} ompd_program;

/* Enumerate the contexts (breadth first from the roots, call sites in
 * order): ctx_proc[k], ctx_site0[k] = second-to-last call site (-1 if none),
 * ctx_site1[k] = last call site (-1 for a root).  *n_contexts receives the
 * count; the arrays (NULL allowed) receive at most `capacity` entries.
 * OMPD_E_INVAL for a malformed program. */
int ompd_program_contexts(ompd_ctx* ctx, const ompd_program* prog, int32_t* n_contexts, int32_t* ctx_proc,
                          int32_t* ctx_site0, int32_t* ctx_site1, int32_t capacity);

/* Outputs of ompd_analyze_program (host pointers, NULL = not requested):
 *   per_context [n_contexts] results of each context's solve, in the order
 *               of ompd_program_contexts, each sized by its procedure
 *   boundaries  per context, in that order, 4*wd words of its procedure:
 *               entry valid host, entry valid device, exit live host, exit
 *               live device (the meet over the contexts' callers)
 *   summaries   [n_procs*16*sw] (sw = ceil((n_globals + max n_params)/64))
 *               summary rows of each procedure over its shared variables
 *               (row order as above; bits past them are 0)
 *   demands     [n_calls*sw] shared variables each call site must make
 *               current on the host (read at the call block) so that the
 *               callee's context has every one valid somewhere, in the
 *               site's layout: bit v < n_globals is global v, bit
 *               n_globals + t the caller variable bound to argument t
 *   rounds      outer rounds until demands and exit-validity caps settled
 *   solves      CFG solves run on the device                              */
typedef struct {
    ompd_result* per_context;
    uint64_t* boundaries;
    uint64_t* summaries;
    uint64_t* demands;
    int32_t rounds;
    int32_t reserved;
    int64_t solves;
} ompd_program_result;

/* Interprocedural solve on the device: summaries bottom-up over the
 * strongly connected components of the call graph (recursion iterates
 * within a component), then contexts top-down in rounds, then host-read
 * demands and exit-validity caps fed back until they settle.  Every CFG
 * solve is a batched device solve of the procedures concerned.  flags:
 * OMPD_F_SWEEP_CAP only.  OMPD_E_NOCONVERGE if the outer rounds do not
 * settle within 64. */
int ompd_analyze_program(ompd_ctx* ctx, const ompd_program* prog, ompd_program_result* out, uint32_t flags);

#ifdef __cplusplus
}
#endif

#endif /* OMPD_H */
