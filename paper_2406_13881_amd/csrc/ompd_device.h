// Device-side descriptors shared by the HIP kernels and the host runtime of
// libompd (internal; the public interface is include/ompd.h).
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace ompd {

enum : int32_t {
    INFO_STATUS = 0,      // 0 ok, else an OMPD_E_* code
    INFO_LEVELS = 1,      // levels of the CFG (level schedule; written by the ingest kernel)
    INFO_SWEEPS = 2,      // [2..7] max sweeps per phase over the CFG's tiles
    // the first wait of the CFG's solve that gave up (status OMPD_E_DEVICE): phase + 1 (0 = none),
    // the tile's index within the CFG, which counter was awaited (WAIT_*), the value last seen,
    // the value awaited, and the wall-clock ticks waited
    INFO_PM_PHASE = 8, INFO_PM_TILE = 9, INFO_PM_WHAT = 10, INFO_PM_SEEN = 11, INFO_PM_TARGET = 12,
    INFO_PM_TICKS = 13,
    // 1: the walk follows the block ids; 0: it follows lorder (positions in loff), written by the
    // ingest kernel when some edge other than BACK goes from a higher to a lower id
    INFO_ORDER = 14,
    INFO_WORDS = 16
};

// What a wait of a phase workgroup waits for (INFO_PM_WHAT).
enum : int32_t {
    WAIT_IN_READY = 1,   // compute: the helper has put a step's inputs in LDS
    WAIT_CONSUMED = 2,   // compute: the helper has read a ring slot
    WAIT_FLUSHED = 3,    // compute: the helper's stores of a step's state have completed
    WAIT_PRODUCED = 4    // helper (idle): the compute wavefront has produced a step
};

// Phases (PH_LIVE: the loop-entry refinement, between the placement and the final validity).
enum : int32_t { PH_NU = 0, PH_AVE = 1, PH_MAYP = 2, PH_LATER = 3, PH_AVF = 4, PH_LIVE = 5 };
constexpr int N_PHASES = 6;

// DevCfg::placement bits.
enum : int32_t {
    PL_EAGER = 1,     // every eager copy stays where it is made
    PL_SUMMARY = 2,   // procedure-summary evaluation (the entry boundary may leave gaps)
    PL_LAZY = 4,      // pure lazy: loop-entry edges do not stop the delay
    PL_REFINE = 8     // loop-entry refinement of the delayed placement
};

// Summary rows of a callee, each a word vector over all variables.
enum : int32_t {
    SUM_MAYR_H = 0, SUM_MAYR_D, SUM_MAYW_H, SUM_MAYW_D,
    SUM_NU0_H, SUM_NU0_D, SUM_NU1_H, SUM_NU1_D,
    SUM_TH = 8, SUM_TD = 12, SUM_ROWS = 16
};

// One CFG as the kernels see it.  Every pointer is a device pointer; inputs
// the caller left NULL and outputs the solve needs internally point into
// scratch owned by the plan.
struct DevCfg {
    int32_t nb, ne, nv, entry, exit, wd;   // wd = 64-bit words per row
    int32_t n_sums, placement, sweep_cap;   // placement: PL_* bits
    int32_t wait_ticks;   // a wait gives up after this many wall-clock ticks without progress (> 0)
    int32_t sched;        // SCHED_WALK or SCHED_LEVEL
    int32_t sched_rule;   // host side: 1 when the default rule chose sched (a launch may revise it)
    const int32_t* succ_ptr;
    const int32_t* succ_idx;
    const uint8_t* kind;
    const uint8_t* space;
    const uint64_t* R;
    const uint64_t* W;
    const uint64_t* ev_h;
    const uint64_t* ev_d;
    const uint64_t* lx_h;
    const uint64_t* lx_d;
    const int32_t* call;        // NULL = no call blocks
    const uint64_t* sums;
    const uint64_t* scalar;     // [wd] variables marked as scalars, or NULL
    uint64_t* fp;               // [wd] firstprivate variables (ingest: marked, written by no DEVICE block)
    uint64_t* fpc;              // [nb*wd] output: each DEVICE block's firstprivate clause, or NULL
    uint64_t* nu_h;  uint64_t* nu_d;
    uint64_t* ave_h; uint64_t* ave_d;
    uint64_t* avf_h; uint64_t* avf_d;      // may be NULL
    uint64_t* ie_h;  uint64_t* ie_d;       // copy into host / device before block
    uint64_t* ig_h;  uint64_t* ig_d;       // copy into host / device on edge
    uint8_t* var_kind;                     // may be NULL
    uint8_t* after_dev;                    // may be NULL
    uint8_t* before_dev;                   // may be NULL
    uint64_t* aveout_h; uint64_t* aveout_d;   // eager validity out; later validity after placement
    uint64_t* mayp_h;   uint64_t* mayp_d;     // pending copies
    uint64_t* later_h;  uint64_t* later_d;    // delayed copies
    uint64_t* eag_h;    uint64_t* eag_d;      // per edge: eager copies
    uint64_t* both;     // per edge: valid in both spaces under the final placement
    uint64_t* flg;      // per tile: [4][nb] words of the flag lane
    uint64_t* vk_acc;   // [4][wd] map-kind masks (to, from, used on the device, firstprivate read);
                        // NULL = no map kinds
    int32_t* pred_ptr;  int32_t* pred_idx; int32_t* pred_eid;
    int32_t* tmp;
    int32_t* rec_f;     // [2*nb] int4: block records with predecessors, in block-id order
    int32_t* rec_b;     // [2*nb] int4: block records with successors, in block-id order
    int32_t* step_f;    // [2*nb] int4: step entries of the forward walk, in walk order (level
                        // schedule: the forward records in level order, the block in word 7)
    int32_t* step_b;    // [2*nb] int4: step entries of the backward walk, in walk order (level
                        // schedule: the backward records in level order)
    int32_t* lorder;    // [nb] the blocks by level (level schedule)
    int32_t* loff;      // [nb + 1] start of each level in lorder
    int32_t* info;
};

// How a CFG's phases visit its blocks: one block after another along the
// block order (the walk), or a level at a time with the blocks of a level in
// parallel.  Results do not depend on it.
enum : int32_t { SCHED_WALK = 0, SCHED_LEVEL = 1 };

// record meta word: neighbour count | flags
constexpr uint32_t REC_COUNT = 0x00FFFFFFu;
constexpr uint32_t REC_ENTRY = 1u << 24, REC_EXIT = 1u << 25, REC_DEV = 1u << 26, REC_CALL = 1u << 27;

// A tile: one CFG and a run of its 64-bit variable words, solved by one
// workgroup (a compute wavefront with two lanes per word, its low and high
// halves, plus the flag lane's two, and a helper wavefront that feeds it and
// stores its results).
// Words per tile slot (LANES, one of them for the flag lane); lane l and
// l + LANES hold the halves of word l, and LDS holds LANES words of every row.
constexpr int LANES = 16;
constexpr int TILE_WORDS = LANES - 1;
constexpr int WORD_BYTES = 8 * LANES;        // one word of every lane in LDS
constexpr int STATE_BYTES = 2 * WORD_BYTES;  // a state (h, d)
struct Tile {
    int32_t cfg;
    int32_t s0;      // first word
    int32_t nw;      // words (0 only when the CFG has no variables)
    int32_t fslot;   // index of the tile within its CFG (flag-lane storage)
};

// Work item of the pass kernels: a CFG, a run of up to PASS_WORDS of its
// words (one per lane of a wavefront, independent of the solve tiles) and the
// first block of a 64-block chunk.
constexpr int PASS_WORDS = 64;
struct EdgeItem {
    int32_t cfg;
    int32_t s0;
    int32_t nw;
    int32_t b0;
};

// Tiles of a CFG with wd words: ceil(wd / TILE_WORDS) (at least one), the
// words split as evenly as possible.
inline int tiles_of(int wd) { return wd <= 0 ? 1 : (wd + TILE_WORDS - 1) / TILE_WORDS; }

// LDS of a phase workgroup: CTL_BYTES of coordination words, the ring of
// the last RS results (STATE_BYTES each), the inputs of the next in_ring(ph)
// steps (phase_inputs(ph) words of WORD_BYTES each), their 16-byte
// descriptors, then one state of identity words (STATE_BYTES).
constexpr int CTL_BYTES = 256;
// Threads of a level-schedule workgroup.
constexpr int LEVEL_THREADS = 64;
// then the blocks of the last BLK_RING planned steps (the helper stores results by them; at least
// the result ring plus the input ring, so that an entry is not reused before its step is stored)
constexpr int BLK_RING = 128;
constexpr int LDS_FIXED = CTL_BYTES + 4 * BLK_RING;
// steps of inputs kept ready per phase (a power of two; more for the phases with fewer inputs).
// The helper wavefront refills them in rounds whose fixed cost is spread over the steps it
// finds free, so a deeper ring means fewer, longer rounds.
constexpr int in_ring(int ph) { return ph == PH_NU || ph == PH_AVE ? 32 : 16; }
inline int phase_inputs(int ph) { return 2 + (ph == PH_NU ? 2 : ph == PH_AVE ? 4 : ph == PH_MAYP ? 6 : 8); }
// Does a CFG run the loop-entry refinement (placement bits)?
constexpr bool refines(int32_t placement) { return (placement & (PL_REFINE | PL_EAGER | PL_LAZY)) == PL_REFINE; }
inline size_t phase_lds(int ph, int ring_slots)
{
    return LDS_FIXED + (size_t)ring_slots * STATE_BYTES + (size_t)in_ring(ph) * (phase_inputs(ph) * WORD_BYTES + 16) +
           STATE_BYTES;
}
// Work counters (int32) of one solve launch: phases 0..5, passes 8..11 and 14 (refinement), map
// kinds 12, per-tile kernel 13, level kernels 16..21.
constexpr int N_COUNTERS = 32;
// Kernels of one solve launch, in launch order (prep excluded; the two of the refinement are
// launched only when a CFG asks for it, their profile marks always).
constexpr int N_SOLVE_KERNELS = 12;

}  // namespace ompd
