"""Pins of the interprocedural oracle driver (whole-procedure summaries,
contexts of the last two call sites, host-read demands) against checks that
share no code with it:

* inlining: on non-recursive programs, next use at every block of the root
  equals that of the program with every call inlined (and eager validity
  never exceeds it), and
  next use of the globals in every context whose call string is at most two
  calls deep equals that of its inlined copy (deeper contexts merge call
  strings, so they may only over-approximate);
* unrolling: on recursive programs, the root's next use is the limit of the
  inlined program unrolled to growing call depth;
* simulation: random walks through calls, recursion and external callees
  never read or copy a stale version;
* schedule independence: Jacobi rounds, FIFO and LIFO worklists over the
  context solves give the same boundaries, demands and placements;
* eager copies: with every eager copy materialised, the validity of every
  block of every context equals that of its inlined copy (both directions)
  when no two call strings meet;
* necessity of demands: dropping any demanded global reopens the gap it
  closes (valid nowhere, yet read) in a context of that call site.
"""
import numpy as np
import pytest

import oracle
import synth
from checkers import inline_program, row_int, simulate_program
from oracle.program import ProgramOracle, tarjan

SMALL = dict(n_procs=6, n_globals=12, n_locals=5, blocks=(4, 14), mean_calls=2.0, max_calls=3, scc_procs=0,
             max_loop_depth=2, device_frac=0.4, p_read=0.25, p_write=0.15, threads=1)


def small_program(seed, **kw):
    prm = dict(SMALL)
    prm.update(kw)
    return synth.program(seed, **prm)


def masked(row, mask):
    return row_int(row) & mask


@pytest.mark.parametrize("seed", range(14))
def test_inlining_equivalence(seed):
    prog = small_program(5000 + seed)
    po = ProgramOracle(prog)
    _, ctx, results = po.analyze()
    big, instances, pos = inline_program(prog, 0, po.demand)
    ref = oracle.solve(big)
    G = prog.n_globals
    gmask = (1 << G) - 1
    root = prog.procs[0]
    rmask = (1 << root.n_vars) - 1
    mine = results[(0, ())]
    for b in range(root.n_blocks):
        for k in ("nu_h", "nu_d"):
            assert masked(mine[k][b], rmask) == masked(ref[k][pos[b]], rmask), \
                "seed %d: %s of root block %d differs from the inlined program" % (seed, k, b)
        # eager validity after a call is capped by what the callee's final
        # placement provides, so it never exceeds the inlined program's
        for k in ("ave_h", "ave_d"):
            assert masked(mine[k][b], rmask) & ~masked(ref[k][pos[b]], rmask) == 0, \
                "seed %d: %s of root block %d exceeds the inlined program" % (seed, k, b)
    checked = 0
    for (P, sigma, off, _) in instances[1:]:
        key = (P, sigma[-2:])
        r = results[key]
        for b in range(prog.procs[P].n_blocks):
            for k in ("nu_h", "nu_d"):
                a = masked(r[k][b], gmask)
                x = masked(ref[k][pos[off + b]], gmask)
                if len(sigma) <= 2:
                    assert a == x, "seed %d: %s of %s block %d" % (seed, k, (P, sigma), b)
                else:
                    assert x & ~a == 0, "seed %d: context %s misses a next use of call string %s" % (seed, key, sigma)
        checked += 1
    assert checked == len(instances) - 1


def test_inlining_covers_calls():
    # the equivalence above is not vacuous: the programs make calls two deep
    deep = 0
    for seed in range(14):
        prog = small_program(5000 + seed)
        _, inst, _ = inline_program(prog, 0, {})
        deep += sum(1 for (_, sg, _, _) in inst if len(sg) >= 2)
    assert deep >= 30


@pytest.mark.parametrize("seed", range(8))
def test_recursive_next_use_is_limit_of_unrolling(seed):
    prog = small_program(7000 + seed, scc_procs=4, scc_size=(2, 3), mean_calls=0.8)
    succ = [[] for _ in prog.procs]
    for j in range(len(prog.call_proc)):
        succ[int(prog.call_proc[j])].append(int(prog.callee[j]))
    assert any(len(c) > 1 for c in tarjan(len(prog.procs), succ))
    po = ProgramOracle(prog)
    _, _, results = po.analyze()
    root = prog.procs[0]
    rmask = (1 << root.n_vars) - 1
    want = [[masked(results[(0, ())][k][b], rmask) for b in range(root.n_blocks)] for k in ("nu_h", "nu_d")]
    prev = None
    for depth in range(0, 7):
        big, _, pos = inline_program(prog, 0, po.demand, cap_depth=depth)
        ref = oracle.solve(big)
        got = [[masked(ref[k][pos[b]], rmask) for b in range(root.n_blocks)] for k in ("nu_h", "nu_d")]
        for s in (0, 1):
            for b in range(root.n_blocks):
                assert got[s][b] & ~want[s][b] == 0, "seed %d depth %d: unrolled next use exceeds the summary" % (seed, depth)
                if prev is not None:
                    assert prev[s][b] & ~got[s][b] == 0
        prev = got
    assert prev == want, "seed %d: unrolling to depth 6 does not reach the summary" % seed


@pytest.mark.parametrize("seed", range(10))
def test_program_walks_are_safe(seed):
    prog = small_program(9000 + seed, n_procs=8, scc_procs=5, scc_size=(2, 3), external_frac=0.3)
    po = ProgramOracle(prog)
    _, ctx, results = po.analyze()
    errs, cut = simulate_program(prog, ctx, results, po.demand, walks=150, seed=seed)
    assert not errs, errs[:5]
    assert cut < 150


def test_external_callee_convention():
    # external calls: the caller must make every global current on the host
    # before each and treat the device copies as stale after it
    single = 0
    for seed in range(4242, 4252):
        prog = small_program(seed, n_procs=1, external_frac=1.0)
        if len(prog.callee) == 0:
            continue
        assert (prog.callee < 0).all()
        po = ProgramOracle(prog)
        _, _, results = po.analyze()
        res = results[(0, ())]
        cfg = prog.procs[0]
        gmask = (1 << prog.n_globals) - 1
        for c in prog.call_block.tolist():
            # the block's own accesses come first: its writes end their next use
            assert masked(res["nu_h"][c], gmask) == (row_int(cfg.R[c]) | ~row_int(cfg.W[c])) & gmask
            # at a successor entered only from the call, eager device validity
            # is just the successor's own next use on the device
            for e in range(int(cfg.succ_ptr[c]), int(cfg.succ_ptr[c + 1])):
                t = int(cfg.succ_idx[e])
                if int((cfg.succ_idx == t).sum()) == 1:
                    assert masked(res["ave_d"][t], gmask) == masked(res["nu_d"][t], gmask)
                    single += 1
        errs, _ = simulate_program(prog, {}, results, po.demand, walks=60, seed=seed)
        assert not errs, errs[:5]
    assert single >= 1


def test_summaries_of_c4_shape():
    # the large-program generator: recursion stays in small components
    prog = synth.program(synth.item_seed(4, 0), **dict(synth.C4, n_procs=300, blocks=(8, 64)))
    succ = [[] for _ in prog.procs]
    for j in range(len(prog.call_proc)):
        if prog.callee[j] >= 0:
            succ[int(prog.call_proc[j])].append(int(prog.callee[j]))
    comps = tarjan(len(prog.procs), succ)
    assert max(len(c) for c in comps) <= 8
    assert sum(1 for c in comps if len(c) > 1) >= 3


# ---------------------------------------------------------------------------
# The context boundaries are fixed points, not artefacts of a schedule
# ---------------------------------------------------------------------------
def _outputs(po, S, ctx, results):
    out = {"S": {p: S[p].tobytes() for p in S}, "demand": {j: po.demand[j].tobytes() for j in po.demand}}
    for key in ctx:
        out[("bnd",) + key] = tuple(np.asarray(x).tobytes() for x in ctx[key])
        out[("res",) + key] = tuple(np.asarray(results[key][k]).tobytes() for k in sorted(results[key])
                                    if k != "visits")
    return out


SCHEDULE_CASES = [("plain", {}), ("recursive", dict(scc_procs=4, scc_size=(2, 3), mean_calls=1.0)),
                  ("external", dict(n_procs=8, scc_procs=5, scc_size=(2, 3), external_frac=0.3)),
                  ("deep", dict(n_procs=9, mean_calls=2.5, max_calls=4))]


@pytest.mark.parametrize("kind,extra", SCHEDULE_CASES, ids=[c[0] for c in SCHEDULE_CASES])
def test_context_solution_does_not_depend_on_the_schedule(kind, extra):
    # Jacobi rounds, a FIFO worklist and a LIFO worklist over the context
    # solves give the same boundaries, demands, summaries and placements
    for seed in range(5):
        prog = small_program(11_000 + 97 * len(kind) + seed, **extra)
        ref = None
        for schedule in ("rounds", "fifo", "lifo"):
            po = ProgramOracle(prog)
            S, ctx, results = po.analyze(schedule=schedule)
            got = _outputs(po, S, ctx, results)
            if ref is None:
                ref = got
            else:
                assert got == ref, "%s seed %d: schedule %s changes the result" % (kind, seed, schedule)


def _shallow(prog):
    # non-recursive, no external callee, and every call string at most two
    # calls deep: no two call strings meet in one context
    if (prog.callee < 0).any():
        return False
    _, inst, _ = inline_program(prog, 0, {})
    return len(prog.roots) == 1 and max(len(sg) for (_, sg, _, _) in inst) <= 2


def test_eager_validity_equals_the_inlined_program():
    # With eager copies everywhere the final validity is the eager one, so no
    # cap can bind; without merged call strings no demand arises; then the
    # validity of every block of every context equals that of its inlined
    # copy, in both directions (the one-sided pin above only bounds it).
    found = deep = 0
    for seed in range(200):
        prog = small_program(13_000 + seed, n_procs=3, mean_calls=2.0, max_calls=3)
        if not _shallow(prog):
            continue
        po = ProgramOracle(prog, placement=1)
        _, ctx, results = po.analyze()
        assert not po.demand, "seed %d: a shallow program needs no demand" % seed
        big, instances, pos = inline_program(prog, 0, {})
        ref = oracle.solve(big, placement=1)
        G = prog.n_globals
        for (P, sigma, off, vmap) in instances:
            cfg = prog.procs[P]
            mask = (1 << (cfg.n_vars if not sigma else G)) - 1
            r = results[(P, sigma)]
            for b in range(cfg.n_blocks):
                # a callee's ENTRY holds its boundary: the inlined program copies
                # on the call edge into it, the context on ENTRY's out-edges, so
                # validity agrees from the first block on
                names = ("nu_h", "nu_d") if (sigma and b == cfg.entry) else \
                    ("ave_h", "ave_d", "avf_h", "avf_d", "nu_h", "nu_d")
                for k in names:
                    assert masked(r[k][b], mask) == masked(ref[k][pos[off + b]], mask), \
                        "seed %d: %s of %s block %d differs from the inlined program" % (seed, k, (P, sigma), b)
        found += 1
        deep += sum(1 for (_, sg, _, _) in instances if len(sg) == 2)
        if found >= 16:
            break
    assert found >= 16 and deep >= 20


def merge_program(seed, n_globals=10):
    """Root calls A at two sites, A calls B, B calls C: the call strings
    (site 0, A->B, B->C) and (site 1, A->B, B->C) meet in C's context.
    Every other block is a random host or device statement over the globals,
    so the two paths into C often leave a global fresh in different spaces."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def stmt(p=0.3):
        dev = int(rng.random() < 0.5)
        rd = [v for v in range(n_globals) if rng.random() < p]
        wr = [v for v in range(n_globals) if rng.random() < p]
        return (dev, rd, wr)

    def chain(body):
        blocks = [(0, [], [])] + body + [(0, [], [])]
        edges = [(i, i + 1, 0) for i in range(len(blocks) - 1)]
        return synth.from_edges(blocks, edges, n_globals)[0]

    host_call = (0, [], [])
    root = chain([stmt(), host_call, stmt(), stmt(), host_call, stmt()])      # calls at blocks 2 and 5
    # nothing is live after the program, so the liveness after the two calls
    # depends on what the root reads next, and may differ
    root.exit_live_h = np.zeros(root.wd, np.uint64)
    # the callees touch few globals, so many pass through all three of them
    a = chain([stmt(0.1), host_call, stmt(0.1)])                               # call at block 2
    b = chain([host_call, stmt(0.1)])                                          # call at block 1
    c = chain([stmt(0.1), stmt(0.1)])
    return synth.Program(procs=[root, a, b, c], n_globals=n_globals,
                         call_proc=np.array([0, 0, 1, 2], np.int32), call_block=np.array([2, 5, 2, 1], np.int32),
                         callee=np.array([1, 1, 2, 3], np.int32), roots=[0])


def test_every_demand_is_needed():
    # Dropping any demanded global of any call site and solving the contexts
    # again leaves that global valid in neither space, and read, in a context
    # the site leads to: the demand is exactly what closes that gap.
    checked = programs = 0
    for seed in range(200):
        prog = merge_program(19_000 + seed)
        po = ProgramOracle(prog)
        po.analyze()
        if not po.demand:
            continue
        programs += 1
        gw = (prog.n_globals + 63) // 64
        for j, m in sorted(po.demand.items()):
            for v in range(64 * gw):
                if not (int(m[v >> 6]) >> (v & 63)) & 1:
                    continue
                po2 = ProgramOracle(prog)
                po2.demand = {jj: mm.copy() for jj, mm in po.demand.items()}
                po2.cap = dict(po.cap)
                po2.demand[j][v >> 6] &= ~np.uint64(1 << (v & 63))
                S2 = po2.summarize()
                po2.contexts(S2)
                gaps = [k for k, nw in po2.nowhere.items()
                        if k[1] and k[1][-1] == j and (int(nw[v >> 6]) >> (v & 63)) & 1]
                assert gaps, "seed %d: demand of global %d at site %d is not needed" % (seed, v, j)
                checked += 1
        # and the demands make the program safe
        _, ctx, results = po.analyze()
        errs, _ = simulate_program(prog, ctx, results, po.demand, walks=20, seed=seed)
        assert not errs, errs[:5]
        if checked >= 40:
            break
    assert programs >= 10 and checked >= 15


def test_c4_digest_file_matches_the_generator():
    """The stored digests of the full whole-program configuration belong to the program the
    generator builds today: same context count and same sorted context list (the context
    graph alone, no solves)."""
    import hashlib
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "c4_digests.json")
    want = json.load(open(path))
    prog = synth.c4()
    keys = sorted(ProgramOracle(prog).context_graph(), key=lambda k: (int(k[0]), tuple(int(s) for s in k[1])))
    h = hashlib.sha256()
    for key in keys:
        h.update(repr((int(key[0]), tuple(int(s) for s in key[1]))).encode())
    assert len(keys) == want["n_contexts"]
    assert h.hexdigest() == want["contexts"]
