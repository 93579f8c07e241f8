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
  never read or copy a stale version.
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
