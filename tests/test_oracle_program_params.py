"""Pins of by-reference pointer parameters in the interprocedural driver
(section "Interprocedural Analysis": data reached through the addresses a
function receives as pointer parameters), against checks that share no code
with it:

* inlining: on non-recursive programs whose host calls bind distinct locals,
  next use at every block of the root, and of every shared variable (the
  globals and the parameters, the latter as the caller variables they are
  bound to) in every context at most two calls deep, equals that of the
  program with every call inlined (a parameter of an inlined copy is the
  bound caller variable itself); deeper contexts may only over-approximate;
  with eager copies and no merged call strings, validity equals it too;
* unrolling: on recursive programs the root's next use is the limit of the
  inlined program unrolled to growing call depth;
* the may rows over the globals and the parameters against a brute-force
  fixed point over the call graph written here (a callee's parameter row
  lands on the caller variable bound to it, if that is one of the caller's
  shared variables);
* random walks over storage cells (a parameter names the cell of its bound
  variable; calls made inside kernels and external calls may bind one datum
  twice, or a global) find no stale read or copy source;
* a call never leaves valid, in the caller, a shared variable that the
  callee context's final validity at its EXIT lacks;
* bindings a host call cannot have (a repeat, a global, the wrong count) are
  rejected;
* planted mistakes in the driver's handling of bindings are caught by these
  pins.
"""
import numpy as np
import pytest

import oracle
import synth
from checkers import inline_program, simulate_program
from oracle.program import ProgramOracle

SMALL = dict(n_procs=6, n_globals=10, n_locals=6, blocks=(4, 14), mean_calls=2.0, max_calls=3, scc_procs=0,
             max_loop_depth=2, device_frac=0.4, p_read=0.25, p_write=0.15, threads=1, max_params=3)


def prog_of(seed, **kw):
    prm = dict(SMALL)
    prm.update(kw)
    return synth.program(seed, **prm)


def bit(row, v):
    return (int(row[v >> 6]) >> (v & 63)) & 1


def bits_of(row, n):
    return {v for v in range(n) if bit(row, v)}


def mapped(row, vmap, n):
    """Bits 0 .. n-1 of a procedure-layout row, read from the inlined program's row through
    the instance's variable map."""
    return {v for v in range(n) if bit(row, vmap[v])}


def test_generator_binds_parameters():
    """The programs below make calls that bind parameters, and their callees use them."""
    used = 0
    for seed in range(14):
        p = prog_of(21_000 + seed)
        assert p.n_params is not None and int(p.n_params.sum()) > 0
        for j in range(len(p.call_proc)):
            q = int(p.callee[j])
            args = p.arg_var[int(p.arg_ptr[j]):int(p.arg_ptr[j + 1])]
            assert len(args) == int(p.n_params[q])
            assert len(set(args.tolist())) == len(args) and (args >= p.n_globals).all()
            c = p.procs[q]
            R = np.asarray(c.R, np.uint64).reshape(c.n_blocks, c.wd)
            W = np.asarray(c.W, np.uint64).reshape(c.n_blocks, c.wd)
            used += sum(1 for i in range(len(args)) for b in range(c.n_blocks)
                        if bit(R[b], p.n_globals + i) or bit(W[b], p.n_globals + i))
    assert used >= 100


@pytest.mark.parametrize("seed", range(14))
def test_inlining_equivalence_with_parameters(seed):
    p = prog_of(21_000 + seed)
    po = ProgramOracle(p)
    _, _, results = po.analyze()
    big, instances, pos = inline_program(p, 0, po.demand)
    ref = oracle.solve(big)
    G = p.n_globals
    root = p.procs[0]
    mine = results[(0, ())]
    for b in range(root.n_blocks):
        for k in ("nu_h", "nu_d"):
            assert bits_of(mine[k][b], root.n_vars) == bits_of(ref[k][pos[b]], root.n_vars), (seed, k, b)
        for k in ("ave_h", "ave_d"):
            assert bits_of(mine[k][b], root.n_vars) <= bits_of(ref[k][pos[b]], root.n_vars), (seed, k, b)
    deep = 0
    for (P, sigma, off, vmap) in instances[1:]:
        r = results[(P, sigma[-2:])]
        ns = G + int(p.n_params[P])
        for b in range(p.procs[P].n_blocks):
            for k in ("nu_h", "nu_d"):
                a = bits_of(r[k][b], ns)
                x = mapped(ref[k][pos[off + b]], vmap, ns)
                if len(sigma) <= 2:
                    assert a == x, (seed, k, P, sigma, b)
                else:
                    assert x <= a, (seed, k, P, sigma, b)
    assert len(instances) > 1


def test_inlining_covers_parameters_two_deep():
    deep = 0
    for seed in range(14):
        p = prog_of(21_000 + seed)
        _, inst, _ = inline_program(p, 0, {})
        deep += sum(1 for (P, sg, _, _) in inst if len(sg) >= 2 and int(p.n_params[P]) > 0)
    assert deep >= 20


@pytest.mark.parametrize("seed", range(8))
def test_recursive_next_use_with_parameters_is_the_limit_of_unrolling(seed):
    p = prog_of(22_000 + seed, scc_procs=4, scc_size=(2, 3), mean_calls=0.8)
    po = ProgramOracle(p)
    _, _, results = po.analyze()
    root = p.procs[0]
    n = root.n_vars
    want = [[bits_of(results[(0, ())][k][b], n) for b in range(root.n_blocks)] for k in ("nu_h", "nu_d")]
    prev = None
    for depth in range(0, 7):
        big, _, pos = inline_program(p, 0, po.demand, cap_depth=depth)
        ref = oracle.solve(big)
        got = [[bits_of(ref[k][pos[b]], n) for b in range(root.n_blocks)] for k in ("nu_h", "nu_d")]
        for s in (0, 1):
            for b in range(root.n_blocks):
                assert got[s][b] <= want[s][b], (seed, depth)
                if prev is not None:
                    assert prev[s][b] <= got[s][b]
        prev = got
    assert prev == want, "seed %d: unrolling to depth 6 does not reach the summary" % seed


def test_eager_validity_with_parameters_equals_the_inlined_program():
    found = 0
    for seed in range(300):
        p = prog_of(23_000 + seed, n_procs=3, mean_calls=2.0, max_calls=3)
        if (p.callee < 0).any() or len(p.roots) != 1:
            continue
        _, inst, _ = inline_program(p, 0, {})
        if max(len(sg) for (_, sg, _, _) in inst) > 2:
            continue
        po = ProgramOracle(p, placement=1)
        _, _, results = po.analyze()
        assert not po.demand
        big, instances, pos = inline_program(p, 0, {})
        ref = oracle.solve(big, placement=1)
        for (P, sigma, off, vmap) in instances:
            cfg = p.procs[P]
            ns = cfg.n_vars if not sigma else p.n_globals + int(p.n_params[P])
            r = results[(P, sigma)]
            for b in range(cfg.n_blocks):
                names = ("nu_h", "nu_d") if (sigma and b == cfg.entry) else \
                    ("ave_h", "ave_d", "avf_h", "avf_d", "nu_h", "nu_d")
                for k in names:
                    assert bits_of(r[k][b], ns) == mapped(ref[k][pos[off + b]], vmap, ns), (seed, k, P, sigma, b)
        found += 1
        if found >= 16:
            break
    assert found >= 16


def brute_may(p, demand):
    """Per procedure, the shared variables (globals, then its parameters) it or anything it
    calls may read / write, per space, by a plain fixed point over the call graph."""
    G, n = p.n_globals, len(p.procs)
    npar = [int(x) for x in p.n_params]
    const = bits_of(p.const_globals, G) if p.const_globals is not None else set()
    cs = p.call_space if p.call_space is not None else np.zeros(len(p.call_proc), np.uint8)
    own = []
    for P, c in enumerate(p.procs):
        ns = G + npar[P]
        m = [set(), set(), set(), set()]   # read H, read D, write H, write D
        R = np.asarray(c.R, np.uint64).reshape(c.n_blocks, c.wd)
        W = np.asarray(c.W, np.uint64).reshape(c.n_blocks, c.wd)
        for b in range(c.n_blocks):
            d = int(c.space[b])
            m[d] |= {v for v in bits_of(R[b], c.n_vars) if v < ns}
            m[2 + d] |= {v for v in bits_of(W[b], c.n_vars) if v < ns}
        own.append(m)
    for j, d in demand.items():
        P = int(p.call_proc[j])
        own[P][0] |= {v for v in bits_of(d, p.procs[P].n_vars) if v < G + npar[P]}
    may = [[set(x) for x in m] for m in own]
    while True:
        changed = False
        for j in range(len(p.call_proc)):
            P, q = int(p.call_proc[j]), int(p.callee[j])
            ns = G + npar[P]
            args = [int(x) for x in p.arg_var[int(p.arg_ptr[j]):int(p.arg_ptr[j + 1])]]
            consts = [bool(x) for x in p.arg_const[int(p.arg_ptr[j]):int(p.arg_ptr[j + 1])]]
            if q < 0:
                r = set(range(G)) | {x for x in args if x < ns}
                w = (set(range(G)) - const) | {x for x, k in zip(args, consts) if x < ns and not k}
                src = [set(), r, set(), w] if cs[j] else [r, set(), w, set()]
            else:
                def to_caller(vs):
                    out = {v for v in vs if v < G}
                    out |= {args[v - G] for v in vs if v >= G and args[v - G] < ns}
                    return out
                src = [to_caller(x) for x in may[q]]
                if cs[j]:
                    w = src[2] | src[3]
                    src = [set(), src[0] | src[1] | w, set(), w]
            for k in range(4):
                if not src[k] <= may[P][k]:
                    may[P][k] |= src[k]
                    changed = True
        if not changed:
            return may


def may_program(seed):
    return prog_of(24_000 + seed, n_procs=8, scc_procs=4 if seed % 2 else 0, scc_size=(2, 3),
                   device_call_frac=0.3 if seed % 3 else 0.0, n_const=2 if seed % 3 == 1 else 0,
                   external_frac=0.25 if seed % 4 == 1 else 0.0, max_ext_args=3)


@pytest.mark.parametrize("seed", range(16))
def test_may_rows_with_parameters_match_a_brute_force_fixed_point(seed):
    p = may_program(seed)
    po = ProgramOracle(p)
    S, _, _ = po.analyze()
    may = brute_may(p, po.demand)
    for P in range(len(p.procs)):
        ns = p.n_globals + int(p.n_params[P])
        for k in range(4):
            assert bits_of(S[P][k], ns) == may[P][k], (seed, P, k)


def walk_program(seed):
    return prog_of(25_000 + seed, n_procs=8, scc_procs=5 if seed % 2 else 0, scc_size=(2, 3),
                   external_frac=0.3, max_ext_args=3, device_call_frac=0.3 if seed % 3 != 2 else 0.0,
                   n_const=2 if seed % 2 else 0)


@pytest.mark.parametrize("seed", range(14))
def test_program_walks_with_parameters_are_safe(seed):
    p = walk_program(seed)
    po = ProgramOracle(p)
    _, ctx, results = po.analyze()
    errs, cut = simulate_program(p, ctx, results, po.demand, walks=120, seed=seed)
    assert not errs, errs[:5]
    assert cut < 120


def test_walk_programs_alias_at_device_and_external_calls():
    """Calls made inside kernels and external calls do bind one datum twice, or a global."""
    rep = glob = 0
    for seed in range(14):
        p = walk_program(seed)
        cs = p.call_space if p.call_space is not None else np.zeros(len(p.call_proc), np.uint8)
        for j in range(len(p.call_proc)):
            a = p.arg_var[int(p.arg_ptr[j]):int(p.arg_ptr[j + 1])].tolist()
            if cs[j] or int(p.callee[j]) < 0:
                rep += len(set(a)) < len(a)
                glob += any(x < p.n_globals for x in a)
    assert rep >= 5 and glob >= 20


@pytest.mark.parametrize("schedule", ["fifo", "lifo"])
def test_parameter_contexts_do_not_depend_on_the_schedule(schedule):
    for seed in range(4):
        p = walk_program(seed)
        a = ProgramOracle(p)
        ra = a.analyze()[2]
        b = ProgramOracle(p)
        rb = b.analyze(schedule=schedule)[2]
        assert ra.keys() == rb.keys()
        assert a.demand.keys() == b.demand.keys()
        for j in a.demand:
            assert np.array_equal(a.demand[j], b.demand[j])
        for k in ra:
            for key in ("ins_entry_h", "ins_entry_d", "ins_edge_h", "ins_edge_d", "avf_h", "avf_d"):
                assert np.array_equal(np.asarray(ra[k][key]), np.asarray(rb[k][key])), (seed, k, key)


def test_bad_bindings_are_rejected():
    p = prog_of(21_001)
    j = next(j for j in range(len(p.call_proc)) if int(p.n_params[int(p.callee[j])]) >= 2)
    lo = int(p.arg_ptr[j])
    for bad in ("repeat", "global", "count"):
        q = prog_of(21_001)
        if bad == "repeat":
            q.arg_var[lo + 1] = q.arg_var[lo]
        elif bad == "global":
            q.arg_var[lo] = 0
        else:
            q.n_params = q.n_params.copy()
            q.n_params[int(q.callee[j])] += 1
        with pytest.raises(ValueError):
            ProgramOracle(q)


def cap_program(seed):
    if seed % 2:
        return walk_program(seed)
    return prog_of(26_000 + seed, n_procs=8, scc_procs=4, scc_size=(2, 3), p_read=0.3, p_write=0.2)


def exceeds_callee_exit(po, p, results):
    """(context, site, variable) triples where the caller's final validity just after a call
    (on an edge into a block with no other predecessor, less what that edge copies) holds a
    shared variable (a global, or the caller variable bound to a parameter) that the
    callee context's final validity at its EXIT does not: a call cannot leave valid what its
    callee does not."""
    G = p.n_globals
    out = []
    for k, edges in po.context_graph().items():
        c = p.procs[k[0]]
        npred = np.zeros(c.n_blocks, np.int64)
        for e in range(c.n_edges):
            npred[int(c.succ_idx[e])] += 1
        for (j, nk) in edges:
            cb, qc = int(p.call_block[j]), p.procs[nk[0]]
            names = [(v, v) for v in range(G)] + [(int(x), G + i) for i, x in
                                                 enumerate(p.arg_var[int(p.arg_ptr[j]):int(p.arg_ptr[j + 1])])]
            for e in range(int(c.succ_ptr[cb]), int(c.succ_ptr[cb + 1])):
                t = int(c.succ_idx[e])
                if npred[t] != 1:
                    continue
                for key, ig in (("avf_h", "ins_edge_h"), ("avf_d", "ins_edge_d")):
                    for x, y in names:
                        if bit(results[k][key][t], x) and not bit(results[k][ig][e], x) \
                                and not bit(results[nk][key][qc.exit], y):
                            out.append((k, j, x))
    return out


@pytest.mark.parametrize("seed", range(16))
def test_validity_after_a_call_never_exceeds_the_callee_exit(seed):
    p = cap_program(seed)
    po = ProgramOracle(p)
    _, _, results = po.analyze()
    assert not exceeds_callee_exit(po, p, results)


def hand_program():
    root, _ = synth.from_edges([(0, [], []), (0, [], []), (0, [0], []), (0, [], [])],
                               [(0, 1, 0), (1, 2, 0), (2, 3, 0)], 1)
    f, _ = synth.from_edges([(0, [], []), (1, [], [0]), (0, [], [])], [(0, 1, 0), (1, 2, 0)], 1)
    return f, synth.Program(procs=[root, f], n_globals=0, call_proc=np.array([0], np.int32),
                            call_block=np.array([1], np.int32), callee=np.array([1], np.int32), roots=[0],
                            n_params=np.array([0, 1], np.int32), arg_ptr=np.array([0, 1], np.int64),
                            arg_var=np.array([0], np.int32), arg_const=np.array([0], np.uint8))


def test_parameter_written_in_a_callee_is_copied_back_for_the_caller():
    """Hand-derived: root R has a local x (variable 0, no globals); R's block 1 calls F
    binding x to F's parameter p; F's kernel block writes p; R's host block 2 reads x.
    F's context gets x's exit liveness on the host, so F copies p back to the host on
    entering its EXIT, and p's map kind in F is "from"; R copies nothing."""
    f, p = hand_program()
    po = ProgramOracle(p)
    _, ctx, results = po.analyze()
    r, c = results[(0, ())], results[(1, (0,))]
    assert not any(np.asarray(r[k]).any() for k in ("ins_entry_h", "ins_entry_d", "ins_edge_h", "ins_edge_d"))
    assert bit(ctx[(1, (0,))][2], 0) == 1                  # p live on the host at F's exit
    assert [int(x) for x in np.asarray(c["ins_entry_h"]).ravel()] == [0, 0, 1]
    assert not np.asarray(c["ins_edge_h"]).any() and not np.asarray(c["ins_entry_d"]).any()
    assert int(c["var_kind"][0]) == 2                      # map(from)
    assert int(c["nu_h"][f.entry][0]) & 1 == 0             # p is written before any host read


def const_arg_program(const):
    """R (local x) calls F(x); F's only block passes its parameter p to an external
    function, as a pointer to const or not."""
    root, _ = synth.from_edges([(0, [], []), (0, [], []), (0, [], [])], [(0, 1, 0), (1, 2, 0)], 1)
    f, _ = synth.from_edges([(0, [], []), (0, [], []), (0, [], [])], [(0, 1, 0), (1, 2, 0)], 1)
    return synth.Program(procs=[root, f], n_globals=0, call_proc=np.array([0, 1], np.int32),
                         call_block=np.array([1, 1], np.int32), callee=np.array([1, -1], np.int32), roots=[0],
                         n_params=np.array([0, 1], np.int32), arg_ptr=np.array([0, 1, 2], np.int64),
                         arg_var=np.array([0, 0], np.int32), arg_const=np.array([0, int(const)], np.uint8))


def test_external_call_through_a_pointer_to_const_does_not_write_the_parameter():
    """Hand-derived: F may read p on the host either way; it may write p only when the
    external function takes it as a pointer to non-const."""
    from oracle import SUM_MAYR_H, SUM_MAYW_D, SUM_MAYW_H
    for const in (False, True):
        S, _, _ = ProgramOracle(const_arg_program(const)).analyze()
        assert bit(S[1][SUM_MAYR_H], 0) == 1
        assert bit(S[1][SUM_MAYW_H], 0) == int(not const)
        assert bit(S[1][SUM_MAYW_D], 0) == 0


def merge_params_program(seed, n_globals=4):
    """Root R passes its local x to A at two sites; A passes its parameter on to B, B to C.
    The call strings (site 0, A->B, B->C) and (site 1, A->B, B->C) meet in C's context, so
    the two paths into C can leave the parameter fresh in different spaces.  Every other
    block is a random host or device statement over the globals and the local or parameter
    (x in R, the parameter in C; A and B only pass it on)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    G = n_globals
    nv = G + 2

    def stmt(p=0.3, par=True):
        dev = int(rng.random() < 0.5)
        pool = list(range(G)) + ([G] if par else [])
        rd = [v for v in pool if rng.random() < p]
        wr = [v for v in pool if rng.random() < p]
        return (dev, rd, wr)

    def chain(body):
        blocks = [(0, [], [])] + body + [(0, [], [])]
        edges = [(i, i + 1, 0) for i in range(len(blocks) - 1)]
        return synth.from_edges(blocks, edges, nv)[0]

    call = (0, [], [])
    root = chain([stmt(), call, stmt(), stmt(), call, stmt()])          # calls at blocks 2 and 5
    root.exit_live_h = np.zeros(root.wd, np.uint64)
    a = chain([stmt(0.1, False), call, stmt(0.1, False)])              # call at block 2
    b = chain([call, stmt(0.1, False)])                                # call at block 1
    c = chain([stmt(0.3), stmt(0.3)])
    return synth.Program(procs=[root, a, b, c], n_globals=G,
                         call_proc=np.array([0, 0, 1, 2], np.int32), call_block=np.array([2, 5, 2, 1], np.int32),
                         callee=np.array([1, 1, 2, 3], np.int32), roots=[0],
                         n_params=np.array([0, 1, 1, 1], np.int32), arg_ptr=np.array([0, 1, 2, 3, 4], np.int32),
                         arg_var=np.array([G, G, G, G], np.int32), arg_const=np.zeros(4, np.uint8))


# seeds (of 1,500 tried) whose program needs a host read of B's parameter at B's call of C
MERGE_PARAM_SEEDS = (44, 156, 260, 319, 371, 550, 586, 596, 727, 973, 1008, 1085, 1494)


def test_parameter_demands_are_needed_and_make_the_program_safe():
    """A parameter valid nowhere at a merged context's entry is demanded at the leading call
    site as a host read of the caller variable bound to it; dropping the demand reopens the gap
    in the callee context; with the demands the walks find nothing stale."""
    seen = 0
    for seed in MERGE_PARAM_SEEDS:
        p = merge_params_program(27_000 + seed)
        po = ProgramOracle(p)
        _, ctx, results = po.analyze()
        G = p.n_globals
        m = po.demand.get(3)
        assert m is not None and bit(m, G), seed
        seen += 1
        po2 = ProgramOracle(p)
        po2.demand = {jj: mm.copy() for jj, mm in po.demand.items()}
        po2.cap = dict(po.cap)
        po2.demand[3][G >> 6] &= ~np.uint64(1 << (G & 63))
        S2 = po2.summarize()
        po2.contexts(S2)
        assert any(k[0] == 3 and bit(nw, G) for k, nw in po2.nowhere.items()), seed
        errs, _ = simulate_program(p, ctx, results, po.demand, walks=40, seed=seed)
        assert not errs, errs[:3]
    assert seen == len(MERGE_PARAM_SEEDS)


# ---------------------------------------------------------------------------
# planted mistakes in a copy of the interprocedural driver must be caught
PARAM_MUTANTS = {
    "arguments_unbound": ("        return [(x, (self.G + i) if q >= 0 else None, c) for i, (x, c) in enumerate(self.args[j])]",
                          "        return []"),
    "boundary_drops_parameters": ("                    t = G + i\n", "                    t = G + i + 64\n"),
    "external_argument_keeps_device_copy": ("                        col[SUM_TD_00 + k4] = const and k4 >= 2",
                                            "                        col[SUM_TD_00 + k4] = k4 >= 2"),
    "external_const_argument_written": ("                        if not const:\n                            m[SUM_MAYW_H, x >> 6] |= b",
                                        "                        if True:\n                            m[SUM_MAYW_H, x >> 6] |= b"),
    "validity_combined_by_or": ("                    for r in T_ROWS:\n                        if not col[r]:\n"
                                "                            s[r, w] &= ~bit",
                                "                    for r in T_ROWS:\n                        if col[r]:\n"
                                "                            s[r, w] |= bit"),
    "demand_kept_on_globals": ("            d |= self._to_caller(jj, q, bits, P2)",
                               "            d[:gw] |= bits[:gw] & _gmask(G, gw)"),
    "argument_cap_ignored": ("                            col[SUM_TH_00 + k4] &= ch\n                            col[SUM_TD_00 + k4] &= cd\n",
                             "                            pass\n"),
}


def _pins_hold(PO):
    from test_oracle_program_device import _mutant_driver  # noqa: F401  (same loader)
    try:
        for seed in range(5):
            p = may_program(seed)
            po = PO(p)
            S, _, _ = po.analyze()
            may = brute_may(p, po.demand)
            for P in range(len(p.procs)):
                ns = p.n_globals + int(p.n_params[P])
                for k in range(4):
                    if bits_of(S[P][k], ns) != may[P][k]:
                        return False
        for seed in range(8):
            p = walk_program(seed)
            po = PO(p)
            _, ctx, results = po.analyze()
            errs, _ = simulate_program(p, ctx, results, po.demand, walks=60, seed=seed)
            if errs:
                return False
        for seed in range(4):
            p = prog_of(21_000 + seed)
            po = PO(p)
            _, _, results = po.analyze()
            big, instances, pos = inline_program(p, 0, po.demand)
            ref = oracle.solve(big)
            for (P, sigma, off, vmap) in instances:
                if len(sigma) > 2:
                    continue
                ns = p.procs[P].n_vars if not sigma else p.n_globals + int(p.n_params[P])
                r = results[(P, sigma)]
                for b in range(p.procs[P].n_blocks):
                    for k in ("nu_h", "nu_d"):
                        if bits_of(r[k][b], ns) != mapped(ref[k][pos[off + b]], vmap, ns):
                            return False
        for seed in (4, 13, 22):
            p = cap_program(seed)
            po = PO(p)
            _, _, results = po.analyze()
            if exceeds_callee_exit(po, p, results):
                return False
        for seed in MERGE_PARAM_SEEDS[:4]:
            p = merge_params_program(27_000 + seed)
            po = PO(p)
            _, ctx, results = po.analyze()
            m = po.demand.get(3)
            if m is None or not bit(m, p.n_globals):
                return False
            errs, _ = simulate_program(p, ctx, results, po.demand, walks=40, seed=seed)
            if errs:
                return False
        from oracle import SUM_MAYW_H
        for const in (False, True):
            S, _, _ = PO(const_arg_program(const)).analyze()
            if bit(S[1][SUM_MAYW_H], 0) != int(not const):
                return False
        f, p = hand_program()
        c = PO(p).analyze()[2][(1, (0,))]
        if [int(x) for x in np.asarray(c["ins_entry_h"]).ravel()] != [0, 0, 1]:
            return False
    except (ValueError, KeyError, AssertionError, RuntimeError, IndexError):
        return False
    return True


def test_unmutated_driver_passes_the_parameter_pins():
    assert _pins_hold(ProgramOracle)


@pytest.mark.parametrize("name", sorted(PARAM_MUTANTS))
def test_parameter_mutant_is_caught(name):
    from test_oracle_program_device import _mutant_driver
    assert not _pins_hold(_mutant_driver(*PARAM_MUTANTS[name])), "the pins did not catch " + name
