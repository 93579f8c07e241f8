"""Pins of the interprocedural refinements (section "Interprocedural
Analysis": accesses on the host or the device; the read-only rule for data
behind a pointer to const, applied per global):

* calls made inside a kernel: the may-read / may-write rows of every
  procedure against a brute-force fixed point over the call graph written
  here; a procedure whose calls all run on the device solves exactly like
  the CFG with each call block turned into a kernel block reading and
  writing the callee's globals; whole-program random walks (the callee run
  on the device) find no stale read or copy source;
* const globals: an external call keeps their device copy (a worked
  example derived by hand), they are never copied to the host, a program
  that writes one is rejected, and without external calls the mark changes
  nothing."""
import numpy as np
import pytest

import oracle
import synth
from checkers import simulate_program
from oracle.program import ProgramOracle

SMALL = dict(n_procs=8, n_globals=12, n_locals=5, blocks=(4, 14), mean_calls=2.0, max_calls=3, scc_procs=0,
             device_frac=0.4, p_read=0.25, p_write=0.15, threads=1)


def prog_of(seed, **kw):
    prm = dict(SMALL)
    prm.update(kw)
    return synth.program(seed, **prm)


def bits_of(row, n):
    return {v for v in range(n) if (int(row[v >> 6]) >> (v & 63)) & 1}


def brute_may(p, demand):
    """Per procedure, the globals it or anything it calls may read / write, per space, by a
    plain fixed point over the call graph (device calls put the callee's everything on the
    device; an external call reads every global and writes every non-const one)."""
    G, n = p.n_globals, len(p.procs)
    const = bits_of(p.const_globals, G) if p.const_globals is not None else set()
    cs = p.call_space if p.call_space is not None else np.zeros(len(p.call_proc), np.uint8)
    own = []
    for P, c in enumerate(p.procs):
        m = [set(), set(), set(), set()]   # read H, read D, write H, write D
        R = np.asarray(c.R, np.uint64).reshape(c.n_blocks, c.wd)
        W = np.asarray(c.W, np.uint64).reshape(c.n_blocks, c.wd)
        for b in range(c.n_blocks):
            d = int(c.space[b])
            m[d] |= {v for v in bits_of(R[b], c.n_vars) if v < G}
            m[2 + d] |= {v for v in bits_of(W[b], c.n_vars) if v < G}
        own.append(m)
    for j, d in demand.items():
        own[int(p.call_proc[j])][0] |= {v for v in bits_of(d, G)}
    may = [[set(x) for x in m] for m in own]
    allg = set(range(G))
    while True:
        changed = False
        for j in range(len(p.call_proc)):
            P, q = int(p.call_proc[j]), int(p.callee[j])
            if q < 0:
                r, w = allg, allg - const
                add = [set(), r, set(), w] if cs[j] else [r, set(), w, set()]
            elif cs[j]:
                w = may[q][2] | may[q][3]
                add = [set(), may[q][0] | may[q][1] | w, set(), w]
            else:
                add = may[q]
            for k in range(4):
                if not add[k] <= may[P][k]:
                    may[P][k] |= add[k]
                    changed = True
        if not changed:
            return may


@pytest.mark.parametrize("seed", range(16))
def test_may_rows_match_a_brute_force_fixed_point(seed):
    p = prog_of(700 + seed, scc_procs=4 if seed % 2 else 0, scc_size=(2, 3), device_call_frac=0.4,
                n_const=3 if seed % 3 else 0, external_frac=0.25 if seed % 4 == 1 else 0.0)
    po = ProgramOracle(p)
    S, _, _ = po.analyze()
    may = brute_may(p, po.demand)
    for P in range(len(p.procs)):
        for k in range(4):
            assert bits_of(S[P][k], p.n_globals) == may[P][k], (P, k)


@pytest.mark.parametrize("seed", range(12))
def test_calls_in_kernels_solve_like_kernel_blocks(seed):
    """Every call made inside a kernel: each procedure is a root whose solve is the plain
    solve of its CFG with each call block reading and writing (on the device) the callee's
    may sets from the brute-force fixed point."""
    p = prog_of(800 + seed, device_call_frac=1.0, scc_procs=4 if seed % 2 else 0, scc_size=(2, 3),
                n_const=2 if seed % 3 else 0, external_frac=0.25 if seed % 4 == 1 else 0.0)
    assert sorted(p.roots) == list(range(len(p.procs)))
    po = ProgramOracle(p)
    S, ctx, results = po.analyze()
    assert not po.demand
    may = brute_may(p, {})
    G = p.n_globals
    allg = set(range(G))
    const = bits_of(p.const_globals, G) if p.const_globals is not None else set()
    for P, c in enumerate(p.procs):
        R = np.array(c.R, np.uint64).reshape(c.n_blocks, c.wd)
        W = np.array(c.W, np.uint64).reshape(c.n_blocks, c.wd)
        for j in range(len(p.call_proc)):
            if int(p.call_proc[j]) != P:
                continue
            q, b = int(p.callee[j]), int(p.call_block[j])
            if q < 0:
                rd, wr = allg, allg - const
            else:
                wr = may[q][2] | may[q][3]
                rd = may[q][0] | may[q][1] | wr
            for v in rd:
                R[b, v >> 6] |= np.uint64(1 << (v & 63))
            for v in wr:
                W[b, v >> 6] |= np.uint64(1 << (v & 63))
        plain = synth.CFG(n_blocks=c.n_blocks, n_vars=c.n_vars, succ_ptr=c.succ_ptr, succ_idx=c.succ_idx,
                          edge_kind=c.edge_kind, space=c.space, R=R, W=W, entry=c.entry, exit=c.exit)
        want = oracle.solve(plain)
        got = results[(P, ())]
        for k in ("nu_h", "nu_d", "ave_h", "ave_d", "avf_h", "avf_d", "ins_entry_h", "ins_entry_d",
                  "ins_edge_h", "ins_edge_d", "var_kind"):
            assert np.array_equal(np.asarray(got[k]), np.asarray(want[k]).reshape(np.asarray(got[k]).shape)), (P, k)


@pytest.mark.parametrize("seed", range(10))
def test_whole_program_walks_with_device_calls_and_const_globals(seed):
    p = prog_of(900 + seed, scc_procs=4 if seed % 2 else 0, scc_size=(2, 3), device_call_frac=0.4,
                n_const=3, external_frac=0.2)
    po = ProgramOracle(p)
    S, ctx, results = po.analyze()
    errs, cut = simulate_program(p, None, results, po.demand, walks=150, seed=seed)
    assert not errs, errs[:4]


@pytest.mark.parametrize("seed", range(10))
def test_const_globals_are_never_copied_to_the_host(seed):
    p = prog_of(1_000 + seed, scc_procs=4 if seed % 2 else 0, scc_size=(2, 3), device_call_frac=0.3,
                n_const=5, external_frac=0.3)
    po = ProgramOracle(p)
    S, ctx, results = po.analyze()
    const = p.const_globals
    for key, r in results.items():
        for k in ("ins_entry_h", "ins_edge_h"):
            rows = np.asarray(r[k])
            if rows.size:
                assert not (rows[:, :const.size] & const).any(), (key, k)


def test_a_program_writing_a_const_global_is_rejected():
    p = prog_of(1_100, n_const=2)
    g = int(np.nonzero([(int(p.const_globals[v >> 6]) >> (v & 63)) & 1 for v in range(p.n_globals)])[0][0])
    c = p.procs[0]
    W = np.array(c.W, np.uint64).reshape(c.n_blocks, c.wd)
    users = [b for b in range(c.n_blocks) if b not in (c.entry, c.exit)]
    W[users[0], g >> 6] |= np.uint64(1 << (g & 63))
    c.W = W
    with pytest.raises(ValueError):
        ProgramOracle(p)


@pytest.mark.parametrize("seed", range(6))
def test_const_marks_matter_only_at_external_calls(seed):
    p = prog_of(1_200 + seed, scc_procs=4 if seed % 2 else 0, scc_size=(2, 3), device_call_frac=0.3, n_const=4)
    a = ProgramOracle(p).analyze()[2]
    p.const_globals = None
    b = ProgramOracle(p).analyze()[2]
    assert a.keys() == b.keys()
    for key in a:
        for k in ("ins_entry_h", "ins_entry_d", "ins_edge_h", "ins_edge_d", "avf_h", "avf_d"):
            assert np.array_equal(np.asarray(a[key][k]), np.asarray(b[key][k])), (key, k)


def test_external_call_keeps_a_const_global_on_the_device():
    """Hand-derived: ENTRY, kernel K1 reads g, host block C calls an external function,
    kernel K2 reads g, EXIT.  g is valid on the host at entry, so a copy to the device goes
    before K1 (map(to)).  The external call may write every global on the host and so leaves
    the device copy stale: K2 needs a second copy (target update to).  With g const the call
    cannot write it, the device copy stays current, and K2 needs nothing."""
    def build(const):
        cfg, _ = synth.from_edges([(0, [], []), (1, [0], []), (0, [], []), (1, [0], []), (0, [], [])],
                                  [(0, 1, 0), (1, 2, 0), (2, 3, 0), (3, 4, 0)], 1)
        return synth.Program(procs=[cfg], n_globals=1, call_proc=np.array([0], np.int32),
                             call_block=np.array([2], np.int32), callee=np.array([-1], np.int32), roots=[0],
                             const_globals=np.array([1], np.uint64) if const else None)
    for const, want in ((False, [1, 3]), (True, [1])):
        _, _, res = ProgramOracle(build(const)).analyze()
        r = res[(0, ())]
        assert [b for b in range(5) if int(r["ins_entry_d"][b, 0]) & 1] == want
        assert not r["ins_edge_d"].any() and not r["ins_entry_h"].any() and not r["ins_edge_h"].any()


# ---------------------------------------------------------------------------
# planted mistakes in a copy of the interprocedural driver must be caught
PROGRAM_MUTANTS = {
    "device_call_writes_nothing": ("                W[blk] |= wr\n", ""),
    "device_call_reads_only_device_reads": (
        "                    r_any = rows[SUM_MAYR_H] | rows[SUM_MAYR_D] | w_any",
        "                    r_any = rows[SUM_MAYR_D]"),
    "external_writes_const": ("    r[SUM_MAYW_H] = gm & ~c ", "    r[SUM_MAYW_H] = gm "),
    "external_stales_const": ("        r[SUM_TD_00 + k] = c if k >= 2 else 0 ",
                              "        r[SUM_TD_00 + k] = 0 "),
    "device_site_as_host_call": ("            (self.dsites if dev else self.sites)[P].append(j)",
                                 "            self.sites[P].append(j)"),
}


def _mutant_driver(old, new):
    import importlib.util
    import os
    import oracle.program as prog_mod
    src = open(prog_mod.__file__).read()
    assert old in src, "mutation site not found"
    spec = importlib.util.spec_from_loader("oracle._program_mutant", loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = "oracle"
    mod.__file__ = os.path.join(os.path.dirname(prog_mod.__file__), "_program_mutant.py")
    exec(compile(src.replace(old, new, 1), mod.__file__, "exec"), mod.__dict__)
    return mod.ProgramOracle


def _pins_hold(PO):
    try:
        for seed in range(6):
            p = prog_of(700 + seed, scc_procs=4 if seed % 2 else 0, scc_size=(2, 3), device_call_frac=0.4,
                        n_const=3 if seed % 3 else 0, external_frac=0.25 if seed % 4 == 1 else 0.0)
            po = PO(p)
            S, _, results = po.analyze()
            may = brute_may(p, po.demand)
            for P in range(len(p.procs)):
                for k in range(4):
                    if bits_of(S[P][k], p.n_globals) != may[P][k]:
                        return False
            errs, _ = simulate_program(p, None, results, po.demand, walks=60, seed=seed)
            if errs:
                return False
        for const, want in ((False, [1, 3]), (True, [1])):
            cfg, _ = synth.from_edges([(0, [], []), (1, [0], []), (0, [], []), (1, [0], []), (0, [], [])],
                                      [(0, 1, 0), (1, 2, 0), (2, 3, 0), (3, 4, 0)], 1)
            p = synth.Program(procs=[cfg], n_globals=1, call_proc=np.array([0], np.int32),
                              call_block=np.array([2], np.int32), callee=np.array([-1], np.int32), roots=[0],
                              const_globals=np.array([1], np.uint64) if const else None)
            r = PO(p).analyze()[2][(0, ())]
            if [b for b in range(5) if int(r["ins_entry_d"][b, 0]) & 1] != want:
                return False
    except (ValueError, KeyError, AssertionError, RuntimeError):
        return False
    return True


def test_unmutated_driver_passes_the_pins():
    assert _pins_hold(ProgramOracle)


@pytest.mark.parametrize("name", sorted(PROGRAM_MUTANTS))
def test_driver_mutant_is_caught(name):
    assert not _pins_hold(_mutant_driver(*PROGRAM_MUTANTS[name])), "the pins did not catch " + name
