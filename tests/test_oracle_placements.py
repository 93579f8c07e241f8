"""Pins of the two placement variants of the oracle.

Loop-entry refinement (Algorithm 1 puts the update a loop's writes make
necessary after the loop nest; the delay of the default placement stops at
loop entries and can leave a copy there that no read uses): checked against a
path search written here from the definition — a copy's value is live when
some path from it reaches a read of that copy (a read in its space, a copy
out of it, the liveness after EXIT) before a write or a copy into the same
space replaces it.  A copy on a loop-entry edge survives iff it is live;
every other copy is the default placement's; the result passes the
placement invariants and random-path simulation.

Pure lazy (the delay without the loop rule): the same as the default
placement on the CFG whose loop-entry edges are relabelled ordinary edges,
and sound (invariants, simulation) on CFGs with loops; the worked examples
carry hand derivations of both variants."""
from collections import deque

import numpy as np
import pytest

import checkers
import oracle
import synth

KEYS = ("nu_h", "nu_d", "ave_h", "ave_d", "avf_h", "avf_d", "ins_entry_h", "ins_entry_d",
        "ins_edge_h", "ins_edge_d", "var_kind", "after_dev", "before_dev", "fp_clause")


def loopy(seed: int, marks: bool = False):
    rng = np.random.Generator(np.random.PCG64(77_000 + seed))
    cfg = synth.make_cfg(77_000 + seed, n_user=int(rng.integers(6, 40)), n_vars=int(rng.choice([1, 5, 64, 70])),
                         max_loop_depth=int(rng.integers(1, 4)), device_frac=0.4,
                         irr_loop_frac=0.2 if seed % 3 == 0 else 0.0, p_read=0.25, p_write=0.15)
    if marks:
        synth.mark_scalars(cfg, seed, frac=0.4, read_only_frac=0.7)
    if seed % 4 == 1:
        m = synth.var_mask(cfg.n_vars)
        cfg.entry_valid_d = np.array([int(x) for x in rng.integers(0, 1 << 62, size=cfg.wd)], dtype=np.uint64) & m
        cfg.entry_valid_h = m.copy()
        cfg.exit_live_d = np.array([int(x) for x in rng.integers(0, 1 << 62, size=cfg.wd)], dtype=np.uint64) & m
    return cfg


def value_read(V, ie, ig, s: int, start: int, v: int) -> bool:
    """Is the value a copy leaves in space s at the entry of `start` (before the
    copies placed there) read before something replaces it?  A search over blocks."""
    o = 1 - s
    bit = 1 << v
    seen = {start}
    todo = deque([start])
    while todo:
        b = todo.popleft()
        if ie[o][b] & bit:          # a copy into the other space reads it
            return True
        if ie[s][b] & bit:          # a copy into s replaces it
            continue
        if V.use(s, b) & bit:       # a read (EXIT: the liveness after the region)
            return True
        if b == V.exit:
            continue
        if V.space[b] == s and V.W[b] & bit:
            continue
        if s == 1 and V.space[b] == 1 and V.R[b] & V.fp & bit:
            continue                # no valid device copy after a kernel's firstprivate read
        for (t, e) in V.succ[b]:
            if ig[o][e] & bit:
                return True
            if ig[s][e] & bit:
                continue
            if t not in seen:
                seen.add(t)
                todo.append(t)
    return False


def rows(r, wd):
    ie = [checkers.rows_int(r["ins_entry_h"]), checkers.rows_int(r["ins_entry_d"])]
    ig = [checkers.rows_int(r["ins_edge_h"].reshape(-1, wd)), checkers.rows_int(r["ins_edge_d"].reshape(-1, wd))]
    return ie, ig


@pytest.mark.parametrize("seed", range(60))
def test_refinement_drops_exactly_the_unread_loop_entry_copies(seed):
    cfg = loopy(seed, marks=seed % 2 == 1)
    base = oracle.solve(cfg)
    ref = oracle.solve(cfg, placement=oracle.PLACEMENT_REFINE)
    V = checkers.View(cfg)
    ie0, ig0 = rows(base, cfg.wd)
    ie1, ig1 = rows(ref, cfg.wd)
    assert ie1 == ie0
    dropped = 0
    for p in range(cfg.n_blocks):
        for (t, e) in V.succ[p]:
            for s in (0, 1):
                if int(cfg.edge_kind[e]) != 2:
                    assert ig1[s][e] == ig0[s][e]
                    continue
                for v in range(cfg.n_vars):
                    if not (ig0[s][e] >> v) & 1:
                        assert not (ig1[s][e] >> v) & 1
                        continue
                    live = value_read(V, ie0, ig0, s, t, v)
                    assert bool((ig1[s][e] >> v) & 1) == live, (e, s, v)
                    dropped += not live
    assert checkers.check_invariants(cfg, ref) == []
    errs, _ = checkers.simulate_paths(cfg, ref, walks=20, seed=seed)
    assert not errs, errs[:3]


def test_refinement_drops_some_copies_in_a_family():
    """The family above does exercise the rule (some loop-entry copies are dropped)."""
    n = 0
    for seed in range(60):
        cfg = loopy(seed)
        a = oracle.solve(cfg)
        b = oracle.solve(cfg, placement=oracle.PLACEMENT_REFINE)
        n += int(np.count_nonzero(a["ins_edge_h"] != b["ins_edge_h"]) + np.count_nonzero(a["ins_edge_d"] != b["ins_edge_d"]))
    assert n > 0


def test_refinement_keeps_config1_sound():
    for i in range(20):
        cfg = synth.c1(i)
        r = oracle.solve(cfg, placement=oracle.PLACEMENT_REFINE)
        assert checkers.check_invariants(cfg, r) == []
        errs, _ = checkers.simulate_paths(cfg, r, walks=20, seed=i)
        assert not errs, errs[:3]


@pytest.mark.parametrize("seed", range(40))
def test_lazy_is_the_default_with_loop_entries_as_ordinary_edges(seed):
    cfg = loopy(seed, marks=seed % 2 == 0)
    r = oracle.solve(cfg, placement=oracle.PLACEMENT_LAZY)
    plain = synth.CFG(**{f: getattr(cfg, f) for f in cfg.__dataclass_fields__})
    plain.edge_kind = np.where(np.asarray(cfg.edge_kind) == 2, 0, np.asarray(cfg.edge_kind)).astype(np.uint8)
    d = oracle.solve(plain)
    for k in KEYS:
        assert np.array_equal(r[k], d[k]), k


@pytest.mark.parametrize("seed", range(30))
def test_lazy_with_loops_is_sound(seed):
    cfg = loopy(seed, marks=seed % 2 == 0)
    r = oracle.solve(cfg, placement=oracle.PLACEMENT_LAZY)
    assert checkers.check_invariants(cfg, r) == []
    errs, _ = checkers.simulate_paths(cfg, r, walks=20, seed=seed)
    assert not errs, errs[:3]


def test_lazy_moves_copies_into_loops_in_a_family():
    """Somewhere in the family the variant does place a copy the loop rule keeps out of a loop."""
    n = 0
    for seed in range(40):
        cfg = loopy(seed)
        a = oracle.solve(cfg)
        b = oracle.solve(cfg, placement=oracle.PLACEMENT_LAZY)
        n += sum(int(np.count_nonzero(a[k] != b[k])) for k in ("ins_entry_h", "ins_entry_d", "ins_edge_h", "ins_edge_d"))
    assert n > 0


def test_variants_leave_the_analyses_alone():
    """Next use, eager validity, labels and firstprivate clauses do not depend on the placement."""
    for seed in range(10):
        cfg = loopy(seed, marks=True)
        a = oracle.solve(cfg)
        for pl in (oracle.PLACEMENT_LAZY, oracle.PLACEMENT_REFINE):
            b = oracle.solve(cfg, placement=pl)
            for k in ("nu_h", "nu_d", "ave_h", "ave_d", "after_dev", "before_dev", "fp_clause"):
                assert np.array_equal(a[k], b[k]), k
