"""Pins of the firstprivate reading (section "Data-Flow Analysis", the
firstprivate paragraph; Table II): a scalar the front end marks and no
DEVICE block writes reaches each kernel that reads it as a firstprivate
argument initialised from the host copy; that read needs the host copy
valid at the launch, and after the kernel the device copy is not valid.

Checked against path enumeration (next use and validity over every path of
small acyclic CFGs), the worked example P12 with and without the mark, the
invariants and random-path simulation (every kernel's firstprivate read
sees the latest host value), and properties that follow from the reading:
marks on nothing change nothing, a marked scalar that a kernel writes is
not firstprivate, and with the default boundaries a firstprivate variable
is never copied into the device."""
import json
import os

import numpy as np
import pytest

import checkers
import oracle
import synth
from test_oracle_pins import GOLDEN, load_golden

KEYS = ("nu_h", "nu_d", "ave_h", "ave_d", "avf_h", "avf_d", "ins_entry_h", "ins_entry_d",
        "ins_edge_h", "ins_edge_d", "var_kind", "after_dev", "before_dev", "fp_clause")


def _same(a, b):
    return all(np.array_equal(np.asarray(a[k]), np.asarray(b[k])) for k in KEYS)


def test_p12_without_the_mark():
    g, cfg, pos = load_golden(os.path.join(GOLDEN, "P12_firstprivate_scalar.json"))
    cfg.scalar = None
    r = oracle.solve(cfg)
    want = g["without_scalar"]
    assert [int(x) for x in r["ins_entry_d"][:, 0]] == want["ins_entry_d"]
    assert [int(x) for x in r["var_kind"]] == [3, 1]
    assert not r["fp_clause"].any()


@pytest.mark.parametrize("seed", range(6))
def test_no_marks_change_nothing(seed):
    cfg = synth.make_cfg(61_000 + seed, n_user=60, n_vars=130, max_loop_depth=4, device_frac=0.4,
                         irr_loop_frac=0.2)
    a = oracle.solve(cfg)
    cfg.scalar = np.zeros(cfg.wd, np.uint64)
    b = oracle.solve(cfg)
    assert _same(a, b)


@pytest.mark.parametrize("seed", range(30))
def test_mop_with_marked_scalars(seed):
    rng = np.random.Generator(np.random.PCG64(3_000 + seed))
    nb = int(rng.integers(3, 12))
    nv = int(rng.choice([3, 31, 64, 65, 70]))
    cfg = synth.mark_scalars(synth.random_dag(900 + seed, nb, nv, p_loop_entry=0.3 if seed % 2 else 0.0),
                             seed, frac=0.5, read_only_frac=0.7)
    if seed % 3 == 0:
        m = synth.var_mask(nv)
        evd = np.array([int(x) for x in rng.integers(0, 1 << 62, size=cfg.wd)], dtype=np.uint64) & m
        cfg.entry_valid_d = evd
        cfg.entry_valid_h = m.copy()
        cfg.exit_live_d = np.array([int(x) for x in rng.integers(0, 1 << 62, size=cfg.wd)], dtype=np.uint64) & m
    r = oracle.solve(cfg)
    wd = cfg.wd
    nu_h, nu_d = checkers.mop_nu(cfg)
    assert checkers.rows_int(r["nu_h"]) == nu_h and checkers.rows_int(r["nu_d"]) == nu_d
    assert (checkers.rows_int(r["ave_h"]), checkers.rows_int(r["ave_d"])) == \
        checkers.mop_valid(cfg, [nu_h, nu_d], [{}, {}])
    ge = [checkers.rows_int(r["ins_entry_h"]), checkers.rows_int(r["ins_entry_d"])]
    gg = [dict(enumerate(checkers.rows_int(r["ins_edge_h"].reshape(-1, wd)))) if cfg.n_edges else {},
          dict(enumerate(checkers.rows_int(r["ins_edge_d"].reshape(-1, wd)))) if cfg.n_edges else {}]
    assert (checkers.rows_int(r["avf_h"]), checkers.rows_int(r["avf_d"])) == checkers.mop_valid(cfg, ge, gg)
    assert checkers.check_invariants(cfg, r) == []
    # the clause of each kernel: its reads of the firstprivate variables
    V = checkers.View(cfg)
    assert checkers.rows_int(r["fp_clause"]) == [V.R[b] & V.fp if V.space[b] == 1 else 0 for b in range(V.nb)]


@pytest.mark.parametrize("seed", range(8))
def test_walks_with_marked_scalars(seed):
    cfgs = [synth.mark_scalars(synth.c1(seed), 40 + seed, frac=0.4, read_only_frac=0.6),
            synth.mark_scalars(synth.make_cfg(62_000 + seed, n_user=120, n_vars=90, max_loop_depth=5,
                                              device_frac=0.4, irr_loop_frac=0.2), seed)]
    for cfg in cfgs:
        r = oracle.solve(cfg)
        assert checkers.check_invariants(cfg, r) == []
        errs, _ = checkers.simulate_paths(cfg, r, walks=60, seed=seed)
        assert not errs, errs[:3]


def test_device_written_scalar_is_not_firstprivate():
    cfg = synth.mark_scalars(synth.make_cfg(63_000, n_user=80, n_vars=100, max_loop_depth=3, device_frac=0.5,
                                            p_read=0.3, p_write=0.2), 5, frac=0.6, read_only_frac=0.5)
    V = checkers.View(cfg)
    a = oracle.solve(cfg)
    # solving with only the read-only marks gives the same result
    fp = np.array([(V.fp >> (64 * w)) & ((1 << 64) - 1) for w in range(cfg.wd)], dtype=np.uint64)
    marked = np.asarray(cfg.scalar).copy()
    assert (marked & ~fp).any()          # some marked scalars are written by a kernel
    cfg.scalar = fp
    b = oracle.solve(cfg)
    assert _same(a, b)


@pytest.mark.parametrize("seed", range(6))
def test_firstprivate_never_copied_to_the_device(seed):
    cfg = synth.mark_scalars(synth.make_cfg(64_000 + seed, n_user=150, n_vars=128, max_loop_depth=4,
                                            device_frac=0.4, irr_loop_frac=0.1), seed, frac=0.5, read_only_frac=1.0)
    V = checkers.View(cfg)
    r = oracle.solve(cfg)
    fp_rows = V.fp
    for k in ("ins_entry_d", "ins_edge_d"):
        for x in checkers.rows_int(r[k].reshape(-1, cfg.wd)):
            assert x & fp_rows == 0, k
    devread = 0
    for b in range(V.nb):
        if V.space[b] == 1:
            devread |= V.R[b]
    for v in range(cfg.n_vars):
        is_fp = (fp_rows >> v) & 1
        assert bool(int(r["var_kind"][v]) & 8) == bool(is_fp and (devread >> v) & 1), v
