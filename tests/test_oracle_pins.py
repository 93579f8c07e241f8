"""Pins of the oracle against facts that do not come from the oracle itself.

* worked examples from the paper's motivation listings, Figure 2 and the
  backprop snippet (tests/golden, each file cites its passage);
* meet-over-all-paths brute force for the gen/kill problems (NU, AVE, AVF);
* brute-force reachability for the label inputs;
* special cases with textbook answers;
* bit independence (permuting variables permutes every output);
* safety / completeness / exclusivity and random-path simulation of the
  placement, for the delayed and the eager variants.
"""
import glob
import json
import os

import numpy as np
import pytest

import checkers
import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SPACE = {"H": 0, "D": 1}
KIND = {"N": 0, "BACK": 1, "LE": 2}
VK = {"NONE": 0, "TO": 1, "FROM": 2, "TOFROM": 3, "ALLOC": 4, "FIRSTPRIVATE": 8}


def load_golden(path):
    g = json.load(open(path))
    blocks = [(SPACE[s], r, w) for (s, r, w) in g["blocks"]]
    edges = [(s, d, KIND[k]) for (s, d, k) in g["edges"]]
    cfg, pos = synth.from_edges(blocks, edges, g["n_vars"])
    if "scalar" in g:
        sc = np.zeros(cfg.wd, np.uint64)
        for v in g["scalar"]:
            sc[v >> 6] |= np.uint64(1 << (v & 63))
        cfg.scalar = sc
    return g, cfg, pos


def bits_of(a, v=0):
    return [int((int(x) >> v) & 1) for x in a[:, 0]]


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(GOLDEN, "P*.json"))), ids=os.path.basename)
def test_worked_example(path):
    g, cfg, pos = load_golden(path)
    check_expect(g, cfg, pos, oracle.solve(cfg), g["expect"])


PLACEMENTS = {"lazy": oracle.PLACEMENT_LAZY, "refine": oracle.PLACEMENT_REFINE}
VARIANT_CASES = [(p, v) for p in sorted(glob.glob(os.path.join(GOLDEN, "P*.json")))
                 for v in sorted(json.load(open(p)).get("variants", {}))]


@pytest.mark.parametrize("path,variant", VARIANT_CASES, ids=lambda x: os.path.basename(str(x)))
def test_worked_example_variant(path, variant):
    """The placement variants (pure lazy, loop-entry refinement) on the worked examples
    whose fixtures carry a hand derivation for them."""
    g, cfg, pos = load_golden(path)
    check_expect(g, cfg, pos, oracle.solve(cfg, placement=PLACEMENTS[variant]), g["variants"][variant])


def check_expect(g, cfg, pos, r, exp):
    for k in ("nu_h", "nu_d", "ave_h", "ave_d", "avf_h", "avf_d"):
        if k in exp:
            assert bits_of(r[k]) == exp[k], k
    if exp is g["expect"]:
        for k, want in g.get("expect_words", {}).items():
            assert [int(x) for x in r[k][:, 0]] == want, k
    # edge indices in the fixture are positions in its own edge list
    inv = {int(pos[i]): i for i in range(len(pos))}
    for k in ("ins_edge_h", "ins_edge_d"):
        got = sorted(inv[e] for e in range(cfg.n_edges) if int(r[k][e, 0]) & 1)
        assert got == sorted(exp[k]), k
    for k in ("ins_entry_h", "ins_entry_d"):
        got = [b for b in range(cfg.n_blocks) if int(r[k][b, 0]) & 1]
        assert got == sorted(exp[k]), k
    for k in ("after_dev", "before_dev"):
        if k in exp:
            assert r[k].tolist() == exp[k]
    assert [int(x) for x in r["var_kind"]] == [VK[x] for x in exp["var_kind"]]
    # labels: map(to) on an edge iff the source is not after a device block, ...
    preds = cfg.preds()
    for k, lab in exp.get("labels", {}).items():
        for where, name in lab.items():
            where = int(where)
            if k == "ins_edge_d":
                e = int(pos[where])
                src = next(p for p in range(cfg.n_blocks) if cfg.succ_ptr[p] <= e < cfg.succ_ptr[p + 1])
                got = "MAP_TO" if not r["after_dev"][src] else "UPDATE_TO"
            elif k == "ins_entry_d":
                got = "MAP_TO" if not any(r["after_dev"][p] for p, _ in preds[where]) else "UPDATE_TO"
            elif k == "ins_edge_h":
                e = int(pos[where])
                got = "MAP_FROM" if not r["before_dev"][int(cfg.succ_idx[e])] else "UPDATE_FROM"
            else:
                got = "MAP_FROM" if not r["before_dev"][where] else "UPDATE_FROM"
            assert got == name, (k, where)


def _mop_case(cfg):
    r = oracle.solve(cfg)
    wd = cfg.wd
    nu_h, nu_d = checkers.mop_nu(cfg)
    assert checkers.rows_int(r["nu_h"]) == nu_h
    assert checkers.rows_int(r["nu_d"]) == nu_d
    # AVE: gens are the eager copies, i.e. NU at block entry (from the MOP, not the oracle)
    ave_h, ave_d = checkers.mop_valid(cfg, [nu_h, nu_d], [{}, {}])
    assert checkers.rows_int(r["ave_h"]) == ave_h
    assert checkers.rows_int(r["ave_d"]) == ave_d
    # AVF: gens are the materialised copies
    ge = [checkers.rows_int(r["ins_entry_h"]), checkers.rows_int(r["ins_entry_d"])]
    gg = [dict(enumerate(checkers.rows_int(r["ins_edge_h"].reshape(-1, wd)))) if cfg.n_edges else {},
          dict(enumerate(checkers.rows_int(r["ins_edge_d"].reshape(-1, wd)))) if cfg.n_edges else {}]
    avf_h, avf_d = checkers.mop_valid(cfg, ge, gg)
    assert checkers.rows_int(r["avf_h"]) == avf_h
    assert checkers.rows_int(r["avf_d"]) == avf_d
    after, before = checkers.reach_labels(cfg)
    assert r["after_dev"].tolist() == after.tolist()
    assert r["before_dev"].tolist() == before.tolist()
    assert checkers.check_invariants(cfg, r) == []


@pytest.mark.parametrize("seed", range(40))
def test_mop_random_dags(seed):
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    nb = int(rng.integers(3, 13))
    nv = int(rng.choice([1, 7, 63, 64, 65, 70]))
    cfg = synth.random_dag(seed, nb, nv, p_loop_entry=0.3 if seed % 2 else 0.0)
    if seed % 3 == 0:
        # non-default boundaries: some variables valid only on the device at entry,
        # some live on the device after exit
        m = synth.var_mask(nv)
        evd = np.array([int(x) for x in rng.integers(0, 1 << 62, size=cfg.wd)], dtype=np.uint64) & m
        cfg.entry_valid_d = evd
        cfg.entry_valid_h = (~evd | np.array([int(x) for x in rng.integers(0, 1 << 62, size=cfg.wd)], dtype=np.uint64)) & m
        cfg.exit_live_d = np.array([int(x) for x in rng.integers(0, 1 << 62, size=cfg.wd)], dtype=np.uint64) & m
    _mop_case(cfg)


@pytest.mark.parametrize("seed", range(12))
def test_mop_structured_acyclic(seed):
    cfg = synth.make_cfg(50_000 + seed, n_user=10, n_vars=66, max_loop_depth=0, device_frac=0.4,
                         p_read=0.3, p_write=0.2)
    _mop_case(cfg)


def test_special_case_all_host():
    """No device block and nothing live on the device after exit: the host
    copy is always valid, the device copy never, and no copy is placed; the
    host next use equals classic live-variable analysis."""
    for seed in range(6):
        cfg = synth.make_cfg(7_000 + seed, n_user=40, n_vars=90, max_loop_depth=3, device_frac=0.0)
        r = oracle.solve(cfg)
        m = synth.var_mask(cfg.n_vars)
        assert (r["ave_h"] == m).all() and (r["ave_d"] == 0).all()
        assert (r["avf_h"] == m).all() and (r["avf_d"] == 0).all()
        for k in ("ins_entry_h", "ins_entry_d", "ins_edge_h", "ins_edge_d"):
            assert not r[k].any()
        assert not r["nu_d"].any()
        # classic liveness by per-variable backward search for a use before a def
        V = checkers.View(cfg)
        for v in range(0, cfg.n_vars, 7):
            bit = 1 << v
            live = [False] * cfg.n_blocks
            for b in range(cfg.n_blocks):
                seen, stack, found = set(), [b], False
                while stack and not found:
                    x = stack.pop()
                    if x in seen:
                        continue
                    seen.add(x)
                    if V.use(0, x) & bit:
                        found = True
                    elif x != V.exit and not (V.W[x] & bit):
                        stack.extend(q for q, _ in V.succ[x])
                live[b] = found
            got = [bool((int(r["nu_h"][b, v >> 6]) >> (v & 63)) & 1) for b in range(cfg.n_blocks)]
            assert got == live


def test_special_case_nothing_used():
    """No variable is ever read and nothing is live after exit: no next use,
    no copy; validity only follows the writes."""
    cfg = synth.make_cfg(8_123, n_user=60, n_vars=40, max_loop_depth=3, device_frac=0.4, p_read=0.0)
    cfg.exit_live_h = np.zeros(cfg.wd, np.uint64)
    r = oracle.solve(cfg)
    assert not r["nu_h"].any() and not r["nu_d"].any()
    for k in ("ins_entry_h", "ins_entry_d", "ins_edge_h", "ins_edge_d"):
        assert not r[k].any()
    assert (r["var_kind"][(r["var_kind"] != 0)] == 4).all()


def _permute(cfg, perm):
    nv = cfg.n_vars

    def prow(a):
        a = a.reshape(-1, cfg.wd)
        bits = np.unpackbits(a.view(np.uint8).reshape(a.shape[0], -1), axis=1, bitorder="little")[:, :nv]
        out_bits = np.zeros((a.shape[0], cfg.wd * 64), dtype=np.uint8)
        out_bits[:, perm] = bits
        return np.packbits(out_bits, axis=1, bitorder="little").view(np.uint64).reshape(a.shape[0], cfg.wd)
    return prow


def test_bit_independence():
    """Bit v of every output depends only on bit v of the inputs."""
    cfg = synth.make_cfg(4242, n_user=80, n_vars=150, max_loop_depth=3, device_frac=0.3)
    rng = np.random.Generator(np.random.PCG64(9))
    perm = rng.permutation(cfg.n_vars)
    pr = _permute(cfg, perm)
    cfg2 = synth.CFG(n_blocks=cfg.n_blocks, n_vars=cfg.n_vars, succ_ptr=cfg.succ_ptr, succ_idx=cfg.succ_idx,
                     edge_kind=cfg.edge_kind, space=cfg.space, R=pr(cfg.R), W=pr(cfg.W))
    a, b = oracle.solve(cfg), oracle.solve(cfg2)
    for k in ("nu_h", "nu_d", "ave_h", "ave_d", "avf_h", "avf_d", "ins_entry_h", "ins_entry_d",
              "ins_edge_h", "ins_edge_d"):
        assert (pr(a[k]) == b[k]).all(), k
    vk = np.zeros(cfg.n_vars, np.uint8)
    vk[perm] = a["var_kind"]
    assert (vk == b["var_kind"]).all()


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("placement", [0, 1])
def test_placement_sound_on_random_paths(seed, placement):
    cfg = synth.c1(seed) if seed < 4 else synth.make_cfg(31_000 + seed, n_user=48, n_vars=70,
                                                          max_loop_depth=3, device_frac=0.4, irr_loop_frac=0.3)
    r = oracle.solve(cfg, placement=placement)
    assert checkers.check_invariants(cfg, r) == []
    errs, _ = checkers.simulate_paths(cfg, r, walks=60, seed=seed)
    assert errs == []


@pytest.mark.parametrize("seed", range(10))
def test_placement_sound_random_loop_entry_kinds(seed):
    """Random LOOP_ENTRY marks on an acyclic graph only restrict the delay;
    the placement must stay safe and complete."""
    cfg = synth.random_dag(500 + seed, 12, 40, p_loop_entry=0.4)
    r = oracle.solve(cfg)
    assert checkers.check_invariants(cfg, r) == []
    errs, _ = checkers.simulate_paths(cfg, r, walks=40, seed=seed)
    assert errs == []


def _p1():
    g, cfg, pos = load_golden(os.path.join(GOLDEN, "P1_listing1_kernel_in_loop.json"))
    return cfg


@pytest.mark.parametrize("mutate", ["entry_pred", "exit_succ", "entry_device", "exit_access",
                                    "bad_kind", "bad_idx", "ptr", "unreachable", "boundary_gap",
                                    "padding", "back_from_entry"])
def test_validation_rejects(mutate):
    cfg = _p1()
    if mutate == "entry_pred":
        cfg.succ_idx = cfg.succ_idx.copy(); cfg.succ_idx[3] = 0      # 3->0
    elif mutate == "exit_succ":
        cfg = synth.from_edges([(0, [], []), (0, [], []), (0, [], [])], [(0, 1, 0), (1, 2, 0), (2, 1, 0)], 1)[0]
    elif mutate == "entry_device":
        cfg.space = cfg.space.copy(); cfg.space[0] = 1
    elif mutate == "exit_access":
        cfg.R = cfg.R.copy(); cfg.R[4, 0] = 1
    elif mutate == "bad_kind":
        cfg.edge_kind = cfg.edge_kind.copy(); cfg.edge_kind[0] = 7
    elif mutate == "bad_idx":
        cfg.succ_idx = cfg.succ_idx.copy(); cfg.succ_idx[0] = 99
    elif mutate == "ptr":
        cfg.succ_ptr = cfg.succ_ptr.copy(); cfg.succ_ptr[2] = 9
    elif mutate == "unreachable":
        cfg = synth.from_edges([(0, [], []), (0, [], []), (0, [], []), (0, [], [])],
                               [(0, 1, 0), (1, 3, 0), (2, 3, 0)], 1)[0]
    elif mutate == "boundary_gap":
        cfg.entry_valid_h = np.zeros(1, np.uint64)
    elif mutate == "padding":
        cfg.R = cfg.R.copy(); cfg.R[1, 0] = 1 << 5
    elif mutate == "back_from_entry":
        cfg.edge_kind = cfg.edge_kind.copy(); cfg.edge_kind[0] = 1
    with pytest.raises(oracle.OracleError):
        oracle.solve(cfg)


def test_degenerate_shapes():
    # no variables at all
    cfg = synth.make_cfg(1, n_user=5, n_vars=0, max_loop_depth=1, device_frac=0.4)
    r = oracle.solve(cfg)
    assert r["nu_h"].shape == (cfg.n_blocks, 0)
    # ENTRY -> EXIT only
    cfg = synth.from_edges([(0, [], []), (0, [], [])], [(0, 1, 0)], 3)[0]
    r = oracle.solve(cfg)
    assert bits_of(r["nu_h"], 0) == [1, 1] and not r["ins_edge_h"].any()
    # exactly 64 variables (no padding word)
    cfg = synth.make_cfg(2, n_user=30, n_vars=64, max_loop_depth=2, device_frac=0.5)
    r = oracle.solve(cfg)
    assert checkers.check_invariants(cfg, r) == []
