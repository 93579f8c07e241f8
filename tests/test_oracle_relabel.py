"""Invariance of the oracle under block relabelling (order independence,
I2): the fixed points are properties of the graph, not of its numbering, so
solving a CFG whose block ids are shuffled (ENTRY and EXIT kept) must give
the original outputs carried through the same shuffle, edge outputs through
the edge map, and identical per-variable map kinds.  Also checks the
shuffling helper of the input generator, which the GPU tests use."""
import numpy as np
import pytest

import oracle
import synth

KEYS_BLOCK = ("nu_h", "nu_d", "ave_h", "ave_d", "avf_h", "avf_d", "ins_entry_h", "ins_entry_d",
              "after_dev", "before_dev")


def _cfgs():
    out = [synth.c1(i) for i in range(6)]
    out += [synth.random_dag(300 + i, 25, 70, p_loop_entry=0.3) for i in range(4)]
    out += [synth.make_cfg(8_800 + i, n_user=120, n_vars=90, max_loop_depth=5, device_frac=0.4,
                           irr_loop_frac=0.3) for i in range(4)]
    return out


@pytest.mark.parametrize("k", range(14))
def test_relabel_invariance(k):
    cfg = _cfgs()[k]
    pc, perm, emap = synth.permute_blocks(cfg, 1234 + k)
    assert sorted(perm.tolist()) == list(range(cfg.n_blocks))
    assert pc.entry == cfg.entry and pc.exit == cfg.exit
    a, b = oracle.solve(cfg), oracle.solve(pc)
    for key in KEYS_BLOCK:
        assert np.array_equal(b[key][perm], a[key]), key
    for key in ("ins_edge_h", "ins_edge_d"):
        assert np.array_equal(b[key][emap], a[key]), key
    assert np.array_equal(a["var_kind"], b["var_kind"])


def test_relabel_changes_the_order():
    cfg = synth.c1(0)
    pc, perm, _ = synth.permute_blocks(cfg, 7)
    assert (perm != np.arange(cfg.n_blocks)).sum() > cfg.n_blocks // 2
    # some forward (non-back) edge now goes from a higher id to a lower one
    sp, si, kd = pc.succ_ptr, pc.succ_idx, pc.edge_kind
    assert any(si[e] < b and kd[e] != 1 for b in range(pc.n_blocks) for e in range(sp[b], sp[b + 1]))
