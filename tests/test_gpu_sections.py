"""GPU parity of array-section facts (section "Array Access Pattern Analysis"),
under the walk and the level schedule:
the section encoding solved on the device gives the oracle's directives and
map kinds on the same encoding, and, for small arrays, exactly the
element-level answer of the oracle (one variable per array element)."""
import os
import sys

import numpy as np
import pytest

import oracle

sys.path.insert(0, os.path.dirname(__file__))
from test_sections import GOLDEN, check_against_elements, element_cfg, load_section_golden, random_model  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2406_13881_amd as ompd
    c = ompd.Context(0)
    yield c
    c.close()


def _bnd(sec):
    return (sec.entry_valid_h, sec.entry_valid_d, sec.exit_live_h, sec.exit_live_d)


def _sched(name):
    import paper_2406_13881_amd as ompd
    return ompd.F_SCHED_WALK if name == "walk" else ompd.F_SCHED_LEVEL


@pytest.mark.parametrize("sched", ["walk", "level"])
def test_sections_match_the_oracle_and_the_elements(ctx, sched):
    models = [random_model(s) for s in range(40)]
    secs = [m.cfg() for m in models]
    got = ctx.analyze_batch(secs, flags=_sched(sched))
    for m, sec, g in zip(models, secs, got):
        ref = oracle.solve(sec, boundary=_bnd(sec))
        assert [d.clause() for d in m.directives(g)] == [d.clause() for d in m.directives(ref)]
        assert m.map_kinds(g) == m.map_kinds(ref)
        el, bnd, base = element_cfg(m)
        check_against_elements(m, g, oracle.solve(el, boundary=bnd), base)


@pytest.mark.parametrize("sched", ["walk", "level"])
def test_large_section_models(ctx, sched):
    """Hundreds of blocks, long arrays and many accesses (thousands of segments)."""
    models = [random_model(100 + s, n_user=400, n_arrays=12, max_len=100_000, n_acc=900) for s in range(6)]
    secs = [m.cfg() for m in models]
    print("segments per model: %s" % [s.n_vars for s in secs], flush=True)
    got = ctx.analyze_batch(secs, flags=_sched(sched))
    for m, sec, g in zip(models, secs, got):
        ref = oracle.solve(sec, boundary=_bnd(sec))
        for k in ("ins_entry_h", "ins_entry_d", "ins_edge_h", "ins_edge_d", "var_kind", "avf_h", "avf_d"):
            assert np.array_equal(np.asarray(g[k]), np.asarray(ref[k]).reshape(np.asarray(g[k]).shape)), k
        assert [d.clause() for d in m.directives(g)] == [d.clause() for d in m.directives(ref)]


def test_section_worked_example_on_the_device(ctx):
    for p in sorted(os.listdir(GOLDEN)):
        if not (p.startswith("S") and p.endswith(".json")):
            continue
        g, m = load_section_golden(os.path.join(GOLDEN, p))
        r = ctx.analyze_cfg(m.cfg())
        assert [d.clause() for d in m.directives(r)] == g["expect"]["clauses"]
