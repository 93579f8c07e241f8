"""GPU parity of the placement variants: the loop-entry refinement
(OMPD_F_PLACEMENT_REFINE: one more backward fixed point and a pass that drops
the copies left on loop-entry edges whose value no read uses) and pure lazy
(OMPD_F_PLACEMENT_LAZY: the delay ignores loop entries).  Every output equals
the oracle's with the same variant, bit for bit, under the walk and the level
schedule, with the per-tile kernel, in resident plans, and through serving;
the families are the worked examples, random DAGs with loop-entry marks,
structured CFGs with irreducible loops and marked scalars, config-1 CFGs,
config-3 items and the full config-2 procedure."""
import glob
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

KEYS = ("nu_h", "nu_d", "ave_h", "ave_d", "avf_h", "avf_d", "ins_entry_h", "ins_entry_d",
        "ins_edge_h", "ins_edge_d", "var_kind", "after_dev", "before_dev", "fp_clause")
VARIANTS = {"refine": ("F_PLACEMENT_REFINE", oracle.PLACEMENT_REFINE),
            "lazy": ("F_PLACEMENT_LAZY", oracle.PLACEMENT_LAZY)}


@pytest.fixture(scope="module")
def ctx():
    import paper_2406_13881_amd as ompd
    c = ompd.Context(0)
    yield c
    c.close()


def _print(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def assert_same(got, ref, tag):
    for k in KEYS:
        g = np.asarray(got[k])
        r = np.asarray(ref[k]).reshape(g.shape)
        if not np.array_equal(g, r):
            bad = np.argwhere(g != r)
            raise AssertionError("%s %s differs at %d places, first %s" % (tag, k, len(bad), bad[0].tolist()))


def _oracle_many(cfgs, placement):
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(lambda c: oracle.solve(c, placement=placement), cfgs))


def family():
    golden = os.path.join(os.path.dirname(__file__), "golden")
    sys.path.insert(0, os.path.dirname(__file__))
    from test_oracle_pins import load_golden
    cfgs = [load_golden(p)[1] for p in sorted(glob.glob(os.path.join(golden, "P*.json")))]
    rng = np.random.Generator(np.random.PCG64(4_242))
    for j in range(30):
        nv = int(rng.choice([1, 31, 64, 65, 130]))
        cfgs.append(synth.random_dag(6_100 + j, int(rng.integers(3, 40)), nv, p_loop_entry=0.4))
    for j in range(30):
        c = synth.make_cfg(6_300 + j, n_user=int(rng.integers(10, 600)), n_vars=int(rng.choice([5, 70, 200, 961])),
                           max_loop_depth=int(rng.integers(1, 5)), device_frac=0.4,
                           irr_loop_frac=0.2 if j % 3 == 0 else 0.0, p_read=0.2, p_write=0.1)
        if j % 2:
            synth.mark_scalars(c, 6_300 + j, frac=0.3, read_only_frac=0.6)
        if j % 4 == 1:
            m = synth.var_mask(c.n_vars)
            c.entry_valid_d = np.array([int(x) for x in rng.integers(0, 1 << 62, size=c.wd)], dtype=np.uint64) & m
            c.entry_valid_h = m.copy()
            c.exit_live_d = np.array([int(x) for x in rng.integers(0, 1 << 62, size=c.wd)], dtype=np.uint64) & m
        cfgs.append(c)
    return cfgs


@pytest.mark.parametrize("variant", sorted(VARIANTS))
@pytest.mark.parametrize("sched", ["walk", "level", "tile"])
def test_variant_families(ctx, variant, sched):
    import paper_2406_13881_amd as ompd
    cfgs = family()
    flag, pl = VARIANTS[variant]
    flags = getattr(ompd, flag) | {"walk": ompd.F_SCHED_WALK, "level": ompd.F_SCHED_LEVEL,
                                   "tile": ompd.F_SCHED_WALK | ompd.F_TILE_KERNEL}[sched]
    _print("%s / %s: %d CFGs" % (variant, sched, len(cfgs)))
    got = ctx.analyze_batch(cfgs, flags=flags)
    refs = _oracle_many(cfgs, pl)
    for i in range(len(cfgs)):
        assert_same(got[i], refs[i], "%s/%s #%d" % (variant, sched, i))


def test_refinement_changes_something(ctx):
    """The family exercises the refinement: some loop-entry copies are dropped on the device."""
    import paper_2406_13881_amd as ompd
    cfgs = family()
    a = ctx.analyze_batch(cfgs)
    b = ctx.analyze_batch(cfgs, flags=ompd.F_PLACEMENT_REFINE)
    n = sum(int(np.count_nonzero(x["ins_edge_h"] != y["ins_edge_h"]) + np.count_nonzero(x["ins_edge_d"] != y["ins_edge_d"]))
            for x, y in zip(a, b))
    assert n > 0


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_variant_config1(ctx, variant):
    import paper_2406_13881_amd as ompd
    flag, pl = VARIANTS[variant]
    cfgs = [synth.c1(i) for i in range(2_000)]
    got = ctx.analyze_batch(cfgs, flags=getattr(ompd, flag))
    refs = _oracle_many(cfgs, pl)
    for i in range(len(cfgs)):
        assert_same(got[i], refs[i], "config-1 %s #%d" % (variant, i))


def test_refine_config3_resident(ctx):
    import paper_2406_13881_amd as ompd
    from paper_2406_13881_amd.resident import ResidentBatch
    cfgs = [synth.c3_item(i) for i in range(128)]
    rb = ResidentBatch(ctx, cfgs, flags=ompd.F_PLACEMENT_REFINE)
    rb.run()
    get = rb.fetch_all()
    refs = _oracle_many(cfgs, oracle.PLACEMENT_REFINE)
    for i in range(len(cfgs)):
        assert_same(get(i), refs[i], "config-3 refine %d" % i)
    rb.close()


@pytest.mark.parametrize("variant", sorted(VARIANTS))
@pytest.mark.parametrize("sched", ["walk", "level"])
def test_variant_config2(ctx, variant, sched):
    import paper_2406_13881_amd as ompd
    flag, pl = VARIANTS[variant]
    cfg = synth.c2()
    flags = getattr(ompd, flag) | (ompd.F_SCHED_WALK if sched == "walk" else ompd.F_SCHED_LEVEL)
    _print("config-2 %s (%s)" % (variant, sched))
    got = ctx.analyze_cfg(cfg, flags=flags)
    assert_same(got, oracle.solve(cfg, placement=pl), "config-2 %s %s" % (variant, sched))


def test_variants_through_serving():
    import paper_2406_13881_amd as ompd
    c = ompd.Context(0, budget_bytes=2 << 30)
    cfgs = [synth.c1(i) for i in range(8)] + [synth.c3_item(i) for i in range(4)]
    work = [(g, v) for g in cfgs for v in sorted(VARIANTS)]
    reqs = [ompd.submit(c, g, flags=getattr(ompd, VARIANTS[v][0])) for g, v in work]
    for r in reqs:
        assert r.admitted
        r.wait(120.0)
    for (g, v), r in zip(work, reqs):
        assert_same(r.out, oracle.solve(g, placement=VARIANTS[v][1]), "served %s" % v)
    c.close()
