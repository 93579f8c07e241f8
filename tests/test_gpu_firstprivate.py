"""GPU parity of the firstprivate reading (section "Data-Flow Analysis", the
firstprivate paragraph; Table II): with scalar marks, every output of the
device solve, the firstprivate clauses included, equals the oracle's bit for
bit, under both schedules (walk and level), through the host batch entry
point, a resident plan over device pointers, and the serving queue.  The
families: the worked example P12, random DAGs with loop-entry marks and ragged
words, structured CFGs with irreducible loops, config-3 items and the full
config-2 procedure."""
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

KEYS = ("nu_h", "nu_d", "ave_h", "ave_d", "avf_h", "avf_d", "ins_entry_h", "ins_entry_d",
        "ins_edge_h", "ins_edge_d", "var_kind", "after_dev", "before_dev", "fp_clause")


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


def _oracle_many(cfgs):
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(oracle.solve, cfgs))


def small_family():
    sys.path.insert(0, os.path.dirname(__file__))
    from test_oracle_pins import GOLDEN, load_golden
    cfgs = [load_golden(os.path.join(GOLDEN, "P12_firstprivate_scalar.json"))[1]]
    rng = np.random.Generator(np.random.PCG64(404))
    for j in range(40):
        nv = int(rng.choice([1, 31, 64, 65, 130, 300]))
        c = synth.random_dag(8_100 + j, int(rng.integers(3, 40)), nv, p_loop_entry=0.3)
        cfgs.append(synth.mark_scalars(c, 8_100 + j, frac=0.5, read_only_frac=0.7))
    for j in range(12):
        c = synth.make_cfg(8_300 + j, n_user=int(rng.integers(20, 400)), n_vars=int(rng.choice([70, 200, 513])),
                           max_loop_depth=4, device_frac=0.4, irr_loop_frac=0.2)
        cfgs.append(synth.mark_scalars(c, 8_300 + j, frac=0.3, read_only_frac=0.6))
    # a mark on every variable, and marks on nothing
    c = synth.random_dag(8_500, 30, 100, p_loop_entry=0.3)
    c.scalar = np.full(c.wd, ~np.uint64(0), np.uint64)
    cfgs.append(c)
    c = synth.random_dag(8_501, 30, 100, p_loop_entry=0.3)
    c.scalar = np.zeros(c.wd, np.uint64)
    cfgs.append(c)
    return cfgs


@pytest.mark.parametrize("sched", ["walk", "level"])
def test_firstprivate_small_families(ctx, sched):
    import paper_2406_13881_amd as ompd
    cfgs = small_family()
    flags = ompd.F_SCHED_WALK if sched == "walk" else ompd.F_SCHED_LEVEL
    _print("firstprivate %s: %d CFGs" % (sched, len(cfgs)))
    got = ctx.analyze_batch(cfgs, flags=flags)
    refs = _oracle_many(cfgs)
    assert refs[0]["fp_clause"].any(), "the worked example has a firstprivate clause"
    for i in range(len(cfgs)):
        assert_same(got[i], refs[i], "%s #%d" % (sched, i))
    one = ctx.analyze_cfg(cfgs[0], flags=flags)
    assert_same(one, refs[0], "%s P12 alone" % sched)


def test_firstprivate_config3_resident(ctx):
    """Config-3 items with marks, packed into a resident plan (device pointers); half the
    items carry no marks, so both kinds share a launch."""
    from paper_2406_13881_amd.resident import ResidentBatch
    cfgs = []
    for i in range(96):
        c = synth.c3_item(i)
        cfgs.append(synth.mark_scalars(c, 9_000 + i, frac=0.2, read_only_frac=0.6) if i % 2 == 0 else c)
    _print("firstprivate config-3: %d items" % len(cfgs))
    rb = ResidentBatch(ctx, cfgs)
    rb.run()
    get = rb.fetch_all()
    refs = _oracle_many(cfgs)
    n_fp = 0
    for i in range(len(cfgs)):
        assert_same(get(i), refs[i], "config-3 item %d" % i)
        n_fp += int(refs[i]["fp_clause"].any())
    assert n_fp > 0
    rb.close()


@pytest.mark.parametrize("sched", ["walk", "level"])
def test_firstprivate_config2(ctx, sched):
    import paper_2406_13881_amd as ompd
    cfg = synth.mark_scalars(synth.c2(), 9_500, frac=0.1, read_only_frac=0.6)
    flags = ompd.F_SCHED_WALK if sched == "walk" else ompd.F_SCHED_LEVEL
    _print("firstprivate config-2 (%s)" % sched)
    got = ctx.analyze_cfg(cfg, flags=flags)
    ref = oracle.solve(cfg)
    assert ref["fp_clause"].any()
    assert_same(got, ref, "config-2 %s" % sched)


def test_firstprivate_serving():
    import paper_2406_13881_amd as ompd
    c = ompd.Context(0, budget_bytes=2 << 30)
    cfgs = [synth.mark_scalars(synth.c1(i), 9_700 + i, frac=0.4, read_only_frac=0.7) for i in range(12)]
    cfgs += [synth.mark_scalars(synth.c3_item(i), 9_800 + i, frac=0.2, read_only_frac=0.6) for i in range(4)]
    reqs = [ompd.submit(c, g) for g in cfgs]
    for r in reqs:
        assert r.admitted
        r.wait(120.0)
    refs = _oracle_many(cfgs)
    for i, r in enumerate(reqs):
        assert_same(r.out, refs[i], "served %d" % i)
    c.close()
