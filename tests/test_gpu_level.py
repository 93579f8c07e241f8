"""GPU parity of the level schedule (OMPD_F_SCHED_LEVEL): the blocks of a
level solved in parallel, a level at a time, give every output of the
oracle, bit for bit, on the same families as the walk: worked examples,
config-1 CFGs (in order and with shuffled block ids), random DAGs with
loop-entry marks, structured CFGs with irreducible loops and ragged words,
non-default boundaries, eager placement, the full config-2 procedure, a
300-way fan-in and call blocks (whole programs)."""
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

KEYS = ("nu_h", "nu_d", "ave_h", "ave_d", "avf_h", "avf_d", "ins_entry_h", "ins_entry_d",
        "ins_edge_h", "ins_edge_d", "var_kind", "after_dev", "before_dev")


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


def _oracle_many(cfgs, placement=0):
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(lambda c: oracle.solve(c, placement=placement), cfgs))


def _check(ctx, cfgs, tag, flags=0, placement=0):
    import paper_2406_13881_amd as ompd
    got = ctx.analyze_batch(cfgs, flags=flags | ompd.F_SCHED_LEVEL)
    refs = _oracle_many(cfgs, placement)
    for i in range(len(cfgs)):
        assert_same(got[i], refs[i], "%s #%d" % (tag, i))
    return got


def test_level_small_families(ctx):
    import glob
    import json
    golden = os.path.join(os.path.dirname(__file__), "golden")
    SPACE = {"H": 0, "D": 1}
    KIND = {"N": 0, "BACK": 1, "LE": 2}
    cfgs = []
    for path in sorted(glob.glob(os.path.join(golden, "P*.json"))):
        g = json.load(open(path))
        cfgs.append(synth.from_edges([(SPACE[s], r, w) for (s, r, w) in g["blocks"]],
                                     [(s, d, KIND[k]) for (s, d, k) in g["edges"]], g["n_vars"])[0])
    cfgs.append(synth.from_edges([(0, [], []), (0, [], [])], [(0, 1, 0)], 3)[0])
    cfgs.append(synth.from_edges([(0, [], []), (1, [0, 65], [0]), (0, [0, 1], [65]), (0, [], [])],
                                 [(0, 1, 2), (1, 1, 1), (1, 2, 0), (2, 3, 0)], 70)[0])
    rng = np.random.Generator(np.random.PCG64(91))
    for j in range(40):
        nv = int(rng.choice([0, 1, 31, 64, 65, 130, 300]))
        cfgs.append(synth.random_dag(7000 + j, int(rng.integers(3, 40)), nv, p_loop_entry=0.3))
    _print("level: %d small CFGs" % len(cfgs))
    _check(ctx, cfgs, "small")


def _self_loops_everywhere(seed, n_user, n_vars):
    """ENTRY, a chain of user blocks each with a self loop (BACK), EXIT; random accesses, some
    blocks on the device."""
    rng = np.random.Generator(np.random.PCG64(seed))
    blocks = [(0, [], [])]
    for _ in range(n_user):
        blocks.append((int(rng.random() < 0.4), [v for v in range(n_vars) if rng.random() < 0.2],
                       [v for v in range(n_vars) if rng.random() < 0.1]))
    blocks.append((0, [], []))
    edges = [(b, b + 1, 0) for b in range(n_user + 1)] + [(b, b, 1) for b in range(1, n_user + 1)]
    return synth.from_edges(blocks, edges, n_vars)[0]


def test_level_recheck_lists_that_do_not_fit(ctx):
    """Every user block reads itself through a self loop, so both re-check lists hold every
    user block and together do not fit in the CFG's scratch words: the level kernels then
    confirm the fixed point with a sweep.  Outputs equal the oracle's (also on the walk, whose
    lists have room for every block)."""
    import paper_2406_13881_amd as ompd
    cfgs = [_self_loops_everywhere(9_500 + k, n, nv) for k, (n, nv) in enumerate(((3, 5), (40, 64), (300, 130)))]
    _check(ctx, cfgs, "self loops everywhere")
    got = ctx.analyze_batch(cfgs, flags=ompd.F_SCHED_WALK)
    for i, cfg in enumerate(cfgs):
        assert_same(got[i], oracle.solve(cfg), "self loops everywhere, walk %d" % i)


def test_level_config1_in_order_and_shuffled(ctx):
    cfgs = [synth.c1(i) for i in range(1000)]
    cfgs += [synth.permute_blocks(synth.c1(i), 70_000 + i)[0] for i in range(1000)]
    _print("level: %d config-1 CFGs" % len(cfgs))
    _check(ctx, cfgs, "c1")


def test_level_structured_irreducible_boundaries(ctx):
    cfgs = [synth.make_cfg(5_000 + j, n_user=50 + 37 * j, n_vars=17 + 23 * j, max_loop_depth=6, device_frac=0.4,
                           irr_loop_frac=0.2, p_read=0.15, p_write=0.08) for j in range(24)]
    rng = np.random.Generator(np.random.PCG64(5))
    for j in range(8):
        cfg = synth.make_cfg(9_100 + j, n_user=80, n_vars=150, max_loop_depth=3, device_frac=0.3)
        m = synth.var_mask(cfg.n_vars)
        r = lambda: np.array([int(x) for x in rng.integers(0, 1 << 63, size=cfg.wd, dtype=np.uint64)], np.uint64) & m
        evd = r()
        cfg.entry_valid_d = evd
        cfg.entry_valid_h = (~evd | r()) & m
        cfg.exit_live_h = r()
        cfg.exit_live_d = r()
        cfgs.append(cfg)
    cfgs += [synth.permute_blocks(synth.c3_item(i), 80_000 + i)[0] for i in (3, 17, 40)]
    _print("level: %d structured CFGs" % len(cfgs))
    _check(ctx, cfgs, "structured")


def test_level_eager_placement(ctx):
    import paper_2406_13881_amd as ompd
    cfgs = [synth.c1(i) for i in range(50)] + [synth.random_dag(40 + i, 20, 70, p_loop_entry=0.3) for i in range(20)]
    _check(ctx, cfgs, "eager", flags=ompd.F_PLACEMENT_EAGER, placement=1)


def test_level_config2_full(ctx):
    cfg = synth.c2(0)
    _print("level: config 2, %d blocks" % cfg.n_blocks)
    got = _check(ctx, [cfg], "c2")
    _print("level: config 2 sweeps %s" % (got[0].get("sweeps"),))


def test_level_wide_fan(ctx):
    rng = np.random.default_rng(2406)
    k, nv = 300, 100
    blocks = [(0, [], [])]
    for _ in range(k + 2):
        rd = sorted(set(rng.integers(0, nv, 6).tolist()))
        wr = sorted(set(rng.integers(0, nv, 3).tolist()))
        blocks.append((int(rng.random() < 0.4), rd, wr))
    blocks.append((0, [], []))
    hdr, join, ex = 1, k + 2, k + 3
    edges = [(0, hdr, 2)] + [(hdr, 2 + c, 0) for c in range(k)] + [(2 + c, join, 0) for c in range(k)]
    edges += [(join, hdr, 1), (join, ex, 0)]
    _check(ctx, [synth.from_edges(blocks, edges, nv)[0]], "fan")


def test_level_programs(ctx):
    """Call blocks (callee summaries, caps, demands, pointer-parameter bindings) under the
    level schedule: the whole interprocedural result equals the oracle's."""
    import paper_2406_13881_amd as ompd
    from oracle.program import ProgramOracle
    progs = [synth.program(31_500 + s, n_procs=8, n_globals=12, n_locals=5, blocks=(4, 14), mean_calls=1.5,
                           max_calls=3, scc_procs=5, scc_size=(2, 3), external_frac=0.3, max_loop_depth=2,
                           device_frac=0.4, p_read=0.25, p_write=0.15, threads=1) for s in range(4)]
    progs.append(synth.c4(n_procs=60))
    # pointer parameters bound at host calls, calls inside kernels and external calls with arguments
    progs += [synth.program(31_600 + s, n_procs=8, n_globals=12, n_locals=6, blocks=(4, 14), mean_calls=1.5,
                            max_calls=3, scc_procs=4, scc_size=(2, 3), external_frac=0.3, max_loop_depth=2,
                            device_frac=0.4, p_read=0.25, p_write=0.15, threads=1, max_params=3, max_ext_args=2,
                            device_call_frac=0.3) for s in range(3)]
    for t, prog in enumerate(progs):
        got = ctx.analyze_program(prog, flags=ompd.F_SCHED_LEVEL)
        po = ProgramOracle(prog)
        S, ctxb, results = po.analyze()
        assert sorted(got["contexts"]) == sorted(results.keys())
        for k, key in enumerate(got["contexts"]):
            assert_same(got["results"][k], results[key], "program %d context %s" % (t, key))
        _print("level: program %d, %d contexts equal" % (t, len(got["contexts"])))


def test_idle_launch_moves_cfgs_to_levels(ctx):
    """With no schedule named, a launch whose walk tiles would leave most CUs idle puts its
    CFGs on the level schedule, and a launch with enough walk tiles to fill the GPU keeps the
    walk; every output equals the oracle's either way."""
    import json
    from paper_2406_13881_amd.resident import ResidentBatch
    nbs, nvs = synth.c3_sizes()
    # (few enough words that one round of level tiles holds all three)
    mid = [int(i) for i in np.nonzero((nbs >= 400) & (nbs <= 3000) & (nvs <= 1280))[0][:3]]
    tiny = [int(i) for i in np.nonzero(nbs < 200)[0][:3]]
    cfgs = [synth.c3_item(i) for i in mid + tiny]
    rb = ResidentBatch(ctx, cfgs)
    try:
        d = json.loads(rb.plan.describe())
        _print("idle launch: blocks %s, plan %s" % ([c.n_blocks for c in cfgs], d))
        assert d["level_cfgs"] == len(cfgs), d
        rb.run()
        import torch
        torch.cuda.synchronize()
        assert (rb.plan.status() == 0).all()
        refs = _oracle_many(cfgs)
        for i in range(len(cfgs)):
            assert_same(rb.fetch(i), refs[i], "idle launch #%d" % i)
    finally:
        rb.close()
    many = [synth.c3_item(i) for i in range(200)]
    rb = ResidentBatch(ctx, many)
    try:
        d = json.loads(rb.plan.describe())
        assert d["level_cfgs"] == 0, d
    finally:
        rb.close()
