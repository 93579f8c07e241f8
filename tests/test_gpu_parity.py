"""GPU parity: every output of the HIP path equals the oracle's, bit for bit.

The inputs are seeded synthetic CFGs (structured programs with loops,
irreducible entries, device kernels; unstructured random DAGs with
loop-entry marks; hand-built worked examples), at sizes that span many
levels, several slices and a ragged last word.  All results are integers,
so the tolerance is zero.
"""
import glob
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
KEYS = ("nu_h", "nu_d", "ave_h", "ave_d", "avf_h", "avf_d", "ins_entry_h", "ins_entry_d",
        "ins_edge_h", "ins_edge_d", "var_kind", "after_dev", "before_dev")


class _Walk:
    """The context, with the walk for every solve that names no schedule: a small launch would
    otherwise move CFGs of a few hundred blocks or more to the level schedule, which
    tests/test_gpu_level.py covers."""

    def __init__(self, c):
        self._c = c

    def __getattr__(self, name):
        return getattr(self._c, name)

    def _flags(self, flags):
        import paper_2406_13881_amd as ompd
        return flags if flags & (ompd.F_SCHED_WALK | ompd.F_SCHED_LEVEL) else flags | ompd.F_SCHED_WALK

    def analyze_batch(self, cfgs, flags=0, **kw):
        return self._c.analyze_batch(cfgs, flags=self._flags(flags), **kw)

    def analyze_cfg(self, cfg, flags=0, **kw):
        return self._c.analyze_cfg(cfg, flags=self._flags(flags), **kw)


@pytest.fixture(scope="module")
def ctx():
    import paper_2406_13881_amd as ompd
    c = ompd.Context(0)
    print("device:", c.device_info(), flush=True)
    yield _Walk(c)
    c.close()


def assert_same(cfg, got, ref, tag=""):
    for k in KEYS:
        g = np.asarray(got[k])
        r = np.asarray(ref[k]).reshape(g.shape)
        if not np.array_equal(g, r):
            bad = np.argwhere(g != r)
            raise AssertionError("%s %s differs at %d places, first %s: got %s want %s" % (
                tag, k, len(bad), bad[0].tolist(), g[tuple(bad[0])], r[tuple(bad[0])]))


def _print(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_worked_examples(ctx):
    SPACE = {"H": 0, "D": 1}
    KIND = {"N": 0, "BACK": 1, "LE": 2}
    cfgs = []
    for path in sorted(glob.glob(os.path.join(GOLDEN, "P*.json"))):
        g = json.load(open(path))
        cfg, _ = synth.from_edges([(SPACE[s], r, w) for (s, r, w) in g["blocks"]],
                                  [(s, d, KIND[k]) for (s, d, k) in g["edges"]], g["n_vars"])
        cfgs.append(cfg)
    _print("worked examples: %d CFGs" % len(cfgs))
    got = ctx.analyze_batch(cfgs)
    for i, cfg in enumerate(cfgs):
        assert_same(cfg, got[i], oracle.solve(cfg), "example %d" % i)


def _oracle_many(cfgs, placement=0):
    """Oracle results of many CFGs on every host core (the oracle is C; ctypes
    releases the interpreter lock while it runs)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(lambda c: oracle.solve(c, placement=placement), cfgs))


def test_config1_sweep(ctx):
    """Config 1 shape: 10,000 seeded CFGs of 64 blocks x 32 variables in one batch."""
    cfgs = [synth.c1(i) for i in range(10_000)]
    _print("c1 sweep: %d CFGs" % len(cfgs))
    got = ctx.analyze_batch(cfgs)
    refs = _oracle_many(cfgs)
    for i, cfg in enumerate(cfgs):
        assert_same(cfg, got[i], refs[i], "c1 #%d" % i)


def test_config1_permuted_ids(ctx):
    """The config-1 sweep with block ids shuffled (ENTRY and EXIT kept): forward edges now
    point backwards in id order, so the walk meets neighbours not yet visited in the sweep
    and steps with two far neighbours.  Every output equals the oracle's on the shuffled CFG."""
    cfgs = [synth.permute_blocks(synth.c1(i), 50_000 + i)[0] for i in range(2_000)]
    _print("c1 permuted: %d CFGs" % len(cfgs))
    got = ctx.analyze_batch(cfgs)
    refs = _oracle_many(cfgs)
    for i, cfg in enumerate(cfgs):
        assert_same(cfg, got[i], refs[i], "c1 permuted #%d" % i)


def test_config3_items_permuted_ids(ctx):
    """Twenty config-3 items (seeded picks of up to 2,048 blocks) with shuffled block ids,
    solved in one batch: every output equals the oracle's."""
    nbs, _ = synth.c3_sizes()
    small = [i for i in range(len(nbs)) if nbs[i] <= 2048]
    picks = sorted(int(i) for i in np.random.default_rng(4242).choice(small, 20, replace=False))
    cfgs = [synth.permute_blocks(synth.c3_item(i), 60_000 + i)[0] for i in picks]
    _print("c3 permuted: items %s, blocks %s" % (picks, [c.n_blocks for c in cfgs]))
    got = ctx.analyze_batch(cfgs)
    refs = _oracle_many(cfgs)
    for i, cfg in enumerate(cfgs):
        assert_same(cfg, got[i], refs[i], "c3 permuted item %d" % picks[i])


def test_permuted_ids_keep_the_sweep_count(ctx):
    """With shuffled block ids the ingest kernel walks in its own order (every edge other than
    BACK forward), so the sweeps per phase stay those of the source order instead of growing
    with the number of blocks; the outputs equal the oracle's.  The largest config-3 items and
    the config-2 procedure, on the walk."""
    import paper_2406_13881_amd as ompd
    nbs, _ = synth.c3_sizes()
    big = [int(i) for i in np.argsort(nbs)[-3:]]
    base = [synth.c3_item(i) for i in big] + [synth.c2()]
    perm = [synth.permute_blocks(c, 70_000 + k)[0] for k, c in enumerate(base)]
    _print("permuted, walk: blocks %s" % [c.n_blocks for c in base])
    a = ctx.analyze_batch(base, flags=ompd.F_SCHED_WALK)
    b = ctx.analyze_batch(perm, flags=ompd.F_SCHED_WALK)
    refs = _oracle_many(perm)
    for k, cfg in enumerate(perm):
        assert_same(cfg, b[k], refs[k], "permuted #%d" % k)
        sa, sb = np.asarray(a[k]["sweeps"][:5]), np.asarray(b[k]["sweeps"][:5])
        _print("sweeps in id order %s, shuffled %s" % (sa.tolist(), sb.tolist()))
        assert (sb <= 2 * sa + 2).all(), (sa.tolist(), sb.tolist())


@pytest.mark.parametrize("seed", range(4))
def test_random_dags_with_loop_entries(ctx, seed):
    rng = np.random.Generator(np.random.PCG64(77 + seed))
    cfgs = []
    for j in range(40):
        nb = int(rng.integers(2, 40)) if j else 2
        nv = int(rng.choice([0, 1, 31, 32, 33, 63, 64, 65, 130, 300]))
        if nb == 2:
            cfgs.append(synth.from_edges([(0, [], []), (0, [], [])], [(0, 1, 0)], nv)[0])
        else:
            cfgs.append(synth.random_dag(1000 * seed + j, nb, nv, p_loop_entry=0.3))
    _print("random dags seed %d" % seed)
    got = ctx.analyze_batch(cfgs)
    for i, cfg in enumerate(cfgs):
        assert_same(cfg, got[i], oracle.solve(cfg), "dag %d/%d" % (seed, i))


def test_acyclic_cfg_settles_in_one_sweep(ctx):
    """Without loops no block reads a neighbour it has not visited in the sweep, so the walk's
    re-check has nothing to evaluate and every phase ends after its first sweep (in id order and
    with the ids shuffled); the outputs equal the oracle's."""
    import paper_2406_13881_amd as ompd
    cfgs = [synth.random_dag(9_100 + j, 30 + 11 * j, 70 + 40 * j) for j in range(6)]
    cfgs += [synth.permute_blocks(c, 9_200 + j)[0] for j, c in enumerate(cfgs)]
    got = ctx.analyze_batch(cfgs, flags=ompd.F_SCHED_WALK)
    for i, cfg in enumerate(cfgs):
        assert_same(cfg, got[i], oracle.solve(cfg), "acyclic %d" % i)
        sw = np.asarray(got[i]["sweeps"][:5])
        assert (sw == 1).all(), (i, sw.tolist())


def _loops_with_self_edges(seed, n_vars):
    """ENTRY, a host loop whose header has two BACK edges (from a device block with a self loop
    and from a host latch), entered through a loop-entry edge, then a host block and EXIT; random
    accesses."""
    rng = np.random.Generator(np.random.PCG64(seed))
    def acc(p):
        return [v for v in range(n_vars) if rng.random() < p]
    blocks = [(0, [], []), (0, acc(0.3), acc(0.1)), (1, acc(0.3), acc(0.2)), (0, acc(0.2), acc(0.3)),
              (0, acc(0.4), []), (0, [], [])]
    edges = [(0, 1, 2), (1, 2, 0), (2, 2, 1), (2, 1, 1), (2, 3, 0), (3, 1, 1), (1, 4, 0), (4, 5, 0)]
    return synth.from_edges(blocks, edges, n_vars)[0]


@pytest.mark.parametrize("seed", range(3))
def test_recheck_with_self_loops_and_two_back_edges(ctx, seed):
    """Blocks that read a neighbour not yet visited in the sweep (a self loop, a header with two
    BACK edges) are re-evaluated after each sweep; the phase ends only when none of them would
    change.  Bit-exact against the oracle on the walk, in id order and shuffled, over 1-3 words."""
    import paper_2406_13881_amd as ompd
    cfgs = [_loops_with_self_edges(9_300 + 10 * seed + k, nv) for k, nv in enumerate((5, 64, 130))]
    cfgs += [synth.permute_blocks(c, 9_400 + k)[0] for k, c in enumerate(cfgs)]
    got = ctx.analyze_batch(cfgs, flags=ompd.F_SCHED_WALK)
    for i, cfg in enumerate(cfgs):
        assert_same(cfg, got[i], oracle.solve(cfg), "loops %d/%d" % (seed, i))
    _print("self loops seed %d: sweeps %s" % (seed, [g["sweeps"][:5].tolist() for g in got]))


def test_structured_irreducible_multiword(ctx):
    """Mid-size structured CFGs with irreducible loop entries, deep nesting
    and 1..9 words of variables (ragged last word), several tiles each."""
    cfgs = []
    for j in range(24):
        cfgs.append(synth.make_cfg(5_000 + j, n_user=50 + 37 * j, n_vars=17 + 23 * j, max_loop_depth=6,
                                   device_frac=0.4, irr_loop_frac=0.2, p_read=0.15, p_write=0.08))
    _print("structured irreducible: %d CFGs" % len(cfgs))
    got = ctx.analyze_batch(cfgs)
    for i, cfg in enumerate(cfgs):
        assert_same(cfg, got[i], oracle.solve(cfg), "struct %d" % i)


def test_boundaries(ctx):
    """Non-default entry validity and exit liveness (callee-style contexts)."""
    rng = np.random.Generator(np.random.PCG64(5))
    cfgs = []
    for j in range(12):
        cfg = synth.make_cfg(9_000 + j, n_user=80, n_vars=150, max_loop_depth=3, device_frac=0.3)
        m = synth.var_mask(cfg.n_vars)
        r = lambda: np.array([int(x) for x in rng.integers(0, 1 << 63, size=cfg.wd, dtype=np.uint64)], np.uint64) & m
        evd = r()
        cfg.entry_valid_d = evd
        cfg.entry_valid_h = (~evd | r()) & m
        cfg.exit_live_h = r()
        cfg.exit_live_d = r()
        cfgs.append(cfg)
    got = ctx.analyze_batch(cfgs)
    for i, cfg in enumerate(cfgs):
        assert_same(cfg, got[i], oracle.solve(cfg), "boundary %d" % i)


def test_eager_placement(ctx):
    import paper_2406_13881_amd as ompd
    cfgs = [synth.c1(i) for i in range(50)] + [synth.random_dag(40 + i, 20, 70, p_loop_entry=0.3) for i in range(20)]
    got = ctx.analyze_batch(cfgs, flags=ompd.F_PLACEMENT_EAGER)
    for i, cfg in enumerate(cfgs):
        assert_same(cfg, got[i], oracle.solve(cfg, placement=1), "eager %d" % i)


def test_config2_full(ctx):
    """Config 2 at full size (16,384 blocks x 2,048 variables), every output."""
    cfg = synth.c2(0)
    _print("c2 full: %d blocks %d vars" % (cfg.n_blocks, cfg.n_vars))
    got = ctx.analyze_cfg(cfg)
    assert_same(cfg, got, oracle.solve(cfg), "c2")


def test_malformed_is_rejected(ctx):
    import paper_2406_13881_amd as ompd
    good = synth.c1(0)
    bad = synth.c1(1)
    bad.succ_idx = bad.succ_idx.copy()
    bad.succ_idx[0] = 0                       # an edge into ENTRY
    with pytest.raises(ompd.OmpdError) as ei:
        ctx.analyze_batch([good, bad])
    assert ei.value.code == ompd.OMPD_E_INVAL
    unreach = synth.from_edges([(0, [], []), (0, [], []), (0, [], []), (0, [], [])],
                               [(0, 1, 0), (1, 3, 0), (2, 3, 0)], 5)[0]
    with pytest.raises(ompd.OmpdError) as ei:
        ctx.analyze_cfg(unreach)
    assert ei.value.code == ompd.OMPD_E_INVAL


def test_sweep_cap_reports_noconverge(ctx):
    """A cap one below the sweeps the slowest phase takes is reported as non-convergence; the
    default cap never triggers."""
    import paper_2406_13881_amd as ompd
    cfg = synth.c1(3)
    got = ctx.analyze_cfg(cfg)
    assert_same(cfg, got, oracle.solve(cfg), "no cap")
    most = int(np.max(got["sweeps"]))
    _print("c1(3) sweeps per phase %s" % got["sweeps"].tolist())
    assert most >= 2   # the CFG has loops that carry facts around
    with pytest.raises(ompd.OmpdError) as ei:
        ctx.analyze_cfg(cfg, flags=ompd.F_SWEEP_CAP(most - 1))
    assert ei.value.code == ompd.OMPD_E_NOCONVERGE
    got = ctx.analyze_cfg(cfg, flags=ompd.F_SWEEP_CAP(most))
    assert_same(cfg, got, oracle.solve(cfg), "cap at the sweeps taken")


def test_tile_kernel_matches_oracle(ctx):
    """The per-tile launch layout (one persistent kernel runs every phase
    and pass of a tile) gives the same results as the default one kernel
    per phase: both equal the oracle on a mixed batch with multi-tile
    CFGs."""
    import paper_2406_13881_amd as ompd
    cfgs = [synth.c1(i) for i in range(20)]
    cfgs += [synth.make_cfg(6_100 + j, n_user=60 + 50 * j, n_vars=40 + 1300 * j, max_loop_depth=4,
                            device_frac=0.4, irr_loop_frac=0.1) for j in range(4)]
    cfgs += [synth.random_dag(77 + j, 30, 90, p_loop_entry=0.3) for j in range(6)]
    refs = [oracle.solve(c) for c in cfgs]
    for flags in (0, ompd.F_TILE_KERNEL):
        got = ctx.analyze_batch(cfgs, flags=flags)
        for i, cfg in enumerate(cfgs):
            assert_same(cfg, got[i], refs[i], "flags=%d #%d" % (flags, i))


def test_ring_sizes_match_oracle(ctx):
    """Results do not depend on the ring of recently solved blocks: with 8 to
    64 ring slots (so that neighbours 9 to 64 steps back move between the
    ring and the far input, and the input lookahead exceeds the ring) every
    output equals the oracle, tiny CFGs (two and four blocks, a self-loop)
    included."""
    import paper_2406_13881_amd as ompd
    cfgs = [synth.c1(i) for i in range(10)]
    cfgs += [synth.make_cfg(6_300 + j, n_user=150 + 120 * j, n_vars=20 + 700 * j, max_loop_depth=4,
                            device_frac=0.4, irr_loop_frac=0.1) for j in range(4)]
    cfgs += [synth.random_dag(91 + j, 40, 120, p_loop_entry=0.3) for j in range(4)]
    tiny, _ = synth.from_edges([(0, [], []), (0, [], [])], [(0, 1, 0)], 3)
    loop, _ = synth.from_edges([(0, [], []), (1, [0, 65], [0]), (0, [0, 1], [65]), (0, [], [])],
                               [(0, 1, 2), (1, 1, 1), (1, 2, 0), (2, 3, 0)], 70)
    cfgs += [tiny, loop]
    refs = [oracle.solve(c) for c in cfgs]
    for rs in (8, 16, 32, 64):
        _print("ring slots %d: %d CFGs" % (rs, len(cfgs)))
        got = ctx.analyze_batch(cfgs, flags=ompd.F_RING_SLOTS(rs))
        for i, cfg in enumerate(cfgs):
            assert_same(cfg, got[i], refs[i], "ring %d #%d" % (rs, i))


def test_config3_batch_resident_full(ctx):
    """Config 3 at full size in the launch configuration the benchmark times:
    the 4,096-CFG batch resident in device memory under one plan, run twice
    (the second run overwrites the first run's outputs).  Every CFG reports
    success and every output of every one of the 4,096 CFGs equals the
    oracle's (the oracle runs on all host cores)."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from paper_2406_13881_amd.resident import ResidentBatch
    cfgs = synth.c3(4096, threads=8)
    nb = np.array([c.n_blocks for c in cfgs])
    _print("c3 batch: %d CFGs, %d blocks" % (len(cfgs), int(nb.sum())))
    rb = ResidentBatch(ctx, cfgs)
    try:
        stream = torch.cuda.current_stream().cuda_stream
        rb.run(stream)
        rb.run(stream)
        torch.cuda.synchronize()
        assert (rb.plan.status() == 0).all()
        host = rb.fetch_all()
        _print("c3 batch: outputs on the host, comparing")

        def check(i):
            assert_same(cfgs[i], host(i), oracle.solve(cfgs[i]), "c3 #%d" % i)
            return i

        order = np.argsort(-nb)          # largest first, so the pool ends on small ones
        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
            done = 0
            for _ in ex.map(check, [int(i) for i in order]):
                done += 1
                if done % 1024 == 0:
                    _print("c3 batch: %d of %d CFGs equal the oracle" % (done, len(cfgs)))
    finally:
        rb.close()


def test_word_counts_at_tile_boundaries(ctx):
    """Variable counts on both sides of the word and tile boundaries (a tile holds up to 15
    64-bit words): 63, 64 and 65 variables; 959, 960 and 961 (15 words, full or with one more
    word, which makes two tiles); 1,024; 1,919 to 1,921 (30 words and 31).  Every output of
    every CFG equals the oracle's, in one batch and each alone."""
    cfgs = [synth.make_cfg(7_100 + k, n_user=70 + 9 * k, n_vars=nv, max_loop_depth=3, device_frac=0.35,
                           irr_loop_frac=0.1)
            for k, nv in enumerate((63, 64, 65, 959, 960, 961, 1024, 1919, 1920, 1921))]
    refs = [oracle.solve(c) for c in cfgs]
    got = ctx.analyze_batch(cfgs)
    for i, cfg in enumerate(cfgs):
        assert_same(cfg, got[i], refs[i], "batch nv=%d" % cfg.n_vars)
    for cfg, ref in zip(cfgs, refs):
        assert_same(cfg, ctx.analyze_cfg(cfg), ref, "alone nv=%d" % cfg.n_vars)


def test_large_cfg_past_16_bit_block_ids(ctx):
    """One CFG of 131,074 blocks (block and edge ids past 16 bits, far neighbours up to the
    whole walk away) and 130 variables (three words, the last ragged): every output equals
    the oracle's."""
    cfg = synth.make_cfg(7_200, n_user=131_072, n_vars=130, max_loop_depth=6, device_frac=0.4,
                         irr_loop_frac=0.01)
    _print("large: %d blocks %d edges %d vars" % (cfg.n_blocks, len(cfg.succ_idx), cfg.n_vars))
    assert_same(cfg, ctx.analyze_cfg(cfg), oracle.solve(cfg), "large")


def test_wide_fan_in_and_fan_out(ctx):
    """A loop whose header branches to 300 cases that all join again (300 successors of one
    block, 300 predecessors of another: neighbours past the first two, in the ring and far
    beyond it), with random accesses on host and device blocks: every output equals the
    oracle's, for several ring sizes."""
    import paper_2406_13881_amd as ompd
    rng = np.random.default_rng(2406)
    k, nv = 300, 100
    blocks = [(0, [], [])]                                   # ENTRY
    for _ in range(k + 2):                                   # header, cases, join
        rd = sorted(set(rng.integers(0, nv, 6).tolist()))
        wr = sorted(set(rng.integers(0, nv, 3).tolist()))
        blocks.append((int(rng.random() < 0.4), rd, wr))
    blocks.append((0, [], []))                               # EXIT
    hdr, join, ex = 1, k + 2, k + 3
    edges = [(0, hdr, 2)] + [(hdr, 2 + c, 0) for c in range(k)] + [(2 + c, join, 0) for c in range(k)]
    edges += [(join, hdr, 1), (join, ex, 0)]
    cfg, _ = synth.from_edges(blocks, edges, nv)
    ref = oracle.solve(cfg)
    for rs in (8, 64):
        got = ctx.analyze_batch([cfg], flags=ompd.F_RING_SLOTS(rs))[0]
        assert_same(cfg, got, ref, "fan ring %d" % rs)


def test_wait_limit_gives_up_and_recovers(ctx):
    """With a wait bound of one nanosecond every wait of the solve kernels that does not succeed
    at once gives up: the kernels still end normally, every CFG of a resident plan reports
    OMPD_E_DEVICE, and the error names the phase, the tile and the counter that did not move.
    With the default bound restored, a new plan over the same CFGs solves them exactly."""
    import torch
    import paper_2406_13881_amd as ompd
    from paper_2406_13881_amd.resident import ResidentBatch
    cfgs = [synth.c1(i) for i in range(40)] + [synth.c3_item(i) for i in range(8)]
    ctx.set_wait_limit(1)
    try:
        with pytest.raises(ompd.OmpdError) as ei:
            ctx.analyze_batch(cfgs[:4])
        assert ei.value.code == ompd.OMPD_E_DEVICE
        assert "gave up" in str(ei.value), str(ei.value)
        _print("give-up message: %s" % ei.value)
        rb = ResidentBatch(ctx, cfgs, flags=ompd.F_SCHED_WALK)
        try:
            rb.run(torch.cuda.current_stream().cuda_stream)
            torch.cuda.synchronize()
            st = rb.plan.status()
            assert (st == ompd.OMPD_E_DEVICE).all(), st.tolist()
        finally:
            rb.close()
    finally:
        ctx.set_wait_limit(0)
    rb = ResidentBatch(ctx, cfgs, flags=ompd.F_SCHED_WALK)
    try:
        rb.run(torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert (rb.plan.status() == 0).all()
        for i, cfg in enumerate(cfgs):
            assert_same(cfg, rb.fetch(i), oracle.solve(cfg), "after the bound is restored #%d" % i)
    finally:
        rb.close()
