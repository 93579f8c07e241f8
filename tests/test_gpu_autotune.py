"""The autotuner and the schedule per size bucket on a resident plan: after
ompd_plan_autotune (schedule of each size bucket, then ring size and
workgroups per CU) and after setting the schedules by hand (all walk, all
level, mixed), every output of a mixed batch equals the oracle's, bit for
bit, and the plan reports the choice."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

KEYS = ("nu_h", "nu_d", "ave_h", "ave_d", "avf_h", "avf_d", "ins_entry_h", "ins_entry_d",
        "ins_edge_h", "ins_edge_d", "var_kind", "after_dev", "before_dev")


def _print(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _mixed():
    cfgs = [synth.c1(i) for i in range(20)]
    cfgs += [synth.c3_item(i, n_user=nb, n_vars=nv) for i, (nb, nv) in
             enumerate([(100, 70), (300, 500), (900, 64), (2000, 200), (5000, 300), (8000, 1000)])]
    cfgs += [synth.make_cfg(4_400 + i, n_user=17_000, n_vars=300, max_loop_depth=6, device_frac=0.4,
                            irr_loop_frac=0.01, p_read=0.05, p_write=0.02) for i in range(1)]
    cfgs += [synth.permute_blocks(synth.c3_item(50), 11)[0]]
    return cfgs


def test_autotune_and_schedules_keep_results():
    import torch
    import paper_2406_13881_amd as ompd
    from concurrent.futures import ThreadPoolExecutor
    from paper_2406_13881_amd.resident import ResidentBatch
    ctx = ompd.Context(0)
    cfgs = _mixed()
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        refs = list(ex.map(oracle.solve, cfgs))
    rb = ResidentBatch(ctx, cfgs)
    stream = torch.cuda.current_stream().cuda_stream

    def check(tag):
        rb.run(stream)
        torch.cuda.synchronize()
        assert (rb.plan.status() == 0).all(), tag
        get = rb.fetch_all()
        for i, c in enumerate(cfgs):
            g = get(i)
            for k in KEYS:
                assert np.array_equal(np.asarray(g[k]), np.asarray(refs[i][k]).reshape(np.asarray(g[k]).shape)), \
                    "%s: CFG %d (%d blocks) output %s differs" % (tag, i, c.n_blocks, k)

    try:
        check("default")
        for sched in ([0] * 5, [1] * 5, [0, 1, 0, 1, 1], [-1] * 5):
            rb.plan.set_schedule(sched)
            d = json.loads(rb.plan.describe())
            _print("schedule %s: %d level CFGs, %d level tiles" % (sched, d["level_cfgs"], d["level_tiles"]))
            assert d["bucket_sched"] == sched
            if sched == [1] * 5:
                assert d["level_cfgs"] == len(cfgs)
            check("schedule %s" % sched)
        best = rb.plan.autotune(stream, trials=1)
        d = json.loads(rb.plan.describe())
        _print("autotune: %.3f ms, %s" % (best, d))
        assert all(s in (0, 1) for s in d["bucket_sched"])
        check("autotuned")
    finally:
        rb.close()
        ctx.close()
