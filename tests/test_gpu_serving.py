"""GPU serving (continuous batching): every request's result is bit-identical
whether solved alone or mixed into a stream of concurrent requests, and the
device-memory budget gates admission (OMPD_E_BUSY) without losing work."""
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

KEYS = ("nu_h", "nu_d", "ave_h", "ave_d", "avf_h", "avf_d", "ins_entry_h", "ins_entry_d",
        "ins_edge_h", "ins_edge_d", "var_kind", "after_dev", "before_dev")


def same(a, b, tag):
    for k in KEYS:
        x = np.asarray(a[k])
        y = np.asarray(b[k]).reshape(x.shape)
        assert np.array_equal(x, y), "%s: %s differs" % (tag, k)


def mixed_requests():
    cfgs = [synth.c1(i) for i in range(20)]
    cfgs += [synth.c3_item(i) for i in range(12)]
    cfgs += [synth.random_dag(900 + i, 25, 130, p_loop_entry=0.3) for i in range(8)]
    cfgs += [synth.make_cfg(77_000 + i, n_user=3000, n_vars=700, max_loop_depth=5, device_frac=0.4,
                            irr_loop_frac=0.05, p_read=0.08, p_write=0.03) for i in range(3)]
    return cfgs


def c5_requests():
    """Config-5 requests: config-2-shaped CFGs (16,384 blocks x 2,048 variables)."""
    return [synth.c5_request(i) for i in range(8)]


def test_serving_mix_matches_alone_and_oracle():
    import paper_2406_13881_amd as ompd
    ctx = ompd.Context(0, budget_bytes=8 << 30)
    small = mixed_requests()
    big = c5_requests()
    # the config-5 requests arrive interleaved with the others
    cfgs = []
    for i, c in enumerate(small):
        cfgs.append(c)
        if i % 5 == 2 and big:
            cfgs.append(big.pop(0))
    cfgs += big
    print("serving mix: %d requests (%d config-5)" % (len(cfgs), sum(c.n_blocks > 16_000 for c in cfgs)), flush=True)
    reqs = []
    for i, c in enumerate(cfgs):
        r = ompd.submit(ctx, c)
        assert r.admitted
        reqs.append(r)
        if i % 7 == 3:
            time.sleep(0.002)          # let some requests start before the next ones arrive
    for r in reqs:
        r.wait(120.0)
    print("serving mix: all requests done", flush=True)
    from concurrent.futures import ThreadPoolExecutor
    import os
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        refs = list(ex.map(oracle.solve, cfgs))
    alone = ctx.analyze_batch(cfgs[:6])
    for i, (c, r) in enumerate(zip(cfgs, reqs)):
        same(r.out, refs[i], "request %d vs oracle" % i)
        if i < 6:
            same(r.out, alone[i], "request %d vs alone" % i)
        if c.n_blocks > 16_000:
            same(r.out, ctx.analyze_cfg(c), "config-5 request %d vs alone" % i)
    st = ompd.serving_stats(ctx)
    assert st["completed"] == len(cfgs) and st["in_flight"] == 0 and st["bytes_in_use"] == 0
    ctx.close()


def test_serving_budget_admission():
    import paper_2406_13881_amd as ompd
    ctx = ompd.Context(0, budget_bytes=5 << 20)       # 5 MiB: two or three of these requests fit at once
    cfgs = [synth.make_cfg(123_000 + i, n_user=1500, n_vars=512, max_loop_depth=3, device_frac=0.3)
            for i in range(10)]
    todo = list(range(len(cfgs)))
    live = {}
    busy = 0
    t0 = time.time()
    while (todo or live) and time.time() - t0 < 120:
        while todo:
            r = ompd.submit(ctx, cfgs[todo[0]])
            if not r.admitted:
                busy += 1
                break
            live[todo.pop(0)] = r
        for i in list(live):
            if live[i].poll():
                same(live[i].out, oracle.solve(cfgs[i]), "budgeted %d" % i)
                del live[i]
        time.sleep(0.001)
    assert not todo and not live
    assert busy > 0, "the budget never pushed back"
    ctx.close()


def test_serving_rejects_malformed_and_unknown_ticket():
    import paper_2406_13881_amd as ompd
    ctx = ompd.Context(0, budget_bytes=256 << 20)
    bad = synth.c1(0)
    bad.succ_idx = bad.succ_idx.copy()
    bad.succ_idx[0] = 0
    r = ompd.submit(ctx, bad)
    assert r.admitted
    with pytest.raises(ompd.OmpdError) as ei:
        r.wait(30.0)
    assert ei.value.code == ompd.OMPD_E_INVAL
    good = ompd.submit(ctx, synth.c1(1))
    same(good.wait(30.0), oracle.solve(synth.c1(1)), "after a bad request")
    d = __import__("ctypes").c_int(0)
    assert ompd.lib().ompd_poll(ctx.h, 987654321, __import__("ctypes").byref(d)) == ompd.OMPD_E_UNKNOWN_TICKET
    ctx.close()
