"""The allocation-free batch entry point (ompd_analyze_batch_noalloc), called
through the C ABI on device buffers, gives exactly the outputs of
ompd_analyze_batch on the same inputs, on two calls in a row (the second
with a smaller batch, so the static scratch holds the first call's
contents), and refuses a batch larger than its scratch without touching
anything."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _print(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _outputs(rb):
    get = rb.fetch_all()
    return [get(i) for i in range(rb.n)]


def test_noalloc_matches_analyze_batch_twice():
    import torch
    import paper_2406_13881_amd as ompd
    from paper_2406_13881_amd.resident import ResidentBatch
    ctx = ompd.Context(0)
    try:
        first = [synth.c1(i) for i in range(30)] + [synth.c3_item(i) for i in range(6)] + [synth.c2(0)]
        second = [synth.c3_item(100 + i) for i in range(3)] + [synth.c1(500 + i) for i in range(4)]
        for tag, cfgs in (("first", first), ("second", second)):
            _print("noalloc %s call: %d CFGs, %d blocks" % (tag, len(cfgs), sum(c.n_blocks for c in cfgs)))
            a = ResidentBatch(ctx, cfgs)
            b = ResidentBatch(ctx, cfgs)
            try:
                s = torch.cuda.current_stream().cuda_stream
                sw_a = ompd.analyze_device(ctx, a.dcfgs, a.dres, stream=s, noalloc=True)
                sw_b = ompd.analyze_device(ctx, b.dcfgs, b.dres, stream=s, noalloc=False)
                torch.cuda.synchronize()
                oa, ob = _outputs(a), _outputs(b)
                for i in range(len(cfgs)):
                    for k in ompd.OUTPUTS:
                        assert np.array_equal(oa[i][k], ob[i][k]), "%s call, CFG %d, %s differs" % (tag, i, k)
                assert np.array_equal(sw_a, sw_b)
            finally:
                a.close()
                b.close()
        # a batch beyond the static scratch is refused (OMPD_E_NOMEM), and the entry point still works
        big = [synth.c2(i) for i in range(8)]
        c = ResidentBatch(ctx, big)
        try:
            with pytest.raises(ompd.OmpdError) as ei:
                ompd.analyze_device(ctx, c.dcfgs, c.dres, stream=torch.cuda.current_stream().cuda_stream,
                                    noalloc=True)
            assert ei.value.code == ompd.OMPD_E_NOMEM, str(ei.value)
            _print("refused: %s" % ei.value)
        finally:
            c.close()
        d = ResidentBatch(ctx, second)
        e = ResidentBatch(ctx, second)
        try:
            s = torch.cuda.current_stream().cuda_stream
            ompd.analyze_device(ctx, d.dcfgs, d.dres, stream=s, noalloc=True)
            ompd.analyze_device(ctx, e.dcfgs, e.dres, stream=s, noalloc=False)
            torch.cuda.synchronize()
            od, oe = _outputs(d), _outputs(e)
            for i in range(len(second)):
                for k in ompd.OUTPUTS:
                    assert np.array_equal(od[i][k], oe[i][k]), "after refusal, CFG %d, %s differs" % (i, k)
        finally:
            d.close()
            e.close()
    finally:
        ctx.close()
