"""GPU parity of the interprocedural solve (ompd_analyze_program): every
context's outputs, every context boundary, every procedure summary and every
call site's host-read demand equal the oracle driver's, bit for bit, on
non-recursive, recursive and external-call programs and on a C4-shaped
program of 300 procedures.  At the full C4 size (2,000 procedures) the
oracle takes minutes, so the device result is compared with digests the
oracle wrote once (tests/golden/c4_digests.json), and checked with
whole-program random walks (no stale read or copy source)."""
import sys

import numpy as np
import pytest

import synth
from checkers import simulate_program
from oracle.program import ProgramOracle
from paper_2406_13881_amd import demand_vars

pytestmark = pytest.mark.gpu

KEYS = ("nu_h", "nu_d", "ave_h", "ave_d", "avf_h", "avf_d", "ins_entry_h", "ins_entry_d",
        "ins_edge_h", "ins_edge_d", "var_kind", "after_dev", "before_dev")


def _print(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2406_13881_amd as ompd
    c = ompd.Context(0)
    yield c
    c.close()


def compare(prog, got, tag):
    po = ProgramOracle(prog)
    S, ctxb, results = po.analyze()
    keys = got["contexts"]
    assert sorted(keys) == sorted(results.keys()), "%s: context sets differ" % tag
    for k, key in enumerate(keys):
        ref, mine = results[key], got["results"][k]
        for name in KEYS:
            a = np.asarray(mine[name])
            b = np.asarray(ref[name]).reshape(a.shape)
            assert np.array_equal(a, b), "%s: context %s output %s differs" % (tag, key, name)
        for i in range(4):
            assert np.array_equal(got["boundaries"][k][i], np.asarray(ctxb[key][i])), \
                "%s: context %s boundary %d differs" % (tag, key, i)
    for p in range(len(prog.procs)):
        w = S[p].shape[1]
        assert np.array_equal(got["summaries"][p][:, :w], S[p]), "%s: summary of procedure %d differs" % (tag, p)
        assert not got["summaries"][p][:, w:].any(), "%s: summary of procedure %d past its width" % (tag, p)
    for j in range(len(prog.call_proc)):
        caller = prog.procs[int(prog.call_proc[j])]
        want = sorted(v for v in range(caller.n_vars) if j in po.demand and (int(po.demand[j][v >> 6]) >> (v & 63)) & 1)
        assert demand_vars(prog, j, got["demands"][j]) == want, "%s: demand of call site %d differs" % (tag, j)
    return po


SMALL = dict(n_procs=6, n_globals=12, n_locals=5, blocks=(4, 14), mean_calls=2.0, max_calls=3, scc_procs=0,
             max_loop_depth=2, device_frac=0.4, p_read=0.25, p_write=0.15, threads=1)


@pytest.mark.parametrize("kind", ["plain", "recursive", "external"])
def test_program_small(ctx, kind):
    extra = {"plain": {}, "recursive": dict(scc_procs=4, scc_size=(2, 3), mean_calls=1.0),
             "external": dict(n_procs=8, scc_procs=5, scc_size=(2, 3), external_frac=0.3)}[kind]
    for seed in range(6):
        prm = dict(SMALL)
        prm.update(extra)
        prog = synth.program(31_000 + 100 * len(kind) + seed, **prm)
        _print("program %s seed %d: %d procs %d calls" % (kind, seed, len(prog.procs), len(prog.call_proc)))
        got = ctx.analyze_program(prog)
        compare(prog, got, "%s/%d" % (kind, seed))


@pytest.mark.parametrize("kind", ["device", "device_recursive", "all_device", "const_external"])
def test_program_device_calls_and_const_globals(ctx, kind):
    """Calls made inside kernels (the callee runs on the device) and const globals, against
    the oracle driver: every context, boundary, summary and demand."""
    extra = {"device": dict(device_call_frac=0.4, n_const=3),
             "device_recursive": dict(device_call_frac=0.4, scc_procs=4, scc_size=(2, 3), mean_calls=1.0),
             "all_device": dict(device_call_frac=1.0, n_const=2, external_frac=0.2),
             "const_external": dict(n_procs=8, n_const=4, external_frac=0.4, device_call_frac=0.2)}[kind]
    for seed in range(5):
        prm = dict(SMALL)
        prm.update(extra)
        prog = synth.program(32_000 + 100 * len(kind) + seed, **prm)
        _print("program %s seed %d: %d procs %d calls (%d in kernels)"
               % (kind, seed, len(prog.procs), len(prog.call_proc), int(np.sum(prog.call_space))
                  if prog.call_space is not None else 0))
        got = ctx.analyze_program(prog)
        compare(prog, got, "%s/%d" % (kind, seed))


@pytest.mark.parametrize("kind", ["plain", "recursive", "device_external", "multiword"])
def test_program_pointer_parameters(ctx, kind):
    """By-reference pointer parameters (host calls bind distinct locals; calls made inside
    kernels and external calls may bind anything), against the oracle driver: every context,
    boundary, summary and demand."""
    extra = {"plain": dict(max_params=3),
             "recursive": dict(max_params=3, scc_procs=4, scc_size=(2, 3), mean_calls=1.0),
             "device_external": dict(n_procs=8, max_params=3, max_ext_args=3, external_frac=0.3,
                                     device_call_frac=0.3, n_const=2, scc_procs=4, scc_size=(2, 3)),
             "multiword": dict(n_procs=8, n_globals=60, n_locals=30, max_params=12, max_ext_args=4,
                               external_frac=0.2, device_call_frac=0.2, scc_procs=2, scc_size=(2, 2))}[kind]
    for seed in range(5):
        prm = dict(SMALL)
        prm.update(extra)
        prog = synth.program(33_000 + 100 * len(kind) + seed, **prm)
        _print("program params %s seed %d: %d procs %d calls %d arguments"
               % (kind, seed, len(prog.procs), len(prog.call_proc), int(prog.arg_ptr[-1])))
        got = ctx.analyze_program(prog)
        compare(prog, got, "params-%s/%d" % (kind, seed))


def test_program_parameter_demands(ctx):
    """Programs whose merged call strings leave a parameter valid nowhere: the demand (a host
    read of the caller variable bound to it) and everything else equal the oracle's."""
    sys.path.insert(0, __import__("os").path.dirname(__file__))
    from test_oracle_program_params import MERGE_PARAM_SEEDS, merge_params_program
    for seed in MERGE_PARAM_SEEDS:
        prog = merge_params_program(27_000 + seed)
        got = ctx.analyze_program(prog)
        po = compare(prog, got, "merge-params/%d" % seed)
        assert demand_vars(prog, 3, got["demands"][3]) and po.demand


def test_program_rejects_aliasing_host_calls(ctx):
    import paper_2406_13881_amd as ompd
    prog = synth.program(33_999, **dict(SMALL, max_params=3))
    j = next(j for j in range(len(prog.call_proc)) if int(prog.n_params[int(prog.callee[j])]) >= 2)
    prog.arg_var = prog.arg_var.copy()
    prog.arg_var[int(prog.arg_ptr[j]) + 1] = prog.arg_var[int(prog.arg_ptr[j])]
    with pytest.raises(ompd.OmpdError):
        ctx.analyze_program(prog)


def test_program_c4_shape_parameters(ctx):
    prog = synth.c4(n_procs=120, max_params=4, max_ext_args=3, device_call_frac=0.1, external_frac=0.05)
    _print("c4-shaped with parameters: %d procs %d calls %d arguments"
           % (len(prog.procs), len(prog.call_proc), int(prog.arg_ptr[-1])))
    got = ctx.analyze_program(prog)
    compare(prog, got, "c4-120-params")


def test_program_c4_shape_device_calls(ctx):
    prog = synth.c4(n_procs=300, device_call_frac=0.25, n_const=32, external_frac=0.05)
    _print("c4-shaped with device calls: %d procs %d calls" % (len(prog.procs), len(prog.call_proc)))
    got = ctx.analyze_program(prog)
    compare(prog, got, "c4-300-device")


def test_program_multiword_globals(ctx):
    # globals spanning words, locals sharing the last global word
    prog = synth.program(4_711, n_procs=10, n_globals=100, n_locals=40, blocks=(6, 30), mean_calls=1.5,
                         max_calls=3, scc_procs=4, scc_size=(2, 2), external_frac=0.2, threads=1)
    got = ctx.analyze_program(prog)
    compare(prog, got, "multiword")


def test_program_c4_shape(ctx):
    prog = synth.c4(n_procs=300)
    _print("c4-shaped: %d procs %d calls %d blocks" % (len(prog.procs), len(prog.call_proc),
                                                        sum(c.n_blocks for c in prog.procs)))
    got = ctx.analyze_program(prog)
    _print("device: %d contexts, %d rounds, %d solves" % (len(got["contexts"]), got["rounds"], got["solves"]))
    compare(prog, got, "c4-300")


def test_program_c4_full_digests(ctx):
    """The full whole-program configuration (2,000 procedures, 20,370 contexts): every
    context's boundaries and 13 outputs, every summary and every demand equal the
    oracle's, compared through SHA-256 digests that tests/golden/make_c4_digests.py wrote
    from the oracle alone (one digest per procedure over its contexts).  Whole-program
    random walks then check that no read or copy source is stale."""
    import json
    import os
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from c4_digest import digests
    want = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c4_digests.json")))
    prog = synth.c4()
    _print("c4: %d procs %d calls" % (len(prog.procs), len(prog.call_proc)))
    got = ctx.analyze_program(prog)
    _print("device: %d contexts, %d rounds, %d solves" % (len(got["contexts"]), got["rounds"], got["solves"]))
    keys = list(got["contexts"])
    results = {key: got["results"][k] for k, key in enumerate(keys)}
    bnds = {key: got["boundaries"][k] for k, key in enumerate(keys)}
    mine = digests(prog, keys, results, bnds, [got["summaries"][p] for p in range(len(prog.procs))],
                   [got["demands"][j] for j in range(len(prog.call_proc))])
    assert mine["n_contexts"] == want["n_contexts"]
    assert mine["contexts"] == want["contexts"], "context sets differ"
    assert mine["summaries"] == want["summaries"], "procedure summaries differ"
    assert mine["demands"] == want["demands"], "host-read demands differ"
    bad = [p for p in want["procedures"] if mine["procedures"].get(p) != want["procedures"][p]]
    assert not bad, "contexts of %d procedures differ, first %s" % (len(bad), bad[:5])
    demands = {j: got["demands"][j] for j in range(len(prog.call_proc)) if got["demands"][j].any()}
    errs, cut = simulate_program(prog, None, results, demands, walks=200, seed=7, max_steps=6000)
    assert not errs, errs[:5]
    assert cut < 200
