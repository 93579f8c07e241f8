"""Benchmark: block x variable facts per second to the fixed point.

Default workload (N = 1): the 4,096-procedure batch (user blocks
log-uniform in [16, 8192], variables log-uniform in [32, 4096], loop depth
<= 3, 30 % device blocks, read p = 0.2, write p = 0.1), resident in HBM,
solved by one resident plan per step (ingest kernel + one persistent solve
launch, replayed from a captured HIP graph; slice/LDS choice by the
autotuner).  A step is one complete pass of the whole path: ingest and
validation, next use, validity, pending copies, delayed placement and its
materialisation, validity after placement, labels and map kinds.

Printed JSON line: the metric of the benchmark plus
  roofline      HBM roofline of the dominant kernel (the persistent solve),
  cpu_baseline  the CPU oracle timed on a bounded sample of the same batch,
  plain         the same CFGs as one plain per-CFG solve each, back to back,
  single        the 16,384-block x 2,048-variable procedure on its own.
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "block×variable facts/sec to fixed point (batched vs plain); p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic_bytes(cfgs, want):
    """Bytes the method must move once per solve: the read/write bitmaps in,
    every requested output out (block vectors, edge vectors, per-variable
    kinds, per-block label facts), in the stored word layout."""
    tot = 0
    for c in cfgs:
        wd = (c.n_vars + 63) // 64
        bv = c.n_blocks * wd * 8
        ev = c.n_edges * wd * 8
        tot += 2 * bv                       # R, W
        for k in want:
            if k.startswith("ins_edge"):
                tot += ev
            elif k == "var_kind":
                tot += c.n_vars
            elif k in ("after_dev", "before_dev"):
                tot += c.n_blocks
            else:
                tot += bv
    return tot


TUNED = os.path.join(ROOT, "paper_2406_13881_amd", "tuned.json")


def load_tuned():
    try:
        return json.load(open(TUNED))
    except (OSError, ValueError):
        return {}


def save_tuned(d):
    with open(TUNED, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)


def cpu_baseline(cfgs, seconds, threads):
    """The oracle as it stands, one CFG per thread, on the first CFGs of the
    batch until `seconds` of wall time have been used."""
    import oracle
    done = []
    t0 = time.perf_counter()
    deadline = t0 + seconds

    def work(i):
        if time.perf_counter() > deadline:
            return None
        oracle.solve(cfgs[i])
        return cfgs[i].facts

    facts = 0
    n = 0
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for r in ex.map(work, range(len(cfgs))):
            if r is None:
                continue
            facts += r
            n += 1
    dt = time.perf_counter() - t0
    return {"value": facts / dt, "unit": "facts/s", "cores": threads, "kind": "oracle",
            "sample": "first %d of %d CFGs of the batch (%d facts, %.1f s wall)" % (n, len(cfgs), facts, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=4096, help="CFGs in the batch")
    ap.add_argument("--autotune", action="store_true",
                    help="re-run the autotuner and store its choice in paper_2406_13881_amd/tuned.json")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_2406_13881_amd as ompd
    from paper_2406_13881_amd.resident import ResidentBatch

    ctx = ompd.Context(0)
    info = ctx.device_info()
    log("device %s" % info)
    t = time.perf_counter()
    cfgs = synth.c3(args.n, threads=min(16, os.cpu_count() or 4))
    facts = sum(c.facts for c in cfgs)
    log("generated %d CFGs, %d facts in %.1f s" % (len(cfgs), facts, time.perf_counter() - t))
    want = ompd.OUTPUTS
    rb = ResidentBatch(ctx, cfgs, want=want)
    stream = torch.cuda.current_stream().cuda_stream
    tuned = load_tuned()
    key = "batch%d" % len(cfgs)
    if args.autotune:
        t = time.perf_counter()
        best = rb.plan.autotune(stream, trials=2)
        d = json.loads(rb.plan.describe())
        tuned[key] = {k: d[k] for k in ("lds_bytes", "wg_per_cu")}
        tuned[key]["best_ms"] = best
        save_tuned(tuned)
        log("autotune: best %.3f ms in %.1f s -> %s" % (best, time.perf_counter() - t, rb.plan.describe()))
    elif key in tuned:
        c = tuned[key]
        rb.plan.configure(c["lds_bytes"], c["wg_per_cu"])
        log("using the stored autotuner choice %s" % c)
    plan_desc = json.loads(rb.plan.describe())
    for _ in range(args.warmup):
        rb.run(stream)
        st = rb.plan.status()
        if (st != 0).any():
            raise SystemExit("solve reported errors for %d CFGs" % int((st != 0).sum()))
    torch.cuda.synchronize()
    solve_ms = []
    total_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rb.run(stream)
        a, b = rb.plan.last_ms()       # HIP events on the launch stream (synchronises)
        total_ms.append(a)
        solve_ms.append(b)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = rb.plan.status()
    assert (st == 0).all()
    value = facts * args.steps / dt
    ms_step = 1e3 * dt / args.steps
    log("batched: %.3f ms/step (device %.3f ms, solve kernel %.3f ms), %.3e facts/s" % (
        ms_step, np.mean(total_ms), np.mean(solve_ms), value))
    alg = algorithmic_bytes(cfgs, want)
    achieved = alg / (np.mean(solve_ms) * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                "algorithmic_bytes_per_launch": alg, "kernel": "ompd_k_solve",
                "kernel_ms": round(float(np.mean(solve_ms)), 4)}
    out = {"metric": METRIC, "value": value, "unit": "facts/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u64", "data": "synthetic (seeded structured CFGs)",
           "config": {"workload": "batch of %d CFGs: user blocks log-uniform [16,8192], variables "
                                  "log-uniform [32,4096], loop depth <= 3, 30%% device, read p=0.2, write p=0.1"
                                  % len(cfgs),
                      "facts": facts, "global_batch": len(cfgs), "parallelism": "single GPU",
                      "plan": plan_desc},
           "roofline": roofline}
    rb.close()
    del rb
    torch.cuda.empty_cache()

    if not args.no_plain:
        # the same CFGs, one resident single-CFG plan each, solved back to back on one stream
        t = time.perf_counter()
        m = len(cfgs)
        plans = [ResidentBatch(ctx, [c], want=want) for c in cfgs[:m]]
        log("plain: built %d single-CFG plans in %.1f s" % (m, time.perf_counter() - t))
        for p in plans:
            p.run(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for p in plans:
            p.run(stream)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t0
        pf = sum(c.facts for c in cfgs[:m])
        out["plain"] = {"value": pf / dtp, "unit": "facts/s", "ms": 1e3 * dtp, "cfgs": m,
                        "batched_speedup": value / (pf / dtp)}
        log("plain: %.1f ms for %d CFGs, %.3e facts/s" % (1e3 * dtp, m, pf / dtp))
        for p in plans:
            p.close()
        del plans
        torch.cuda.empty_cache()

    if not args.no_single:
        c2 = synth.c2(0)
        sb = ResidentBatch(ctx, [c2], want=want)
        if "single" in tuned:
            c = tuned["single"]
            sb.plan.configure(c["lds_bytes"], c["wg_per_cu"])
        elif args.autotune:
            sb.plan.autotune(stream, trials=1)
            d = json.loads(sb.plan.describe())
            tuned["single"] = {k: d[k] for k in ("lds_bytes", "wg_per_cu")}
            save_tuned(tuned)
        for _ in range(2):
            sb.run(stream)
        torch.cuda.synchronize()
        lat = []
        for _ in range(5):
            sb.run(stream)
            a, b = sb.plan.last_ms()
            lat.append(a)
        assert (sb.plan.status() == 0).all()
        out["single"] = {"workload": "one CFG, 16,384 user blocks x 2,048 variables, loop depth <= 6, "
                                     "40% device, 1% irreducible loops", "ms": float(np.median(lat)),
                         "value": c2.facts / (np.median(lat) * 1e-3), "unit": "facts/s",
                         "plan": json.loads(sb.plan.describe())}
        log("single c2: %.3f ms, %.3e facts/s" % (np.median(lat), out["single"]["value"]))
        sb.close()

    if not args.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(cfgs, args.cpu_seconds, threads)
        log("cpu baseline: %s" % out["cpu_baseline"])
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
