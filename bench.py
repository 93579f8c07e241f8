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
  single        the 16,384-block x 2,048-variable procedure on its own,
  serving       a stream of requests shaped like that procedure through the
                serving loop (submit / poll): capacity in saturated mode,
                then Poisson arrivals at 0.5, 0.8 and 1.0 x capacity with
                p50 / p99 of completion minus arrival time.
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


def fact_bytes(cfgs, with_ave=True):
    """Algorithmic bytes of one pass of the path: per fact (user block x
    variable) the R and W bits in and the next-use, final-validity,
    copy-before-block (and, when requested, eager-validity) bits out, one
    bit per space each; per (edge x variable) the two copy-on-edge bits; the
    successor CSR, edge kinds and block spaces; per variable its map kind
    and per block its two label facts.  That is the minimum the method moves
    once, with every iteration on chip (1.325 B per fact, 1.575 B with
    eager validity, plus the exact CSR and label bytes)."""
    bits_per_fact = 2 + 2 + 2 + 2 + (2 if with_ave else 0)
    tot = 0.0
    for c in cfgs:
        nb, ne, nv = c.n_blocks, c.n_edges, c.n_vars
        tot += (nb - 2) * nv * bits_per_fact / 8.0 + ne * nv * 2 / 8.0
        tot += 4 * (nb + 1) + 4 * ne + ne + nb          # successor CSR, edge kinds, spaces
        tot += nv + 2 * nb                              # map kinds, label facts
    return int(tot)


def cpu_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count() or 1, "cpu_model": model}


TUNED = os.path.join(ROOT, "paper_2406_13881_amd", "tuned.json")


def load_tuned():
    try:
        return json.load(open(TUNED))
    except (OSError, ValueError):
        return {}


def apply_tuned(plan, c):
    """Apply a stored autotuner choice: the schedule per size bucket, then the launch configuration."""
    if "bucket_sched" in c:
        plan.set_schedule(c["bucket_sched"])
    plan.configure(c["lds_bytes"], c["wg_per_cu"])


def save_tuned(d):
    with open(TUNED, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)


# What a serving request asks for: the placement and its labels.
SERVE_WANT = ("ins_entry_h", "ins_entry_d", "ins_edge_h", "ins_edge_d", "var_kind", "after_dev", "before_dev")


def serving(ctx, n_pool, n_cap, n_warm, n_meas, loads):
    """Capacity (requests/s with the queue kept full) and latency percentiles
    under Poisson arrivals, on C2-shaped requests drawn from a pool of
    distinct seeded CFGs."""
    import numpy as np
    import synth
    import paper_2406_13881_amd as ompd
    pool = [synth.c5_request(i) for i in range(n_pool)]

    def drive(arrivals_s):
        """Submit request k at arrivals_s[k] (None = as fast as admission allows);
        returns per-request (arrival_ns, done_ns)."""
        n = len(arrivals_s)
        t0 = time.monotonic_ns()
        arr_ns = [t0 + (0 if a is None else int(a * 1e9)) for a in arrivals_s]
        live, out = [], [None] * n
        i = 0
        while i < n or live:
            now = time.monotonic_ns()
            while i < n and arr_ns[i] <= now:
                r = ompd.submit(ctx, pool[i % n_pool], want=SERVE_WANT)
                if not r.admitted:
                    break                   # budget full: retry after completions (latency keeps counting)
                live.append((i, r))
                i += 1
            still = []
            for k, r in live:
                if r.poll():
                    out[k] = (arr_ns[k], r.done_ns)
                else:
                    still.append((k, r))
            live = still
            time.sleep(0.0002)
        return out

    burst = drive([None] * n_cap)
    t_first = min(a for a, _ in burst)
    cap = n_cap / ((max(d for _, d in burst) - t_first) * 1e-9)
    res = {"workload": "requests shaped like the 16,384-block x 2,048-variable procedure (pool of %d seeded "
                       "CFGs), placement and labels returned to host memory" % n_pool,
           "capacity_rps": round(cap, 2), "capacity_requests": n_cap, "warmup": n_warm, "measured": n_meas,
           "loads": []}
    log("serving capacity: %.1f requests/s over %d requests" % (cap, n_cap))
    for f in loads:
        lam = f * cap
        arrivals = list(synth.poisson_arrivals(lam, n_warm + n_meas, seed=int(1000 * f)))
        got = drive(arrivals)[n_warm:]
        lat = np.array([(d - a) * 1e-6 for a, d in got])
        row = {"load": f, "offered_rps": round(lam, 2), "p50_ms": round(float(np.percentile(lat, 50)), 3),
               "p99_ms": round(float(np.percentile(lat, 99)), 3), "mean_ms": round(float(lat.mean()), 3)}
        res["loads"].append(row)
        log("serving load %.1f: %s" % (f, row))
    return res


TRAFFIC = os.path.join(ROOT, "profiles", "hbm_traffic_c3_batch4096.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2406_13881_amd", "csrc", "ompd_kernels.hip")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    record (FETCH_SIZE and WRITE_SIZE, scaled by a copy of known size), or
    None when the kernel source has changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC))
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != sha or kernel not in rec.get("per_launch", {}):
        return None
    return rec["per_launch"][kernel]["total_bytes"]


def kernel_bytes(cfgs):
    """Algorithmic bytes of each kernel per launch over the batch: every array
    the kernel must read or write, once (bv = a block vector, ev = an edge
    vector, both in the stored 64-bit word layout).  Iteration traffic (state
    rows revisited by later sweeps) is not algorithmic."""
    # (the loop-entry refinement, ompd_k_live and ompd_k_post_live, is not requested here: no launch)
    out = dict.fromkeys(("ompd_k_prep", "ompd_k_nu", "ompd_k_ave", "ompd_k_post_ave", "ompd_k_mayp",
                         "ompd_k_post_mayp", "ompd_k_later", "ompd_k_post_later", "ompd_k_live",
                         "ompd_k_post_live", "ompd_k_avf", "ompd_k_post_avf", "ompd_k_varkind"), 0)
    for c in cfgs:
        wd = (c.n_vars + 63) // 64
        nb, ne = c.n_blocks, c.n_edges
        bv, ev = nb * wd * 8, ne * wd * 8
        out["ompd_k_prep"] += 4 * (nb + 1) + 5 * ne + nb + 4 * (nb + 1) + 8 * ne + 128 * nb   # + records, step entries
        out["ompd_k_nu"] += 2 * bv + 2 * bv                    # R, W in; next use H/D out
        out["ompd_k_ave"] += 3 * bv + 2 * bv + 2 * nb          # NU H/D, W in; validity after each block H/D, labels out
        out["ompd_k_post_ave"] += 4 * bv + 2 * bv + 4 * ev     # NU, validity after in; validity before, EAG, valid-after-edge out
        out["ompd_k_mayp"] += 2 * bv + 2 * ev + 2 * bv         # R, W, EAG in; pending H/D out
        out["ompd_k_post_mayp"] += 4 * ev + 2 * bv + ev        # EAG, valid-after-edge, pending in; both-valid out
        out["ompd_k_later"] += 2 * bv + 3 * ev + 2 * bv        # R, W, EAG, both in; delayed H/D out
        out["ompd_k_post_later"] += 3 * ev + 3 * bv + 2 * bv + 2 * ev   # EAG, both, delayed, R in; copies out
        out["ompd_k_avf"] += 3 * bv + 2 * ev + 2 * bv          # copies before blocks, W, copies on edges in; validity after out
        out["ompd_k_post_avf"] += 2 * bv + 2 * ev + 4 * bv + 2 * bv + 3 * wd * 8   # copies, validity after, R, W in; validity before, map masks out
        out["ompd_k_varkind"] += 3 * wd * 8 + c.n_vars         # map masks in; map kinds out
    # the per-tile kernel runs every phase and pass
    out["ompd_k_solve"] = sum(v for k, v in out.items() if k != "ompd_k_prep")
    return out


def cpu_baseline(cfgs, seconds, threads, c1=None, c2=None):
    """The oracle as it stands, one CFG per thread on every host core, on the
    first CFGs of the batch until `seconds` of wall time have been used; and,
    single-threaded, its time on the 64-block procedure (median of 50) and on
    the 16,384-block procedure (one solve)."""
    import numpy as np
    import oracle
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
    out = {"value": facts / dt, "unit": "facts/s", "cores": threads, "kind": "oracle",
           "sample": "first %d of %d CFGs of the batch, one per thread (%d facts, %.1f s wall)" % (
               n, len(cfgs), facts, dt)}
    out.update(cpu_info())
    if c1 is not None:
        ts = []
        for _ in range(50):
            t = time.perf_counter()
            oracle.solve(c1)
            ts.append(time.perf_counter() - t)
        out["c1_ms"] = round(1e3 * float(np.median(ts)), 4)
    if c2 is not None:
        t = time.perf_counter()
        oracle.solve(c2)
        out["c2_ms"] = round(1e3 * (time.perf_counter() - t), 1)
    return out


def c1_leg(out, p1, c1, stream):
    """The 64-block procedure alone: one plan, graph replays timed one by one."""
    import numpy as np
    import torch
    for _ in range(5):
        p1.run(stream)
    torch.cuda.synchronize()
    lat1 = []
    for _ in range(50):
        p1.run(stream)
        a, _b = p1.plan.last_ms()
        lat1.append(a)
    assert (p1.plan.status() == 0).all()
    out["c1"] = {"workload": "one CFG, 64 user blocks x 32 variables, loop depth <= 3, 30% device",
                 "ms": round(float(np.median(lat1)), 4), "p99_ms": round(float(np.percentile(lat1, 99)), 4),
                 "value": c1.facts / (np.median(lat1) * 1e-3), "unit": "facts/s"}
    log("c1: %.4f ms per solve (median of 50)" % np.median(lat1))


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
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-program", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES of device memory (a device-to-device copy of known size, "
                         "to calibrate the HBM byte counters of a profiler) and exit")
    ap.add_argument("--serve-requests", type=int, default=2000, help="measured requests per offered load")
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--progress", action="store_true",
                    help="synchronise and print a line after every timed step (for profiler runs)")
    ap.add_argument("--no-c1", action="store_true", help="skip the 64-block procedure leg")
    ap.add_argument("--no-kernel-times", action="store_true",
                    help="skip the separate pass that times every kernel with events")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.copy_calibration:
        n = args.copy_calibration // 8
        x = torch.ones(n, dtype=torch.int64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        log("copied %d bytes" % (8 * n))
        return
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
    # the synthetic CFGs carry no scalar marks: no firstprivate clause to write
    want = tuple(k for k in ompd.OUTPUTS if k != "fp_clause")
    rb = ResidentBatch(ctx, cfgs, want=want)
    stream = torch.cuda.current_stream().cuda_stream
    tuned = load_tuned()
    key = "batch%d" % len(cfgs)
    if args.autotune:
        t = time.perf_counter()
        best = rb.plan.autotune(stream, trials=2)
        d = json.loads(rb.plan.describe())
        tuned[key] = {k: d[k] for k in ("lds_bytes", "wg_per_cu", "bucket_sched")}
        tuned[key]["best_ms"] = best
        save_tuned(tuned)
        log("autotune: best %.3f ms in %.1f s -> %s" % (best, time.perf_counter() - t, rb.plan.describe()))
    elif key in tuned:
        apply_tuned(rb.plan, tuned[key])
        log("using the stored autotuner choice %s" % tuned[key])
    for _ in range(args.warmup):
        rb.run(stream)
        st = rb.plan.status()
        if (st != 0).any():
            raise SystemExit("solve reported errors for %d CFGs" % int((st != 0).sum()))
    torch.cuda.synchronize()
    plan_desc = json.loads(rb.plan.describe())
    if not plan_desc.get("graph_captured"):
        raise SystemExit("the solve was not captured into a HIP graph: %s" % plan_desc)
    # timed: K replays of the captured graphs (ingest, then every phase and pass), back to back
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for k in range(args.steps):
        rb.run(stream)
        if args.progress:
            torch.cuda.synchronize()
            log("timed step %d of %d done" % (k + 1, args.steps))
    e1.record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dev_ms = e0.elapsed_time(e1) / args.steps
    st = rb.plan.status()
    assert (st == 0).all()
    value = facts * args.steps / dt
    ms_step = 1e3 * dt / args.steps
    log("batched (graph replay): %.3f ms/step (device %.3f ms), %.3e facts/s" % (ms_step, dev_ms, value))
    # separately: every kernel timed with HIP events recorded after it on the launch stream
    # (direct launches, not the graph)
    kms = {}
    if not args.no_kernel_times:
        rb.plan.profile(True)
        per_kernel = []
        for k in range(3):
            rb.run(stream)
            rb.plan.last_ms()
            per_kernel.append(rb.plan.kernel_ms())
            log("kernel-timing step %d of 3 done" % (k + 1))
        rb.plan.profile(False)
        torch.cuda.synchronize()
        kms = {k: float(np.mean([d[k] for d in per_kernel])) for k in per_kernel[0]}
        log("kernel ms: " + ", ".join("%s %.3f" % (k, v) for k, v in kms.items()))
    path_bytes = fact_bytes(cfgs, with_ave="ave_h" in want)
    dom = max(kms, key=kms.get) if kms else None
    dom_ms = kms[dom] if kms else dev_ms
    achieved = path_bytes / (dom_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": measured_traffic(dom) if dom else None,
                "kernel": dom, "kernel_ms": round(dom_ms, 4),
                "algorithmic_bytes_per_launch": path_bytes,
                "bytes_rule": "1.575 B per fact (R, W in; next use, eager and final validity, copies before "
                              "blocks out; one bit per space) + 2 bits per edge x variable + exact CSR and "
                              "label bytes; every phase kernel processes every fact of the batch per launch",
                "kernels_ms": {k: round(v, 4) for k, v in kms.items()},
                "kernel_model_bytes": kernel_bytes(cfgs).get(dom) if dom else None,
                "path_achieved_gbs": round(path_bytes / (dev_ms * 1e-3) / 1e9, 3),
                "path_frac": round(path_bytes / (dev_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 6)}
    out = {"metric": METRIC, "value": value, "unit": "facts/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u64", "data": "synthetic (seeded structured CFGs)",
           "config": {"workload": "batch of %d CFGs: user blocks log-uniform [16,8192], variables "
                                  "log-uniform [32,4096], loop depth <= 3, 30%% device, read p=0.2, write p=0.1"
                                  % len(cfgs),
                      "facts": facts, "global_batch": len(cfgs), "parallelism": "single GPU",
                      "device_ms_per_step": round(dev_ms, 4), "plan": plan_desc},
           "roofline": roofline}
    rb.close()
    del rb
    torch.cuda.empty_cache()

    # the 64-block procedure alone: one plan, graph replays timed one by one
    c1 = synth.c1(0)
    p1 = ResidentBatch(ctx, [c1], want=want) if not args.no_c1 else None
    if p1 is not None:
        c1_leg(out, p1, c1, stream)
        p1.close()

    if not args.no_plain:
        # the same CFGs, one resident single-CFG plan each, solved back to back on one stream
        t = time.perf_counter()
        m = len(cfgs)
        plans = [ResidentBatch(ctx, [c], want=want) for c in cfgs[:m]]
        log("plain: built %d single-CFG plans in %.1f s" % (m, time.perf_counter() - t))
        def run_all(tag):
            # one stream, back to back; a synchronisation every 512 plans only to report progress
            for j, p in enumerate(plans):
                p.run(stream)
                if (j + 1) % 512 == 0:
                    torch.cuda.synchronize()
                    log("plain %s: %d of %d CFGs solved" % (tag, j + 1, m))
            torch.cuda.synchronize()
        run_all("warm-up")
        t0 = time.perf_counter()
        run_all("timed")
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
        if args.autotune:
            sb.plan.autotune(stream, trials=1)
            d = json.loads(sb.plan.describe())
            tuned["single"] = {k: d[k] for k in ("lds_bytes", "wg_per_cu", "bucket_sched")}
            save_tuned(tuned)
        elif "single" in tuned:
            apply_tuned(sb.plan, tuned["single"])
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

    if not args.no_program:
        # whole-program analysis: summaries bottom-up, then every (procedure, call string <= 2)
        # context solved; synchronous, host arrays in and out, so the time includes the copies
        prog = synth.c4()
        t0 = time.perf_counter()
        got = ctx.analyze_program(prog)
        first = time.perf_counter() - t0
        t0 = time.perf_counter()
        got = ctx.analyze_program(prog)
        dt = time.perf_counter() - t0
        pf = sum(prog.procs[p].n_blocks * prog.procs[p].n_vars for (p, _) in got["contexts"])
        out["program"] = {"workload": "%d procedures (%d-%d blocks, %d globals + %d locals), %d call sites, "
                                      "contexts = call strings of length <= 2" % (
                                          len(prog.procs), synth.C4["blocks"][0], synth.C4["blocks"][1],
                                          prog.n_globals, synth.C4["n_locals"], len(prog.call_proc)),
                          "ms": 1e3 * dt, "first_ms": 1e3 * first, "contexts": len(got["contexts"]),
                          "solves": int(got["solves"]), "rounds": int(got["rounds"]), "facts": int(pf),
                          "value": pf / dt, "unit": "facts/s (host arrays in and out)"}
        try:
            rec = json.load(open(os.path.join(ROOT, "tests", "golden", "c4_digests.json")))
            out["program"]["oracle_s"] = rec.get("oracle_seconds")
            out["program"]["oracle_note"] = ("the interprocedural oracle (one thread) on the same program, timed "
                                             "when its digests were written (%s)" % rec.get("oracle_host", "?"))
        except (OSError, ValueError):
            pass
        log("program c4: %.1f ms (first %.1f ms), %d contexts, %d solves, %d rounds, %.3e facts/s" % (
            1e3 * dt, 1e3 * first, len(got["contexts"]), got["solves"], got["rounds"], pf / dt))
        del got

    if not args.no_serve:
        sctx = ompd.Context(0, budget_bytes=64 << 30)
        out["serving"] = serving(sctx, n_pool=32, n_cap=256, n_warm=args.serve_warmup, n_meas=args.serve_requests,
                                 loads=(0.5, 0.8, 1.0))
        sctx.close()

    if not args.no_cpu:
        threads = os.cpu_count() or 1
        out["cpu_baseline"] = cpu_baseline(cfgs, args.cpu_seconds, threads, c1=c1,
                                           c2=None if args.no_single else synth.c2(0))
        log("cpu baseline: %s" % out["cpu_baseline"])
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
