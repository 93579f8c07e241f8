"""Summaries of rocprofv3 runs of the solve kernels (kernel-trace durations
and HBM traffic from the FETCH_SIZE / WRITE_SIZE counters).

    python -m paper_2406_13881_amd.rocprof_summary trace DB
    python -m paper_2406_13881_amd.rocprof_summary counters DB [DB ...]
    python -m paper_2406_13881_amd.rocprof_summary traffic --fetch DB --write DB \\
        --cal-fetch DB --cal-write DB --cal-bytes N --json OUT.json --workload TEXT

Each DB is the `*_results.db` SQLite file rocprofv3 (ROCm 7) writes.  The
counters are in KiB per counter instance; a dispatch's value is the sum over
its instances.  FETCH_SIZE and WRITE_SIZE are scaled by what they read for a
plain device-to-device copy of --cal-bytes bytes (the largest dispatch of
the calibration runs), so that the reported bytes are HBM bytes.  The JSON
record carries the sha256 of the kernel source it was measured on; the
benchmark reports it only while that source is unchanged.
"""
import argparse
import collections
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(HERE, "csrc", "ompd_kernels.hip")


def kernel_durations(db_path):
    """{kernel: (calls, average us)} from a kernel-trace run (the top_kernels view, microseconds)."""
    db = sqlite3.connect(db_path)
    out = {}
    for name, calls, _total, avg, _pct in db.execute("select * from top_kernels"):
        out[name] = (int(calls), float(avg))
    return out


def counter_per_dispatch(db_path, counter):
    """{kernel: (dispatches, average value per dispatch)} of one counter."""
    db = sqlite3.connect(db_path)
    rows = db.execute("select kernel_name, dispatch_id, value from counters_collection where counter_name = ?",
                      (counter,)).fetchall()
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    for name, did, v in rows:
        agg[name][did] += v
    return {k: (len(d), sum(d.values()) / len(d)) for k, d in agg.items()}


def counters(db_paths, prefix="ompd_k_"):
    """{kernel: {counter: average per dispatch}} over every counter of the given runs."""
    out = collections.defaultdict(dict)
    for path in db_paths:
        db = sqlite3.connect(path)
        names = [r[0] for r in db.execute("select distinct counter_name from counters_collection")]
        for c in names:
            for k, (_n, avg) in counter_per_dispatch(path, c).items():
                if k.startswith(prefix):
                    out[k.split("(")[0]][c] = avg
    return dict(out)


def traffic(fetch_db, write_db, cal_fetch_db, cal_write_db, cal_bytes, prefix="ompd_k_"):
    fetch = counter_per_dispatch(fetch_db, "FETCH_SIZE")
    write = counter_per_dispatch(write_db, "WRITE_SIZE")
    cf = max(v for _, v in counter_per_dispatch(cal_fetch_db, "FETCH_SIZE").values())
    cw = max(v for _, v in counter_per_dispatch(cal_write_db, "WRITE_SIZE").values())
    kib = cal_bytes / 1024.0
    ff, fw = kib / cf, kib / cw
    per = {}
    for k in sorted(set(fetch) | set(write)):
        if not k.startswith(prefix):
            continue
        r = fetch.get(k, (0, 0.0))[1] * ff * 1024.0
        w = write.get(k, (0, 0.0))[1] * fw * 1024.0
        per[k] = {"fetch_kib": round(fetch.get(k, (0, 0.0))[1], 1), "write_kib": round(write.get(k, (0, 0.0))[1], 1),
                  "dispatches": fetch.get(k, (0, 0))[0], "read_bytes": int(r), "written_bytes": int(w),
                  "total_bytes": int(r + w)}
    return {"fetch_factor": ff, "write_factor": fw, "cal_fetch_kib": cf, "cal_write_kib": cw, "per_launch": per}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    c = sub.add_parser("counters")
    c.add_argument("dbs", nargs="+")
    f = sub.add_parser("traffic")
    for a in ("--fetch", "--write", "--cal-fetch", "--cal-write", "--json", "--workload"):
        f.add_argument(a, required=True)
    f.add_argument("--cal-bytes", type=int, required=True)
    args = ap.parse_args(argv)
    if args.cmd == "trace":
        print("| kernel | calls | average ms |")
        print("|---|---|---|")
        for k, (n, avg) in sorted(kernel_durations(args.db).items(), key=lambda kv: -kv[1][1]):
            print("| %s | %d | %.3f |" % (k[:60], n, avg / 1e3))
        return 0
    if args.cmd == "counters":
        per = counters(args.dbs)
        cols = sorted({n for v in per.values() for n in v})
        print("| kernel | " + " | ".join(cols) + " |")
        print("|---|" + "---|" * len(cols))
        for k in sorted(per):
            print("| %s | " % k + " | ".join("%.4g" % per[k].get(n, float("nan")) for n in cols) + " |")
        return 0
    rec = traffic(args.fetch, args.write, args.cal_fetch, args.cal_write, args.cal_bytes)
    rec = dict({"workload": args.workload,
                "kernel_source_sha256": hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()}, **rec)
    with open(args.json, "w") as fh:
        json.dump(rec, fh, indent=1)
    print("calibration: a copy of %d bytes reads %.1f KiB (FETCH_SIZE) and writes %.1f KiB (WRITE_SIZE): "
          "factors %.4f and %.4f" % (args.cal_bytes, rec["cal_fetch_kib"], rec["cal_write_kib"],
                                    rec["fetch_factor"], rec["write_factor"]))
    print("| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | read GB | written GB | total GB |")
    print("|---|---|---|---|---|---|")
    for k, v in rec["per_launch"].items():
        print("| %s | %.0f | %.0f | %.2f | %.2f | %.2f |" % (k, v["fetch_kib"], v["write_kib"], v["read_bytes"] / 1e9,
                                                          v["written_bytes"] / 1e9, v["total_bytes"] / 1e9))
    return 0


if __name__ == "__main__":
    sys.exit(main())
