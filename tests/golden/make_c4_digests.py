"""Writes c4_digests.json: SHA-256 digests of the interprocedural oracle's
full result on the 2,000-procedure whole-program configuration (synth.c4()).

Test infrastructure: calls only the oracle (oracle.program.ProgramOracle)
and the seeded input generator.  Per procedure, one digest over all of its
contexts (sorted by call string), each context contributing its four
boundary vectors and its 13 outputs; one digest over every procedure
summary; one over every call site's host-read demand; the sorted context
list.  The GPU test hashes the device result the same way (c4_digest.py).

Usage: python tests/golden/make_c4_digests.py   (takes tens of minutes)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, HERE)

import synth  # noqa: E402
from oracle.program import ProgramOracle  # noqa: E402
from c4_digest import digests  # noqa: E402


def main():
    t0 = time.time()
    prog = synth.c4()
    po = ProgramOracle(prog)
    S, bnd, results = po.analyze()
    gw = (prog.n_globals + 63) // 64
    demands = [po.demand.get(j) for j in range(len(prog.call_proc))]
    d = digests(prog, list(results.keys()), results, bnd, [S[p] for p in range(len(prog.procs))],
                [None if x is None else x[:gw] for x in demands])
    d["oracle_seconds"] = round(time.time() - t0, 1)
    d["oracle_solves"] = po.visits
    model = ""
    try:
        model = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
    except (OSError, IndexError):
        pass
    d["oracle_host"] = "%s, one thread" % model
    with open(os.path.join(HERE, "c4_digests.json"), "w") as f:
        json.dump(d, f, indent=0, sort_keys=True)
    print("contexts %d, %.0f s" % (d["n_contexts"], time.time() - t0))


if __name__ == "__main__":
    main()
