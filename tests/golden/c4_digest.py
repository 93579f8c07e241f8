"""Digests of a whole-program result (contexts, boundaries, outputs,
summaries, demands) in one canonical byte layout, so that the oracle's
result and the device's can be compared without storing either.  Holds no
analysis arithmetic: it only serialises arrays."""
import hashlib

import numpy as np

KEYS = ("nu_h", "nu_d", "ave_h", "ave_d", "avf_h", "avf_d", "ins_entry_h", "ins_entry_d",
        "ins_edge_h", "ins_edge_d", "var_kind", "after_dev", "before_dev")
BYTE_KEYS = ("var_kind", "after_dev", "before_dev")


def _canon(name, a):
    dt = np.uint8 if name in BYTE_KEYS else np.uint64
    return np.ascontiguousarray(np.asarray(a).reshape(-1), dtype=dt).tobytes()


def context_bytes(key, result, boundary):
    h = hashlib.sha256()
    h.update(repr((int(key[0]), tuple(int(s) for s in key[1]))).encode())
    for i in range(4):
        h.update(_canon("b", boundary[i]))
    for k in KEYS:
        h.update(k.encode())
        h.update(_canon(k, result[k]))
    return h.digest()


def digests(prog, keys, results, boundaries, summaries, demands):
    """keys: context keys (proc, call string); results / boundaries: per key;
    summaries: per procedure [16][gw]; demands: per call site [gw] or None."""
    gw = (int(prog.n_globals) + 63) // 64
    by_proc = {}
    for key in sorted(keys, key=lambda k: (int(k[0]), tuple(int(s) for s in k[1]))):
        by_proc.setdefault(int(key[0]), hashlib.sha256()).update(context_bytes(key, results[key], boundaries[key]))
    hs = hashlib.sha256()
    for s in summaries:
        hs.update(_canon("s", s))
    hd = hashlib.sha256()
    for d in demands:
        hd.update(_canon("d", np.zeros(gw, np.uint64) if d is None else np.asarray(d)[:gw]))
    hk = hashlib.sha256()
    for key in sorted(keys, key=lambda k: (int(k[0]), tuple(int(s) for s in k[1]))):
        hk.update(repr((int(key[0]), tuple(int(s) for s in key[1]))).encode())
    return {"n_contexts": len(keys), "contexts": hk.hexdigest(), "summaries": hs.hexdigest(),
            "demands": hd.hexdigest(), "procedures": {str(p): h.hexdigest()[:32] for p, h in sorted(by_proc.items())}}
