"""ORACLE — test infrastructure only.

Python binding of the plain C worklist solver in ``oracle.c`` (and, in
``program.py``, of the interprocedural driver).  Only ``tests/``, the smoke
check and the CPU-baseline leg of the benchmark may import this package; the
GPU library never does.  See ``oracle.c`` for the equations and the passages
of the paper they follow.

Parity status per function (pins live in ``tests/``):

* NU, AVE, AVF: pinned by brute-force meet-over-all-paths on tiny acyclic
  CFGs, by textbook special cases and by the worked examples of the paper's
  motivation listings.
* EAG, MAYP, LATER and the materialised copies: pinned by the worked
  examples (Listings 1-3, the backprop snippet) and by the safety,
  completeness and exclusivity invariants plus random-path simulation;
  beyond those, "parity unpinned" (the definition itself is the reference).
* labels: pinned by brute-force reachability and the worked examples.
* placement variants: the loop-entry refinement by a path search for the
  readers of each loop-entry copy's value (and worked examples P1, P3, P4,
  P9); pure lazy by the default placement on relabelled loop entries (and
  the same worked examples).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

SUM_ROWS = 16
(SUM_MAYR_H, SUM_MAYR_D, SUM_MAYW_H, SUM_MAYW_D, SUM_NU0_H, SUM_NU0_D, SUM_NU1_H, SUM_NU1_D,
 SUM_TH_00, SUM_TH_01, SUM_TH_10, SUM_TH_11, SUM_TD_00, SUM_TD_01, SUM_TD_10, SUM_TD_11) = range(16)

MAP_TO, MAP_FROM, MAP_ALLOC = 1, 2, 4

# placement variants (the ``placement`` argument of solve)
PLACEMENT_EAGER = 1     # every eager copy stays where it is made
PLACEMENT_LAZY = 2      # pure lazy: the delay also enters loops
PLACEMENT_REFINE = 4    # loop-entry refinement: drop loop-entry copies whose value is never read


class OracleError(RuntimeError):
    def __init__(self, rc: int):
        super().__init__("oracle_solve failed with %d" % rc)
        self.rc = rc


def build() -> str:
    """Compile the oracle with gcc (always recompiles)."""
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
    os.replace(tmp, _SO)
    return _SO


_lock = threading.Lock()
_handle = None


def _lib():
    global _handle
    with _lock:
        if _handle is None:
            if not os.path.exists(_SO):
                build()
            lib = ctypes.CDLL(_SO)
            vp = ctypes.c_void_p
            i32 = ctypes.c_int32
            lib.oracle_solve.restype = ctypes.c_int
            lib.oracle_solve.argtypes = [i32, i32, i32, i32, i32] + [vp] * 4 + [vp, vp] + [vp] * 4 + \
                [vp, vp, i32] + [vp] * 10 + [vp, vp, vp, vp]
            _handle = lib
        return _handle


def use_library(path: str):
    """Load the solver from another build of oracle.c (used by the mutation
    tests that plant mistakes in a copy); returns the previous handle."""
    global _handle
    with _lock:
        prev = _handle
        lib = ctypes.CDLL(path)
        vp = ctypes.c_void_p
        i32 = ctypes.c_int32
        lib.oracle_solve.restype = ctypes.c_int
        lib.oracle_solve.argtypes = [i32, i32, i32, i32, i32] + [vp] * 4 + [vp, vp] + [vp] * 4 + \
            [vp, vp, i32] + [vp] * 10 + [vp, vp, vp, vp]
        _handle = lib
        return prev


def restore_library(prev):
    global _handle
    with _lock:
        _handle = prev


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def solve(cfg, placement: int = 0, call: Optional[np.ndarray] = None,
          sums: Optional[np.ndarray] = None, boundary=None) -> Dict[str, np.ndarray]:
    """Solve one CFG (a ``synth.CFG``).  Raises OracleError on malformed input.

    ``call``: [n_blocks] int32 summary index per call block (-1 otherwise).
    ``sums``: [n_summaries, 16, words] uint64 callee summaries.
    ``boundary``: optional (ev_h, ev_d, lx_h, lx_d) overriding the CFG's own.
    """
    lib = _lib()
    nb, ne, nv, wd = cfg.n_blocks, cfg.n_edges, cfg.n_vars, cfg.wd
    evh, evd, lxh, lxd = cfg.boundary() if boundary is None else [np.ascontiguousarray(x, dtype=np.uint64) for x in boundary]
    sp = np.ascontiguousarray(cfg.succ_ptr, dtype=np.int32)
    si = np.ascontiguousarray(cfg.succ_idx, dtype=np.int32)
    kd = np.ascontiguousarray(cfg.edge_kind, dtype=np.uint8)
    spc = np.ascontiguousarray(cfg.space, dtype=np.uint8)
    R = np.ascontiguousarray(cfg.R, dtype=np.uint64).reshape(nb, wd)
    W = np.ascontiguousarray(cfg.W, dtype=np.uint64).reshape(nb, wd)
    if si.size == 0:
        si = np.zeros(1, dtype=np.int32)
        kd = np.zeros(1, dtype=np.uint8)
    if call is not None:
        call = np.ascontiguousarray(call, dtype=np.int32)
        sums = np.ascontiguousarray(sums, dtype=np.uint64)
    out = {
        "nu_h": np.zeros((nb, wd), np.uint64), "nu_d": np.zeros((nb, wd), np.uint64),
        "ave_h": np.zeros((nb, wd), np.uint64), "ave_d": np.zeros((nb, wd), np.uint64),
        "avf_h": np.zeros((nb, wd), np.uint64), "avf_d": np.zeros((nb, wd), np.uint64),
        "ins_entry_h": np.zeros((nb, wd), np.uint64), "ins_entry_d": np.zeros((nb, wd), np.uint64),
        "ins_edge_h": np.zeros((max(ne, 1), wd), np.uint64), "ins_edge_d": np.zeros((max(ne, 1), wd), np.uint64),
        "var_kind": np.zeros(max(nv, 1), np.uint8), "after_dev": np.zeros(nb, np.uint8),
        "before_dev": np.zeros(nb, np.uint8), "fp_clause": np.zeros((nb, wd), np.uint64),
        "visits": np.zeros(6, np.int64),
    }
    scalar = getattr(cfg, "scalar", None)
    if scalar is not None:
        scalar = np.ascontiguousarray(scalar, dtype=np.uint64).reshape(wd)
        if scalar.size == 0:
            scalar = None
    # keep buffers of at least one element so every pointer is valid
    evh_, evd_, lxh_, lxd_ = [x if x.size else np.zeros(1, np.uint64) for x in (evh, evd, lxh, lxd)]
    R_ = R if R.size else np.zeros((nb, 1), np.uint64)
    W_ = W if W.size else np.zeros((nb, 1), np.uint64)
    bufs = {k: (v if v.size else np.zeros(1, v.dtype)) for k, v in out.items()}
    rc = lib.oracle_solve(nb, ne, nv, int(cfg.entry), int(cfg.exit), _p(sp), _p(si), _p(kd), _p(spc),
                          _p(R_), _p(W_), _p(evh_), _p(evd_), _p(lxh_), _p(lxd_), _p(call), _p(sums),
                          int(placement), _p(scalar),
                          _p(bufs["nu_h"]), _p(bufs["nu_d"]), _p(bufs["ave_h"]), _p(bufs["ave_d"]),
                          _p(bufs["avf_h"]), _p(bufs["avf_d"]), _p(bufs["ins_entry_h"]), _p(bufs["ins_entry_d"]),
                          _p(bufs["ins_edge_h"]), _p(bufs["ins_edge_d"]), _p(bufs["var_kind"]),
                          _p(bufs["after_dev"]), _p(bufs["before_dev"]), _p(bufs["fp_clause"]),
                          _p(bufs["visits"]))
    if rc != 0:
        raise OracleError(rc)
    out["ins_edge_h"] = out["ins_edge_h"][:ne]
    out["ins_edge_d"] = out["ins_edge_d"][:ne]
    out["var_kind"] = out["var_kind"][:nv]
    return out
