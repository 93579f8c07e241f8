"""MI355X (gfx950) solver for the OMPDart data-flow problems — Python binding.

Thin ctypes binding of ``libompd.so`` (``include/ompd.h``): argument
marshalling only.  Every step of the solve runs in the library's HIP
kernels; there is no CPU fallback, and importing a function whose library is
not built raises ``OmpdNotBuilt``.

Entry points (same names as the C ABI): ``ctx_create``, ``analyze_cfg``,
``analyze_batch``, ``plan_create`` / ``plan_run`` / ``plan_status`` /
``plan_autotune`` / ``plan_last_ms`` / ``plan_describe``, ``submit`` /
``poll`` / ``wait``, ``analyze_program``.  CFG arguments are any objects
with the attributes of ``synth.CFG`` (numpy arrays), or ``DeviceCFG`` for
device pointers.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libompd.so")
_SOURCES = ["csrc/ompd_kernels.hip", "csrc/ompd_runtime.hip", "csrc/ompd_serving.hip", "csrc/ompd_program.hip"]

OMPD_OK = 0
OMPD_E_INVAL = -1
OMPD_E_NOMEM = -2
OMPD_E_DEVICE = -3
OMPD_E_NOCONVERGE = -4
OMPD_E_BUSY = -5
OMPD_E_UNKNOWN_TICKET = -6
OMPD_E_TIMEOUT = -7

F_DEVICE_PTRS = 1 << 0
F_PLACEMENT_EAGER = 1 << 1
F_TILE_KERNEL = 1 << 3
F_SCHED_LEVEL = 1 << 4
F_SCHED_WALK = 1 << 5
F_PLACEMENT_LAZY = 1 << 6
F_PLACEMENT_REFINE = 1 << 7


def F_RING_SLOTS(n: int) -> int:
    """Ring of recently solved blocks per solve workgroup (8, 16, 32 or 64;
    0 = default) for the one-shot entry points."""
    return (4 if n >= 64 else 3 if n >= 32 else 2 if n >= 16 else 1 if n >= 8 else 0) << 8


def F_SWEEP_CAP(n: int) -> int:
    return (int(n) & 0xFFFF) << 16


OUTPUTS = ("nu_h", "nu_d", "ave_h", "ave_d", "avf_h", "avf_d", "ins_entry_h", "ins_entry_d",
           "ins_edge_h", "ins_edge_d", "var_kind", "after_dev", "before_dev", "fp_clause")


def build() -> str:
    """Compile libompd.so for gfx950 with hipcc (always recompiles)."""
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-o", tmp] + [os.path.join(_HERE, s) for s in _SOURCES]
    subprocess.check_call(cmd, cwd=_HERE)
    os.replace(tmp, _SO)
    return _SO


class OmpdNotBuilt(RuntimeError):
    pass


class OmpdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("ompd error %d: %s" % (code, msg))
        self.code = code


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32


class _Cfg(ctypes.Structure):
    _fields_ = [("n_blocks", _i32), ("n_edges", _i32), ("n_vars", _i32), ("entry", _i32), ("exit", _i32),
                ("succ_ptr", _vp), ("succ_idx", _vp), ("edge_kind", _vp), ("space", _vp),
                ("read_bits", _vp), ("write_bits", _vp),
                ("entry_valid_host", _vp), ("entry_valid_dev", _vp), ("exit_live_host", _vp),
                ("exit_live_dev", _vp), ("call_summary", _vp), ("summaries", _vp),
                ("n_summaries", _i32), ("reserved", _i32), ("scalar", _vp)]


class _Res(ctypes.Structure):
    _fields_ = [("nu_host", _vp), ("nu_dev", _vp), ("ave_host", _vp), ("ave_dev", _vp),
                ("avf_host", _vp), ("avf_dev", _vp), ("ins_entry_to_dev", _vp), ("ins_entry_to_host", _vp),
                ("ins_edge_to_dev", _vp), ("ins_edge_to_host", _vp), ("var_kind", _vp),
                ("after_dev", _vp), ("before_dev", _vp), ("fp_clause", _vp), ("sweeps", _i32 * 6)]


class _Prog(ctypes.Structure):
    _fields_ = [("n_procs", _i32), ("n_globals", _i32), ("procs", _vp), ("n_calls", _i32),
                ("call_proc", _vp), ("call_block", _vp), ("callee", _vp), ("n_roots", _i32), ("roots", _vp),
                ("call_space", _vp), ("const_globals", _vp), ("n_params", _vp), ("arg_ptr", _vp),
                ("arg_var", _vp), ("arg_const", _vp)]


class _ProgRes(ctypes.Structure):
    _fields_ = [("per_context", _vp), ("boundaries", _vp), ("summaries", _vp), ("demands", _vp),
                ("rounds", _i32), ("reserved", _i32), ("solves", ctypes.c_int64)]


_RES_FIELD = {"nu_h": "nu_host", "nu_d": "nu_dev", "ave_h": "ave_host", "ave_d": "ave_dev",
              "avf_h": "avf_host", "avf_d": "avf_dev", "ins_entry_h": "ins_entry_to_host",
              "ins_entry_d": "ins_entry_to_dev", "ins_edge_h": "ins_edge_to_host",
              "ins_edge_d": "ins_edge_to_dev", "var_kind": "var_kind", "after_dev": "after_dev",
              "before_dev": "before_dev", "fp_clause": "fp_clause"}

_lock = threading.Lock()
_handle = None


def lib():
    """The loaded library; raises OmpdNotBuilt if libompd.so is missing."""
    global _handle
    with _lock:
        if _handle is None:
            if not os.path.exists(_SO):
                raise OmpdNotBuilt("libompd.so is not built (run __graft_entry__.build())")
            # torch ships its own HIP runtime under the same library name: it has to be loaded
            # before libompd, which then binds to it.  In the other order the process holds the
            # system runtime first and torch, when it is used later (device buffers, streams),
            # finds no GPU.
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
            L = ctypes.CDLL(_SO)
            P = ctypes.POINTER
            L.ompd_ctx_create.argtypes = [P(_vp), ctypes.c_int, ctypes.c_uint64]
            L.ompd_ctx_destroy.argtypes = [_vp]
            L.ompd_ctx_destroy.restype = None
            L.ompd_last_error.argtypes = [_vp]
            L.ompd_last_error.restype = ctypes.c_char_p
            L.ompd_device_info.argtypes = [_vp, P(_i32), P(_i32), P(ctypes.c_int64)]
            L.ompd_set_wait_limit.argtypes = [_vp, ctypes.c_int64]
            L.ompd_analyze_cfg.argtypes = [_vp, P(_Cfg), P(_Res), ctypes.c_uint32, _vp]
            L.ompd_analyze_batch.argtypes = [_vp, P(_Cfg), P(_Res), _i32, ctypes.c_uint32, _vp]
            L.ompd_analyze_batch_noalloc.argtypes = [_vp, P(_Cfg), P(_Res), _i32, ctypes.c_uint32, _vp]
            L.ompd_plan_create.argtypes = [_vp, P(_Cfg), P(_Res), _i32, ctypes.c_uint32, P(_vp)]
            L.ompd_plan_run.argtypes = [_vp, _vp]
            L.ompd_plan_status.argtypes = [_vp, _vp]
            L.ompd_plan_autotune.argtypes = [_vp, _vp, _i32, P(ctypes.c_float)]
            L.ompd_plan_set_schedule.argtypes = [_vp, _vp]
            L.ompd_plan_describe.argtypes = [_vp, ctypes.c_char_p, _i32]
            L.ompd_plan_configure.argtypes = [_vp, ctypes.c_int64, _i32]
            L.ompd_plan_profile.argtypes = [_vp, _i32]
            L.ompd_plan_split_kernels.argtypes = [_vp, _i32]
            L.ompd_plan_kernel_ms.argtypes = [_vp, P(ctypes.c_float), _i32, P(_i32)]
            L.ompd_plan_last_ms.argtypes = [_vp, P(ctypes.c_float), P(ctypes.c_float)]
            L.ompd_plan_destroy.argtypes = [_vp]
            L.ompd_plan_destroy.restype = None
            L.ompd_submit.argtypes = [_vp, P(_Cfg), P(_Res), ctypes.c_uint32, P(ctypes.c_uint64)]
            L.ompd_poll.argtypes = [_vp, ctypes.c_uint64, P(ctypes.c_int)]
            L.ompd_poll_ex.argtypes = [_vp, ctypes.c_uint64, P(ctypes.c_int), P(ctypes.c_int64)]
            L.ompd_wait.argtypes = [_vp, ctypes.c_uint64, ctypes.c_int64, P(ctypes.c_int)]
            L.ompd_serving_stats.argtypes = [_vp, P(ctypes.c_int64), P(ctypes.c_int64), P(ctypes.c_int64),
                                             P(ctypes.c_int64)]
            L.ompd_program_contexts.argtypes = [_vp, P(_Prog), P(_i32), _vp, _vp, _vp, _i32]
            L.ompd_analyze_program.argtypes = [_vp, P(_Prog), P(_ProgRes), ctypes.c_uint32]
            _handle = L
        return _handle


def _check(rc: int):
    if rc != 0:
        msg = lib().ompd_last_error(None)
        raise OmpdError(rc, msg.decode() if msg else "")


def _np_ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return _vp(a.ctypes.data)


@dataclass
class DeviceCFG:
    """A CFG whose arrays are device pointers (e.g. torch tensors' data_ptr())."""
    n_blocks: int
    n_edges: int
    n_vars: int
    entry: int
    exit: int
    succ_ptr: int
    succ_idx: int
    edge_kind: int
    space: int
    read_bits: int
    write_bits: int
    entry_valid_host: int = 0
    entry_valid_dev: int = 0
    exit_live_host: int = 0
    exit_live_dev: int = 0
    call_summary: int = 0
    summaries: int = 0
    n_summaries: int = 0
    scalar: int = 0


def _cfg_struct(cfg, keep: list) -> _Cfg:
    if isinstance(cfg, DeviceCFG):
        s = _Cfg()
        for f in ("n_blocks", "n_edges", "n_vars", "entry", "exit", "n_summaries"):
            setattr(s, f, int(getattr(cfg, f)))
        for f in ("succ_ptr", "succ_idx", "edge_kind", "space", "read_bits", "write_bits", "entry_valid_host",
                  "entry_valid_dev", "exit_live_host", "exit_live_dev", "call_summary", "summaries", "scalar"):
            v = int(getattr(cfg, f))
            setattr(s, f, v if v else None)
        return s
    nb, nv = int(cfg.n_blocks), int(cfg.n_vars)
    wd = (nv + 63) // 64

    def arr(a, dt, shape=None):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dt)
        if shape is not None:
            a = a.reshape(shape)
        keep.append(a)
        return a
    sp = arr(cfg.succ_ptr, np.int32)
    si = arr(cfg.succ_idx, np.int32)
    kd = arr(cfg.edge_kind, np.uint8)
    spc = arr(cfg.space, np.uint8)
    R = arr(cfg.R, np.uint64, (nb, wd))
    W = arr(cfg.W, np.uint64, (nb, wd))
    s = _Cfg()
    s.n_blocks, s.n_edges, s.n_vars = nb, int(si.shape[0]), nv
    s.entry, s.exit = int(cfg.entry), int(cfg.exit)
    s.succ_ptr, s.succ_idx, s.edge_kind, s.space = _np_ptr(sp), _np_ptr(si), _np_ptr(kd), _np_ptr(spc)
    s.read_bits, s.write_bits = _np_ptr(R), _np_ptr(W)
    for f_api, f_cfg in (("entry_valid_host", "entry_valid_h"), ("entry_valid_dev", "entry_valid_d"),
                         ("exit_live_host", "exit_live_h"), ("exit_live_dev", "exit_live_d")):
        v = getattr(cfg, f_cfg, None)
        setattr(s, f_api, _np_ptr(arr(v, np.uint64)) if v is not None else None)
    call = getattr(cfg, "call_summary", None)
    if call is not None:
        sums = arr(cfg.summaries, np.uint64)
        s.call_summary = _np_ptr(arr(call, np.int32))
        s.summaries = _np_ptr(sums)
        s.n_summaries = int(sums.size // (16 * max(wd, 1))) if wd else int(getattr(cfg, "n_summaries", 1))
    sc = getattr(cfg, "scalar", None)
    if sc is not None:
        s.scalar = _np_ptr(arr(sc, np.uint64))
    return s


def _alloc_outputs(cfg, want: Sequence[str]) -> Dict[str, np.ndarray]:
    nb, nv = int(cfg.n_blocks), int(cfg.n_vars)
    ne = int(np.asarray(cfg.succ_idx).shape[0])
    wd = (nv + 63) // 64
    out = {}
    for k in want:
        if k.startswith("ins_edge"):
            out[k] = np.zeros((ne, wd), np.uint64)
        elif k == "var_kind":
            out[k] = np.zeros(nv, np.uint8)
        elif k in ("after_dev", "before_dev"):
            out[k] = np.zeros(nb, np.uint8)
        else:
            out[k] = np.zeros((nb, wd), np.uint64)
    return out


_RES_INDEX = {k: [f[0] for f in _Res._fields_].index(v) for k, v in _RES_FIELD.items()}


def _alloc_outputs_many(cfgs: Sequence, want: Sequence[str], R) -> List[Dict[str, np.ndarray]]:
    """Output arrays of many CFGs (as _alloc_outputs), one zeroed buffer per output with each
    CFG's arrays as views into it; writes their addresses into the result structs R."""
    n = len(cfgs)
    nb = np.array([int(c.n_blocks) for c in cfgs], np.int64)
    nv = np.array([int(c.n_vars) for c in cfgs], np.int64)
    ne = np.array([int(np.asarray(c.succ_idx).shape[0]) for c in cfgs], np.int64)
    wd = (nv + 63) // 64
    words = np.frombuffer(R, dtype=np.uint64).reshape(len(R), ctypes.sizeof(_Res) // 8)
    outs: List[Dict[str, np.ndarray]] = [dict() for _ in range(n)]
    for k in want:
        if k.startswith("ins_edge") or k not in ("var_kind", "after_dev", "before_dev"):
            rows, dt = (ne if k.startswith("ins_edge") else nb), np.uint64
            size = rows * wd
        else:
            rows, dt = (nv if k == "var_kind" else nb), np.uint8
            size = rows
        off = np.zeros(n + 1, np.int64)
        np.cumsum(size, out=off[1:])
        buf = np.zeros(max(int(off[-1]), 1), dt)
        words[:n, _RES_INDEX[k]] = np.uint64(buf.ctypes.data) + (off[:n] * buf.itemsize).astype(np.uint64)
        for i in range(n):
            a = buf[off[i]:off[i + 1]]
            outs[i][k] = a.reshape(int(rows[i]), int(wd[i])) if dt is np.uint64 else a
    return outs


def _sweeps_of(R, n: int) -> np.ndarray:
    """[n, 6] int32 copy of the sweeps fields of the first n result structs."""
    ints = np.frombuffer(R, dtype=np.int32).reshape(len(R), ctypes.sizeof(_Res) // 4)
    at = _Res.sweeps.offset // 4
    return ints[:n, at:at + 6].copy()


def _res_struct(out: Dict[str, np.ndarray]) -> _Res:
    r = _Res()
    for k, a in out.items():
        setattr(r, _RES_FIELD[k], _vp(a.ctypes.data) if a.size else _vp(a.ctypes.data))
    return r


class Context:
    """An ompd context on one GPU (ompd_ctx_create / ompd_ctx_destroy)."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        h = _vp()
        _check(lib().ompd_ctx_create(ctypes.byref(h), int(device), int(budget_bytes)))
        self.h = h

    def close(self):
        if self.h:
            lib().ompd_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_info(self) -> Dict[str, int]:
        cu, lds, mem = _i32(0), _i32(0), ctypes.c_int64(0)
        _check(lib().ompd_device_info(self.h, ctypes.byref(cu), ctypes.byref(lds), ctypes.byref(mem)))
        return {"n_cu": cu.value, "lds_bytes": lds.value, "mem_bytes": mem.value}

    def set_wait_limit(self, ns: int = 0):
        """ompd_set_wait_limit: bound of a solve kernel's wait without progress (0 = default)."""
        _check(lib().ompd_set_wait_limit(self.h, int(ns)))

    # -- one-shot, host pointers ------------------------------------------------
    def analyze_cfg(self, cfg, flags: int = 0, want: Sequence[str] = OUTPUTS) -> Dict[str, np.ndarray]:
        return self.analyze_batch([cfg], flags, want)[0]

    def analyze_batch(self, cfgs: Sequence, flags: int = 0, want: Sequence[str] = OUTPUTS) -> List[Dict[str, np.ndarray]]:
        keep: list = []
        n = len(cfgs)
        C = (_Cfg * max(n, 1))()
        R = (_Res * max(n, 1))()
        for i, g in enumerate(cfgs):
            C[i] = _cfg_struct(g, keep)
        outs = _alloc_outputs_many(cfgs, want, R)
        _check(lib().ompd_analyze_batch(self.h, C, R, n, int(flags), None))
        sweeps = _sweeps_of(R, n)
        for i in range(n):
            outs[i]["sweeps"] = sweeps[i]
        return outs


def _prog_struct(prog, keep: list) -> _Prog:
    """Marshal a program (procs, n_globals, call_proc, call_block, callee, roots)."""
    n = len(prog.procs)
    C = (_Cfg * n)()
    for i, c in enumerate(prog.procs):
        C[i] = _cfg_struct(c, keep)
    keep.append(C)
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.int32)) for a in (prog.call_proc, prog.call_block,
                                                                         prog.callee, prog.roots)]
    keep.extend(arrs)
    P = _Prog()
    P.n_procs, P.n_globals = n, int(prog.n_globals)
    P.procs = _vp(ctypes.addressof(C))
    P.n_calls = int(arrs[0].size)
    P.call_proc, P.call_block, P.callee = (_np_ptr(a) if a.size else None for a in arrs[:3])
    P.n_roots, P.roots = int(arrs[3].size), _np_ptr(arrs[3])
    cs = getattr(prog, "call_space", None)
    if cs is not None:
        cs = np.ascontiguousarray(np.asarray(cs, dtype=np.uint8))
        keep.append(cs)
        P.call_space = _np_ptr(cs) if cs.size else None
    cg = getattr(prog, "const_globals", None)
    if cg is not None:
        cg = np.ascontiguousarray(np.asarray(cg, dtype=np.uint64))
        keep.append(cg)
        P.const_globals = _np_ptr(cg)
    for name, dt in (("n_params", np.int32), ("arg_ptr", np.int32), ("arg_var", np.int32), ("arg_const", np.uint8)):
        a = getattr(prog, name, None)
        if a is not None:
            a = np.ascontiguousarray(np.asarray(a, dtype=dt))
            keep.append(a)
            setattr(P, name, _np_ptr(a) if a.size else None)
    return P


def shared_words(prog) -> int:
    """Words of a program's summary and demand rows: the globals and the most pointer parameters
    of any procedure."""
    npar = getattr(prog, "n_params", None)
    mx = int(np.max(npar)) if npar is not None and len(npar) else 0
    return (int(prog.n_globals) + mx + 63) // 64


def demand_vars(prog, j: int, row) -> List[int]:
    """The caller variables a call site's demand row (the site's layout: globals, then one bit
    per argument) asks to make current on the host."""
    G = int(prog.n_globals)
    ap, av = getattr(prog, "arg_ptr", None), getattr(prog, "arg_var", None)
    args = [] if ap is None else [int(x) for x in av[int(ap[j]):int(ap[j + 1])]]
    out = set()
    for v in range(64 * len(row)):
        if (int(row[v >> 6]) >> (v & 63)) & 1:
            out.add(v if v < G else args[v - G])
    return sorted(out)


def _sigma(s0: int, s1: int) -> tuple:
    return () if s1 < 0 else ((s1,) if s0 < 0 else (s0, s1))


def _program_contexts(self, prog) -> List[tuple]:
    """Contexts of a program as (procedure, call string of at most two sites), in library order."""
    keep: list = []
    P = _prog_struct(prog, keep)
    n = _i32(0)
    _check(lib().ompd_program_contexts(self.h, ctypes.byref(P), ctypes.byref(n), None, None, None, 0))
    cp = np.zeros(max(n.value, 1), np.int32)
    c0 = np.zeros_like(cp)
    c1 = np.zeros_like(cp)
    _check(lib().ompd_program_contexts(self.h, ctypes.byref(P), ctypes.byref(n), _np_ptr(cp), _np_ptr(c0),
                                       _np_ptr(c1), n.value))
    return [(int(cp[k]), _sigma(int(c0[k]), int(c1[k]))) for k in range(n.value)]


def _analyze_program(self, prog, flags: int = 0, want: Sequence[str] = OUTPUTS[:-1]) -> Dict:
    """ompd_analyze_program: per-context results, boundaries, summaries and demands."""
    keys = self.program_contexts(prog)
    keep: list = []
    P = _prog_struct(prog, keep)
    R = (_Res * max(len(keys), 1))()
    outs = _alloc_outputs_many([prog.procs[p] for (p, _) in keys], want, R)
    wds = [(prog.procs[p].n_vars + 63) // 64 for (p, _) in keys]
    bnd = np.zeros(max(4 * sum(wds), 1), np.uint64)
    sw = shared_words(prog)
    summ = np.zeros((len(prog.procs), 16, sw), np.uint64)
    nc = int(np.asarray(prog.call_proc).size)
    dem = np.zeros((nc, sw), np.uint64)
    out = _ProgRes()
    out.per_context = _vp(ctypes.addressof(R))
    out.boundaries = _np_ptr(bnd)
    out.summaries = _np_ptr(summ) if summ.size else None
    out.demands = _np_ptr(dem) if dem.size else None
    _check(lib().ompd_analyze_program(self.h, ctypes.byref(P), ctypes.byref(out), int(flags)))
    bounds, off = [], 0
    for wdk in wds:
        bounds.append([bnd[off + i * wdk: off + (i + 1) * wdk] for i in range(4)])
        off += 4 * wdk
    sweeps = _sweeps_of(R, len(keys))
    for k in range(len(keys)):
        outs[k]["sweeps"] = sweeps[k]
    return {"contexts": keys, "results": outs, "boundaries": bounds, "summaries": summ, "demands": dem,
            "rounds": out.rounds, "solves": out.solves}


Context.program_contexts = _program_contexts
Context.analyze_program = _analyze_program


class Request:
    """A submitted analysis request (ompd_submit): the host buffers its
    results land in stay referenced here until the request is collected."""

    def __init__(self, ctx: "Context", cfg, flags: int = 0, want: Sequence[str] = OUTPUTS):
        self.ctx = ctx
        self._keep: list = []
        self._C = _cfg_struct(cfg, self._keep)
        self.out = _alloc_outputs(cfg, want)
        self._R = _res_struct(self.out)
        t = ctypes.c_uint64(0)
        rc = lib().ompd_submit(ctx.h, ctypes.byref(self._C), ctypes.byref(self._R), int(flags), ctypes.byref(t))
        self.rc = rc
        self.ticket = t.value
        self.done = False
        self.done_ns = 0
        self.status = 0

    @property
    def admitted(self) -> bool:
        return self.rc == 0

    def poll(self) -> bool:
        """True once the request has completed (raises on its error)."""
        if self.done:
            return True
        d = ctypes.c_int(0)
        ns = ctypes.c_int64(0)
        _check(lib().ompd_poll_ex(self.ctx.h, ctypes.c_uint64(self.ticket), ctypes.byref(d), ctypes.byref(ns)))
        if d.value == 0:
            return False
        self.done = True
        self.done_ns = ns.value
        self.status = 0 if d.value == 1 else d.value
        self.out["sweeps"] = np.array(list(self._R.sweeps), dtype=np.int32)
        if self.status:
            raise OmpdError(self.status, "request failed")
        return True

    def wait(self, timeout_s: float = -1.0) -> Dict[str, np.ndarray]:
        if not self.done:
            d = ctypes.c_int(0)
            _check(lib().ompd_wait(self.ctx.h, ctypes.c_uint64(self.ticket),
                                   int(timeout_s * 1e9) if timeout_s >= 0 else -1, ctypes.byref(d)))
            self.done = True
            self.status = 0 if d.value == 1 else d.value
            self.out["sweeps"] = np.array(list(self._R.sweeps), dtype=np.int32)
            if self.status:
                raise OmpdError(self.status, "request failed")
        return self.out


def submit(ctx: "Context", cfg, flags: int = 0, want: Sequence[str] = OUTPUTS) -> Request:
    """ompd_submit; check .admitted (False = OMPD_E_BUSY, retry later)."""
    r = Request(ctx, cfg, flags, want)
    if r.rc not in (0, OMPD_E_BUSY):
        _check(r.rc)
    return r


def serving_stats(ctx: "Context") -> Dict[str, int]:
    a, c, f, b = (ctypes.c_int64(0) for _ in range(4))
    _check(lib().ompd_serving_stats(ctx.h, ctypes.byref(a), ctypes.byref(c), ctypes.byref(f), ctypes.byref(b)))
    return {"admitted": a.value, "completed": c.value, "in_flight": f.value, "bytes_in_use": b.value}


def ctx_create(device: int = 0, budget_bytes: int = 0) -> Context:
    return Context(device, budget_bytes)


def analyze_cfg(ctx: Context, cfg, flags: int = 0, want: Sequence[str] = OUTPUTS):
    return ctx.analyze_cfg(cfg, flags, want)


def analyze_batch(ctx: Context, cfgs: Sequence, flags: int = 0, want: Sequence[str] = OUTPUTS):
    return ctx.analyze_batch(cfgs, flags, want)


@dataclass
class DeviceResult:
    """Device pointers for one CFG's outputs (0 = not requested)."""
    nu_h: int = 0
    nu_d: int = 0
    ave_h: int = 0
    ave_d: int = 0
    avf_h: int = 0
    avf_d: int = 0
    ins_entry_h: int = 0
    ins_entry_d: int = 0
    ins_edge_h: int = 0
    ins_edge_d: int = 0
    var_kind: int = 0
    after_dev: int = 0
    before_dev: int = 0
    fp_clause: int = 0


def analyze_device(ctx: Context, cfgs: Sequence[DeviceCFG], results: Sequence[DeviceResult], flags: int = 0,
                   stream: int = 0, noalloc: bool = False) -> np.ndarray:
    """One synchronous batch solve over device-pointer CFGs and outputs: ompd_analyze_batch
    with OMPD_F_DEVICE_PTRS, or (noalloc) ompd_analyze_batch_noalloc, which allocates no
    device memory.  Returns the [n, 6] sweeps per phase."""
    n = len(cfgs)
    C = (_Cfg * max(n, 1))()
    R = (_Res * max(n, 1))()
    keep: list = []
    for i in range(n):
        C[i] = _cfg_struct(cfgs[i], keep)
        r = _Res()
        for k, f in _RES_FIELD.items():
            v = int(getattr(results[i], k))
            setattr(r, f, v if v else None)
        R[i] = r
    fn = lib().ompd_analyze_batch_noalloc if noalloc else lib().ompd_analyze_batch
    _check(fn(ctx.h, C, R, n, int(flags) | F_DEVICE_PTRS, _vp(stream) if stream else None))
    return _sweeps_of(R, n)


class Plan:
    """A resident batch (ompd_plan_*) over device-pointer CFGs."""

    def __init__(self, ctx: Context, cfgs: Sequence[DeviceCFG], results: Sequence[DeviceResult], flags: int = 0):
        n = len(cfgs)
        self.ctx = ctx
        self.n = n
        self._C = (_Cfg * max(n, 1))()
        self._R = (_Res * max(n, 1))()
        keep: list = []
        for i in range(n):
            self._C[i] = _cfg_struct(cfgs[i], keep)
            r = _Res()
            for k, f in _RES_FIELD.items():
                v = int(getattr(results[i], k))
                setattr(r, f, v if v else None)
            self._R[i] = r
        h = _vp()
        _check(lib().ompd_plan_create(ctx.h, self._C, self._R, n, int(flags) | F_DEVICE_PTRS, ctypes.byref(h)))
        self.h = h

    def run(self, stream: int = 0):
        _check(lib().ompd_plan_run(self.h, _vp(stream) if stream else None))

    def status(self) -> np.ndarray:
        per = np.zeros(max(self.n, 1), np.int32)
        per[:] = 1   # a HIP failure before the per-CFG words are read leaves this (not a status)
        rc = lib().ompd_plan_status(self.h, _vp(per.ctypes.data))
        if rc not in (0, OMPD_E_INVAL, OMPD_E_NOCONVERGE, OMPD_E_DEVICE) or (per[:self.n] == 1).any():
            _check(rc)
        return per[:self.n]

    def autotune(self, stream: int = 0, trials: int = 2) -> float:
        best = ctypes.c_float(0)
        _check(lib().ompd_plan_autotune(self.h, _vp(stream) if stream else None, int(trials), ctypes.byref(best)))
        return best.value

    def configure(self, lds_bytes: int = 0, wg_per_cu: int = 0):
        """LDS ring bytes per solve wavefront (0 = default) and wavefronts per CU (0 = as many as fit)."""
        _check(lib().ompd_plan_configure(self.h, int(lds_bytes), int(wg_per_cu)))

    KERNELS = ("ompd_k_prep", "ompd_k_nu", "ompd_k_ave", "ompd_k_post_ave", "ompd_k_mayp", "ompd_k_post_mayp",
               "ompd_k_later", "ompd_k_post_later", "ompd_k_live", "ompd_k_post_live", "ompd_k_avf",
               "ompd_k_post_avf", "ompd_k_varkind")
    KERNELS_TILE = ("ompd_k_prep", "ompd_k_solve")

    def split_kernels(self, split: bool = True):
        """One kernel per phase and pass (the default), or one per-tile kernel for every phase."""
        _check(lib().ompd_plan_split_kernels(self.h, 1 if split else 0))

    def profile(self, enable: bool = True):
        """Time every kernel of the following runs with HIP events on their stream."""
        _check(lib().ompd_plan_profile(self.h, 1 if enable else 0))

    def kernel_ms(self) -> Dict[str, float]:
        """Per-kernel durations (ms) of the last profiled run."""
        buf = (ctypes.c_float * 16)()
        n = _i32(0)
        _check(lib().ompd_plan_kernel_ms(self.h, buf, 16, ctypes.byref(n)))
        names = self.KERNELS if n.value == len(self.KERNELS) else self.KERNELS_TILE
        return {k: float(buf[i]) for i, k in enumerate(names[:n.value])}

    def set_schedule(self, per_bucket):
        """ompd_plan_set_schedule: -1 (rule), 0 (walk) or 1 (level) per size bucket (5)."""
        v = np.asarray(list(per_bucket), np.int32)
        assert v.size == 5
        _check(lib().ompd_plan_set_schedule(self.h, _vp(v.ctypes.data)))

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(1024)
        _check(lib().ompd_plan_describe(self.h, buf, 1024))
        return buf.value.decode()

    def last_ms(self):
        a, b = ctypes.c_float(0), ctypes.c_float(0)
        _check(lib().ompd_plan_last_ms(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def close(self):
        if getattr(self, "h", None):
            lib().ompd_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_create(ctx: Context, cfgs: Sequence[DeviceCFG], results: Sequence[DeviceResult], flags: int = 0) -> Plan:
    return Plan(ctx, cfgs, results, flags)
