"""Seeded synthetic inputs for the OMPDart data-flow solve.

This package only produces inputs (structured CFGs with host/device blocks,
read/write bitmaps, call graphs, request arrival times) and the plain
container that carries them.  It holds none of the analysis arithmetic: the
oracle and the GPU library both consume what it returns.

Workload recipes (all seeded from ``MASTER_SEED``):

* ``c1``  one procedure, 64 user blocks, loop depth <= 3, 30 % device blocks,
  32 variables, read p=0.2, write p=0.1.
* ``c2``  one procedure, 16,384 user blocks, loop depth <= 6, 40 % device
  blocks, 1 % of loops made irreducible, 2,048 variables, p=0.05 / 0.02.
* ``c3``  4,096 procedures, user blocks log-uniform in [16, 8192], variables
  log-uniform in [32, 4096], otherwise as ``c1``.
* ``c4``  a program of 2,000 procedures (see ``program``).
* ``c5``  a Poisson stream of ``c2``-shaped requests (see ``poisson_arrivals``).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_SO = os.path.join(_HERE, "libsynth.so")

MASTER_SEED = 240613881
MASK64 = (1 << 64) - 1

KIND_NORMAL, KIND_BACK, KIND_LOOP_ENTRY = 0, 1, 2
HOST, DEVICE = 0, 1


def build() -> str:
    """Compile the generator with gcc (always recompiles)."""
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _SO)
    return _SO


_lib_lock = threading.Lock()
_lib_handle = None


class _Params(ctypes.Structure):
    _fields_ = [
        ("n_user", ctypes.c_int32),
        ("n_vars", ctypes.c_int32),
        ("max_loop_depth", ctypes.c_int32),
        ("n_call_sites", ctypes.c_int32),
        ("device_frac", ctypes.c_double),
        ("irr_loop_frac", ctypes.c_double),
        ("thr_read", ctypes.c_uint32),
        ("thr_write", ctypes.c_uint32),
    ]


def _lib():
    global _lib_handle
    with _lib_lock:
        if _lib_handle is None:
            if not os.path.exists(_SO):
                build()
            lib = ctypes.CDLL(_SO)
            lib.synth_splitmix64.restype = ctypes.c_uint64
            lib.synth_splitmix64.argtypes = [ctypes.c_uint64]
            lib.synth_log_uniform_int.restype = ctypes.c_int64
            lib.synth_log_uniform_int.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64]
            lib.synth_cfg_edges.restype = ctypes.c_int64
            lib.synth_cfg_edges.argtypes = [ctypes.c_uint64, ctypes.POINTER(_Params)]
            vp = ctypes.c_void_p
            lib.synth_cfg_fill.restype = ctypes.c_int
            lib.synth_cfg_fill.argtypes = [ctypes.c_uint64, ctypes.POINTER(_Params), vp, vp, vp, vp, vp, vp, vp, vp]
            _lib_handle = lib
        return _lib_handle


def splitmix64(x: int) -> int:
    return int(_lib().synth_splitmix64(ctypes.c_uint64(x & MASK64)))


def config_seed(k: int) -> int:
    return splitmix64(MASTER_SEED ^ k)


def item_seed(k: int, i: int) -> int:
    return splitmix64((config_seed(k) + i) & MASK64)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def words(n_vars: int) -> int:
    return (n_vars + 63) // 64


def var_mask(n_vars: int) -> np.ndarray:
    """[words] mask of the valid variable bits."""
    wd = words(n_vars)
    m = np.full(wd, np.uint64(MASK64), dtype=np.uint64)
    if n_vars % 64 and wd:
        m[-1] = np.uint64((1 << (n_vars % 64)) - 1)
    return m


@dataclass
class CFG:
    """One procedure: successor CSR, edge kinds, block spaces and R/W bitmaps.

    ``n_blocks`` includes the access-free HOST blocks ``entry`` and ``exit``.
    Bit v of word (v >> 6) of row b of ``R``/``W`` is the access of
    variable v in block b.  Boundary vectors left ``None`` take the defaults:
    everything valid on the host and nothing on the device at ENTRY, and
    every variable live on the host (none on the device) after EXIT.
    """

    n_blocks: int
    n_vars: int
    succ_ptr: np.ndarray
    succ_idx: np.ndarray
    edge_kind: np.ndarray
    space: np.ndarray
    R: np.ndarray
    W: np.ndarray
    entry: int = 0
    exit: int = -1
    entry_valid_h: Optional[np.ndarray] = None
    entry_valid_d: Optional[np.ndarray] = None
    exit_live_h: Optional[np.ndarray] = None
    exit_live_d: Optional[np.ndarray] = None
    loop_depth: Optional[np.ndarray] = None
    call_blocks: Optional[np.ndarray] = None
    seed: Optional[int] = None
    scalar: Optional[np.ndarray] = None   # [wd] variables the front end marks as scalars (None = none)

    def __post_init__(self):
        if self.exit < 0:
            self.exit = self.n_blocks - 1

    @property
    def n_edges(self) -> int:
        return int(self.succ_idx.shape[0])

    @property
    def wd(self) -> int:
        return words(self.n_vars)

    @property
    def facts(self) -> int:
        return (self.n_blocks - 2) * self.n_vars

    def boundary(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
        """(entry_valid_h, entry_valid_d, exit_live_h, exit_live_d) with defaults filled."""
        m = var_mask(self.n_vars)
        z = np.zeros(self.wd, dtype=np.uint64)
        evh = m.copy() if self.entry_valid_h is None else np.ascontiguousarray(self.entry_valid_h, dtype=np.uint64)
        evd = z.copy() if self.entry_valid_d is None else np.ascontiguousarray(self.entry_valid_d, dtype=np.uint64)
        lxh = m.copy() if self.exit_live_h is None else np.ascontiguousarray(self.exit_live_h, dtype=np.uint64)
        lxd = z.copy() if self.exit_live_d is None else np.ascontiguousarray(self.exit_live_d, dtype=np.uint64)
        return evh, evd, lxh, lxd

    def preds(self) -> List[List[Tuple[int, int]]]:
        """Per block: list of (pred block, successor-CSR edge id)."""
        out: List[List[Tuple[int, int]]] = [[] for _ in range(self.n_blocks)]
        for p in range(self.n_blocks):
            for e in range(int(self.succ_ptr[p]), int(self.succ_ptr[p + 1])):
                out[int(self.succ_idx[e])].append((p, e))
        return out


def make_cfg(seed: int, n_user: int, n_vars: int, max_loop_depth: int, device_frac: float,
             irr_loop_frac: float = 0.0, p_read: float = 0.2, p_write: float = 0.1,
             n_call_sites: int = 0, with_bits: bool = True) -> CFG:
    """Generate one structured CFG (deterministic in every argument)."""
    p = _Params(n_user, n_vars, max_loop_depth, n_call_sites, device_frac, irr_loop_frac,
                int(round(p_read * 65536)), int(round(p_write * 65536)))
    lib = _lib()
    ne = int(lib.synth_cfg_edges(ctypes.c_uint64(seed & MASK64), ctypes.byref(p)))
    if ne < 0:
        raise ValueError("bad generator parameters")
    nb = n_user + 2
    wd = words(n_vars)
    succ_ptr = np.zeros(nb + 1, dtype=np.int32)
    succ_idx = np.zeros(max(ne, 1), dtype=np.int32)[:ne]
    kind = np.zeros(max(ne, 1), dtype=np.uint8)[:ne]
    space = np.zeros(nb, dtype=np.uint8)
    ldepth = np.zeros(nb, dtype=np.int32)
    R = np.zeros((nb, wd), dtype=np.uint64)
    W = np.zeros((nb, wd), dtype=np.uint64)
    calls = np.zeros(max(n_call_sites, 1), dtype=np.int32)
    nc = lib.synth_cfg_fill(ctypes.c_uint64(seed & MASK64), ctypes.byref(p), _ptr(succ_ptr), _ptr(succ_idx),
                            _ptr(kind), _ptr(space), _ptr(R) if with_bits else None,
                            _ptr(W) if with_bits else None, _ptr(ldepth), _ptr(calls))
    if nc < 0:
        raise ValueError("generator failed")
    return CFG(n_blocks=nb, n_vars=n_vars, succ_ptr=succ_ptr, succ_idx=succ_idx, edge_kind=kind,
               space=space, R=R, W=W, loop_depth=ldepth, call_blocks=calls[:nc].copy(), seed=seed)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
C1 = dict(n_user=64, n_vars=32, max_loop_depth=3, device_frac=0.30, irr_loop_frac=0.0, p_read=0.2, p_write=0.1)
C2 = dict(n_user=16384, n_vars=2048, max_loop_depth=6, device_frac=0.40, irr_loop_frac=0.01,
          p_read=0.05, p_write=0.02)
C3_BLOCKS = (16, 8192)
C3_VARS = (32, 4096)
C3_COUNT = 4096


def c1(i: int = 0) -> CFG:
    """Config 1 (i = 0 is the benchmark instance; others feed the parity sweep)."""
    return make_cfg(item_seed(1, i), **C1)


def c2(i: int = 0) -> CFG:
    return make_cfg(item_seed(2, i), **C2)


def c3_sizes(n: int = C3_COUNT) -> Tuple[np.ndarray, np.ndarray]:
    """(user blocks, variables) of the first n items of config 3."""
    lib = _lib()
    nu = np.zeros(n, dtype=np.int64)
    nv = np.zeros(n, dtype=np.int64)
    for i in range(n):
        s = item_seed(3, i)
        nu[i] = lib.synth_log_uniform_int(ctypes.c_uint64(splitmix64(s ^ 0xB10C5)), C3_BLOCKS[0], C3_BLOCKS[1])
        nv[i] = lib.synth_log_uniform_int(ctypes.c_uint64(splitmix64(s ^ 0x7A125)), C3_VARS[0], C3_VARS[1])
    return nu, nv


def c3_item(i: int, n_user: Optional[int] = None, n_vars: Optional[int] = None) -> CFG:
    if n_user is None or n_vars is None:
        nu, nv = c3_sizes(i + 1)
        n_user, n_vars = int(nu[i]), int(nv[i])
    prm = dict(C1)
    prm.update(n_user=int(n_user), n_vars=int(n_vars))
    return make_cfg(item_seed(3, i), **prm)


def c3(n: int = C3_COUNT, threads: int = 0, indices: Optional[Sequence[int]] = None) -> List[CFG]:
    """Items of config 3, generated in parallel threads (the C code releases the GIL)."""
    nu, nv = c3_sizes(n if indices is None else max(indices) + 1)
    idx = list(range(n)) if indices is None else list(indices)
    threads = threads or min(16, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda i: c3_item(i, int(nu[i]), int(nv[i])), idx))


def c5_request(i: int) -> CFG:
    """Request i of the serving stream: a config-2-shaped CFG with its own seed."""
    return make_cfg(item_seed(5, i), **C2)


def poisson_arrivals(rate_per_s: float, n: int, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson stream of n requests at the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


def from_edges(blocks: Sequence[Tuple[int, Sequence[int], Sequence[int]]],
               edges: Sequence[Tuple[int, int, int]], n_vars: int) -> Tuple[CFG, np.ndarray]:
    """Hand-built CFG.

    ``blocks``: per block (space, read vars, written vars); block 0 is ENTRY and
    the last block is EXIT.  ``edges``: (src, dst, kind) in any order.
    Returns the CFG and, for each input edge, its id in successor-CSR order
    (edges are grouped by source, keeping the given order within a source).
    """
    nb = len(blocks)
    wd = words(n_vars)
    order = sorted(range(len(edges)), key=lambda k: (edges[k][0], k))
    csr_pos = np.zeros(len(edges), dtype=np.int64)
    succ_idx = np.zeros(len(edges), dtype=np.int32)
    kind = np.zeros(len(edges), dtype=np.uint8)
    ptr = np.zeros(nb + 1, dtype=np.int32)
    for pos, k in enumerate(order):
        s, d, kd = edges[k]
        csr_pos[k] = pos
        succ_idx[pos] = d
        kind[pos] = kd
        ptr[s + 1] += 1
    ptr = np.cumsum(ptr).astype(np.int32)
    space = np.array([b[0] for b in blocks], dtype=np.uint8)
    R = np.zeros((nb, wd), dtype=np.uint64)
    W = np.zeros((nb, wd), dtype=np.uint64)
    for b, (_, rd, wr) in enumerate(blocks):
        for v in rd:
            R[b, v >> 6] |= np.uint64(1 << (v & 63))
        for v in wr:
            W[b, v >> 6] |= np.uint64(1 << (v & 63))
    return CFG(n_blocks=nb, n_vars=n_vars, succ_ptr=ptr, succ_idx=succ_idx, edge_kind=kind,
               space=space, R=R, W=W), csr_pos


def mark_scalars(cfg: CFG, seed: int, frac: float = 0.3, read_only_frac: float = 0.5) -> CFG:
    """Mark a seeded fraction `frac` of the variables as scalars (cfg.scalar).  For
    `read_only_frac` of the marked ones, device writes are removed from W so that they are
    read-only on the device (firstprivate candidates the analysis will accept); the others
    keep their accesses.  Returns the CFG (modified in place)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nv, wd = cfg.n_vars, cfg.wd
    pick = rng.random(nv) < frac
    ro = pick & (rng.random(nv) < read_only_frac)
    sc = np.zeros(wd, np.uint64)
    rom = np.zeros(wd, np.uint64)
    for v in np.nonzero(pick)[0]:
        sc[v >> 6] |= np.uint64(1 << (int(v) & 63))
    for v in np.nonzero(ro)[0]:
        rom[v >> 6] |= np.uint64(1 << (int(v) & 63))
    dev = np.asarray(cfg.space) == 1
    W = np.array(cfg.W, dtype=np.uint64).reshape(cfg.n_blocks, wd)
    W[dev] &= ~rom
    cfg.W = W
    cfg.scalar = sc
    return cfg


def permute_blocks(cfg: CFG, seed: int) -> Tuple[CFG, np.ndarray, np.ndarray]:
    """The same CFG with its block ids shuffled (ENTRY and EXIT keep theirs).

    Returns (permuted CFG, perm, edge_map): block b of ``cfg`` is block
    perm[b] of the result, and edge e of ``cfg`` (successor-CSR order) is
    edge edge_map[e] of the result.  Each block keeps its successors in their
    order, kinds and accesses; boundaries are carried over."""
    nb = cfg.n_blocks
    rng = np.random.Generator(np.random.PCG64(seed))
    others = np.array([b for b in range(nb) if b not in (cfg.entry, cfg.exit)], dtype=np.int64)
    perm = np.arange(nb, dtype=np.int64)
    perm[others] = others[rng.permutation(len(others))]
    inv = np.empty(nb, dtype=np.int64)
    inv[perm] = np.arange(nb)
    sp = np.asarray(cfg.succ_ptr, dtype=np.int64)
    si = np.asarray(cfg.succ_idx, dtype=np.int64)
    deg = np.diff(sp)
    ptr = np.zeros(nb + 1, dtype=np.int64)
    np.cumsum(deg[inv], out=ptr[1:])
    succ_idx = np.zeros(si.shape[0], dtype=np.int32)
    kind = np.zeros(si.shape[0], dtype=np.uint8)
    edge_map = np.zeros(si.shape[0], dtype=np.int64)
    for nbk in range(nb):
        o = int(inv[nbk])
        a, z = int(sp[o]), int(sp[o + 1])
        succ_idx[ptr[nbk]:ptr[nbk] + (z - a)] = perm[si[a:z]]
        kind[ptr[nbk]:ptr[nbk] + (z - a)] = np.asarray(cfg.edge_kind)[a:z]
        edge_map[a:z] = np.arange(ptr[nbk], ptr[nbk] + (z - a))
    out = CFG(n_blocks=nb, n_vars=cfg.n_vars, succ_ptr=ptr.astype(np.int32), succ_idx=succ_idx, edge_kind=kind,
              space=np.ascontiguousarray(np.asarray(cfg.space)[inv]), R=np.ascontiguousarray(np.asarray(cfg.R)[inv]),
              W=np.ascontiguousarray(np.asarray(cfg.W)[inv]), entry=int(perm[cfg.entry]), exit=int(perm[cfg.exit]),
              entry_valid_h=cfg.entry_valid_h, entry_valid_d=cfg.entry_valid_d, exit_live_h=cfg.exit_live_h,
              exit_live_d=cfg.exit_live_d, seed=cfg.seed, scalar=cfg.scalar)
    return out, perm, edge_map


def random_dag(seed: int, n_blocks: int, n_vars: int, p_extra: float = 0.3, p_dev: float = 0.4,
               p_read: float = 0.3, p_write: float = 0.2, p_loop_entry: float = 0.0) -> CFG:
    """Small random acyclic CFG (unstructured).  Every block has a
    predecessor of lower id and a successor of higher id, so every block is
    reachable from ENTRY (0) and reaches EXIT (n_blocks - 1).  Optionally
    marks random edges LOOP_ENTRY to stress the loop rule of the placement."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = n_blocks
    E = set()
    for i in range(1, nb - 1):
        E.add((int(rng.integers(0, i)), i))
        E.add((i, int(rng.integers(i + 1, nb))))
    for i in range(0, nb - 1):
        for j in range(i + 1, nb):
            if rng.random() < p_extra / max(1, nb - i - 1) * 2:
                if not (i == 0 and j == nb - 1):
                    E.add((i, j))
    if not any(s == 0 for (s, _) in E):
        E.add((0, nb - 1))
    edges = []
    for (s, d) in sorted(E):
        k = KIND_LOOP_ENTRY if (d != nb - 1 and rng.random() < p_loop_entry) else KIND_NORMAL
        edges.append((s, d, k))
    blocks = []
    for b in range(nb):
        if b == 0 or b == nb - 1:
            blocks.append((HOST, [], []))
            continue
        sp = DEVICE if rng.random() < p_dev else HOST
        rd = [v for v in range(n_vars) if rng.random() < p_read]
        wr = [v for v in range(n_vars) if rng.random() < p_write]
        blocks.append((sp, rd, wr))
    cfg, _ = from_edges(blocks, edges, n_vars)
    return cfg


# --------------------------------------------------------------------------
# programs (config 4)
# --------------------------------------------------------------------------
@dataclass
class Program:
    """Procedures sharing ``n_globals`` global variables (vars [0, n_globals)
    of every procedure; the rest are locals).  Call site j is block
    ``call_block[j]`` of procedure ``call_proc[j]``; ``callee[j]`` is the
    called procedure or -1 for an external function."""
    procs: List[CFG]
    n_globals: int
    call_proc: np.ndarray
    call_block: np.ndarray
    callee: np.ndarray
    roots: List[int]
    call_space: Optional[np.ndarray] = None      # [n_calls] 1: the call runs on the device (None: all host)
    const_globals: Optional[np.ndarray] = None   # [words of globals] globals never written (None: none)
    n_params: Optional[np.ndarray] = None        # [n_procs] pointer parameters: vars [G, G + n_params)
    arg_ptr: Optional[np.ndarray] = None         # [n_calls + 1] into arg_var / arg_const
    arg_var: Optional[np.ndarray] = None         # caller variable bound to each argument
    arg_const: Optional[np.ndarray] = None       # 1: an external callee's pointer-to-const argument


C4 = dict(n_procs=2000, n_globals=256, n_locals=16, blocks=(32, 1024), mean_calls=3.0, max_calls=8,
          scc_procs=100, scc_size=(2, 8), max_loop_depth=3, device_frac=0.30, p_read=0.2, p_write=0.1)


def program(seed: int, n_procs: int = 2000, n_globals: int = 256, n_locals: int = 16,
            blocks: Tuple[int, int] = (32, 1024), mean_calls: float = 3.0, max_calls: int = 8,
            scc_procs: int = 100, scc_size: Tuple[int, int] = (2, 8), max_loop_depth: int = 3,
            device_frac: float = 0.30, p_read: float = 0.2, p_write: float = 0.1,
            external_frac: float = 0.0, threads: int = 0, device_call_frac: float = 0.0,
            n_const: int = 0, max_params: int = 0, max_ext_args: int = 0) -> Program:
    """A random call graph: procedure i calls Poisson(mean_calls) (at most
    max_calls) procedures of higher index; then scc_procs procedures are
    grouped into cycles of U{scc_size} members (a call from each member to the
    next), which makes recursive SCCs.  Procedure 0 and every procedure that
    no host call reaches are roots.  Each procedure is a structured CFG whose
    call sites are distinct host statements; a seeded fraction
    device_call_frac of them become calls made inside a kernel (their block
    turns DEVICE), and n_const seeded globals become const (every write of
    them is removed).  With max_params > 0 each procedure gets U{0..max_params}
    pointer parameters (its first locals) and every call binds them to caller
    variables: a host call distinct non-global ones (so no frame sees one datum
    under two names), a call made inside a kernel any, with repeats (globals
    passed by pointer too).  An external call gets up to max_ext_args
    arguments, any caller variables, some pointers to const."""
    rng = np.random.Generator(np.random.PCG64(seed))
    calls: List[List[int]] = [[] for _ in range(n_procs)]
    for i in range(n_procs - 1):
        k = min(int(rng.poisson(mean_calls)), max_calls)
        if k:
            calls[i].extend(int(x) for x in rng.integers(i + 1, n_procs, size=k))
    # recursive groups are runs of consecutive procedures: calls of the random
    # DAG only go to higher indices, so a cycle closed inside a run cannot pull
    # procedures outside the run into its strongly connected component
    placed = 0
    taken = np.zeros(n_procs, bool)
    attempts = 0
    while placed < scc_procs and attempts < 100 * max(scc_procs, 1):
        attempts += 1
        sz = min(int(rng.integers(scc_size[0], scc_size[1] + 1)), scc_procs - placed)
        if sz < 2:
            break
        start = int(rng.integers(0, n_procs - sz + 1))
        if taken[start:start + sz].any():
            continue
        taken[start:start + sz] = True
        grp = list(range(start, start + sz))
        for a, b in zip(grp, grp[1:] + grp[:1]):
            calls[a].append(int(b))
        placed += sz
    if external_frac > 0:
        for i in range(n_procs):
            if rng.random() < external_frac:
                calls[i].append(-1)
    lo, hi = blocks
    sizes = [int(round(math.exp(math.log(lo) + rng.random() * (math.log(hi) - math.log(lo))))) for _ in range(n_procs)]
    nv = n_globals + n_locals
    seeds = [int(x) for x in rng.integers(0, 1 << 62, size=n_procs)]

    def gen(i):
        # a procedure too small to hold all its call statements is regrown
        # (deterministically) until it does, so every call of the graph exists
        n = sizes[i]
        for attempt in range(64):
            c = make_cfg(seeds[i] + attempt, n_user=n, n_vars=nv, max_loop_depth=max_loop_depth,
                         device_frac=device_frac, p_read=p_read, p_write=p_write, n_call_sites=len(calls[i]))
            if len(c.call_blocks) == len(calls[i]):
                return c
            n += max(2, n // 4)
        raise RuntimeError("procedure %d cannot hold %d call sites" % (i, len(calls[i])))
    threads = threads or min(16, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        procs = list(ex.map(gen, range(n_procs)))
    cp, cb, ce = [], [], []
    for i, c in enumerate(procs):
        for j, blk in enumerate(c.call_blocks.tolist()):
            cp.append(i)
            cb.append(int(blk))
            ce.append(calls[i][j])
    cs = np.zeros(len(cp), np.uint8)
    if device_call_frac > 0:
        pick = rng.random(len(cp)) < device_call_frac
        for j in np.nonzero(pick)[0]:
            c = procs[cp[j]]
            c.space = np.array(c.space, np.uint8)
            c.space[cb[j]] = 1
            cs[j] = 1
    gw = words(n_globals)
    const = np.zeros(gw, np.uint64)
    if n_const > 0:
        for v in rng.choice(n_globals, size=min(n_const, n_globals), replace=False):
            const[int(v) >> 6] |= np.uint64(1 << (int(v) & 63))
        for c in procs:
            W = np.array(c.W, np.uint64).reshape(c.n_blocks, c.wd)
            W[:, :gw] &= ~const
            c.W = W
    # pointer parameters and their bindings
    npar = np.zeros(n_procs, np.int32)
    ap = np.zeros(len(cp) + 1, np.int64)
    av: List[int] = []
    acn: List[int] = []
    if max_params > 0 or max_ext_args > 0:
        if max_params > 0:
            npar = rng.integers(0, max_params + 1, size=n_procs).astype(np.int32)
            npar = np.minimum(npar, n_locals).astype(np.int32)
        for j in range(len(cp)):
            P, q = cp[j], ce[j]
            nv_p = n_globals + n_locals
            k = int(npar[q]) if q >= 0 else int(rng.integers(0, max_ext_args + 1))
            if q >= 0 and not cs[j]:
                pool = np.arange(n_globals, nv_p)
                pick = rng.choice(pool, size=min(k, pool.size), replace=False)
            else:
                pick = rng.integers(0, nv_p, size=k)
            av.extend(int(x) for x in pick)
            acn.extend(int(rng.random() < 0.5) if q < 0 else 0 for _ in range(len(pick)))
            ap[j + 1] = len(av)
    # roots: procedure 0 and every procedure no host call reaches (a procedure called only from
    # kernels is a device function and gets no context of its own)
    called = set(x for x, d in zip(ce, cs) if x >= 0 and not d)
    roots = sorted(set([0]) | set(i for i in range(n_procs) if i not in called))
    return Program(procs=procs, n_globals=n_globals, call_proc=np.array(cp, np.int32),
                   call_block=np.array(cb, np.int32), callee=np.array(ce, np.int32), roots=roots,
                   call_space=cs if device_call_frac > 0 else None,
                   const_globals=const if n_const > 0 else None,
                   n_params=npar if (max_params > 0 or max_ext_args > 0) else None,
                   arg_ptr=ap if (max_params > 0 or max_ext_args > 0) else None,
                   arg_var=np.array(av, np.int32) if (max_params > 0 or max_ext_args > 0) else None,
                   arg_const=np.array(acn, np.uint8) if (max_params > 0 or max_ext_args > 0) else None)


def c4(n_procs: int = 2000, **kw) -> Program:
    prm = dict(C4)
    prm.update(n_procs=n_procs)
    prm.update(kw)
    return program(item_seed(4, 0), **prm)
