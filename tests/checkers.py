"""Independent checkers that pin the oracle (no code shared with it).

* ``mop_nu`` / ``mop_valid``: meet-over-all-paths by explicit path
  enumeration on acyclic CFGs.  The data-flow problems are gen/kill, hence
  distributive, so the fixed point must equal the MOP solution.
* ``reach_after_dev`` / ``reach_before_dev``: boolean transitive closure.
* ``simulate_paths``: random walks with per-variable version counters in each
  memory space; every read must see the latest version and every copy must
  read from a space that holds it.
* ``check_invariants``: static safety, completeness and exclusivity.

Variables are handled as Python integers of n_vars bits, so every check is
written per path, not per word.
"""
from __future__ import annotations

from collections import deque
from typing import Dict, List, Sequence, Tuple

import numpy as np

KIND_LOOP_ENTRY = 2


def row_int(row: np.ndarray) -> int:
    v = 0
    for w, x in enumerate(row.tolist()):
        v |= int(x) << (64 * w)
    return v


def int_row(v: int, wd: int) -> np.ndarray:
    return np.array([(v >> (64 * w)) & ((1 << 64) - 1) for w in range(wd)], dtype=np.uint64)


def rows_int(a: np.ndarray) -> List[int]:
    return [row_int(a[i]) for i in range(a.shape[0])]


class View:
    """Big-int view of a CFG for path-level checks."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.nb = cfg.n_blocks
        self.full = (1 << cfg.n_vars) - 1
        self.R = rows_int(cfg.R.reshape(cfg.n_blocks, cfg.wd))
        self.W = rows_int(cfg.W.reshape(cfg.n_blocks, cfg.wd))
        evh, evd, lxh, lxd = cfg.boundary()
        self.ev = [row_int(evh), row_int(evd)]
        self.lx = [row_int(lxh), row_int(lxd)]
        self.space = [int(x) for x in cfg.space]
        # firstprivate variables: marked scalars no DEVICE block writes
        sc = getattr(cfg, "scalar", None)
        dev_w = 0
        for b in range(self.nb):
            if self.space[b] == 1:
                dev_w |= self.W[b]
        self.fp = (row_int(np.asarray(sc, dtype=np.uint64)) & ~dev_w & self.full) if sc is not None else 0
        self.succ: List[List[Tuple[int, int]]] = [[] for _ in range(self.nb)]
        for p in range(self.nb):
            for e in range(int(cfg.succ_ptr[p]), int(cfg.succ_ptr[p + 1])):
                self.succ[p].append((int(cfg.succ_idx[e]), e))
        self.entry, self.exit = cfg.entry, cfg.exit

    def use(self, s: int, b: int) -> int:
        """Reads of b that need the copy in space s (a kernel's read of a firstprivate
        variable needs the host copy: the kernel is launched with the host value)."""
        if b == self.exit:
            return self.lx[s]
        if self.space[b] == 1:
            return self.R[b] & ~self.fp if s == 1 else self.R[b] & self.fp
        return self.R[b] if s == 0 else 0

    def after(self, s: int, b: int, val: int) -> int:
        """Validity of the copy in space s after block b's own accesses (a write makes the
        other copy stale; a kernel leaves no valid device copy of a firstprivate it reads)."""
        w = self.W[b]
        val = (val | w) if self.space[b] == s else (val & ~w)
        if s == 1 and self.space[b] == 1:
            val &= ~(self.R[b] & self.fp)
        return val

    def paths_from(self, b: int) -> List[List[Tuple[int, int]]]:
        """All paths b -> EXIT as lists of (block, edge taken from it; -1 at EXIT)."""
        out = []

        def rec(x, acc):
            if x == self.exit:
                out.append(acc + [(x, -1)])
                return
            for (q, e) in self.succ[x]:
                rec(q, acc + [(x, e)])
        rec(b, [])
        return out

    def paths_to(self, q: int) -> List[List[Tuple[int, int]]]:
        """All paths ENTRY -> q as lists of (block, edge that entered it; -1 at ENTRY)."""
        out = []

        def rec(x, acc):
            if x == q:
                out.append(acc)
                return
            for (y, e) in self.succ[x]:
                rec(y, acc + [(y, e)])
        rec(self.entry, [(self.entry, -1)])
        return out


def mop_nu(cfg) -> Tuple[List[int], List[int]]:
    """Next use per space: some path from b to EXIT reads v in s before any
    write of v (reads of a block precede its writes), or reaches EXIT without
    a write while v is live in s after the region."""
    V = View(cfg)
    res = [[0] * V.nb, [0] * V.nb]
    for b in range(V.nb):
        for path in V.paths_from(b):
            for s in (0, 1):
                live, alive = 0, V.full
                for (x, _) in path:
                    live |= alive & V.use(s, x)
                    if x != V.exit:
                        alive &= ~V.W[x]
                res[s][b] |= live
    return res[0], res[1]


def mop_valid(cfg, gen_entry: Sequence[List[int]], gen_edge: Sequence[Dict[int, int]]) -> Tuple[List[int], List[int]]:
    """Must-validity at block entry over every ENTRY->q path.

    Along a path the copy in space s is valid after a write in s, stale after
    a write in the other space, and made valid by the gens: ``gen_entry[s][b]``
    just before block b and ``gen_edge[s][e]`` on edge e.  At ENTRY the
    validity is the boundary.
    """
    V = View(cfg)
    res = [[V.full] * V.nb, [V.full] * V.nb]
    for q in range(V.nb):
        for path in V.paths_to(q):
            for s in (0, 1):
                val = None
                for i, (x, e) in enumerate(path):
                    if i == 0:
                        val = V.ev[s]
                    else:
                        val = val | gen_edge[s].get(e, 0) | gen_entry[s][x]
                    if x == q:
                        break
                    val = V.after(s, x, val)
                res[s][q] &= val
    return res[0], res[1]


def closure(cfg) -> np.ndarray:
    """reach[a, b] = b is reachable from a by a path of >= 0 edges."""
    nb = cfg.n_blocks
    M = np.eye(nb, dtype=bool)
    for p in range(nb):
        for e in range(int(cfg.succ_ptr[p]), int(cfg.succ_ptr[p + 1])):
            M[p, int(cfg.succ_idx[e])] = True
    for k in range(nb):
        M = M | (M[:, k:k + 1] & M[k:k + 1, :])
    return M


def reach_labels(cfg) -> Tuple[np.ndarray, np.ndarray]:
    M = closure(cfg)
    dev = np.asarray(cfg.space) == 1
    after = (M[dev, :].any(axis=0)).astype(np.uint8)
    before = (M[:, dev].any(axis=1)).astype(np.uint8)
    return after, before


def check_invariants(cfg, res) -> List[str]:
    """Static checks of a placement (empty list = all hold).

    safety:       a copy into s on p->q needs o valid at the end of p
                  (after copies placed on p's own entry); a copy before q
                  needs o valid on every in-edge.
    completeness: every read (and the liveness after EXIT) is valid.
    exclusivity:  never a copy into both spaces at one location.
    """
    V = View(cfg)
    nb = V.nb
    wd = cfg.wd
    errs = []
    avf = [rows_int(res["avf_h"]), rows_int(res["avf_d"])]
    ie = [rows_int(res["ins_entry_h"]), rows_int(res["ins_entry_d"])]
    ig = [rows_int(res["ins_edge_h"].reshape(-1, wd)) if cfg.n_edges else [],
          rows_int(res["ins_edge_d"].reshape(-1, wd)) if cfg.n_edges else []]

    def out_valid(s, b):
        return V.after(s, b, avf[s][b])

    preds = cfg.preds()
    for p in range(nb):
        for (q, e) in V.succ[p]:
            for s in (0, 1):
                o = 1 - s
                if ig[s][e] & ~out_valid(o, p):
                    errs.append("safety edge %d space %d" % (e, s))
                if ig[0][e] & ig[1][e]:
                    errs.append("exclusive edge %d" % e)
    for q in range(nb):
        for s in (0, 1):
            o = 1 - s
            if ie[s][q]:
                src = V.full
                for (p, e) in preds[q]:
                    src &= out_valid(o, p) | ig[o][e]
                if q == V.entry:
                    src = V.ev[o]
                if ie[s][q] & ~src:
                    errs.append("safety entry %d space %d" % (q, s))
            if V.use(s, q) & ~avf[s][q]:
                errs.append("completeness block %d space %d" % (q, s))
        if ie[0][q] & ie[1][q]:
            errs.append("exclusive entry %d" % q)
    return errs


def simulate_paths(cfg, res, walks: int, seed: int, cap_factor: int = 50) -> Tuple[List[str], float]:
    """Random-path soundness check of a placement.

    Each walk picks successors uniformly (loops run a geometric number of
    times, including zero), is capped at cap_factor * n_blocks steps and
    then finishes along a shortest path to EXIT.  Versions: a write in x
    makes ``ver += 1; ver_x = ver``; a copy into s asserts ``ver_o == ver``
    and sets ``ver_s = ver``; a read in x asserts ``ver_x == ver``; at EXIT
    the live spaces must hold ``ver``.  Returns (errors, copies per walk).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nb, nv, wd = cfg.n_blocks, cfg.n_vars, cfg.wd
    V = View(cfg)

    def bits(v: int) -> np.ndarray:
        return np.array([(v >> i) & 1 for i in range(nv)], dtype=bool)

    R = [bits(x) for x in V.R]
    Wb = [bits(x) for x in V.W]
    FP = bits(V.fp)
    ie = [[bits(x) for x in rows_int(res["ins_entry_h"])], [bits(x) for x in rows_int(res["ins_entry_d"])]]
    ig = [[bits(x) for x in rows_int(res["ins_edge_h"].reshape(-1, wd))] if cfg.n_edges else [],
          [bits(x) for x in rows_int(res["ins_edge_d"].reshape(-1, wd))] if cfg.n_edges else []]
    ev = [bits(V.ev[0]), bits(V.ev[1])]
    lx = [bits(V.lx[0]), bits(V.lx[1])]
    # distance to EXIT for the finishing leg
    dist = [-1] * nb
    dist[V.exit] = 0
    rev: List[List[int]] = [[] for _ in range(nb)]
    for p in range(nb):
        for (q, _) in V.succ[p]:
            rev[q].append(p)
    dq = deque([V.exit])
    while dq:
        q = dq.popleft()
        for p in rev[q]:
            if dist[p] < 0:
                dist[p] = dist[q] + 1
                dq.append(p)
    errs: List[str] = []
    copies = 0
    for wk in range(walks):
        ver = np.zeros(nv, dtype=np.int64)
        vs = [np.where(ev[0], 0, -1).astype(np.int64), np.where(ev[1], 0, -1).astype(np.int64)]

        def copy(mask, s, where):
            nonlocal copies
            if not mask.any():
                return
            o = 1 - s
            bad = mask & (vs[o] != ver)
            if bad.any():
                errs.append("walk %d: stale copy source into space %d at %s, vars %s" % (wk, s, where, np.nonzero(bad)[0][:4].tolist()))
            vs[s] = np.where(mask, ver, vs[s])
            copies += int(mask.sum())

        b = V.entry
        steps = 0
        while True:
            for s in (0, 1):
                copy(ie[s][b], s, "entry %d" % b)
            if b == V.exit:
                for s in (0, 1):
                    bad = lx[s] & (vs[s] != ver)
                    if bad.any():
                        errs.append("walk %d: stale live-out in space %d, vars %s" % (wk, s, np.nonzero(bad)[0][:4].tolist()))
                break
            x = V.space[b]
            # a kernel reads a firstprivate variable from the host copy (its launch value)
            rfp = R[b] & FP if x == 1 else np.zeros(nv, dtype=bool)
            bad = (R[b] & ~rfp & (vs[x] != ver)) | (rfp & (vs[0] != ver))
            if bad.any():
                errs.append("walk %d: stale read in block %d space %d, vars %s" % (wk, b, x, np.nonzero(bad)[0][:4].tolist()))
            if Wb[b].any():
                ver = ver + Wb[b].astype(np.int64)
                vs[x] = np.where(Wb[b], ver, vs[x])
            if rfp.any():
                vs[1] = np.where(rfp, -1, vs[1])   # no valid device copy after the kernel
            steps += 1
            succ = V.succ[b]
            if steps < cap_factor * nb:
                q, e = succ[int(rng.integers(len(succ)))]
            else:
                q, e = min(succ, key=lambda t: dist[t[0]])
            for s in (0, 1):
                copy(ig[s][e], s, "edge %d" % e)
            b = q
        if len(errs) > 20:
            break
    return errs, copies / max(walks, 1)


# --------------------------------------------------------------------------
# interprocedural checks
# --------------------------------------------------------------------------
def _bitset(v: int, n: int) -> np.ndarray:
    return np.array([(v >> i) & 1 for i in range(n)], dtype=bool)


def _vars_of(row: np.ndarray) -> List[int]:
    v = row_int(row)
    out = []
    i = 0
    while v:
        if v & 1:
            out.append(i)
        v >>= 1
        i += 1
    return out


def inline_program(prog, root: int, demands: Dict[int, np.ndarray], cap_depth: int = -1):
    """Inline every call reached from ``root``.

    Each call block keeps its own accesses (plus the host reads that
    ``demands`` adds at that call site) and then branches into a fresh copy of
    the callee, whose EXIT branches to the call block's successors.  Globals
    (the first ``prog.n_globals`` variables) are shared; a pointer parameter
    of an inlined copy is the caller variable bound to it at that call site;
    every other local of the copy is a fresh variable, not live after the
    program, and a host block that writes them (and reads nothing) precedes
    the copy's ENTRY: each activation starts with new storage, valid on the
    host, that no earlier activation's accesses reach (a call in a loop
    re-enters the same copy).  Returns (cfg, instances, pos) where instances lists
    (procedure, call string, block offset, variable map) in creation order and
    ``pos`` maps an instance block id to its id in the returned CFG.

    With ``cap_depth >= 0`` a call made at that nesting depth is not expanded:
    a host block that writes every global and every argument (and reads
    none) stands in for it,
    so no next use crosses it.  Unrolling recursion this way gives the next
    use of the paths with at most ``cap_depth`` nested calls, a lower bound
    that grows to the exact solution."""
    import synth
    G = prog.n_globals
    site_at: Dict[Tuple[int, int], int] = {}
    for j in range(len(prog.call_proc)):
        site_at[(int(prog.call_proc[j]), int(prog.call_block[j]))] = j
    ap, av = getattr(prog, "arg_ptr", None), getattr(prog, "arg_var", None)

    def args(j):
        return [] if ap is None else [int(av[t]) for t in range(int(ap[j]), int(ap[j + 1]))]
    blocks: List[Tuple[int, List[int], List[int]]] = []
    edges: List[Tuple[int, int, int]] = []
    instances = []
    nvars = [G]

    def add(P: int, sigma: tuple, bound: List[int]) -> int:
        cfg = prog.procs[P]
        off = len(blocks)
        nfresh = cfg.n_vars - G - len(bound)
        vmap = list(range(G)) + list(bound) + list(range(nvars[0], nvars[0] + nfresh))
        nvars[0] += nfresh
        instances.append((P, sigma, off, vmap))
        fresh = vmap[G + len(bound):]
        R = cfg.R.reshape(cfg.n_blocks, cfg.wd)
        W = cfg.W.reshape(cfg.n_blocks, cfg.wd)
        for b in range(cfg.n_blocks):
            rd = set(_vars_of(R[b]))
            j = site_at.get((P, b))
            if j is not None and j in demands:
                rd |= set(_vars_of(demands[j]))
            blocks.append((int(cfg.space[b]), sorted(vmap[v] for v in rd), sorted(vmap[v] for v in _vars_of(W[b]))))
        for b in range(cfg.n_blocks):
            outs = [(int(cfg.succ_idx[e]) + off, int(cfg.edge_kind[e]))
                    for e in range(int(cfg.succ_ptr[b]), int(cfg.succ_ptr[b + 1]))]
            j = site_at.get((P, b))
            if j is not None:
                q = int(prog.callee[j])
                assert q >= 0, "inlining needs every callee's body"
                if len(sigma) == cap_depth:
                    cap = len(blocks)
                    blocks.append((0, [], sorted(set(range(G)) | {vmap[v] for v in args(j)})))
                    edges.append((b + off, cap, 0))
                    for (t, k) in outs:
                        edges.append((cap, t, k))
                    continue
                kill = len(blocks)
                blocks.append((0, [], []))
                qoff, qfresh = add(q, sigma + (j,), [vmap[v] for v in args(j)])
                blocks[kill] = (0, [], sorted(qfresh))
                qc = prog.procs[q]
                edges.append((b + off, kill, 0))
                edges.append((kill, qc.entry + qoff, 0))
                for (t, k) in outs:
                    edges.append((qc.exit + qoff, t, k))
            else:
                for (t, k) in outs:
                    edges.append((b + off, t, k))
        return off, fresh

    add(root, (), [])
    rc = prog.procs[root]
    nb = len(blocks)
    order = [rc.entry] + [b for b in range(nb) if b not in (rc.entry, rc.exit)] + [rc.exit]
    pos = {b: i for i, b in enumerate(order)}
    cfg, _ = synth.from_edges([blocks[b] for b in order], [(pos[s], pos[d], k) for (s, d, k) in edges], nvars[0])
    lx = synth.var_mask(nvars[0]).copy()
    nroot = rc.n_vars
    for v in range(nroot, nvars[0]):
        lx[v >> 6] &= ~np.uint64(1 << (v & 63))
    cfg.exit_live_h = lx
    return cfg, instances, pos


class _CtxBits:
    """Per-context placement as boolean rows, built on first use."""

    def __init__(self, cfg, res):
        nv, wd = cfg.n_vars, cfg.wd
        self.ie = [[_bitset(x, nv) for x in rows_int(res[k].reshape(-1, wd))] for k in ("ins_entry_h", "ins_entry_d")]
        self.ig = [[_bitset(x, nv) for x in rows_int(res[k].reshape(-1, wd))] if cfg.n_edges else []
                   for k in ("ins_edge_h", "ins_edge_d")]


def simulate_program(prog, ctx, results, demands: Dict[int, np.ndarray], walks: int, seed: int,
                     max_steps: int = 3000, max_depth: int = 30) -> Tuple[List[str], int]:
    """Random walks over a whole program, checking the per-context placements.

    Data lives in cells, each with a version and, per memory space, the
    version its copy holds: the globals' cells are shared by all frames, an
    activation gets fresh cells for its locals (valid in the space it runs in), and a
    pointer parameter names the cell of the caller variable bound to it (so
    one datum may have several names).  A call block runs its own accesses
    (and the host reads that ``demands`` adds there), then the callee from
    ENTRY to EXIT in the context named by the last two call sites, then the
    caller takes a successor.  An external callee reads every global and its
    arguments on the host and writes them there (but the const globals and
    the pointer-to-const arguments).  A call made inside a kernel
    (``prog.call_space``) runs the callee on the device: a walk through it
    (and whatever it calls) in which every read must see a current device
    copy and every write makes the device copy the only current one; no copy
    fires inside it.  Copies placed in the running context fire as walked;
    every read, and every copy's source, must hold the latest version; at
    the program's exit the live copies must be current.  A walk that exceeds
    ``max_steps`` or ``max_depth`` stops where it is (everything it did so
    far was checked).  Returns (violations, walks cut short)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    G = prog.n_globals
    nc = len(prog.call_proc)
    site_at: Dict[Tuple[int, int], int] = {}
    for j in range(nc):
        site_at[(int(prog.call_proc[j]), int(prog.call_block[j]))] = j
    cspace = getattr(prog, "call_space", None)
    cspace = np.zeros(nc, np.uint8) if cspace is None else np.asarray(cspace)
    cg = getattr(prog, "const_globals", None)
    const = _bitset(row_int(np.asarray(cg, np.uint64)), G) if cg is not None else np.zeros(G, bool)
    npar = getattr(prog, "n_params", None)
    npar = [0] * len(prog.procs) if npar is None else [int(x) for x in npar]
    ap, av, ac = getattr(prog, "arg_ptr", None), getattr(prog, "arg_var", None), getattr(prog, "arg_const", None)

    def args(j):
        if ap is None:
            return []
        return [(int(av[t]), bool(ac[t]) if ac is not None else False) for t in range(int(ap[j]), int(ap[j + 1]))]
    views: Dict[int, View] = {}
    rw: Dict[int, Tuple[list, list]] = {}
    bits: Dict[tuple, _CtxBits] = {}
    dem = {j: _bitset(row_int(m), prog.procs[int(prog.call_proc[j])].n_vars) for j, m in demands.items()}

    def view(P):
        if P not in views:
            V = View(prog.procs[P])
            views[P] = V
            rw[P] = ([_bitset(x, V.cfg.n_vars) for x in V.R], [_bitset(x, V.cfg.n_vars) for x in V.W])
        return views[P]

    def cbits(key):
        if key not in bits:
            bits[key] = _CtxBits(prog.procs[key[0]], results[key])
        return bits[key]

    errs: List[str] = []
    cut = 0
    for wk in range(walks):
        root = prog.roots[int(rng.integers(len(prog.roots)))]
        rv = view(root)
        nv0 = rv.cfg.n_vars
        ev = [_bitset(rv.ev[0], nv0), _bitset(rv.ev[1], nv0)]
        # cells: version and per space the version held (-1: never valid)
        ver: List[int] = [0] * G
        hold = [[0 if ev[s][v] else -1 for v in range(G)] for s in (0, 1)]
        counter = [1]

        def new_cell(valid_h: bool, valid_d: bool) -> int:
            ver.append(0)
            hold[0].append(0 if valid_h else -1)
            hold[1].append(0 if valid_d else -1)
            return len(ver) - 1

        def frame(P, key, cells_of_params, on_device=False):
            n = prog.procs[P].n_vars
            cell = list(range(G)) + [0] * (n - G)
            for i in range(n - G):
                if i < len(cells_of_params):
                    cell[G + i] = cells_of_params[i]
                elif P == root and key == (root, ()):
                    cell[G + i] = new_cell(bool(ev[0][G + i]), bool(ev[1][G + i]))
                else:
                    cell[G + i] = new_cell(not on_device, on_device)
            return dict(P=P, key=key, b=prog.procs[P].entry, after=False, cell=cell)

        def bump(c):
            ver[c] = counter[0]
            counter[0] += 1

        def read(c, s, what):
            if hold[s][c] != ver[c]:
                errs.append("walk %d: stale %s (cell %d, space %d)" % (wk, what, c, s))

        def write(c, s):
            bump(c)
            hold[s][c] = ver[c]

        def copy(c, s, what):
            if hold[1 - s][c] != ver[c]:
                errs.append("walk %d: stale copy source into space %d at %s (cell %d)" % (wk, s, what, c))
            hold[s][c] = ver[c]

        def device_call(q, cells_of_args, consts, depth):
            """The callee q run on the device (an external one: every global and its arguments)."""
            if q < 0:
                for c in list(range(G)) + list(cells_of_args):
                    read(c, 1, "device external read")
                for c in range(G):
                    if not const[c]:
                        write(c, 1)
                for c, k in zip(cells_of_args, consts):
                    if not k:
                        write(c, 1)
                return
            Vq = view(q)
            Rq, Wq = rw[q]
            fq = frame(q, None, cells_of_args, on_device=True)
            bq, n = Vq.entry, 0
            while bq != Vq.exit and n < max_steps and depth < max_depth:
                for v in np.nonzero(Rq[bq])[0]:
                    read(fq["cell"][v], 1, "device function %d read in block %d" % (q, bq))
                for v in np.nonzero(Wq[bq])[0]:
                    write(fq["cell"][v], 1)
                jj = site_at.get((q, bq))
                if jj is not None:
                    aa = args(jj)
                    device_call(int(prog.callee[jj]), [fq["cell"][x] for x, _ in aa], [k for _, k in aa], depth + 1)
                sq = Vq.succ[bq]
                bq = sq[int(rng.integers(len(sq)))][0]
                n += 1

        stack = [frame(root, (root, ()), [])]
        steps = 0
        while stack and len(errs) <= 20:
            fr = stack[-1]
            P, key, b = fr["P"], fr["key"], fr["b"]
            V = view(P)
            Rb, Wb = rw[P]
            cb = cbits(key)
            cell = fr["cell"]
            if not fr["after"]:
                for s in (0, 1):
                    for v in np.nonzero(cb.ie[s][b])[0]:
                        copy(cell[v], s, "%s entry of %d" % (key, b))
                if b == V.exit:
                    if len(stack) == 1:
                        for s in (0, 1):
                            for v in np.nonzero(_bitset(V.lx[s], V.cfg.n_vars))[0]:
                                read(cell[v], s, "live-out")
                    stack.pop()
                    continue
                x = V.space[b]
                j = site_at.get((P, b))
                rd = Rb[b] | dem[j] if j is not None and j in dem else Rb[b]
                for v in np.nonzero(rd)[0]:
                    read(cell[v], x, "%s read in block %d" % (key, b))
                for v in np.nonzero(Wb[b])[0]:
                    write(cell[v], x)
                fr["after"] = True
                if j is not None and cspace[j]:
                    aa = args(j)
                    device_call(int(prog.callee[j]), [cell[v] for v, _ in aa], [k for _, k in aa], len(stack))
                    j = None
                if j is not None:
                    q = int(prog.callee[j])
                    aa = args(j)
                    if q < 0:
                        for c in list(range(G)) + [cell[v] for v, _ in aa]:
                            read(c, 0, "%s external call at %d" % (key, b))
                        for c in range(G):
                            if not const[c]:
                                write(c, 0)
                        for v, k in aa:
                            if not k:
                                write(cell[v], 0)
                    else:
                        if len(stack) >= max_depth or steps >= max_steps:
                            cut += 1
                            break
                        stack.append(frame(q, (q, (key[1] + (j,))[-2:]), [cell[v] for v, _ in aa]))
                        continue
            steps += 1
            if steps >= max_steps:
                cut += 1
                break
            succ = V.succ[b]
            t, e = succ[int(rng.integers(len(succ)))]
            for s in (0, 1):
                for v in np.nonzero(cb.ig[s][e])[0]:
                    copy(cell[v], s, "%s edge %d" % (key, e))
            fr["b"] = t
            fr["after"] = False
    return errs, cut
