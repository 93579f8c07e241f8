"""ORACLE — test infrastructure only: the interprocedural driver.

Follows the interprocedural section of the paper (side effects of a call on
global variables, read or write, host or device; repeat over the functions
up to the maximum call depth and stop early when nothing changes; external
functions are treated pessimistically), made exact for the bit-vector
problems of ``oracle.c``:

* Bottom-up over the strongly connected components of the call graph
  (callees first), each procedure Q gets, per global variable and memory
  space, its exact transfer functions: next use at Q's entry for exit
  liveness 0 and 1 (NU0, NU1), validity at Q's exit for the four
  (entry valid, exit live) combinations (T), and flow-insensitive may-read /
  may-write bits, transitively over callees (MAYR, MAYW).  Inside a
  recursive component the next-use summaries iterate from 0, then the
  validity tables from all-ones, then the may bits from 0, until no bit
  changes.  Each problem is gen/kill per bit, so two (resp. four) boundary
  evaluations define the function exactly.
* Top-down, contexts are (procedure, last two call sites).  Solving a
  context gives, at each call site, the caller's next use after the call
  (exit liveness of the callee) and the validity after the call block's own
  accesses under eager copies (entry validity of the callee).  Several calls
  that reach one context meet: liveness by OR, validity by AND.  Next use
  grows with exit liveness and eager validity shrinks with entry validity,
  so the exit liveness of every context is one least fixed point and, given
  it, the entry validity one greatest fixed point: any order of the context
  solves reaches them.  A global that the AND leaves valid in neither space
  (host-fresh and device-fresh callers meeting) and that the context reads
  before writing it is demanded as a host read at the call site that leads
  to the context (the last of its call string), unless a calling context
  lacks that global at its own entry (its demand comes first); a global the
  context never reads may stay valid nowhere.  Demands feed back into the
  summaries, and the whole computation repeats until no demand changes.
* The validity tables describe the callee under eager copies; a context's
  final placement delays copies and can leave a copy stale at the callee's
  exit where the eager one would be current.  So when a context is solved,
  each of its calls is capped by the validity at EXIT, under the final
  placement, of the callee context that the call leads to: the caller's
  validity after the call is the table's value ANDed with that cap.  The
  callee keeps valid at its exit whatever the caller reads next (its exit
  liveness), so a cap never removes a needed copy.  Caps are taken afresh
  from the latest context solutions, and the whole computation repeats
  until neither the demands nor the caps change.

External callees (index -1): may read and write every global on the host,
need every global on the host on entry, leave the host copy valid and the
device copy stale.

Two refinements of the model (the interprocedural section: accesses on the
host or the device, and the read-only rule for data behind a pointer to
``const``):

* A call made inside a kernel (``call_space[j] = 1``, a device function) runs
  on the device: the call block is a DEVICE block that reads every global
  the callee may read or write (in either space) and writes every global it
  may write; such a call gets no context of its own (a device function
  carries no mapping directives) and no summary table.  An external device
  function may read and write every global.
* Globals marked ``const_globals`` are never written: no block may write
  them, and an external callee neither writes them nor leaves their device
  copy stale.

By-reference pointer parameters ("data at the address of pointer
parameters"): procedure Q's first ``n_params[Q]`` locals (variables
[G, G + n_params[Q])) are its pointer parameters, and call site j binds them
to caller variables (``arg_var[arg_ptr[j]:arg_ptr[j + 1]]``).  A procedure's
summary covers its globals and its parameters (its shared variables); at a
call site the callee's row of parameter i applies to the caller variable it
is bound to, combined with any other row that reaches that variable (the
global's own, another parameter's): may and next-use rows by OR, validity
tables by AND.  A callee context's boundary takes, for parameter i, the
caller's facts on the bound variable, and its gaps and caps map back the
same way.  The callee is solved name by name, so a host call's arguments
must be distinct locals of the caller (no global, no repeat): then no frame
sees one datum under two names.  A call made inside a kernel may bind any
caller variables, repeats and globals included, since only its may rows
cross it.  An external callee may take arguments too: it reads them on the
host and writes them there unless the argument is a pointer to const
(``arg_const``).
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

from . import (SUM_MAYR_D, SUM_MAYR_H, SUM_MAYW_D, SUM_MAYW_H, SUM_NU0_D, SUM_NU0_H, SUM_NU1_D,
               SUM_NU1_H, SUM_ROWS, SUM_TD_00, SUM_TH_00, solve)

SUMMARY_MODE = 1 << 8


def _gmask(n_globals: int, wd: int) -> np.ndarray:
    m = np.zeros(wd, np.uint64)
    for w in range(wd):
        lo = 64 * w
        if n_globals >= lo + 64:
            m[w] = np.uint64((1 << 64) - 1)
        elif n_globals > lo:
            m[w] = np.uint64((1 << (n_globals - lo)) - 1)
    return m


def _vmask(nv: int, wd: int) -> np.ndarray:
    return _gmask(nv, wd)


def tarjan(n: int, succ: List[List[int]]) -> List[List[int]]:
    """Strongly connected components, in reverse topological order of the
    condensation (a component is listed after every component it calls)."""
    index = [-1] * n
    low = [0] * n
    on = [False] * n
    st: List[int] = []
    out: List[List[int]] = []
    counter = [0]
    for root in range(n):
        if index[root] >= 0:
            continue
        work = [(root, 0)]
        while work:
            v, i = work.pop()
            if i == 0:
                index[v] = low[v] = counter[0]
                counter[0] += 1
                st.append(v)
                on[v] = True
            recurse = False
            while i < len(succ[v]):
                w = succ[v][i]
                i += 1
                if index[w] < 0:
                    work.append((v, i))
                    work.append((w, 0))
                    recurse = True
                    break
                if on[w]:
                    low[v] = min(low[v], index[w])
            if recurse:
                continue
            if low[v] == index[v]:
                comp = []
                while True:
                    w = st.pop()
                    on[w] = False
                    comp.append(w)
                    if w == v:
                        break
                out.append(comp)
            if work:
                u, _ = work[-1]
                low[u] = min(low[u], low[v])
    return out


class Summary:
    """Per-procedure summary over the globals: rows [16][words of globals]."""

    def __init__(self, gw: int):
        self.rows = np.zeros((SUM_ROWS, gw), np.uint64)


def external_summary(gm: np.ndarray, const=None) -> np.ndarray:
    c = np.zeros(gm.size, np.uint64) if const is None else (np.asarray(const, np.uint64)[:gm.size] & gm)
    r = np.zeros((SUM_ROWS, gm.size), np.uint64)
    for k in (SUM_MAYR_H, SUM_NU0_H, SUM_NU1_H, SUM_NU1_D):
        r[k] = gm
    r[SUM_MAYW_H] = gm & ~c                 # a const global is never written
    for k in range(4):
        r[SUM_TH_00 + k] = gm               # host copy valid after the call
        r[SUM_TD_00 + k] = c if k >= 2 else 0   # device copy stale after the call, but a const one kept
    return r


class ProgramOracle:
    def __init__(self, prog, placement: int = 0):
        """``placement``: 0 delayed copies (the method), 1 eager copies only
        (every solve of the driver materialises each eager copy)."""
        self.p = prog
        self.placement = placement
        self.n = len(prog.procs)
        self.G = prog.n_globals
        gw = (self.G + 63) // 64
        nc = len(prog.call_proc)
        cs = getattr(prog, "call_space", None)
        self.call_space = np.zeros(nc, np.uint8) if cs is None else np.asarray(cs, np.uint8)
        cg = getattr(prog, "const_globals", None)
        self.const = np.zeros(gw, np.uint64) if cg is None else (np.asarray(cg, np.uint64)[:gw] & _gmask(self.G, gw))
        self.sites: List[List[int]] = [[] for _ in range(self.n)]      # host call-site ids per caller
        self.dsites: List[List[int]] = [[] for _ in range(self.n)]     # device call-site ids per caller
        for j in range(nc):
            P, b = int(prog.call_proc[j]), int(prog.call_block[j])
            dev = bool(self.call_space[j])
            if int(prog.procs[P].space[b]) != int(dev):
                raise ValueError("call site %d: its block's space is not the call's" % j)
            (self.dsites if dev else self.sites)[P].append(j)
        for P, c in enumerate(prog.procs):
            if (np.asarray(c.W, np.uint64)[:, :gw] & self.const).any():
                raise ValueError("procedure %d writes a const global" % P)
        npar = getattr(prog, "n_params", None)
        self.np = [0] * self.n if npar is None else [int(x) for x in npar]
        ap = getattr(prog, "arg_ptr", None)
        av = getattr(prog, "arg_var", None)
        ac = getattr(prog, "arg_const", None)
        self.args: List[List[Tuple[int, bool]]] = []
        for j in range(nc):
            a = [] if ap is None else [(int(av[t]), bool(ac[t]) if ac is not None else False)
                                       for t in range(int(ap[j]), int(ap[j + 1]))]
            q, P = int(prog.callee[j]), int(prog.call_proc[j])
            if q >= 0 and len(a) != self.np[q]:
                raise ValueError("call site %d binds %d arguments to %d parameters" % (j, len(a), self.np[q]))
            if any(not (0 <= x < prog.procs[P].n_vars) for x, _ in a):
                raise ValueError("call site %d: argument is not a caller variable" % j)
            if q >= 0 and not self.call_space[j] and (len(set(x for x, _ in a)) < len(a)
                                                      or any(x < self.G for x, _ in a)):
                raise ValueError("call site %d: a host call's arguments must be distinct locals" % j)
            self.args.append(a)
        for P, c in enumerate(prog.procs):
            if self.G + self.np[P] > c.n_vars:
                raise ValueError("procedure %d has more parameters than locals" % P)
        self.demand: Dict[int, np.ndarray] = {}                          # call site -> host-read mask (caller words)
        self.cap: Dict[tuple, Tuple[np.ndarray, np.ndarray]] = {}        # callee context -> (host, device) validity at EXIT
        self.sum_rows: Dict[int, np.ndarray] = {}
        self.nowhere: Dict[tuple, np.ndarray] = {}                       # last contexts(): globals valid nowhere
        self.visits = 0

    # -- shared variables and argument bindings ---------------------------------------
    def shared(self, P: int) -> int:
        """Number of P's shared variables: the globals, then its pointer parameters."""
        return self.G + self.np[P]

    def _smask(self, P: int, wd: int) -> np.ndarray:
        return _vmask(self.shared(P), wd)

    def _rows(self, j: int, q: int, summaries) -> np.ndarray:
        """The callee side of call site j: q's summary rows over its shared variables, or an
        external callee's rows over the globals and, past them, its arguments."""
        if q >= 0:
            return summaries[q]
        gw = (self.G + 63) // 64
        return external_summary(_gmask(self.G, gw), self.const)

    def _sources(self, j: int, q: int):
        """(caller variable, callee row index or None for an external argument, const) for
        every argument of call site j."""
        return [(x, (self.G + i) if q >= 0 else None, c) for i, (x, c) in enumerate(self.args[j])]

    # -- call tables in a caller's variable layout ------------------------------------
    def _caller_tables(self, P: int, summaries: Dict[int, np.ndarray], sigma=None):
        cfg = self.p.procs[P]
        wd = cfg.wd
        gw = (self.G + 63) // 64
        gm = _gmask(self.G, wd)
        vm = _vmask(cfg.n_vars, wd)
        call = np.full(cfg.n_blocks, -1, np.int32)
        sums = np.zeros((max(len(self.sites[P]), 1), SUM_ROWS, wd), np.uint64)
        OR_ROWS = list(range(SUM_MAYR_H, SUM_NU1_D + 1))
        T_ROWS = list(range(SUM_TH_00, SUM_TD_00 + 4))
        for k, j in enumerate(self.sites[P]):
            call[int(self.p.call_block[j])] = k
            q = int(self.p.callee[j])
            rows = self._rows(j, q, summaries)
            ckey = None if (sigma is None or q < 0) else (q, (tuple(sigma) + (j,))[-2:])
            cap = self.cap.get(ckey)
            # identity for every caller variable (NU1 = 1, T[e][l] = e), then the globals' rows
            s = np.zeros((SUM_ROWS, wd), np.uint64)
            for r in (SUM_NU1_H, SUM_NU1_D, SUM_TH_00 + 2, SUM_TH_00 + 3, SUM_TD_00 + 2, SUM_TD_00 + 3):
                s[r] = vm & ~gm
            s[:, :gw] |= rows[:, :gw] & gm[:gw]
            if cap is not None:
                for k4 in range(4):
                    s[SUM_TH_00 + k4, :gw] &= cap[0][:gw] | ~gm[:gw]
                    s[SUM_TD_00 + k4, :gw] &= cap[1][:gw] | ~gm[:gw]
            # arguments: the row of the parameter (or of an external argument) applies to the bound
            # caller variable, combined with whatever already reaches it
            seen = set(range(self.G))
            for (x, src, const) in self._sources(j, q):
                col = np.zeros(SUM_ROWS, bool)
                if src is not None:
                    for r in range(SUM_ROWS):
                        col[r] = bool((int(rows[r][src >> 6]) >> (src & 63)) & 1)
                    if cap is not None:
                        ch = bool((int(cap[0][src >> 6]) >> (src & 63)) & 1)
                        cd = bool((int(cap[1][src >> 6]) >> (src & 63)) & 1)
                        for k4 in range(4):
                            col[SUM_TH_00 + k4] &= ch
                            col[SUM_TD_00 + k4] &= cd
                else:   # an external argument: read on the host, written there unless const
                    for r in (SUM_MAYR_H, SUM_NU0_H, SUM_NU1_H, SUM_NU1_D):
                        col[r] = True
                    col[SUM_MAYW_H] = not const
                    for k4 in range(4):
                        col[SUM_TH_00 + k4] = True
                        col[SUM_TD_00 + k4] = const and k4 >= 2
                bit = np.uint64(1 << (x & 63))
                w = x >> 6
                if x in seen:
                    for r in OR_ROWS:
                        if col[r]:
                            s[r, w] |= bit
                    for r in T_ROWS:
                        if not col[r]:
                            s[r, w] &= ~bit
                else:
                    for r in range(SUM_ROWS):
                        s[r, w] = (s[r, w] | bit) if col[r] else (s[r, w] & ~bit)
                    seen.add(x)
            sums[k] = s
        return call, sums

    def _to_caller(self, j: int, q: int, row: np.ndarray, P: int) -> np.ndarray:
        """A row over callee q's shared variables (an external callee: its rows over the
        globals and arguments) moved to caller P's layout through the bindings of site j
        (OR where several reach one caller variable)."""
        cfg = self.p.procs[P]
        gw = (self.G + 63) // 64
        out = np.zeros(cfg.wd, np.uint64)
        out[:gw] = row[:gw] & _gmask(self.G, gw)
        for (x, src, _) in self._sources(j, q):
            if src is not None and (int(row[src >> 6]) >> (src & 63)) & 1:
                out[x >> 6] |= np.uint64(1 << (x & 63))
        return out

    def _cfg_with_demands(self, P: int, S):
        """P's read and write rows with the host reads demanded at its call blocks and, at each
        device call block, the variables the callee may read and write (either space), moved to
        P's layout (an external device function: every global and its arguments)."""
        cfg = self.p.procs[P]
        R, W = cfg.R, cfg.W
        dem = [(int(self.p.call_block[j]), self.demand[j]) for j in self.sites[P] if j in self.demand]
        if dem or self.dsites[P]:
            R, W = R.copy(), W.copy()
            for blk, m in dem:
                R[blk] |= m
            gw = (self.G + 63) // 64
            gm = _gmask(self.G, gw)
            for j in self.dsites[P]:
                q, blk = int(self.p.callee[j]), int(self.p.call_block[j])
                if q < 0:
                    rd = np.zeros(cfg.wd, np.uint64)
                    rd[:gw] = gm
                    wr = rd.copy()
                    wr[:gw] &= ~self.const
                    for (x, _, const) in self._sources(j, q):
                        rd[x >> 6] |= np.uint64(1 << (x & 63))
                        if not const:
                            wr[x >> 6] |= np.uint64(1 << (x & 63))
                else:
                    rows = S[q]
                    w_any = rows[SUM_MAYW_H] | rows[SUM_MAYW_D]
                    r_any = rows[SUM_MAYR_H] | rows[SUM_MAYR_D] | w_any
                    rd = self._to_caller(j, q, r_any, P)
                    wr = self._to_caller(j, q, w_any, P)
                R[blk] |= rd
                W[blk] |= wr
        return cfg, R, W

    def _solve(self, P, summaries, boundary, summary_mode=False, sigma=None):
        cfg, R, W = self._cfg_with_demands(P, summaries)
        call, sums = self._caller_tables(P, summaries, sigma)
        view = type(cfg)(n_blocks=cfg.n_blocks, n_vars=cfg.n_vars, succ_ptr=cfg.succ_ptr, succ_idx=cfg.succ_idx,
                         edge_kind=cfg.edge_kind, space=cfg.space, R=R, W=W, entry=cfg.entry, exit=cfg.exit)
        self.visits += 1
        res = solve(view, placement=(SUMMARY_MODE if summary_mode else 0) | self.placement,
                    call=call if self.sites[P] else None, sums=sums if self.sites[P] else None,
                    boundary=boundary)
        return view, call, sums, res

    # -- bottom-up ----------------------------------------------------------------
    def summarize(self) -> Dict[int, np.ndarray]:
        n, G = self.n, self.G
        gw = (G + 63) // 64
        succ = [[] for _ in range(n)]
        for j in range(len(self.p.call_proc)):
            q = int(self.p.callee[j])
            if q >= 0:
                succ[int(self.p.call_proc[j])].append(q)
        comps = tarjan(n, succ)
        # a component is recursive when it has several members or a call to itself
        S: Dict[int, np.ndarray] = {}
        for comp in comps:
            if len(comp) == 1 and comp[0] not in succ[comp[0]]:
                # not recursive: every callee is final, one evaluation is exact
                q = comp[0]
                S[q] = self._evaluate(q, S)
                S[q][:4] = self._may(q, S)
                continue
            for q in comp:
                sw = (self.shared(q) + 63) // 64
                r = np.zeros((SUM_ROWS, sw), np.uint64)
                for k in range(4):
                    r[SUM_TH_00 + k] = self._smask(q, sw)
                    r[SUM_TD_00 + k] = self._smask(q, sw)
                S[q] = r
            # may bits from 0 (device calls read them into the callers' rows), then next use
            # from 0, then validity tables from all-ones
            while True:
                changed = False
                for q in comp:
                    m = self._may(q, S)
                    if not np.array_equal(S[q][:4], m):
                        S[q][:4] = m
                        changed = True
                if not changed:
                    break
            for stage in ("nu", "t"):
                while True:
                    changed = False
                    for q in comp:
                        new = self._evaluate(q, S)
                        rows = list(range(SUM_NU0_H, SUM_NU1_D + 1)) if stage == "nu" else \
                            list(range(SUM_TH_00, SUM_TD_00 + 4))
                        if not np.array_equal(S[q][rows], new[rows]):
                            S[q][rows] = new[rows]
                            changed = True
                    if not changed:
                        break
        self.sum_rows = S
        return S

    def _evaluate(self, Q: int, S) -> np.ndarray:
        """NU0/NU1 and the four T tables of Q, over its shared variables (globals and
        parameters), from four boundary evaluations."""
        cfg = self.p.procs[Q]
        wd = cfg.wd
        gw = (self.shared(Q) + 63) // 64
        gm = self._smask(Q, wd)
        lm = _vmask(cfg.n_vars, wd) & ~gm
        out = np.zeros((SUM_ROWS, gw), np.uint64)
        for eps in (0, 1):
            for ell in (0, 1):
                ev_h = (gm if eps else 0) | lm
                ev_d = gm if eps else np.zeros(wd, np.uint64)
                lx = gm if ell else np.zeros(wd, np.uint64)
                _, _, _, res = self._solve(Q, S, (np.asarray(ev_h, np.uint64), np.asarray(ev_d, np.uint64),
                                                  lx.copy(), lx.copy()), summary_mode=True)
                if eps == 0:
                    base = SUM_NU1_H if ell else SUM_NU0_H
                    out[base] = res["nu_h"][cfg.entry][:gw] & gm[:gw]
                    out[base + 1] = res["nu_d"][cfg.entry][:gw] & gm[:gw]
                out[SUM_TH_00 + 2 * eps + ell] = res["ave_h"][cfg.exit][:gw] & gm[:gw]
                out[SUM_TD_00 + 2 * eps + ell] = res["ave_d"][cfg.exit][:gw] & gm[:gw]
        return out

    def _may(self, Q: int, S) -> np.ndarray:
        """May-read / may-write rows of Q over its shared variables: its own blocks (reads
        including the demanded ones, and device calls' rows) and its host calls' callees,
        through the argument bindings."""
        cfg, R, W = self._cfg_with_demands(Q, S)
        gw = (self.shared(Q) + 63) // 64
        gm = self._smask(Q, gw)
        m = np.zeros((4, gw), np.uint64)
        dev = np.asarray(cfg.space) == 1
        if (~dev).any():
            m[0] = np.bitwise_or.reduce(R[~dev][:, :gw], axis=0)
            m[2] = np.bitwise_or.reduce(W[~dev][:, :gw], axis=0)
        if dev.any():
            m[1] = np.bitwise_or.reduce(R[dev][:, :gw], axis=0)
            m[3] = np.bitwise_or.reduce(W[dev][:, :gw], axis=0)
        G = self.G
        ggw = (G + 63) // 64
        for j in self.sites[Q]:
            q = int(self.p.callee[j])
            if q < 0:
                rows = external_summary(_gmask(G, ggw), self.const)
                m[:, :ggw] |= rows[:4]
                for (x, _, const) in self._sources(j, q):
                    if x < self.shared(Q):
                        b = np.uint64(1 << (x & 63))
                        m[SUM_MAYR_H, x >> 6] |= b
                        if not const:
                            m[SUM_MAYW_H, x >> 6] |= b
            else:
                for r in range(4):
                    m[r] |= self._to_caller(j, q, S[q][r], Q)[:gw]
        return m & gm

    # -- top-down -------------------------------------------------------------------
    def context_graph(self):
        """Contexts reachable from the roots and the call edges between them:
        {key: [(site, callee key), ...]} with key = (procedure, last <= 2 sites)."""
        out: Dict[Tuple[int, tuple], List[Tuple[int, Tuple[int, tuple]]]] = {}
        todo = [(r, ()) for r in self.p.roots]
        while todo:
            key = todo.pop()
            if key in out:
                continue
            P, sigma = key
            edges = []
            for j in self.sites[P]:
                q = int(self.p.callee[j])
                if q >= 0:
                    nk = (q, (sigma + (j,))[-2:])
                    edges.append((j, nk))
                    todo.append(nk)
            out[key] = edges
        return out

    def _call_values(self, P, cfg, res, j):
        """What call site j of a solved context of P gives its callee: the
        validity after the call block's own accesses under eager copies, and
        the next use after the call (successor entries), over the globals."""
        c = int(self.p.call_block[j])
        w = cfg.W[c]
        a1_h = res["ave_h"][c] | w
        a1_d = res["ave_d"][c] & ~w
        l_h = np.zeros(cfg.wd, np.uint64)
        l_d = np.zeros(cfg.wd, np.uint64)
        for e in range(int(cfg.succ_ptr[c]), int(cfg.succ_ptr[c + 1])):
            t = int(cfg.succ_idx[e])
            l_h |= res["nu_h"][t]
            l_d |= res["nu_d"][t]
        return a1_h, a1_d, l_h, l_d

    def _iterate(self, graph, keys, value, contrib, meet, identity, schedule):
        """Chaotic iteration of one monotone boundary system over the context
        graph: the value of a non-root context is the meet, over its incoming
        call edges, of the latest contribution of each (identity while the
        caller is unsolved); roots keep theirs.  ``contrib(key, bnd)`` solves a
        context and returns {(site, callee key): contribution}.  Every schedule
        reaches the same fixed point because the contributions move one way."""
        into: Dict[Tuple[int, tuple], List[Tuple[Tuple[int, tuple], int]]] = {k: [] for k in keys}
        for k in keys:
            for (j, nk) in graph[k]:
                into[nk].append((k, j))
        latest: Dict[Tuple[Tuple[int, tuple], int], np.ndarray] = {}

        def recompute(nk):
            v = identity(nk)
            for (k, j) in into[nk]:
                if (k, j) in latest:
                    v = meet(v, latest[(k, j)])
            return v

        order = sorted(keys)
        if schedule == "rounds":
            dirty = order
            while dirty:
                touched = set()
                for k in dirty:
                    for (j, nk), v in contrib(k, value[k]).items():
                        latest[(k, j)] = v
                        touched.add(nk)
                dirty = []
                for nk in sorted(touched):
                    if nk[1] == () and nk[0] in self.roots_set:
                        continue
                    v = recompute(nk)
                    if any(not np.array_equal(a, b) for a, b in zip(v, value[nk])):
                        value[nk] = v
                        dirty.append(nk)
        elif schedule in ("fifo", "lifo"):
            queue = list(order) if schedule == "fifo" else list(reversed(order))
            queued = set(queue)
            while queue:
                k = queue.pop(0) if schedule == "fifo" else queue.pop()
                queued.discard(k)
                for (j, nk), v in contrib(k, value[k]).items():
                    latest[(k, j)] = v
                    if nk[1] == () and nk[0] in self.roots_set:
                        continue
                    w = recompute(nk)
                    if any(not np.array_equal(a, b) for a, b in zip(w, value[nk])):
                        value[nk] = w
                        if nk not in queued:
                            queued.add(nk)
                            queue.append(nk)
        else:
            raise ValueError(schedule)
        return value

    def contexts(self, S, schedule: str = "rounds"):
        """Context boundaries {(proc, sigma): (ev_h, ev_d, lx_h, lx_d)}, the
        host-read demands they require, per context its validity at EXIT under
        the final placement (the caps of the next outer round), and the
        contexts' final solutions.

        Two monotone systems over the context graph, solved one after the
        other (each has one fixed point, whatever the order of the solves):
        * exit liveness, least fixed point: a context's host / device exit
          liveness is the OR, over the calls that lead to it, of the caller's
          next use after the call; next use only grows with exit liveness;
        * entry validity, greatest fixed point given that liveness: the AND,
          over the calls, of the caller's eager validity after the call
          block's own accesses; eager validity only shrinks with entry
          validity.
        A global that the AND leaves valid in neither space and that the
        context reads before writing it needs its host copy made current by
        the callers: it is demanded, as a host read, at the call site that
        leads to the context (the last site of its call string), unless a
        caller context is itself missing that global at entry (the caller's
        own demand comes first); if every remaining gap is of that kind (a
        cycle of recursive contexts), all of them are demanded.  A global the
        context never reads may stay valid nowhere (its solve allows it)."""
        G = self.G
        gw = (G + 63) // 64
        graph = self.context_graph()
        keys = sorted(graph)
        self.roots_set = set(self.p.roots)
        is_root = {k: (k[1] == () and k[0] in self.roots_set) for k in keys}

        def masks(q):
            qc = self.p.procs[q]
            gq = self._smask(q, qc.wd)
            return gq, _vmask(qc.n_vars, qc.wd) & ~gq

        def to_callee(x, nk):
            """A caller-layout row moved to the callee context nk through the bindings of its
            leading call site: the globals, and parameter i from the bound caller variable."""
            q, j = nk[0], nk[1][-1]
            qc = self.p.procs[q]
            m = np.zeros(qc.wd, np.uint64)
            m[:gw] = x[:gw]
            m &= _gmask(G, qc.wd)
            for i, (v, _) in enumerate(self.args[j]):
                if (int(x[v >> 6]) >> (v & 63)) & 1:
                    t = G + i
                    m[t >> 6] |= np.uint64(1 << (t & 63))
            return m

        bnd: Dict[Tuple[int, tuple], List[np.ndarray]] = {}
        for k in keys:
            if is_root[k]:
                bnd[k] = [np.asarray(x, np.uint64).copy() for x in self.p.procs[k[0]].boundary()]
            else:
                gq, lq = masks(k[0])
                wd = self.p.procs[k[0]].wd
                bnd[k] = [gq | lq, gq.copy(), np.zeros(wd, np.uint64), np.zeros(wd, np.uint64)]

        # exit liveness (least fixed point); entry validity does not enter next use
        live = {k: (bnd[k][2], bnd[k][3]) for k in keys}

        def contrib_live(k, lv):
            P, sigma = k
            b = bnd[k]
            cfg, _, _, res = self._solve(P, S, (b[0], b[1], lv[0], lv[1]), summary_mode=True, sigma=sigma)
            out = {}
            for (j, nk) in graph[k]:
                _, _, l_h, l_d = self._call_values(P, cfg, res, j)
                out[(j, nk)] = (to_callee(l_h, nk), to_callee(l_d, nk))
            return out

        live = self._iterate(graph, keys, live, contrib_live, lambda a, b: (a[0] | b[0], a[1] | b[1]),
                             lambda nk: (np.zeros(self.p.procs[nk[0]].wd, np.uint64),
                                         np.zeros(self.p.procs[nk[0]].wd, np.uint64)), schedule)
        for k in keys:
            bnd[k][2], bnd[k][3] = live[k]

        # entry validity (greatest fixed point) with that liveness
        valid = {k: (bnd[k][0], bnd[k][1]) for k in keys}

        def top(nk):
            gq, lq = masks(nk[0])
            return (gq | lq, gq.copy())

        def contrib_valid(k, ev):
            P, sigma = k
            b = bnd[k]
            cfg, _, _, res = self._solve(P, S, (ev[0], ev[1], b[2], b[3]), summary_mode=True, sigma=sigma)
            out = {}
            for (j, nk) in graph[k]:
                a1_h, a1_d, _, _ = self._call_values(P, cfg, res, j)
                gq, lq = masks(nk[0])
                out[(j, nk)] = (to_callee(a1_h, nk) | lq, to_callee(a1_d, nk))
            return out

        valid = self._iterate(graph, keys, valid, contrib_valid, lambda a, b: (a[0] & b[0], a[1] & b[1]), top,
                              schedule)
        for k in keys:
            bnd[k][0], bnd[k][1] = valid[k]

        # final solves (a non-root context may leave globals valid nowhere), and the caps they give
        results = {}
        caps: Dict[tuple, Tuple[np.ndarray, np.ndarray]] = {}
        for k in keys:
            res = self._solve(k[0], S, tuple(bnd[k]), summary_mode=not is_root[k], sigma=k[1])[3]
            results[k] = res
            if k[1]:
                qc = self.p.procs[k[0]]
                sm = self._smask(k[0], qc.wd)
                caps[k] = ((res["avf_h"][qc.exit] & sm).copy(), (res["avf_d"][qc.exit] & sm).copy())

        # globals valid nowhere that the context reads before writing them (next
        # use at its ENTRY, which does not depend on entry validity): host-read
        # demands at the leading call site; a gap the context never reads stays
        gaps = {}
        for k in keys:
            if not is_root[k]:
                qc = self.p.procs[k[0]]
                gq, _ = masks(k[0])
                need = results[k]["nu_h"][qc.entry] | results[k]["nu_d"][qc.entry]
                nw = gq & ~(bnd[k][0] | bnd[k][1]) & need
                if nw.any():
                    gaps[k] = nw
        callers: Dict[Tuple[int, tuple], List[Tuple[int, tuple]]] = {k: [] for k in keys}
        for k in keys:
            for (j, nk) in graph[k]:
                callers[nk].append(k)
        new_demand: Dict[int, np.ndarray] = {}

        def demand(k, bits):
            """Gaps of context k (its layout) as host reads of the bound caller variables at its
            leading call site."""
            jj = k[1][-1]
            q = k[0]
            P2 = int(self.p.call_proc[jj])
            d = new_demand.get(jj, np.zeros(self.p.procs[P2].wd, np.uint64))
            d |= self._to_caller(jj, q, bits, P2)
            new_demand[jj] = d

        for k, nw in gaps.items():
            inherited = np.zeros(self.p.procs[k[0]].wd, np.uint64)
            for x in callers[k]:
                if x in gaps:
                    inherited |= to_callee(gaps[x], k)
            own = nw & ~inherited
            if own.any():
                demand(k, own)
        if gaps and not new_demand:
            for k, nw in gaps.items():
                demand(k, nw)
        self.nowhere = {k: nw.copy() for k, nw in gaps.items()}
        return bnd, new_demand, caps, results

    def analyze(self, max_rounds: int = 64, schedule: str = "rounds"):
        """Summaries, context boundaries and per-context results, after the
        outer rounds (summaries, then contexts) have settled the demands and
        the caps.  ``schedule`` orders the context solves inside a round
        ("rounds", "fifo" or "lifo"); the result does not depend on it."""
        for _ in range(max_rounds):
            S = self.summarize()
            ctx, nd, caps, results = self.contexts(S, schedule)
            grew = False
            for j, m in nd.items():
                old = self.demand.get(j)
                cur = m if old is None else (old | m)
                if old is None or not np.array_equal(old, cur):
                    self.demand[j] = cur
                    grew = True
            # (caps are over each callee context's shared variables)
            if caps.keys() != self.cap.keys() or any(
                    not (np.array_equal(caps[k][0], self.cap[k][0]) and np.array_equal(caps[k][1], self.cap[k][1]))
                    for k in caps):
                self.cap = caps
                grew = True
            if not grew:
                return S, ctx, results
        raise RuntimeError("demands and caps did not settle")
