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
  context gives, at each call site, the validity after the caller's own
  accesses in the final placement (entry validity of the callee) and the
  caller's next use after the call (exit liveness of the callee).  Several
  callers that reach one context meet: validity by AND, liveness by OR,
  over everything contributed so far, in rounds that re-solve every context
  whose boundary changed.  A variable that the meet leaves valid in neither
  space is assumed valid on the host in that context, and the call site that
  leads to the context (the last of its call string) must then make it valid
  on the host before the call (a host read at the call block); such demands
  feed back into the summaries, and the whole computation repeats until no
  demand changes.
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


def external_summary(gm: np.ndarray) -> np.ndarray:
    r = np.zeros((SUM_ROWS, gm.size), np.uint64)
    for k in (SUM_MAYR_H, SUM_MAYW_H, SUM_NU0_H, SUM_NU1_H, SUM_NU1_D):
        r[k] = gm
    for k in range(4):
        r[SUM_TH_00 + k] = gm       # host copy valid after the call
        r[SUM_TD_00 + k] = 0        # device copy stale after the call
    return r


class ProgramOracle:
    def __init__(self, prog):
        self.p = prog
        self.n = len(prog.procs)
        self.G = prog.n_globals
        self.sites: List[List[int]] = [[] for _ in range(self.n)]      # call-site ids per caller
        for j in range(len(prog.call_proc)):
            self.sites[int(prog.call_proc[j])].append(j)
        self.demand: Dict[int, np.ndarray] = {}                          # call site -> host-read mask (caller words)
        self.cap: Dict[tuple, Tuple[np.ndarray, np.ndarray]] = {}        # callee context -> (host, device) validity at EXIT
        self.sum_rows: Dict[int, np.ndarray] = {}
        self.visits = 0

    # -- call tables in a caller's variable layout ------------------------------------
    def _caller_tables(self, P: int, summaries: Dict[int, np.ndarray], sigma=None):
        cfg = self.p.procs[P]
        wd = cfg.wd
        gw = (self.G + 63) // 64
        gm = _gmask(self.G, wd)
        lm = _vmask(cfg.n_vars, wd) & ~gm
        call = np.full(cfg.n_blocks, -1, np.int32)
        sums = np.zeros((max(len(self.sites[P]), 1), SUM_ROWS, wd), np.uint64)
        for k, j in enumerate(self.sites[P]):
            call[int(self.p.call_block[j])] = k
            q = int(self.p.callee[j])
            rows = external_summary(_gmask(self.G, gw)) if q < 0 else summaries[q]
            s = np.zeros((SUM_ROWS, wd), np.uint64)
            s[:, :gw] = rows
            s &= gm
            # identity for the caller's locals: NU1 = 1, T[e][l] = e
            s[SUM_NU1_H] |= lm
            s[SUM_NU1_D] |= lm
            for base in (SUM_TH_00, SUM_TD_00):
                s[base + 2] |= lm
                s[base + 3] |= lm
            ckey = None if (sigma is None or q < 0) else (q, (tuple(sigma) + (j,))[-2:])
            if ckey in self.cap:
                ch, cd = self.cap[ckey]
                for k4 in range(4):
                    s[SUM_TH_00 + k4, :gw] &= ch | ~gm[:gw]
                    s[SUM_TD_00 + k4, :gw] &= cd | ~gm[:gw]
            sums[k] = s
        return call, sums

    def _cfg_with_demands(self, P: int):
        cfg = self.p.procs[P]
        R = cfg.R
        dem = [(int(self.p.call_block[j]), self.demand[j]) for j in self.sites[P] if j in self.demand]
        if dem:
            R = R.copy()
            for blk, m in dem:
                R[blk] |= m
        return cfg, R

    def _solve(self, P, summaries, boundary, summary_mode=False, sigma=None):
        cfg, R = self._cfg_with_demands(P)
        call, sums = self._caller_tables(P, summaries, sigma)
        view = type(cfg)(n_blocks=cfg.n_blocks, n_vars=cfg.n_vars, succ_ptr=cfg.succ_ptr, succ_idx=cfg.succ_idx,
                         edge_kind=cfg.edge_kind, space=cfg.space, R=R, W=cfg.W, entry=cfg.entry, exit=cfg.exit)
        self.visits += 1
        res = solve(view, placement=SUMMARY_MODE if summary_mode else 0,
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
        S: Dict[int, np.ndarray] = {}
        for comp in comps:
            if len(comp) == 1 and comp[0] not in succ[comp[0]]:
                # not recursive: every callee is final, one evaluation is exact
                q = comp[0]
                S[q] = self._evaluate(q, S)
                S[q][:4] = self._may(q, S)
                continue
            for q in comp:
                r = np.zeros((SUM_ROWS, gw), np.uint64)
                for k in range(4):
                    r[SUM_TH_00 + k] = _gmask(G, gw)
                    r[SUM_TD_00 + k] = _gmask(G, gw)
                S[q] = r
            # next use from 0, then validity tables from all-ones, then may bits from 0
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
            while True:
                changed = False
                for q in comp:
                    m = self._may(q, S)
                    if not np.array_equal(S[q][:4], m):
                        S[q][:4] = m
                        changed = True
                if not changed:
                    break
        self.sum_rows = S
        return S

    def _evaluate(self, Q: int, S) -> np.ndarray:
        """NU0/NU1 and the four T tables of Q from four boundary evaluations."""
        cfg = self.p.procs[Q]
        wd = cfg.wd
        gw = (self.G + 63) // 64
        gm = _gmask(self.G, wd)
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
        cfg, R = self._cfg_with_demands(Q)
        gw = (self.G + 63) // 64
        gm = _gmask(self.G, gw)
        m = np.zeros((4, gw), np.uint64)
        dev = np.asarray(cfg.space) == 1
        if (~dev).any():
            m[0] = np.bitwise_or.reduce(R[~dev][:, :gw], axis=0)
            m[2] = np.bitwise_or.reduce(cfg.W[~dev][:, :gw], axis=0)
        if dev.any():
            m[1] = np.bitwise_or.reduce(R[dev][:, :gw], axis=0)
            m[3] = np.bitwise_or.reduce(cfg.W[dev][:, :gw], axis=0)
        for j in self.sites[Q]:
            q = int(self.p.callee[j])
            rows = external_summary(gm) if q < 0 else S[q]
            m |= rows[:4]
        return m & gm

    # -- top-down -------------------------------------------------------------------
    def contexts(self, S):
        """Context boundaries {(proc, sigma): (ev_h, ev_d, lx_h, lx_d)}, the
        host-read demands they require and, per context, its validity at EXIT
        under the final placement (the caps of the next round).

        Rounds: every context whose boundary is new or changed is solved;
        each of its calls contributes the validity after the call block's own
        accesses and the next use after the call to the callee context (the
        last two call sites); a context's boundary is the meet of everything
        contributed to it so far (validity AND, liveness OR), so boundaries
        only move one way and the rounds end.  Bits left valid in neither
        space are then assumed valid on the host and demanded, as a host read,
        at the call site that leads to the context (the last site of its call
        string)."""
        G = self.G
        gw = (G + 63) // 64
        ctx: Dict[Tuple[int, tuple], List[np.ndarray]] = {}
        last: Dict[Tuple[int, tuple], dict] = {}
        for r in self.p.roots:
            ctx[(r, ())] = list(self.p.procs[r].boundary())
        dirty = sorted(ctx)
        new_demand: Dict[int, np.ndarray] = {}
        while dirty:
            acc: Dict[Tuple[int, tuple], List[np.ndarray]] = {}
            for key in dirty:
                P, sigma = key
                cfg, call, sums, res = self._solve(P, S, ctx[key], sigma=sigma)
                last[key] = res
                wd = cfg.wd
                for j in self.sites[P]:
                    q = int(self.p.callee[j])
                    if q < 0:
                        continue
                    c = int(self.p.call_block[j])
                    # validity after the call block's own accesses (final placement)
                    w = cfg.W[c]
                    a1_h = res["avf_h"][c] | w
                    a1_d = res["avf_d"][c] & ~w
                    l_h = np.zeros(wd, np.uint64)
                    l_d = np.zeros(wd, np.uint64)
                    for e in range(int(cfg.succ_ptr[c]), int(cfg.succ_ptr[c + 1])):
                        t = int(cfg.succ_idx[e])
                        l_h |= res["nu_h"][t]
                        l_d |= res["nu_d"][t]
                    qc = self.p.procs[q]
                    qwd = qc.wd
                    gq = _gmask(G, qwd)
                    lq = _vmask(qc.n_vars, qwd) & ~gq
                    m = [np.zeros(qwd, np.uint64) for _ in range(4)]
                    m[0][:gw] = a1_h[:gw]
                    m[1][:gw] = a1_d[:gw]
                    m[2][:gw] = l_h[:gw]
                    m[3][:gw] = l_d[:gw]
                    m = [(m[0] & gq) | lq, m[1] & gq, m[2] & gq, m[3] & gq]
                    nkey = (q, (sigma + (j,))[-2:])
                    if nkey in acc:
                        a = acc[nkey]
                        acc[nkey] = [a[0] & m[0], a[1] & m[1], a[2] | m[2], a[3] | m[3]]
                    else:
                        acc[nkey] = m
            dirty = []
            for nkey in sorted(acc):
                a = acc[nkey]
                if nkey in ctx:
                    old = ctx[nkey]
                    m = [old[0] & a[0], old[1] & a[1], old[2] | a[2], old[3] | a[3]]
                else:
                    m = a
                q = nkey[0]
                gq = _gmask(G, self.p.procs[q].wd)
                # variables valid in neither space (must-validity is empty after a
                # join of host-fresh and device-fresh paths, or after a meet of
                # callers): assume the host copy and make the call site that leads
                # here provide it
                nowhere = gq & ~(m[0] | m[1])
                if nowhere.any():
                    m[0] = m[0] | nowhere
                    jj = nkey[1][-1]
                    P2 = int(self.p.call_proc[jj])
                    d = new_demand.get(jj, np.zeros(self.p.procs[P2].wd, np.uint64))
                    d[:gw] |= nowhere[:gw]
                    new_demand[jj] = d
                if nkey not in ctx or any(not np.array_equal(x, y) for x, y in zip(ctx[nkey], m)):
                    ctx[nkey] = m
                    dirty.append(nkey)
        caps: Dict[tuple, Tuple[np.ndarray, np.ndarray]] = {}
        for key, res in last.items():
            if key[1]:
                qc = self.p.procs[key[0]]
                caps[key] = (res["avf_h"][qc.exit][:gw].copy(), res["avf_d"][qc.exit][:gw].copy())
        return ctx, new_demand, caps

    def analyze(self, max_rounds: int = 64):
        """Summaries, contexts and per-context results (with demands settled)."""
        gm = _gmask(self.G, (self.G + 63) // 64)
        for _ in range(max_rounds):
            S = self.summarize()
            ctx, nd, caps = self.contexts(S)
            grew = False
            for j, m in nd.items():
                old = self.demand.get(j)
                cur = m if old is None else (old | m)
                if old is None or not np.array_equal(old, cur):
                    self.demand[j] = cur
                    grew = True
            caps = {k: (ch & gm, cd & gm) for k, (ch, cd) in caps.items()}
            if caps.keys() != self.cap.keys() or any(
                    not (np.array_equal(caps[k][0], self.cap[k][0]) and np.array_equal(caps[k][1], self.cap[k][1]))
                    for k in caps):
                self.cap = caps
                grew = True
            if not grew:
                results = {}
                for key, b in ctx.items():
                    results[key] = self._solve(key[0], S, b, sigma=key[1])[3]
                return S, ctx, results
        raise RuntimeError("demands and caps did not settle")
