"""Array-section facts (section "Array Access Pattern Analysis").

The paper bounds each array access by the loops around it (the lower bound
from the loop's initialisation, the upper one from its condition, minus one
for a strict comparison) and maps only the section of the array that the
program touches.  Here an access is a half-open range [lo, hi) of element
indices (row-major for arrays of several dimensions); `affine_range` gives
it for an index expression that is affine in the loop indices, from the
corners of the loops' bounds.

The bit-vector solve stays as it is: every array's index space is cut at the
bounds of all its accesses (and of the boundary sections) into segments, each
segment becomes one variable, so all elements of a segment are accessed by the
same blocks and get the same facts.  The copies the solve places are read back
as array sections: the segments of one array copied at the same place merge
into maximal ranges, and each copy carries its map/update label (Table II).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

Section = Tuple[str, int, int]   # (array, lo, hi): elements lo .. hi - 1


def affine_range(const: int, terms: Sequence[Tuple[int, int, int]]) -> Tuple[int, int]:
    """[lo, hi) of const + sum(c * i) over loops i in [first, last] (inclusive bounds), one
    (c, first, last) per loop: each term's extreme values sit at the loop's first or last index."""
    lo = hi = int(const)
    for c, first, last in terms:
        a, b = c * first, c * last
        lo += min(a, b)
        hi += max(a, b)
    return lo, hi + 1


@dataclass
class Access:
    block: int
    array: str
    lo: int
    hi: int
    mode: str = "r"     # "r", "w" or "rw" (reads precede writes within a block)


@dataclass
class Directive:
    where: Tuple[str, int]          # ("edge", index in the caller's edge list) or ("entry", block)
    into: str                       # "device" or "host"
    label: str                      # "map" or "update" (Table II)
    sections: List[Section]

    def clause(self) -> str:
        body = ", ".join("%s[%d:%d]" % (a, lo, hi - lo) for a, lo, hi in self.sections)
        d = "to" if self.into == "device" else "from"
        return ("map(%s: %s)" % (d, body)) if self.label == "map" else ("target update %s(%s)" % (d, body))


@dataclass
class SectionCFG:
    """The bit-vector problem of a section model, in the form the solver's entry points take."""
    n_blocks: int
    n_vars: int
    entry: int
    exit: int
    succ_ptr: np.ndarray
    succ_idx: np.ndarray
    edge_kind: np.ndarray
    space: np.ndarray
    R: np.ndarray
    W: np.ndarray
    entry_valid_h: Optional[np.ndarray] = None
    entry_valid_d: Optional[np.ndarray] = None
    exit_live_h: Optional[np.ndarray] = None
    exit_live_d: Optional[np.ndarray] = None

    @property
    def wd(self) -> int:
        return (self.n_vars + 63) // 64

    @property
    def n_edges(self) -> int:
        return int(self.succ_idx.shape[0])


@dataclass
class SectionModel:
    """A CFG (blocks with their memory space, edges with their kinds) whose accesses are
    array sections.  `arrays` maps each array to its length in elements (a scalar is an
    array of length 1).  Boundary sections default to the whole arrays valid on the host at
    entry and live on the host after exit, none on the device."""
    space: Sequence[int]
    edges: Sequence[Tuple[int, int, int]]            # (source, target, kind)
    arrays: Dict[str, int]
    accesses: Sequence[Access]
    entry: int = 0
    exit: int = -1
    entry_valid_d: Sequence[Section] = ()
    exit_live_d: Sequence[Section] = ()
    exit_dead_h: Sequence[Section] = ()               # sections not read on the host after exit
    segments: List[Section] = field(default_factory=list, init=False)
    csr_pos: np.ndarray = field(default=None, init=False)   # edge list index -> CSR position

    def __post_init__(self):
        nb = len(self.space)
        if self.exit < 0:
            self.exit = nb - 1
        for a in self.accesses:
            n = self.arrays[a.array]
            if not (0 <= a.lo < a.hi <= n) or a.mode not in ("r", "w", "rw") or not (0 <= a.block < nb):
                raise ValueError("bad access %r" % (a,))
        cuts: Dict[str, set] = {name: {0, n} for name, n in self.arrays.items()}
        for a in self.accesses:
            cuts[a.array] |= {a.lo, a.hi}
        for name, lo, hi in list(self.entry_valid_d) + list(self.exit_live_d) + list(self.exit_dead_h):
            n = self.arrays[name]
            if not (0 <= lo < hi <= n):
                raise ValueError("bad boundary section %r" % ((name, lo, hi),))
            cuts[name] |= {lo, hi}
        self.segments = []
        for name in self.arrays:
            c = sorted(cuts[name])
            self.segments += [(name, c[i], c[i + 1]) for i in range(len(c) - 1)]
        self._first = {}
        for v, (name, lo, hi) in enumerate(self.segments):
            self._first.setdefault(name, v)

    def bits(self, name: str, lo: int, hi: int) -> List[int]:
        """The variables (segments) that make up the section [lo, hi) of an array."""
        out = []
        v = self._first[name]
        while v < len(self.segments) and self.segments[v][0] == name:
            s = self.segments[v]
            if s[1] >= lo and s[2] <= hi:
                out.append(v)
            v += 1
        return out

    def cfg(self) -> SectionCFG:
        nb, nv = len(self.space), len(self.segments)
        wd = (nv + 63) // 64
        order = sorted(range(len(self.edges)), key=lambda i: (self.edges[i][0], i))
        succ_ptr = np.zeros(nb + 1, np.int32)
        for s, _, _ in self.edges:
            succ_ptr[s + 1] += 1
        np.cumsum(succ_ptr, out=succ_ptr)
        succ_idx = np.array([self.edges[i][1] for i in order], np.int32)
        kind = np.array([self.edges[i][2] for i in order], np.uint8)
        self.csr_pos = np.empty(len(self.edges), np.int64)
        self.csr_pos[order] = np.arange(len(self.edges))
        R = np.zeros((nb, wd), np.uint64)
        W = np.zeros((nb, wd), np.uint64)

        def setb(M, b, v):
            M[b, v >> 6] |= np.uint64(1 << (v & 63))
        for a in self.accesses:
            for v in self.bits(a.array, a.lo, a.hi):
                if "r" in a.mode:
                    setb(R, a.block, v)
                if "w" in a.mode:
                    setb(W, a.block, v)

        def vec(secs, default_all: bool):
            x = np.zeros(wd, np.uint64)
            if default_all:
                for v in range(nv):
                    x[v >> 6] |= np.uint64(1 << (v & 63))
            for name, lo, hi in secs:
                for v in self.bits(name, lo, hi):
                    m = np.uint64(1 << (v & 63))
                    x[v >> 6] = (x[v >> 6] | m) if not default_all else (x[v >> 6] & ~m)
            return x
        evd = vec(self.entry_valid_d, False)
        return SectionCFG(n_blocks=nb, n_vars=nv, entry=self.entry, exit=self.exit, succ_ptr=succ_ptr,
                          succ_idx=succ_idx, edge_kind=kind, space=np.asarray(self.space, np.uint8), R=R, W=W,
                          entry_valid_h=vec((), True), entry_valid_d=evd,
                          exit_live_h=vec(self.exit_dead_h, True), exit_live_d=vec(self.exit_live_d, False))

    def _merge(self, row: np.ndarray) -> List[Section]:
        out: List[Section] = []
        for v, (name, lo, hi) in enumerate(self.segments):
            if not (int(row[v >> 6]) >> (v & 63)) & 1:
                continue
            if out and out[-1][0] == name and out[-1][2] == lo:
                out[-1] = (name, out[-1][1], hi)
            else:
                out.append((name, lo, hi))
        return out

    def directives(self, res) -> List[Directive]:
        """The copies of a solve result (the solver's output arrays for cfg()) as directives on
        array sections, labelled by Table II's rule (one target data region per function)."""
        nb = len(self.space)
        after, before = np.asarray(res["after_dev"]), np.asarray(res["before_dev"])
        preds: List[List[int]] = [[] for _ in range(nb)]
        for s, t, _ in self.edges:
            preds[t].append(s)
        out: List[Directive] = []
        for q in range(nb):
            for into, key in (("device", "ins_entry_d"), ("host", "ins_entry_h")):
                secs = self._merge(np.asarray(res[key])[q])
                if secs:
                    if into == "device":
                        lab = "update" if any(after[p] for p in preds[q]) else "map"
                    else:
                        lab = "update" if before[q] else "map"
                    out.append(Directive(("entry", q), into, lab, secs))
        for i, (s, t, _) in enumerate(self.edges):
            e = int(self.csr_pos[i])
            for into, key in (("device", "ins_edge_d"), ("host", "ins_edge_h")):
                secs = self._merge(np.asarray(res[key])[e])
                if secs:
                    lab = ("update" if after[s] else "map") if into == "device" else ("update" if before[t] else "map")
                    out.append(Directive(("edge", i), into, lab, secs))
        return out

    def map_kinds(self, res) -> Dict[str, List[Tuple[str, int, int]]]:
        """Per array, its sections by map kind ("to", "from", "tofrom", "alloc", "firstprivate")."""
        vk = np.asarray(res["var_kind"])
        names = {1: "to", 2: "from", 3: "tofrom", 4: "alloc"}
        out: Dict[str, List[Tuple[str, int, int]]] = {}
        for v, (name, lo, hi) in enumerate(self.segments):
            k = int(vk[v])
            kind = names.get(k & 7) if k & 7 else ("firstprivate" if k & 8 else None)
            if kind is None:
                continue
            lst = out.setdefault(name, [])
            if lst and lst[-1][0] == kind and lst[-1][2] == lo:
                lst[-1] = (kind, lst[-1][1], hi)
            else:
                lst.append((kind, lo, hi))
        return out
