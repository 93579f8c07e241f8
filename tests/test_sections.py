"""Array-section facts (section "Array Access Pattern Analysis") on the CPU:
the affine bounds against enumeration of the loop indices, the segmentation
against the element ranges it must cover, and the whole encoding against the
element-level problem (one variable per array element, built here directly
from the accesses) solved by the oracle: every element is copied at exactly
the places, in the direction and with the label that the section directives
give, and gets the map kind of its section.  The worked example is the
paper's for-bounds listing (a kernel that writes a[0:N/2])."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import synth
from paper_2406_13881_amd.sections import Access, SectionModel, affine_range

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("seed", range(30))
def test_affine_range_is_the_extreme_of_the_loop_corners(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    k = int(rng.integers(1, 4))
    const = int(rng.integers(-5, 6))
    terms = []
    for _ in range(k):
        first = int(rng.integers(-3, 4))
        terms.append((int(rng.integers(-4, 5)), first, first + int(rng.integers(0, 4))))
    vals = [const + sum(c * i for (c, _, _), i in zip(terms, idx))
            for idx in itertools.product(*[range(f, l + 1) for (_, f, l) in terms])]
    assert affine_range(const, terms) == (min(vals), max(vals) + 1)


def random_model(seed, n_user=None, n_arrays=3, max_len=24, n_acc=None):
    rng = np.random.Generator(np.random.PCG64(90_000 + seed))
    n_user = n_user or int(rng.integers(4, 30))
    sk = synth.make_cfg(90_000 + seed, n_user=n_user, n_vars=1, max_loop_depth=int(rng.integers(1, 4)),
                        device_frac=0.4, irr_loop_frac=0.2 if seed % 3 == 0 else 0.0)
    nb = sk.n_blocks
    edges = []
    for p in range(nb):
        for e in range(int(sk.succ_ptr[p]), int(sk.succ_ptr[p + 1])):
            edges.append((p, int(sk.succ_idx[e]), int(sk.edge_kind[e])))
    order = rng.permutation(len(edges))            # the caller's edge list need not be in CSR order
    edges = [edges[i] for i in order]
    arrays = {"a%d" % i: int(rng.integers(1, max_len + 1)) for i in range(n_arrays)}
    acc = []
    users = [b for b in range(nb) if b not in (sk.entry, sk.exit)]
    for _ in range(n_acc or int(rng.integers(1, 3 * n_user))):
        name = "a%d" % int(rng.integers(n_arrays))
        n = arrays[name]
        lo = int(rng.integers(0, n))
        hi = int(rng.integers(lo + 1, n + 1))
        acc.append(Access(int(rng.choice(users)), name, lo, hi, ["r", "w", "rw"][int(rng.integers(3))]))
    kw = {}
    if seed % 4 == 1:
        name = "a0"
        kw["entry_valid_d"] = [(name, 0, arrays[name])]
        kw["exit_live_d"] = [(name, 0, (arrays[name] + 1) // 2)]
    if seed % 5 == 2:
        kw["exit_dead_h"] = [("a1", 0, arrays["a1"])]
    return SectionModel(space=[int(x) for x in sk.space], edges=edges, arrays=arrays, accesses=acc,
                        entry=sk.entry, exit=sk.exit, **kw)


def element_cfg(m: SectionModel):
    """The element-level problem of a section model: one variable per array element."""
    names = list(m.arrays)
    base = {}
    nv = 0
    for name in names:
        base[name] = nv
        nv += m.arrays[name]
    sec = m.cfg()          # the block/edge skeleton is shared; the variables are not
    nb, wd = sec.n_blocks, (nv + 63) // 64
    R = np.zeros((nb, wd), np.uint64)
    W = np.zeros((nb, wd), np.uint64)

    def put(M, b, v):
        M[b, v >> 6] |= np.uint64(1 << (v & 63))
    for a in m.accesses:
        for i in range(a.lo, a.hi):
            if "r" in a.mode:
                put(R, a.block, base[a.array] + i)
            if "w" in a.mode:
                put(W, a.block, base[a.array] + i)

    def vec(secs):
        x = np.zeros(wd, np.uint64)
        for name, lo, hi in secs:
            for i in range(lo, hi):
                put(x[None, :], 0, base[name] + i)
        return x
    allv = vec([(n, 0, m.arrays[n]) for n in names])
    evh = allv.copy()
    lxh = allv & ~vec(m.exit_dead_h)
    cfg = synth.CFG(n_blocks=nb, n_vars=nv, succ_ptr=sec.succ_ptr, succ_idx=sec.succ_idx, edge_kind=sec.edge_kind,
                    space=sec.space, R=R, W=W, entry=sec.entry, exit=sec.exit)
    bnd = (evh, vec(m.entry_valid_d), lxh, vec(m.exit_live_d))
    return cfg, bnd, base


def element_copies(m, res_el, base):
    """{(where, into): set of (array, element)} and labels from the element-level result."""
    out = {}
    inv = {}
    for name, b in base.items():
        for i in range(m.arrays[name]):
            inv[b + i] = (name, i)

    def elems(row):
        return {inv[v] for v in inv if (int(row[v >> 6]) >> (v & 63)) & 1}
    nb = len(m.space)
    for q in range(nb):
        for into, key in (("device", "ins_entry_d"), ("host", "ins_entry_h")):
            s = elems(res_el[key][q])
            if s:
                out[(("entry", q), into)] = s
    for i in range(len(m.edges)):
        e = int(m.csr_pos[i])
        for into, key in (("device", "ins_edge_d"), ("host", "ins_edge_h")):
            s = elems(res_el[key][e])
            if s:
                out[(("edge", i), into)] = s
    return out


def check_against_elements(m, res_sec, res_el, base):
    got = {}
    for d in m.directives(res_sec):
        key = (d.where, d.into)
        assert key not in got
        got[key] = {(name, i) for name, lo, hi in d.sections for i in range(lo, hi)}
        # sections are maximal and disjoint ranges
        for (n1, l1, h1), (n2, l2, h2) in zip(d.sections, d.sections[1:]):
            assert (n1, h1) != (n2, l2)
    assert got == element_copies(m, res_el, base)
    # labels: the element-level labelling facts are the section-level ones (block facts)
    assert np.array_equal(res_sec["after_dev"], res_el["after_dev"])
    assert np.array_equal(res_sec["before_dev"], res_el["before_dev"])
    kinds = m.map_kinds(res_sec)
    names = {1: "to", 2: "from", 3: "tofrom", 4: "alloc"}
    for name, b in base.items():
        for i in range(m.arrays[name]):
            k = int(res_el["var_kind"][b + i])
            want = names.get(k & 7)
            have = [kd for kd, lo, hi in kinds.get(name, []) if lo <= i < hi]
            assert have == ([want] if want else []), (name, i, k, have)


@pytest.mark.parametrize("seed", range(40))
def test_sections_equal_the_element_level_problem(seed):
    m = random_model(seed)
    sec = m.cfg()
    res_sec = oracle.solve(sec, boundary=(sec.entry_valid_h, sec.entry_valid_d, sec.exit_live_h, sec.exit_live_d))
    el, bnd, base = element_cfg(m)
    res_el = oracle.solve(el, boundary=bnd)
    check_against_elements(m, res_sec, res_el, base)


def test_segments_cover_the_accesses_exactly():
    for seed in range(20):
        m = random_model(seed)
        for a in m.accesses:
            covered = sorted(i for v in m.bits(a.array, a.lo, a.hi) for i in range(m.segments[v][1], m.segments[v][2]))
            assert covered == list(range(a.lo, a.hi))
        for name, n in m.arrays.items():
            segs = [s for s in m.segments if s[0] == name]
            assert segs[0][1] == 0 and segs[-1][2] == n
            assert all(x[2] == y[1] for x, y in zip(segs, segs[1:]))


def load_section_golden(path):
    g = json.load(open(path))
    SPACE = {"H": 0, "D": 1}
    KIND = {"N": 0, "BACK": 1, "LE": 2}
    m = SectionModel(space=[SPACE[x] for x in g["blocks"]], edges=[(s, d, KIND[k]) for s, d, k in g["edges"]],
                     arrays=g["arrays"], accesses=[Access(*a) for a in g["accesses"]])
    return g, m


@pytest.mark.parametrize("path", sorted(p for p in os.listdir(GOLDEN) if p.startswith("S") and p.endswith(".json")))
def test_section_worked_example(path):
    g, m = load_section_golden(os.path.join(GOLDEN, path))
    sec = m.cfg()
    r = oracle.solve(sec, boundary=(sec.entry_valid_h, sec.entry_valid_d, sec.exit_live_h, sec.exit_live_d))
    assert [d.clause() for d in m.directives(r)] == g["expect"]["clauses"]
    assert {k: [list(x) for x in v] for k, v in m.map_kinds(r).items()} == g["expect"]["map_kinds"]


def test_bad_accesses_are_rejected():
    with pytest.raises(ValueError):
        SectionModel(space=[0, 1, 0], edges=[(0, 1, 0), (1, 2, 0)], arrays={"a": 4}, accesses=[Access(1, "a", 2, 5)])
    with pytest.raises(ValueError):
        SectionModel(space=[0, 1, 0], edges=[(0, 1, 0), (1, 2, 0)], arrays={"a": 4}, accesses=[Access(1, "a", 3, 3)])
