"""The re-check that ends a phase without a confirming sweep, on a model.

After a Gauss-Seidel sweep the next sweep can only see other states than this
one through blocks that read a neighbour not yet visited in the sweep (walk
order) or not at a lower level (level schedule, Jacobi within a level).  If
each of those, evaluated again against the states the sweep left, keeps its
state, the states are the fixed point.  This holds for any graph and any
order, which these tests check against a plain worklist fixed point of the
same equations (gen/kill problems over 64-bit words, forward must and backward
may, on random graphs with self loops, irreducible cycles and unreachable
cycles), and the re-check must never end a phase early.  The model shares
nothing with the device code; it tests the argument, not the kernels.
"""
import numpy as np
import pytest

ALL = (1 << 64) - 1


def _graph(rng, nb):
    """Random digraph over blocks 0..nb-1 (0 = entry): a spanning path plus random edges
    (forward, backward and self loops)."""
    edges = {(b, b + 1) for b in range(nb - 1)}
    for _ in range(int(rng.integers(nb // 2, 2 * nb + 1))):
        a, b = int(rng.integers(0, nb)), int(rng.integers(1, nb))
        edges.add((a, b))
    preds = [[] for _ in range(nb)]
    succs = [[] for _ in range(nb)]
    for a, b in sorted(edges):
        succs[a].append(b)
        preds[b].append(a)
    return preds, succs


def _problem(rng, nb, forward):
    gen = [int(rng.integers(0, 1 << 63)) & int(rng.integers(0, 1 << 63)) for _ in range(nb)]
    kill = [int(rng.integers(0, 1 << 63)) | int(rng.integers(0, 1 << 63)) for _ in range(nb)]
    top = ALL if forward else 0

    def f(b, st, nbr):
        if forward:
            if b == 0:
                return gen[0]
            m = ALL
            for p in nbr[b]:
                m &= st[p]
            return gen[b] | (m & ~kill[b] & ALL)
        m = 0
        for q in nbr[b]:
            m |= st[q]
        return gen[b] | (m & ~kill[b] & ALL)
    return f, top


def _worklist(nb, f, top, nbr, dep):
    st = [top] * nb
    work = list(range(nb))
    while work:
        b = work.pop()
        v = f(b, st, nbr)
        if v != st[b]:
            st[b] = v
            work.extend(dep[b])
    return st


def _walk(nb, f, top, nbr, order):
    """Gauss-Seidel in `order`, ended by the re-check; returns states and sweeps."""
    pos = {b: k for k, b in enumerate(order)}
    listed = [b for b in order if any(pos[p] >= pos[b] for p in nbr[b])]
    st = [top] * nb
    sweeps = 0
    while True:
        changed = False
        for b in order:
            v = f(b, st, nbr)
            changed |= v != st[b]
            st[b] = v
        sweeps += 1
        if not changed or all(f(b, st, nbr) == st[b] for b in listed):
            return st, sweeps
        assert sweeps <= 2 * nb + 2


def _levels(nb, f, top, nbr, level, rng):
    """Levels in order, the blocks of a level from the same states (Jacobi), in a random
    order of writes; ended by the re-check over blocks with a neighbour at a level not below."""
    by = {}
    for b in range(nb):
        by.setdefault(level[b], []).append(b)
    listed = [b for b in range(nb) if any(level[p] >= level[b] for p in nbr[b])]
    st = [top] * nb
    sweeps = 0
    while True:
        changed = False
        for lv in sorted(by):
            new = {b: f(b, st, nbr) for b in by[lv]}
            for b in rng.permutation(by[lv]):
                changed |= new[int(b)] != st[int(b)]
                st[int(b)] = new[int(b)]
        sweeps += 1
        if not changed or all(f(b, st, nbr) == st[b] for b in listed):
            return st, sweeps
        assert sweeps <= 2 * nb + 2


@pytest.mark.parametrize("seed", range(40))
def test_recheck_ends_at_the_fixed_point(seed):
    rng = np.random.default_rng(5_000 + seed)
    nb = int(rng.integers(2, 40))
    preds, succs = _graph(rng, nb)
    for forward in (True, False):
        f, top = _problem(rng, nb, forward)
        nbr, dep = (preds, succs) if forward else (succs, preds)
        ref = _worklist(nb, f, top, nbr, dep)
        ids = list(range(nb)) if forward else list(range(nb - 1, -1, -1))
        shuffled = [int(b) for b in rng.permutation(nb)]
        for order in (ids, shuffled):
            got, _ = _walk(nb, f, top, nbr, order)
            assert got == ref, (seed, forward, order)
        level = [int(x) for x in rng.integers(0, max(1, nb // 3), nb)]
        got, _ = _levels(nb, f, top, nbr, level, rng)
        assert got == ref, (seed, forward, "levels")


def test_acyclic_in_forward_order_needs_one_sweep():
    rng = np.random.default_rng(77)
    nb = 30
    preds = [[] for _ in range(nb)]
    for b in range(1, nb):
        for a in rng.choice(b, size=min(b, 2), replace=False):
            preds[b].append(int(a))
    f, top = _problem(rng, nb, True)
    got, sweeps = _walk(nb, f, top, preds, list(range(nb)))
    succs = [[] for _ in range(nb)]
    for b in range(nb):
        for p in preds[b]:
            succs[p].append(b)
    assert got == _worklist(nb, f, top, preds, succs) and sweeps == 1


def test_a_missing_listed_block_would_stop_early():
    """Planted mistake: leaving a block with a BACK edge into it out of the list ends the
    walk before the fixed point on some graph, so the list is what makes it exact."""
    rng = np.random.default_rng(3)
    early = 0
    for _ in range(200):
        nb = int(rng.integers(3, 20))
        preds, succs = _graph(rng, nb)
        f, top = _problem(rng, nb, True)
        ref = _worklist(nb, f, top, preds, succs)
        order = list(range(nb))
        pos = {b: k for k, b in enumerate(order)}
        listed = [b for b in order if any(pos[p] >= pos[b] for p in preds[b])]
        if not listed:
            continue
        drop = listed[0]
        st = [top] * nb
        for _sweep in range(2 * nb + 2):
            changed = False
            for b in order:
                v = f(b, st, preds)
                changed |= v != st[b]
                st[b] = v
            if not changed or all(f(b, st, preds) == st[b] for b in listed if b != drop):
                break
        early += st != ref
    assert early > 0
