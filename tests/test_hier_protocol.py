"""Host model of the descending-core hierarchy construction (the two-pass
"TE" build), run under random interleavings.

After a peel without linking, the device builds the same union-find uf
(same-core components) and nearest-lower-core table L as Algorithm 5, level
by level from the largest core number down. Inside a level many pair
operations run concurrently; a second union-find (tuf) groups r-cliques by
partial tree and `bottom` names each tree's lowest component. This model of
the device routine makes every shared access a scheduling point and lets a
seeded random scheduler interleave all pairs of one level; the canonical tree
built from the final uf and L must equal the oracle's whatever the
interleaving.
"""
import random

import pytest

import brute
import oracle
from paper_2306_08623_amd import inputs as I
from test_link_protocol import NONE, find, run_interleaved, tree_from, unite


class Mem:
    def __init__(self, n):
        self.uf = list(range(n))
        self.L = [NONE] * n


class TMem:
    """tuf in the layout find/unite expect (attribute uf)."""
    def __init__(self, n):
        self.uf = list(range(n))


def hier_pair(mem, tmem, bottom, nd, R, R2, c):
    if nd[R2] == c:
        yield from unite(mem, R, R2)
        yield from unite(tmem, R, R2)
        return
    T = yield from find(tmem, R2)
    B = bottom[T]; yield
    if nd[B] == c:
        yield from unite(mem, B, R)
        yield from unite(tmem, T, R)
        return
    Bs = yield from find(mem, B)
    old = mem.L[Bs]
    if old == NONE:
        mem.L[Bs] = R
    yield
    if old == NONE:
        yield from unite(tmem, T, R)
        w = yield from find(tmem, R)
        bottom[w] = R
        yield
    else:
        yield from unite(mem, old, R)
        yield from unite(tmem, T, R)


def check(g, r, s, seed):
    d = oracle.decompose(g, r, s)
    adj = brute.adjacency_sets(g)
    Rs, S, deg, members = brute.s_clique_degrees(adj, r, s)
    n_r = len(Rs)
    nd = [int(x) for x in d.coreness]
    k = max(nd) if nd else 0
    rng = random.Random(seed)
    mem, tmem = Mem(n_r), TMem(n_r)
    bottom = list(range(n_r))
    inc = [[] for _ in range(n_r)]
    for si, ids in enumerate(members):
        for x in ids:
            inc[x].append(si)
    for c in range(k, 0, -1):
        gens = []
        for R in (x for x in range(n_r) if nd[x] == c):
            for si in inc[R]:
                for R2 in members[si]:
                    if R2 != R and nd[R2] >= c:
                        gens.append(hier_pair(mem, tmem, bottom, nd, R, R2, c))
        rng.shuffle(gens)
        run_interleaved(gens, rng)
    parent, level = tree_from(mem, nd, n_r)
    return parent == d.parent.tolist() and level == d.level.tolist()


@pytest.mark.parametrize("rs", [(1, 2), (2, 3), (3, 4), (2, 4)])
def test_random_interleavings(rs):
    r, s = rs
    for gi in range(120):
        n = random.Random(gi).randint(6, 24)
        p = random.Random(gi + 1).uniform(0.15, 0.65)
        g = I.gnp(n, p, seed=gi)
        for seed in range(3):
            assert check(g, r, s, seed), (gi, n, p, rs, seed)


def test_planted_interleavings():
    g = I.er_planted(40, 0.1, 3, 5, 9, seed=4)
    for r, s in [(1, 2), (2, 3), (3, 4), (2, 4)]:
        for seed in range(4):
            assert check(g, r, s, seed), (r, s, seed)


def test_two_k5_bridge():
    for seed in range(10):
        assert check(I.two_k5_bridge(), 2, 3, seed)
        assert check(I.two_k5_bridge(), 1, 2, seed)
