"""Pins of the oracle's approximate decomposition (Section 6, Algorithm 2)
and of the hierarchy built on its values:

* the approximation bound of the paper's theorem against the exact core
  numbers: core <= approx <= (C(s,r) + delta)(1 + delta) core, on every
  r-clique of many graphs, every pair, three deltas;
* a pure-Python round-by-round run of Algorithm 2 on brute-force cliques
  (same bucket ends and round cap), equal value by value;
* closed forms on complete graphs;
* the tree of the approximate values equals the per-level BFS hierarchy of
  those values (brute force)."""
from __future__ import annotations

import math
from itertools import combinations
from math import comb

import numpy as np
import pytest

import oracle
from paper_2306_08623_amd import inputs as I

from brute import adjacency_sets, hierarchy_bfs, s_clique_degrees

PAIRS = [(1, 2), (2, 3), (1, 3), (2, 4), (3, 4), (1, 4)]
DELTAS = [0.1, 0.5, 1.0]


def bucket_ends(C: int, delta: float, upto: int) -> list[int]:
    """floor((C + delta)(1 + delta)^(i+1)), i = 0, 1, ..., until one is
    >= upto (the product built by repeated multiplication)."""
    out, t = [], C + delta
    while True:
        t *= 1.0 + delta
        out.append(math.floor(t))
        if out[-1] >= upto:
            return out


def round_cap(C: int, delta: float, nr: int) -> int:
    return 1 if nr <= 1 else int(math.log(nr) / math.log(1.0 + delta / C)) + 1


def brute_approx(csr, r, s, delta):
    """Algorithm 2 with synchronous rounds, on explicit clique lists."""
    adj = adjacency_sets(csr)
    R, S, deg, members = s_clique_degrees(adj, r, s)
    nr = len(R)
    C = comb(s, r)
    ends = bucket_ends(C, delta, max(deg, default=0) + 1)
    cap = round_cap(C, delta, nr)
    cur = list(deg)
    rnd = [None] * nr
    val = [0] * nr
    t = 0
    zero = [i for i in range(nr) if cur[i] == 0]
    for i in zero:
        rnd[i] = 0
    if zero:
        t = 1
    b, here = 0, 0
    by_member = [[] for _ in range(nr)]
    for si, ids in enumerate(members):
        for i in ids:
            by_member[i].append(si)
    while any(x is None for x in rnd):
        lvl = ends[b]
        A = [i for i in range(nr) if rnd[i] is None and cur[i] <= lvl]
        if not A:
            b, here = b + 1, 0
            continue
        for i in A:
            rnd[i] = t
            val[i] = lvl
        removed = set()
        for i in A:
            for si in by_member[i]:
                ids = members[si]
                if any(rnd[j] is not None and rnd[j] < t for j in ids):
                    continue        # destroyed in an earlier round
                removed.add(si)
        for si in removed:
            for j in members[si]:
                if rnd[j] is None:
                    cur[j] -= 1
        t += 1
        here += 1
        if here >= cap:
            b, here = b + 1, 0
    return val, members


def _graphs():
    rng = np.random.default_rng(7)
    out = [I.complete(6), I.two_k5_bridge(),
           I.disjoint_union(I.complete(5), I.complete(7), I.cycle(6))]
    for _ in range(5):
        n = int(rng.integers(6, 12))
        out.append(I.gnp(n, float(rng.uniform(0.3, 0.8)), seed=int(rng.integers(1 << 30))))
    out.append(I.er_planted(14, 0.2, 2, 4, 7, seed=5))
    return out


@pytest.mark.parametrize("r,s", PAIRS)
@pytest.mark.parametrize("delta", DELTAS)
def test_approx_matches_brute_rounds_and_tree(r, s, delta):
    for g in _graphs():
        a = oracle.approx_decompose(g, r, s, delta)
        val, members = brute_approx(g, r, s, delta)
        assert a.coreness.tolist() == val, (r, s, delta, g.n)
        # the tree of these values is the per-level component hierarchy
        parent, level = hierarchy_bfs(a.n_r, members, val)
        assert a.parent.tolist() == parent and a.level.tolist() == level
        # peeled in non-decreasing order of the assigned values
        pv = a.coreness[a.peel_order]
        assert np.all(pv[1:] >= pv[:-1])


@pytest.mark.parametrize("r,s", PAIRS)
@pytest.mark.parametrize("delta", DELTAS)
def test_approx_bound_against_exact(r, s, delta):
    C = comb(s, r)
    for g in _graphs() + [I.workload_er2k() if (r, s) in ((1, 2), (2, 3)) else
                          I.er_planted(400, 0.04, 5, 5, 12, seed=9)]:
        e = oracle.decompose(g, r, s)
        a = oracle.approx_decompose(g, r, s, delta)
        assert a.n_r == e.n_r and np.array_equal(a.count, e.count)
        core, apx = e.coreness.astype(np.float64), a.coreness.astype(np.float64)
        assert np.all((core == 0) == (apx == 0))
        assert np.all(apx >= core)
        assert np.all(apx <= (C + delta) * (1 + delta) * core + 1e-9)


@pytest.mark.parametrize("r,s", PAIRS)
def test_approx_complete_graph(r, s):
    """K_n: every r-clique lies in D = C(n-r, s-r) s-cliques; one round at
    the first bucket whose end reaches D peels all of them."""
    for n in range(s, 9):
        D = comb(n - r, s - r)
        for delta in DELTAS:
            a = oracle.approx_decompose(I.complete(n), r, s, delta)
            want = next(e for e in bucket_ends(comb(s, r), delta, D) if e >= D)
            assert set(a.coreness.tolist()) == {want}
            assert a.n_int == 1 and a.level.tolist() == [want]


def test_approx_rejects_bad_delta():
    for d in (0.0, -0.5):
        with pytest.raises(oracle.OracleError):
            oracle.approx_decompose(I.complete(5), 2, 3, d)
