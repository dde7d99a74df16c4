"""Pins of the oracle's hierarchy cut (the c-(r,s) nuclei from the
definition: components of the r-cliques of core >= c under s-clique
adjacency, with their vertex sets and induced edges) against breadth-first
search on brute-force cliques and core numbers, closed forms, and the
paper's pairwise-adjacency reading on two K5 joined at a vertex plus a
bridge."""
from __future__ import annotations

from math import comb

import numpy as np
import pytest

import oracle
from paper_2306_08623_amd import inputs as I

from brute import nuclei_bfs

PAIRS = [(1, 2), (2, 3), (1, 3), (2, 4), (3, 4), (1, 4)]


def _as_list(x):
    out = []
    off = x["vert_off"]
    for i in range(x["n_nuclei"]):
        verts = tuple(int(v) for v in x["verts"][int(off[i]):int(off[i + 1])])
        out.append((int(x["min_leaf"][i]), int(x["level"][i]), int(x["n_rcliques"][i]), verts,
                    int(x["n_edges"][i])))
    return out


def _check(g, r, s):
    d = oracle.decompose(g, r, s)
    for c in range(1, int(d.k) + 2):
        x = oracle.nuclei(g, r, s, d.coreness, c)
        got = _as_list(x)
        assert got == nuclei_bfs(g, r, s, c), (r, s, c)
        # consistency of the per-r-clique map with the lists
        leaf = x["leaf_nucleus"]
        assert np.array_equal(leaf >= 0, d.coreness >= c)
        for i, (ml, lv, nrc, verts, ne) in enumerate(got):
            assert int((leaf == i).sum()) == nrc
            assert leaf[ml] == i
            assert len(verts) == int(x["n_vertices"][i])


@pytest.mark.parametrize("r,s", PAIRS)
def test_nuclei_match_bfs_on_small_graphs(r, s):
    rng = np.random.default_rng(100 + 10 * r + s)
    for trial in range(6):
        n = int(rng.integers(5, 11))
        p = float(rng.uniform(0.3, 0.8))
        _check(I.gnp(n, p, seed=int(rng.integers(1 << 30))), r, s)
    _check(I.er_planted(13, 0.25, 2, 4, 6, seed=3), r, s)


@pytest.mark.parametrize("r,s", PAIRS)
def test_nuclei_closed_forms(r, s):
    for n in range(s, 8):
        g = I.complete(n)
        d = oracle.decompose(g, r, s)
        top = comb(n - r, s - r)
        x = oracle.nuclei(g, r, s, d.coreness, top)
        assert x["n_nuclei"] == 1
        assert int(x["n_rcliques"][0]) == comb(n, r)
        assert int(x["n_vertices"][0]) == n and int(x["n_edges"][0]) == comb(n, 2)
        assert oracle.nuclei(g, r, s, d.coreness, top + 1)["n_nuclei"] == 0
    # disjoint cliques are separate nuclei until the smaller one's level is passed
    g = I.disjoint_union(I.complete(5), I.complete(7))
    d = oracle.decompose(g, r, s)
    lo, hi = comb(5 - r, s - r), comb(7 - r, s - r)
    x = oracle.nuclei(g, r, s, d.coreness, lo)
    assert x["n_nuclei"] == 2
    assert sorted(int(v) for v in x["n_vertices"]) == [5, 7]
    assert sorted(int(e) for e in x["n_edges"]) == [10, 21]
    if hi > lo:
        x = oracle.nuclei(g, r, s, d.coreness, lo + 1)
        assert x["n_nuclei"] == 1 and int(x["n_vertices"][0]) == 7


def test_nuclei_pairwise_reading_two_k5():
    """Two K5 sharing vertex v plus the edge (a,b) between them, (2,3): the
    K5 edges (v,a) and (v,b) share triangle {v,a,b} of G, so at c = 3 all 20
    K5 edges form one nucleus (pairwise adjacency); its 9 vertices span 21
    edges of G (the bridge included, though the bridge's own core is 1)."""
    g = I.two_k5_bridge()
    d = oracle.decompose(g, 2, 3)
    x = oracle.nuclei(g, 2, 3, d.coreness, 3)
    assert x["n_nuclei"] == 1
    assert int(x["n_rcliques"][0]) == 20 and int(x["level"][0]) == 3
    assert int(x["n_vertices"][0]) == 9 and int(x["n_edges"][0]) == 21
    x = oracle.nuclei(g, 2, 3, d.coreness, 1)
    assert x["n_nuclei"] == 1 and int(x["n_rcliques"][0]) == 21 and int(x["level"][0]) == 1
    assert oracle.nuclei(g, 2, 3, d.coreness, 4)["n_nuclei"] == 0


def test_nuclei_rejects_level_zero():
    g = I.complete(4)
    d = oracle.decompose(g, 2, 3)
    with pytest.raises(oracle.OracleError):
        oracle.nuclei(g, 2, 3, d.coreness, 0)
