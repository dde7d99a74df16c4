"""Full-size parity on the Chung-Lu workload (n = 4,000,000, exponent 2.1,
~40M sampled edges + 1,000 dense communities, seed 3; m = 44,187,397), for
(3,4) and (2,4), in the configuration the library runs by default (Algorithm
5 linking for (3,4), the descending-core build for (2,4)).

A full oracle run would take days (7.1e9 4-cliques). The r-clique listing is
compared in full with the oracle's own listing; counts and core numbers are
checked on sampled r-cliques against values the oracle computes one r-clique
at a time, with the certificates of tests/certify.py; the tree is checked for
the properties that hold at any size, for adjacency closure on sampled
r-cliques and for connectivity of sampled small nodes. Sampled r-cliques are
drawn among those in at most 200,000 s-cliques (the oracle lists every
incident s-clique of a sampled r-clique; hub edges are in millions).
"""
from __future__ import annotations

from math import comb

import numpy as np
import pytest

import certify
import oracle
from paper_2306_08623_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    from conftest import progress
    progress(msg)


@pytest.fixture(scope="module")
def cl4m():
    _say("[cl4m] generating the graph")
    return I.workload_chung_lu_4m()


def _run(g, r, s, hierarchy="auto"):
    from paper_2306_08623_amd import nucleus
    with nucleus.Context(device=0, progress=True, hierarchy=hierarchy) as ctx:
        ctx.load_csr(g)
        ctx.nd_set_rs(r, s)
        ctx.nd_decompose()
        info = ctx.nd_get_info()
        out = dict(info=info, rcl=ctx.nd_get_rcliques(), counts=ctx.nd_get_counts(),
                   core=ctx.nd_get_coreness(), rounds=ctx.nd_get_peel_rounds())
        out["parent"], out["level"] = ctx.nd_get_tree()
    return out


def _check(g, r, s, res, n_sample):
    info, counts, core = res["info"], res["counts"], res["core"]
    n_r = info["n_r"]
    assert int(counts.astype(np.uint64).sum()) == comb(s, r) * info["n_s"]
    assert info["visits"] == comb(s, r) * info["n_s"]
    assert int(core.max()) == info["k"]
    assert np.all(core <= counts)
    _say(f"[cl4m] ({r},{s}): oracle listing of the r-cliques")
    G = oracle.Graph(g, r, s)
    _say(f"[cl4m] ({r},{s}): oracle listed {G.n_r} r-cliques")
    assert G.n_r == n_r
    assert np.array_equal(G.rcliques(), res["rcl"])
    _say(f"[cl4m] ({r},{s}): listings equal")
    rng = np.random.default_rng(10 * r + s)
    small = np.nonzero(counts <= 200_000)[0]
    sample = rng.choice(small, size=min(small.size, n_sample), replace=False)
    extremes = [int(np.argmin(core))]
    light = small[np.argmax(core[small])]          # highest core among the light ones
    sample = np.unique(np.concatenate([sample, extremes, [light]]))
    _say(f"[cl4m] ({r},{s}): certificates on {sample.size} r-cliques")
    certify.check_core_certificates(G, core, res["rounds"], counts, sample)
    _say(f"[cl4m] ({r},{s}): tree properties")
    certify.check_tree_properties(res["parent"], res["level"], core, n_r)
    closure = sample[counts[sample] <= 5000][:400]
    _say(f"[cl4m] ({r},{s}): adjacency closure from {closure.size} r-cliques")
    npairs = certify.check_adjacency_closure(G, res["parent"], res["level"], core, n_r, closure)
    _say(f"[cl4m] ({r},{s}): small nodes")
    nodes = certify.check_small_nodes_connected(G, res["parent"], res["level"], core, n_r,
                                                max_nodes=10)
    _say(f"[cl4m] ({r},{s}): {npairs} adjacent pairs closed, {nodes} small nodes connected")
    G.close()


@pytest.mark.timeout(1200)
def test_chunglu4m_34(cl4m):
    _say("[cl4m] (3,4): GPU decomposition")
    res = _run(cl4m, 3, 4)
    # the hierarchy built after the peel instead of during it: identical
    # results, element by element
    _say("[cl4m] (3,4): GPU decomposition, descending-core hierarchy")
    te = _run(cl4m, 3, 4, hierarchy="te")
    assert res["info"]["hier_te"] == 0 and te["info"]["hier_te"] == 1
    for f in ("counts", "core", "parent", "level"):
        assert np.array_equal(res[f], te[f]), f
    del te
    _check(cl4m, 3, 4, res, 3000)


@pytest.mark.timeout(1200)
def test_chunglu4m_24(cl4m):
    _say("[cl4m] (2,4): GPU decomposition")
    res = _run(cl4m, 2, 4)
    assert res["info"]["hier_te"] == 1
    _check(cl4m, 2, 4, res, 3000)
