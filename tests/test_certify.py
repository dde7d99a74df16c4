"""The full-size checks in certify.py accept the oracle's exact outputs and
reject planted mistakes (mistakes are planted in copies of the oracle's
outputs, on the CPU)."""
import numpy as np
import pytest

import certify
import oracle
from paper_2306_08623_amd import inputs as I


def _setup(r, s, seed=5):
    g = I.er_planted(160, 0.06, 5, 6, 14, seed)
    d = oracle.decompose(g, r, s)
    G = oracle.Graph(g, r, s)
    rounds = np.empty(d.n_r, dtype=np.int64)
    rounds[d.peel_order.astype(np.int64)] = np.arange(d.n_r)   # sequential peel positions
    return g, d, G, rounds


@pytest.mark.parametrize("r,s", [(1, 2), (2, 3), (3, 4)])
def test_accepts_exact_outputs(r, s):
    g, d, G, rounds = _setup(r, s)
    allr = np.arange(d.n_r)
    certify.check_core_certificates(G, d.coreness, rounds, d.count, allr)
    certify.check_tree_properties(d.parent, d.level, d.coreness, d.n_r)
    assert certify.check_adjacency_closure(G, d.parent, d.level, d.coreness, d.n_r, allr) > 0
    assert certify.check_small_nodes_connected(G, d.parent, d.level, d.coreness, d.n_r) > 0


@pytest.mark.parametrize("r,s", [(2, 3), (3, 4)])
def test_rejects_wrong_core(r, s):
    g, d, G, rounds = _setup(r, s)
    allr = np.arange(d.n_r)
    x = int(np.argmax(d.coreness))
    for delta in (+1, -1):
        bad = d.coreness.astype(np.int64).copy()
        bad[x] += delta
        with pytest.raises(AssertionError):
            certify.check_core_certificates(G, bad, rounds, d.count, allr)


@pytest.mark.parametrize("r,s", [(2, 3), (3, 4)])
def test_rejects_wrong_tree(r, s):
    g, d, G, rounds = _setup(r, s)
    allr = np.arange(d.n_r)
    n_r = d.n_r
    # move one leaf of the deepest node to the root-most node of another tree
    par = d.parent.copy()
    leaf = int(np.nonzero(par[:n_r] != certify.NONE)[0][0])
    top = [z for z in range(n_r, n_r + d.n_int)
           if par[z] == certify.NONE and z != par[leaf]]
    if top:
        par[leaf] = top[0]
        with pytest.raises(AssertionError):
            certify.check_tree_properties(par, d.level, d.coreness, n_r)
            certify.check_adjacency_closure(G, par, d.level, d.coreness, n_r, allr)
    # split: detach a whole node from its parent
    par = d.parent.copy()
    inner = [z for z in range(n_r, n_r + d.n_int) if par[z] != certify.NONE]
    if inner:
        par[inner[0]] = certify.NONE
        with pytest.raises(AssertionError):
            certify.check_tree_properties(par, d.level, d.coreness, n_r)
            certify.check_adjacency_closure(G, par, d.level, d.coreness, n_r, allr)
