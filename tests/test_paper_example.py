"""The paper's worked (1,3) example: the tree of Algorithm 1 (Section 5) and
the tree of Algorithm 5 (Section 7.3) must be the same canonical tree once
parents with one child are removed. This pins the canonical form that the
oracle and the GPU path both emit."""
import json
import os

import brute

HERE = os.path.dirname(os.path.abspath(__file__))
NONE = brute.NONE


def _load():
    with open(os.path.join(HERE, "golden", "paper_example_trees.json")) as f:
        return json.load(f)


def _canon(spec, leaves):
    ids = {name: i for i, name in enumerate(leaves)}
    nxt = len(leaves)
    for name in spec["nodes"]:
        ids[name] = nxt
        nxt += 1
    parent = {ids[c]: ids[p] for c, p in spec["parent"].items()}
    level = {ids[nm]: lv for nm, lv in spec["nodes"].items()}
    return brute.canonicalize_forest(len(leaves), parent, level)


def test_alg1_and_alg5_trees_agree():
    g = _load()
    p1, l1 = _canon(g["alg1_tree"], g["leaves"])
    p5, l5 = _canon(g["alg5_tree"], g["leaves"])
    assert (p1, l1) == (p5, l5)
    # expected canonical form: three nodes at levels 1, 2, 3
    assert l1 == [1, 2, 3]
    n = len(g["leaves"])
    lv1, lv2, lv3 = n, n + 1, n + 2
    name = {nm: i for i, nm in enumerate(g["leaves"])}
    assert p1[name["1a"]] == lv1 and p1[name["2a"]] == lv2 and p1[name["4d"]] == lv2
    for nm in ("3a", "3b", "3c", "4a", "4b", "4c"):
        assert p1[name[nm]] == lv3
    assert p1[lv3] == lv2 and p1[lv2] == lv1 and p1[lv1] == NONE
