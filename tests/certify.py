"""Checks of a decomposition that hold at any size (host side, numpy).

Used on full-size graphs where the oracle cannot run to the end. Every check
either follows from a definition in the paper or compares against values the
oracle computes one r-clique at a time (``oracle.Graph.incident``: the other
r-cliques of every s-clique containing a given r-clique).

Core numbers (Section 3 definition, sequential-peeling characterisation of
Section 6): for a sampled r-clique R with core c and peel round t,
  (1) at least c s-cliques containing R have all members of core >= c, and
  (2) at most c s-cliques containing R have all members peeled in round >= t;
with core numbers non-decreasing in the peel round, (1) for every R shows each
set {core >= c} is a c-nucleus set (cores are not too high) and (2) for every
R shows no r-clique could stay in a larger nucleus (cores are not too low).

Hierarchy (canonical tree): node levels decrease towards the root; each node's
level is the smallest core below it and it has >= 2 children; nodes are
numbered by (level, smallest leaf); for every sampled pair of s-clique-adjacent
r-cliques R, R' the node of level <= min(core) that contains R also contains
R' (no missing merge); sampled small nodes are connected at their level (no
spurious merge).
"""
from __future__ import annotations

import numpy as np

NONE = np.uint64(0xFFFFFFFFFFFFFFFF)


def check_core_certificates(G, core, rounds, counts, sample):
    core = core.astype(np.int64)
    rounds = rounds.astype(np.int64)
    order = np.argsort(rounds, kind="stable")
    assert np.all(np.diff(core[order]) >= 0), "core numbers decrease along the peel rounds"
    for rid in sample:
        inc = G.incident(int(rid)).astype(np.int64)
        assert inc.shape[0] == int(counts[rid]), ("count", rid)
        c = core[rid]
        if inc.shape[0] == 0:
            assert c == 0, ("core of an r-clique in no s-clique", rid)
            continue
        inside = int((core[inc].min(axis=1) >= c).sum())
        present = int((rounds[inc].min(axis=1) >= rounds[rid]).sum())
        assert inside >= c, ("certificate (1)", rid, inside, c)
        assert present <= c, ("certificate (2)", rid, present, c)


def _node_arrays(parent, level, core, n_r):
    n_int = level.size
    par = parent.astype(np.int64)
    par[parent == NONE] = -1
    lev = level.astype(np.int64)
    core = core.astype(np.int64)
    # direct children
    leaf_par = par[:n_r]
    node_par = par[n_r:]
    return n_int, par, lev, core, leaf_par, node_par


def check_tree_properties(parent, level, core, n_r):
    n_int, par, lev, core, leaf_par, node_par = _node_arrays(parent, level, core, n_r)
    assert par.size == n_r + n_int
    hl = leaf_par >= 0
    assert np.all(leaf_par[hl] >= n_r)
    assert np.all(lev[leaf_par[hl] - n_r] <= core[hl]), "a leaf sits below a node above its core"
    assert np.all(core[~hl] >= 0)
    hn = node_par >= 0
    assert np.all(node_par[hn] >= n_r)
    assert np.all(lev[node_par[hn] - n_r] < lev[np.arange(n_int)[hn]]), "levels must decrease upwards"
    # children counts, min core and min leaf per node, bottom-up by level
    nkids = np.zeros(n_int, dtype=np.int64)
    np.add.at(nkids, leaf_par[hl] - n_r, 1)
    np.add.at(nkids, node_par[hn] - n_r, 1)
    assert np.all(nkids >= 2), "a node with a single child"
    big = np.iinfo(np.int64).max
    mcore = np.full(n_int, big)
    mleaf = np.full(n_int, big)
    leaves = np.arange(n_r, dtype=np.int64)
    np.minimum.at(mcore, leaf_par[hl] - n_r, core[hl])
    np.minimum.at(mleaf, leaf_par[hl] - n_r, leaves[hl])
    for lv in np.unique(lev)[::-1]:
        idx = np.nonzero((lev == lv) & hn)[0]
        if idx.size:
            np.minimum.at(mcore, node_par[idx] - n_r, mcore[idx])
            np.minimum.at(mleaf, node_par[idx] - n_r, mleaf[idx])
    assert np.array_equal(mcore, lev), "node level differs from the smallest core below it"
    key = lev * (n_r + 1) + mleaf
    assert np.all(np.diff(key) > 0), "nodes are not numbered by (level, smallest leaf)"
    return mleaf


def ancestor_at(parent, level, n_r, x, c):
    """Deepest ancestor node of leaves x with level <= c (-1 if none).

    Levels strictly decrease towards the root, so the answer is found by
    binary lifting: jump tables of 2^j-th ancestors over the internal nodes
    (hierarchies can be tens of thousands of levels deep)."""
    par = parent.astype(np.int64)
    par[parent == NONE] = -1
    lev = level.astype(np.int64)
    n_int = lev.size
    node = par[np.asarray(x, dtype=np.int64)]          # first internal node (or -1)
    c = np.asarray(c, dtype=np.int64)
    if n_int == 0:
        return node
    up = [np.where(par[n_r:] >= 0, par[n_r:] - n_r, -1)]   # parent among nodes, -1 at roots
    while len(up) < 64:
        prev = up[-1]
        nxt = np.where(prev >= 0, prev[np.maximum(prev, 0)], -1)
        if np.array_equal(nxt, prev):
            break
        up.append(nxt)
    cur = np.where(node >= 0, node - n_r, -1)
    # climb while the node's level is above c: highest jumps first, only to
    # ancestors still above c; then one more step to the parent
    above = np.zeros(cur.shape, dtype=bool)
    ok = cur >= 0
    above[ok] = lev[cur[ok]] > c[ok]
    for tab in reversed(up):
        cand = np.where(above, tab[np.maximum(cur, 0)], -1)
        take = above & (cand >= 0)
        take[take] = lev[cand[take]] > c[take]
        cur = np.where(take, cand, cur)
    step = np.where(above, up[0][np.maximum(cur, 0)], cur)
    res = np.where(step >= 0, step + n_r, -1)
    return res


def check_adjacency_closure(G, parent, level, core, n_r, sample):
    """Every s-clique-adjacent pair (R, R') is inside one node at level
    min(core R, core R')."""
    core = core.astype(np.int64)
    xs, ys = [], []
    for rid in sample:
        inc = G.incident(int(rid)).astype(np.int64).ravel()
        if inc.size:
            xs.append(np.full(inc.size, int(rid), dtype=np.int64))
            ys.append(inc)
    if not xs:
        return 0
    x = np.concatenate(xs)
    y = np.concatenate(ys)
    c = np.minimum(core[x], core[y])
    ax = ancestor_at(parent, level, n_r, x, c)
    ay = ancestor_at(parent, level, n_r, y, c)
    bad = (ax < 0) | (ax != ay)
    assert not bad.any(), ("adjacent r-cliques not merged at their level",
                           int(x[bad][0]), int(y[bad][0]), int(c[bad][0]))
    return x.size


def check_small_nodes_connected(G, parent, level, core, n_r, max_leaves=300, max_nodes=20,
                                seed=0):
    """Sampled nodes with few leaves: their leaves are connected through
    s-cliques whose members all have core >= the node's level."""
    par = parent.astype(np.int64)
    par[parent == NONE] = -1
    n_int = level.size
    core = core.astype(np.int64)
    order = np.argsort(par, kind="stable")
    sp = par[order]
    starts = np.searchsorted(sp, np.arange(n_r, n_r + n_int), side="left")
    ends = np.searchsorted(sp, np.arange(n_r, n_r + n_int), side="right")

    def leaves_of(node):
        out, stack = [], [node]
        while stack:
            z = stack.pop()
            for ch in order[starts[z - n_r]:ends[z - n_r]]:
                if ch < n_r:
                    out.append(int(ch))
                else:
                    stack.append(int(ch))
                if len(out) > max_leaves:
                    return None
        return out

    rng = np.random.default_rng(seed)
    checked = 0
    for z in rng.permutation(np.arange(n_r, n_r + n_int)):
        if checked >= max_nodes:
            break
        lv = int(level[z - n_r])
        lf = leaves_of(int(z))
        if lf is None or len(lf) < 2:
            continue
        members = set(lf)
        adj = {x: set() for x in lf}
        for x in lf:
            inc = G.incident(x).astype(np.int64)
            for y in np.unique(inc.ravel()):
                y = int(y)
                if core[y] < lv:                # pairwise adjacency at level lv
                    continue
                assert y in members, ("node not closed", int(z), x, y)
                adj[x].add(y)
                adj[y].add(x)
        seen = {lf[0]}
        stack = [lf[0]]
        while stack:
            u = stack.pop()
            for w in adj[u]:
                if w not in seen:
                    seen.add(w)
                    stack.append(w)
        assert seen == members, ("node not connected at its level", int(z))
        checked += 1
    return checked
