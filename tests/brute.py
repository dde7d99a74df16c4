"""Brute-force references for tiny graphs (pure Python, itertools).

These pin the oracle with algorithms that differ from its own:

* cliques by testing every vertex subset;
* core numbers by the fixed-point definition of a c-(r,s) nucleus
  (Section 3): Y_c is the largest set of r-cliques in which every member lies
  in at least c s-cliques whose r-cliques all belong to Y_c, found by
  iterated deletion; the core number of R is the largest c with R in Y_c;
* the hierarchy by the "vanilla" method the paper contrasts with Algorithm 1
  (end of Section 5): breadth-first components of the s-clique-adjacency graph
  restricted to core >= c, separately for every c;
* canonical form of any rooted forest over the r-cliques (the paper's
  remark in Section 7.3 that parents with one child can be removed).
"""
from __future__ import annotations

from itertools import combinations

import numpy as np

NONE = 0xFFFFFFFFFFFFFFFF


def adjacency_sets(csr) -> list[set[int]]:
    rp = csr.row_ptr.astype(np.int64)
    return [set(int(x) for x in csr.col[rp[u]:rp[u + 1]]) for u in range(csr.n)]


def cliques(adj: list[set[int]], q: int) -> list[tuple[int, ...]]:
    n = len(adj)
    out = []
    for t in combinations(range(n), q):
        if all(b in adj[a] for a, b in combinations(t, 2)):
            out.append(t)
    return out


def s_clique_degrees(adj, r, s):
    R = cliques(adj, r)
    idx = {t: i for i, t in enumerate(R)}
    S = cliques(adj, s)
    deg = [0] * len(R)
    members = []
    for sc in S:
        ids = [idx[sub] for sub in combinations(sc, r)]
        members.append(ids)
        for i in ids:
            deg[i] += 1
    return R, S, deg, members


def coreness_fixpoint(n_r: int, members: list[list[int]]) -> list[int]:
    """ND[R] = max{c : R in Y_c}, Y_c by iterated deletion."""
    nd = [0] * n_r
    c = 1
    while True:
        alive = [True] * n_r
        changed = True
        while changed:
            changed = False
            cnt = [0] * n_r
            for ids in members:
                if all(alive[i] for i in ids):
                    for i in ids:
                        cnt[i] += 1
            for i in range(n_r):
                if alive[i] and cnt[i] < c:
                    alive[i] = False
                    changed = True
        if not any(alive):
            return nd
        for i in range(n_r):
            if alive[i]:
                nd[i] = c
        c += 1


def hierarchy_bfs(n_r: int, members: list[list[int]], nd: list[int]):
    """Canonical tree from per-level BFS components.

    Returns (parent list of length n_r + n_int, level list of length n_int).
    """
    nbrs = [set() for _ in range(n_r)]
    for ids in members:
        for a, b in combinations(ids, 2):
            nbrs[a].add(b)
            nbrs[b].add(a)
    k = max(nd) if nd else 0
    nodes: dict[frozenset, int] = {}
    for c in range(1, k + 1):
        seen = set()
        for v in range(n_r):
            if nd[v] < c or v in seen:
                continue
            comp = {v}
            stack = [v]
            seen.add(v)
            while stack:
                x = stack.pop()
                for y in nbrs[x]:
                    if nd[y] >= c and y not in seen:
                        seen.add(y)
                        comp.add(y)
                        stack.append(y)
            if len(comp) >= 2:
                fs = frozenset(comp)
                nodes[fs] = max(nodes.get(fs, 0), c)
    return canonical_from_sets(n_r, nodes)


def canonical_from_sets(n_r: int, nodes: dict[frozenset, int]):
    order = sorted(nodes.items(), key=lambda kv: (kv[1], min(kv[0])))
    canon = {fs: n_r + i for i, (fs, _) in enumerate(order)}
    parent = [NONE] * (n_r + len(order))
    level = [lv for _, lv in order]
    # smallest strictly containing set
    sets = [fs for fs, _ in order]
    for x in range(n_r):
        best = None
        for fs in sets:
            if x in fs and (best is None or len(fs) < len(best)):
                best = fs
        if best is not None:
            parent[x] = canon[best]
    for fs in sets:
        best = None
        for gs in sets:
            if gs is not fs and fs < gs and (best is None or len(gs) < len(best)):
                best = gs
        if best is not None:
            parent[canon[fs]] = canon[best]
    return parent, level


def canonicalize_forest(n_leaves: int, parent: dict, level: dict):
    """Canonical form of a forest given by ``parent`` (node -> parent node or
    None) and ``level`` (internal node -> level), leaves ``0..n_leaves-1``.

    Unary internal nodes are removed (their child goes to their parent);
    internal nodes are renumbered n_leaves + rank of (level, min leaf)."""
    parent = dict(parent)
    internal = [x for x in level]
    children: dict = {x: [] for x in internal}
    for x, p in parent.items():
        if p is not None:
            children[p].append(x)
    # remove unary nodes repeatedly
    changed = True
    while changed:
        changed = False
        for x in list(children):
            if len(children[x]) == 1:
                (ch,) = children[x]
                px = parent.get(x)
                parent[ch] = px
                if px is not None:
                    children[px].remove(x)
                    children[px].append(ch)
                del children[x]
                parent.pop(x, None)
                changed = True
            elif len(children[x]) == 0:
                px = parent.get(x)
                if px is not None:
                    children[px].remove(x)
                del children[x]
                parent.pop(x, None)
                changed = True

    def leaves(x):
        if x not in children:
            return [x]
        out = []
        for c in children[x]:
            out.extend(leaves(c))
        return out

    sets = {x: frozenset(leaves(x)) for x in children}
    order = sorted(children, key=lambda x: (level[x], min(sets[x])))
    canon = {x: n_leaves + i for i, x in enumerate(order)}
    out_parent = [NONE] * (n_leaves + len(order))
    for x in range(n_leaves):
        p = parent.get(x)
        out_parent[x] = NONE if p is None else canon[p]
    for x in order:
        p = parent.get(x)
        out_parent[canon[x]] = NONE if p is None else canon[p]
    return out_parent, [level[x] for x in order]


def brute_all(csr, r: int, s: int):
    adj = adjacency_sets(csr)
    R, S, deg, members = s_clique_degrees(adj, r, s)
    nd = coreness_fixpoint(len(R), members)
    parent, level = hierarchy_bfs(len(R), members, nd)
    return {"rcliques": R, "n_s": len(S), "count": deg, "coreness": nd,
            "parent": parent, "level": level}


def nuclei_bfs(csr, r: int, s: int, c: int):
    """The c-(r,s) nuclei by breadth-first search over s-clique adjacency
    among the r-cliques of core >= c (core numbers by the fixed point above):
    a list, ordered by smallest member, of (smallest member, smallest core
    inside, r-clique count, sorted vertex tuple, edges of G among those
    vertices)."""
    adj = adjacency_sets(csr)
    R, S, deg, members = s_clique_degrees(adj, r, s)
    nd = coreness_fixpoint(len(R), members)
    nbrs = [set() for _ in range(len(R))]
    for ids in members:
        for a, b in combinations(ids, 2):
            nbrs[a].add(b)
            nbrs[b].add(a)
    out, seen = [], set()
    for v in range(len(R)):
        if nd[v] < c or v in seen:
            continue
        comp, stack = {v}, [v]
        seen.add(v)
        while stack:
            x = stack.pop()
            for y in nbrs[x]:
                if nd[y] >= c and y not in seen:
                    seen.add(y)
                    comp.add(y)
                    stack.append(y)
        verts = sorted({u for i in comp for u in R[i]})
        vs = set(verts)
        edges = sum(1 for a in verts for b in adj[a] if b > a and b in vs)
        out.append((min(comp), min(nd[i] for i in comp), len(comp), tuple(verts), edges))
    return out
