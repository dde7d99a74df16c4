"""GPU hierarchy cut (nd_cut / nd_get_cut: the c-(r,s) nuclei read off the
canonical tree) against the oracle's nuclei from the definition (components
of the r-cliques of core >= c, no tree), element by element at every level:
nucleus, level, r-clique count, vertex set, induced edges, and every
r-clique's nucleus."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2306_08623_amd import inputs as I

pytestmark = pytest.mark.gpu

RS = [(1, 2), (2, 3), (3, 4), (2, 4), (1, 3), (1, 4)]


def _say(msg):
    from conftest import progress
    progress(msg)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2306_08623_amd import nucleus
    c = nucleus.Context(device=0)
    yield c
    c.close()


def check_cut(ctx, g, r, s, levels, tag):
    _say(f"[cut] {tag} n={g.n} m={g.m} (r,s)=({r},{s}) levels={len(levels)}")
    res = ctx.decompose(g, r, s)
    d = oracle.decompose(g, r, s)
    assert np.array_equal(res.coreness.astype(np.uint64), d.coreness), tag
    for c in levels:
        got = ctx.cut(c)
        want = oracle.nuclei(g, r, s, d.coreness, c)
        nuc = got["nuclei"]
        nn = want["n_nuclei"]
        assert len(nuc) == nn, (tag, c)
        # nuclei come in node order on the GPU and by smallest leaf in the
        # oracle: match them by smallest leaf (unique per nucleus)
        order = np.argsort(nuc["min_leaf"], kind="stable")
        g_sorted = nuc[order]
        assert np.array_equal(g_sorted["min_leaf"], want["min_leaf"]), (tag, c)
        assert np.array_equal(g_sorted["level"].astype(np.uint64), want["level"]), (tag, c)
        assert np.array_equal(g_sorted["n_rcliques"], want["n_rcliques"]), (tag, c)
        assert np.array_equal(g_sorted["n_vertices"], want["n_vertices"]), (tag, c)
        assert np.array_equal(g_sorted["n_edges"], want["n_edges"]), (tag, c)
        off = want["vert_off"]
        for i in range(nn):
            q = g_sorted[i]
            gv = got["verts"][int(q["vert_off"]):int(q["vert_off"] + q["n_vertices"])]
            assert np.array_equal(gv, want["verts"][int(off[i]):int(off[i + 1])]), (tag, c, i)
            # the nucleus is a tree node of level >= c
            assert q["node"] >= res.info["n_r"] and q["level"] >= c
        # every r-clique's nucleus, mapped to the oracle's numbering
        rank = np.empty(nn, dtype=np.int64)
        rank[order] = np.arange(nn)
        gl = got["leaf_nucleus"]
        mapped = np.full(gl.shape, -1, dtype=np.int64)
        mapped[gl >= 0] = rank[gl[gl >= 0]]
        assert np.array_equal(mapped, want["leaf_nucleus"]), (tag, c)
        # the vertex lists tile exactly
        assert int(nuc["n_vertices"].sum()) == len(got["verts"])


@pytest.mark.parametrize("r,s", RS)
def test_cut_every_level_small(ctx, r, s):
    for name, g in [("two-K5", I.two_k5_bridge()),
                    ("K5+K7+C6", I.disjoint_union(I.complete(5), I.complete(7), I.cycle(6))),
                    ("planted300", I.er_planted(300, 0.03, 6, 5, 14, seed=21)),
                    ("edgeless", I.empty(6))]:
        d = oracle.decompose(g, r, s)
        check_cut(ctx, g, r, s, list(range(1, int(d.k) + 2)), name)


@pytest.mark.parametrize("r,s", [(2, 3), (3, 4), (1, 2)])
def test_cut_er2k(ctx, r, s):
    g = I.workload_er2k()
    d = oracle.decompose(g, r, s)
    k = int(d.k)
    levels = sorted({1, 2, max(1, k // 4), max(1, k // 2), max(1, 3 * k // 4), k, k + 1})
    check_cut(ctx, g, r, s, levels, "er2k")


def test_cut_rmat12_34(ctx):
    g = I.rmat(12, 16, 2)
    d = oracle.decompose(g, 3, 4)
    k = int(d.k)
    check_cut(ctx, g, 3, 4, sorted({1, k // 3 or 1, 2 * k // 3 or 1, k}), "rmat12")


def test_cut_errors(ctx):
    from paper_2306_08623_amd import nucleus
    g = I.complete(5)
    ctx.decompose(g, 2, 3)
    with pytest.raises(nucleus.NucleusError) as e:
        ctx.nd_cut(0)
    assert e.value.code == nucleus.ND_E_INVALID_ARG
    with nucleus.Context(device=0) as fresh:
        with pytest.raises(nucleus.NucleusError) as e:
            fresh.nd_cut(1)
        assert e.value.code == nucleus.ND_E_STATE
    # the context stays usable
    check_cut(ctx, g, 2, 3, [1, 2, 3, 4], "K5 after errors")
