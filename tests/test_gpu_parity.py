"""GPU parity: the HIP path through the C ABI against the CPU oracle,
element by element and bit-exact (integers throughout): r-clique listing,
initial s-clique counts, core numbers and the canonical tree."""
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


def check(ctx, g, r, s, tag=""):
    _say(f"[parity] {tag} n={g.n} m={g.m} (r,s)=({r},{s})")
    res = ctx.decompose(g, r, s)
    d = oracle.decompose(g, r, s)
    assert res.info["n_r"] == d.n_r, tag
    assert res.info["n_s"] == d.n_s, tag
    assert np.array_equal(res.rcliques, d.rcliques.reshape(d.n_r, r)), tag
    assert np.array_equal(res.counts.astype(np.uint64), d.count), tag
    assert np.array_equal(res.coreness.astype(np.uint64), d.coreness), tag
    assert res.info["k"] == d.k, tag
    assert res.info["n_int"] == d.n_int, tag
    assert np.array_equal(res.parent, d.parent), tag
    assert np.array_equal(res.level.astype(np.uint64), d.level), tag
    # every (r-clique, s-clique) incidence is visited once while peeling
    from math import comb
    assert res.info["visits"] == comb(s, r) * d.n_s, tag
    return res, d


@pytest.mark.parametrize("r,s", RS)
def test_closed_forms(ctx, r, s):
    for n in range(1, 9):
        check(ctx, I.complete(n), r, s, f"K{n}")
    check(ctx, I.two_k5_bridge(), r, s, "two-K5")
    check(ctx, I.disjoint_union(I.complete(5), I.complete(7), I.cycle(6)), r, s, "K5+K7+C6")
    check(ctx, I.star(9), r, s, "star")
    check(ctx, I.empty(5), r, s, "edgeless")


@pytest.mark.parametrize("r,s", RS)
def test_random_small(ctx, r, s):
    rng = np.random.default_rng(r * 10 + s)
    for i in range(40):
        n = int(rng.integers(2, 40))
        p = float(rng.uniform(0.05, 0.7))
        check(ctx, I.gnp(n, p, seed=1000 + i), r, s, f"gnp{i}")


@pytest.mark.parametrize("r,s", RS)
def test_planted_medium(ctx, r, s):
    for seed in (1, 2, 3):
        g = I.er_planted(600, 0.015, 8, 5, 18, seed)
        check(ctx, g, r, s, f"planted600/{seed}")


@pytest.mark.parametrize("r,s", RS)
def test_er2k_workload(ctx, r, s):
    """G(2000, 0.01) + 20 planted cliques of sizes 5..30 (several tiles of
    every kernel, ragged tails)."""
    check(ctx, I.workload_er2k(), r, s, "er2k")


@pytest.mark.parametrize("r,s", [(2, 3), (3, 4), (2, 4), (1, 3), (1, 4)])
def test_rmat_small(ctx, r, s):
    """Skewed degrees: R-MAT scale 12, edge factor 16."""
    check(ctx, I.rmat(12, 16, seed=7), r, s, "rmat12")


def test_schedule_invariance(ctx):
    """Same input under different persistent-grid sizes: identical canonical
    outputs (the lock-free link and the atomic counts must not depend on the
    interleaving)."""
    from paper_2306_08623_amd import nucleus
    g = I.er_planted(800, 0.02, 10, 6, 20, 5)
    for r, s in [(2, 3), (3, 4), (2, 4), (1, 3), (1, 4)]:
        d = oracle.decompose(g, r, s)
        for nb in (1, 3, 16, 64, 0):
            with nucleus.Context(device=0, peel_blocks=nb) as c2:
                _say(f"[schedule] (r,s)=({r},{s}) peel_blocks={nb}")
                res = c2.decompose(g, r, s)
                assert np.array_equal(res.coreness.astype(np.uint64), d.coreness)
                assert np.array_equal(res.parent, d.parent)
                assert np.array_equal(res.level.astype(np.uint64), d.level)


def test_schedule_table(ctx):
    """nd_set_schedule: a table that sends every (3,4) decomposition to a
    grid of 8 workgroups gives the oracle's results (the grid changes no
    result); malformed entries are refused."""
    from paper_2306_08623_amd import nucleus
    g = I.er_planted(800, 0.02, 10, 6, 20, 5)
    tab = [{"kind": nucleus.ND_SCHED_SINGLE, "r": 3, "s": 4, "n_r_max": 10, "peel_blocks": 1024},
           {"kind": nucleus.ND_SCHED_SINGLE, "r": 3, "s": 4, "n_r_max": (1 << 64) - 1,
            "peel_blocks": 8},
           {"kind": nucleus.ND_SCHED_BATCH, "r": 2, "s": 3, "n_r_max": (1 << 64) - 1,
            "peel_blocks": 3}]
    with nucleus.Context(device=0, schedule=tab) as c2:
        check(c2, g, 3, 4, "schedule 8 blocks")
        out = c2.decompose_batch([(I.er_planted(300, 0.03, 4, 5, 12, i), 2, 3) for i in range(6)])
        for i, b in enumerate(out):
            d = oracle.decompose(I.er_planted(300, 0.03, 4, 5, 12, i), 2, 3)
            assert np.array_equal(b.coreness.astype(np.uint64), d.coreness), i
            assert np.array_equal(b.parent, d.parent), i
        for bad in ({"kind": 0, "r": 3, "s": 3, "n_r_max": 1, "peel_blocks": 1},
                    {"kind": 0, "r": 1, "s": 9, "n_r_max": 1, "peel_blocks": 1},
                    {"kind": 7, "r": 1, "s": 2, "n_r_max": 1, "peel_blocks": 1}):
            with pytest.raises(nucleus.NucleusError) as e:
                c2.set_schedule([bad])
            assert e.value.code == nucleus.ND_E_INVALID_ARG
        c2.set_schedule([])
        check(c2, g, 3, 4, "schedule cleared")


def test_error_paths(ctx):
    from paper_2306_08623_amd import nucleus
    bad = I.CSR(3, np.array([0, 1, 1, 1], dtype=np.uint64), np.array([1], dtype=np.uint32))
    with pytest.raises(nucleus.NucleusError) as e:
        ctx.load_csr(bad)
    assert e.value.code == nucleus.ND_E_BAD_GRAPH
    loop = I.CSR(2, np.array([0, 1, 2], dtype=np.uint64), np.array([0, 1], dtype=np.uint32))
    with pytest.raises(nucleus.NucleusError) as e:
        ctx.load_csr(loop)
    assert e.value.code == nucleus.ND_E_BAD_GRAPH
    ctx.load_csr(I.complete(5))
    with pytest.raises(nucleus.NucleusError) as e:
        ctx.nd_set_rs(3, 3)
    assert e.value.code == nucleus.ND_E_INVALID_ARG
    with pytest.raises(nucleus.NucleusError) as e:
        ctx.nd_set_rs(4, 8)
    assert e.value.code == nucleus.ND_E_UNSUPPORTED
    with nucleus.Context(device=0, mem_limit=4096) as small:
        with pytest.raises(nucleus.NucleusError) as e:
            small.decompose(I.complete(30), 2, 3)
        assert e.value.code == nucleus.ND_E_OOM
    # the context is still usable after errors
    check(ctx, I.complete(6), 2, 3, "after-errors")


def _bipartite_plus_clique(a: int, q: int):
    """K_{a,a} plus a clique on q vertices of each side: an orientation with
    out-degree above 1024 (degeneracy about a) whose s-cliques all touch
    the planted clique."""
    left = list(range(a))
    right = list(range(a, 2 * a))
    edges = [(u, v) for u in left for v in right]
    planted = left[:q] + right[:q]
    edges += [(planted[i], planted[j]) for i in range(len(planted))
              for j in range(i + 1, len(planted))]
    return I.from_edges(2 * a, edges)


def test_outdegree_above_lds_cap(ctx):
    """s = 4 on a graph whose oriented out-degree passes 1024 (the on-chip
    C2 buffer): the heavy rows go to the global-memory counter; results
    equal the oracle's. The context stays usable."""
    g = _bipartite_plus_clique(1030, 4)
    for r, s in [(3, 4), (2, 4), (1, 4)]:
        res, d = check(ctx, g, r, s, "K1030,1030+K8")
        assert res.info["max_outdeg"] > 1024
    check(ctx, I.complete(7), 3, 4, "after-outdegree-limit")


@pytest.mark.parametrize("r,s", [(3, 4), (2, 4), (1, 4)])
def test_count_global_c2(r, s):
    """Every row through the global-memory C2 slices (ND_FLAG_COUNT_GLOBAL):
    the same counts, cores and trees as the oracle."""
    from paper_2306_08623_amd import nucleus
    with nucleus.Context(device=0, count_global=True) as c2:
        for g, name in [(I.workload_er2k(), "er2k"), (I.rmat(12, 16, seed=7), "rmat12"),
                        (I.complete(9), "K9"), (I.two_k5_bridge(), "two-K5")]:
            check(c2, g, r, s, f"{name}/global-C2")


def test_progress_reports(capfd):
    """ND_FLAG_PROGRESS prints the end of every phase to stderr."""
    from paper_2306_08623_amd import nucleus
    g = I.workload_er2k()
    with nucleus.Context(device=0, progress=True) as c2:
        res = c2.decompose(g, 3, 4)
    err = capfd.readouterr().err
    for tag in ("prep queued", "count done", "peel done", "tree done"):
        assert f"[nd] {tag}" in err, err
    assert f"n_s={res.info['n_s']}" in err


@pytest.mark.parametrize("mode", ["el", "te"])
@pytest.mark.parametrize("r,s", RS)
def test_hierarchy_modes(r, s, mode):
    """Algorithm 5 during the peel (EL) and the descending-core build after
    it (TE) give the oracle's canonical tree for every pair."""
    from paper_2306_08623_amd import nucleus
    graphs = [(I.workload_er2k(), "er2k"), (I.er_planted(600, 0.015, 8, 5, 18, 2), "planted600"),
              (I.two_k5_bridge(), "two-K5"), (I.complete(7), "K7")]
    if (r, s) != (2, 4):
        graphs.append((I.rmat(12, 16, seed=7), "rmat12"))
    with nucleus.Context(device=0, hierarchy=mode) as c2:
        for g, name in graphs:
            res, d = check(c2, g, r, s, f"{name}/{mode}")
            assert res.info["hier_te"] == (1 if mode == "te" else 0)
