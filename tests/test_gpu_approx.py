"""GPU approximate decomposition (nd_set_approx: Algorithm 2's geometric
buckets in the persistent peel) against the oracle's round-synchronous
Algorithm 2, bit-exact: counts, approximate core numbers and the canonical
tree of those values, in both hierarchy modes. (The theorem's bound at full
R-MAT size is checked in test_gpu_fullsize.py.)"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2306_08623_amd import inputs as I

pytestmark = pytest.mark.gpu

RS = [(1, 2), (2, 3), (3, 4), (2, 4), (1, 3), (1, 4)]
DELTAS = [0.1, 0.5, 1.0]


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


def check(ctx, g, r, s, delta, tag, hierarchy="auto"):
    _say(f"[approx] {tag} n={g.n} m={g.m} (r,s)=({r},{s}) delta={delta} {hierarchy}")
    from paper_2306_08623_amd import nucleus
    if hierarchy != "auto":
        with nucleus.Context(device=0, hierarchy=hierarchy) as c2:
            res = c2.decompose_approx(g, r, s, delta)
    else:
        res = ctx.decompose_approx(g, r, s, delta)
    d = oracle.approx_decompose(g, r, s, delta)
    assert res.info["n_r"] == d.n_r and res.info["n_s"] == d.n_s, tag
    assert np.array_equal(res.counts.astype(np.uint64), d.count), tag
    assert np.array_equal(res.coreness.astype(np.uint64), d.coreness), tag
    assert res.info["k"] == d.k, tag
    assert np.array_equal(res.parent, d.parent), tag
    assert np.array_equal(res.level.astype(np.uint64), d.level), tag
    assert res.info["approx_delta"] == delta
    return res, d


@pytest.mark.parametrize("r,s", RS)
def test_approx_small(ctx, r, s):
    for delta in DELTAS:
        for name, g in [("K7", I.complete(7)), ("two-K5", I.two_k5_bridge()),
                        ("K5+K7+C6", I.disjoint_union(I.complete(5), I.complete(7), I.cycle(6))),
                        ("planted300", I.er_planted(300, 0.03, 6, 5, 14, seed=21)),
                        ("edgeless", I.empty(5))]:
            check(ctx, g, r, s, delta, name)


@pytest.mark.parametrize("r,s", [(1, 2), (2, 3), (3, 4), (2, 4)])
def test_approx_er2k_rmat12(ctx, r, s):
    for delta in DELTAS:
        check(ctx, I.workload_er2k(), r, s, delta, "er2k")
    check(ctx, I.rmat(12, 16, 2), r, s, 0.1, "rmat12")


@pytest.mark.parametrize("r,s", [(2, 3), (3, 4)])
def test_approx_both_hierarchy_modes(r, s):
    g = I.er_planted(600, 0.02, 8, 5, 16, seed=44)
    for mode in ("el", "te"):
        check(None, g, r, s, 0.5, "planted600", hierarchy=mode)


def test_approx_rounds_fewer_and_exact_mode_restored(ctx):
    """Geometric buckets need far fewer rounds than exact levels; after
    delta = 0 the context peels exactly again."""
    g = I.rmat(13, 16, 2)
    ex = ctx.decompose(g, 2, 3)
    ap = ctx.decompose_approx(g, 2, 3, 0.5)
    assert ap.info["rounds"] < ex.info["rounds"]
    again = ctx.decompose(g, 2, 3)
    assert np.array_equal(again.coreness, ex.coreness)
    d = oracle.decompose(g, 2, 3)
    assert np.array_equal(again.coreness.astype(np.uint64), d.coreness)


def test_approx_errors(ctx):
    from paper_2306_08623_amd import nucleus
    for bad in (-1.0, float("nan"), 1e9):
        with pytest.raises(nucleus.NucleusError) as e:
            ctx.nd_set_approx(bad)
        assert e.value.code == nucleus.ND_E_INVALID_ARG
    ctx.nd_set_approx(0.5)
    with pytest.raises(nucleus.NucleusError) as e:
        ctx.decompose_batch([(I.complete(5), 2, 3)])
    assert e.value.code == nucleus.ND_E_UNSUPPORTED
    ctx.nd_set_approx(0.0)
    assert len(ctx.decompose_batch([(I.complete(5), 2, 3)])) == 1
