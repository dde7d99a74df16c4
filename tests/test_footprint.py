"""Host-side checks of the admission estimate (nd_estimate_footprint needs no
GPU for host inputs): its r-clique bound never falls below the true number of
r-cliques (the oracle's count), and the estimate grows with the graph."""
from __future__ import annotations

import pytest

import oracle
from paper_2306_08623_amd import inputs as I


def _bound_nr(res_bytes, r):
    return (res_bytes - 256) // (4 * r + 28)


@pytest.mark.parametrize("r,s", [(1, 2), (2, 3), (3, 4)])
def test_rclique_bound_holds(r, s):
    from paper_2306_08623_amd import nucleus
    graphs = [I.complete(9), I.empty(4), I.two_k5_bridge(), I.workload_er2k(),
              I.rmat(10, 16, 2)] + [I.serve_graph(i, m_hi=20_000)[0] for i in range(6)]
    for g in graphs:
        ws, res = nucleus.estimate_footprint(g, r, s)
        d = oracle.count(g, r, s)
        assert _bound_nr(res, r) >= d.n_r, (g.n, g.m, r, s)
        assert ws >= 32 * g.m


def test_estimate_grows_with_size():
    from paper_2306_08623_amd import nucleus
    a = nucleus.estimate_footprint(I.rmat(10, 8, 3), 3, 4)
    b = nucleus.estimate_footprint(I.rmat(12, 8, 3), 3, 4)
    assert b[0] > a[0] and b[1] > a[1]
