"""Batched decomposition through the C ABI (nd_batch_decompose / nd_batch_get).

Each graph of a batch must come out exactly as when decomposed alone, and as
the oracle computes it: r-cliques, counts, core numbers and canonical tree
(union decomposition is exact, see include/nucleus.h). The full 4,096-graph
mixed batch is compared per graph with digests the oracle wrote
(tests/golden/make_batch_golden.py).
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2306_08623_amd import inputs as I

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))


def _say(msg):
    from conftest import progress
    progress(msg)


@pytest.fixture(scope="module")
def ctx():
    from paper_2306_08623_amd import nucleus
    c = nucleus.Context(device=0)
    yield c
    c.close()


def _degenerate():
    return [
        (I.empty(0), 2, 3),
        (I.empty(5), 3, 4),
        (I.complete(6), 3, 4),
        (I.complete(7), 2, 3),
        (I.two_k5_bridge(), 1, 2),
        (I.cycle(10), 2, 3),
        (I.star(9), 1, 2),
        (I.complete(2), 3, 4),
        (I.complete(7), 2, 4),
        (I.batch_graph(0)[0], 2, 4),
        (I.batch_graph(3)[0], 2, 4),
        (I.batch_graph(5)[0], 1, 3),
        (I.two_k5_bridge(), 1, 3),
        (I.batch_graph(7)[0], 1, 4),
        (I.complete(7), 1, 4),
    ]


def _small_batch():
    gs = [I.batch_graph(i) for i in range(40)]
    deg = _degenerate()
    # degenerate members interleaved with the random ones
    out = []
    for j, g in enumerate(gs):
        out.append(g)
        if j % 5 == 0 and deg:
            out.append(deg.pop())
    return out + deg


def _assert_same(res, d, tag):
    r = d.r
    assert res.rcliques.shape == (d.n_r, r), tag
    assert np.array_equal(res.rcliques, d.rcliques), (tag, "rcliques")
    assert np.array_equal(res.counts.astype(np.uint64), d.count), (tag, "counts")
    assert np.array_equal(res.coreness.astype(np.uint64), d.coreness), (tag, "coreness")
    assert np.array_equal(res.parent, d.parent), (tag, "parent")
    assert np.array_equal(res.level.astype(np.uint64), d.level), (tag, "level")


@pytest.mark.timeout(300)
def test_batch_host_vs_oracle_and_solo(ctx):
    graphs = _small_batch()
    _say(f"[batch] {len(graphs)} graphs, host inputs")
    out = ctx.decompose_batch(graphs)
    info = ctx.nd_get_info()
    assert info["r"] == 0 and info["s"] == 0            # mixed pairs
    tot_ns = 0
    for i, ((g, r, s), res) in enumerate(zip(graphs, out)):
        d = oracle.decompose(g, r, s)
        _assert_same(res, d, ("oracle", i, g.n, r, s))
        assert res.info["n_s"] == d.n_s and res.info["k"] == d.k
        assert res.info["n_int"] == d.n_int and res.info["status"] == 0
        tot_ns += d.n_s
    assert info["n_s"] == tot_ns
    # a few members decomposed alone give the same arrays
    for i in (0, 1, 2, 3, len(graphs) - 1):
        g, r, s = graphs[i]
        solo = ctx.decompose(g, r, s)
        for name in ("rcliques", "counts", "coreness", "parent", "level"):
            assert np.array_equal(getattr(solo, name), getattr(out[i], name)), (i, name)


@pytest.mark.timeout(300)
def test_batch_device_inputs_and_reuse(ctx):
    import torch
    from paper_2306_08623_amd import nucleus
    graphs = _small_batch()
    host = ctx.decompose_batch(graphs)
    dev = []
    for g, r, s in graphs:
        rp = torch.from_numpy(g.row_ptr.astype(np.int64)).cuda()
        col = torch.from_numpy(g.col.astype(np.int32)).cuda()
        dev.append((g.n, rp, col, r, s))
    torch.cuda.synchronize()
    _say(f"[batch] {len(graphs)} graphs, device inputs")
    out = ctx.decompose_batch(dev, where=nucleus.ND_MEM_DEVICE)
    for i, (a, b) in enumerate(zip(host, out)):
        for name in ("rcliques", "counts", "coreness", "parent", "level"):
            assert np.array_equal(getattr(a, name), getattr(b, name)), (i, name)
    # a second, smaller batch right after reuses the slots
    small = [(I.batch_graph(100 + i)) for i in range(6)]
    _say("[batch] second, smaller batch")
    out2 = ctx.decompose_batch(small)
    for i, ((g, r, s), res) in enumerate(zip(small, out2)):
        _assert_same(res, oracle.decompose(g, r, s), ("second", i))


def test_batch_errors(ctx):
    from paper_2306_08623_amd import nucleus
    ok = I.complete(5)
    # a column outside the member's own vertex range
    bad = I.CSR(n=3, row_ptr=np.array([0, 1, 2, 2], np.uint64), col=np.array([1, 3], np.uint32))
    with pytest.raises(nucleus.NucleusError) as e:
        ctx.decompose_batch([(ok, 2, 3), (bad, 2, 3)])
    assert e.value.code == nucleus.ND_E_BAD_GRAPH
    with pytest.raises(nucleus.NucleusError) as e:
        ctx.decompose_batch([(ok, 2, 8)])
    assert e.value.code == nucleus.ND_E_UNSUPPORTED
    with pytest.raises(nucleus.NucleusError) as e:
        ctx.decompose_batch([(ok, 3, 3)])
    assert e.value.code == nucleus.ND_E_INVALID_ARG
    # after a batch, the single-graph getters have nothing to return
    ctx.decompose_batch([(ok, 2, 3)])
    with pytest.raises(nucleus.NucleusError) as e:
        ctx.nd_get_rcliques()
    assert e.value.code == nucleus.ND_E_STATE
    # an empty batch is fine
    assert ctx.decompose_batch([]) == []


@pytest.mark.timeout(900)
def test_batch4096_golden(ctx):
    from make_batch_golden import result_digest
    with open(os.path.join(HERE, "golden", "batch4096.json")) as f:
        gold = json.load(f)
    _say("[batch] generating the 4,096 graphs")
    graphs = I.batch_graphs(gold["count"], gold["base_seed"])
    _say("[batch] decomposing them in one batch")
    out = ctx.decompose_batch(graphs)
    bad = []
    for i, ((g, r, s), res, row) in enumerate(zip(graphs, out, gold["graphs"])):
        n_r, n_s, k, n_int, csr12, dig = row
        assert g.sha256()[:12] == csr12, ("input differs", i)
        got = (res.info["n_r"], res.info["n_s"], res.info["k"], res.info["n_int"],
               result_digest(res.rcliques, res.counts, res.coreness, res.parent, res.level))
        if got != (n_r, n_s, k, n_int, dig):
            bad.append(i)
    assert not bad, f"{len(bad)} graphs differ from the oracle, first {bad[:10]}"
