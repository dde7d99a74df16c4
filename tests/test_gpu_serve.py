"""Serving loop through the C ABI (nd_server_*).

A request's result must be exactly the same whether it is served alone or in
a mix with other requests, and equal to the oracle's (integers: tolerance 0).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2306_08623_amd import inputs as I

pytestmark = pytest.mark.gpu

FIELDS = ("rcliques", "counts", "coreness", "parent", "level")


def _say(msg):
    from conftest import progress
    progress(msg)


def _requests(count=48, m_hi=40_000):
    reqs = [I.serve_graph(i, m_hi=m_hi) for i in range(count)]
    reqs[5:5] = [(I.empty(0), 2, 3), (I.complete(6), 3, 4), (I.empty(7), 1, 2),
                 (I.two_k5_bridge(), 2, 3), (I.complete(8), 2, 4),
                 (I.serve_graph(1, m_hi=m_hi)[0], 2, 4), (I.serve_graph(2, m_hi=m_hi)[0], 1, 3),
                 (I.serve_graph(3, m_hi=m_hi)[0], 1, 4)]
    return reqs


def _same(a, b, tag):
    for f in FIELDS:
        assert np.array_equal(getattr(a, f), getattr(b, f)), (tag, f)


def _vs_oracle(res, csr, r, s, tag):
    d = oracle.decompose(csr, r, s)
    assert np.array_equal(res.rcliques, d.rcliques), (tag, "rcliques")
    assert np.array_equal(res.counts.astype(np.uint64), d.count), (tag, "counts")
    assert np.array_equal(res.coreness.astype(np.uint64), d.coreness), (tag, "coreness")
    assert np.array_equal(res.parent, d.parent), (tag, "parent")
    assert np.array_equal(res.level.astype(np.uint64), d.level), (tag, "level")
    assert res.info["n_s"] == d.n_s and res.info["k"] == d.k


@pytest.mark.timeout(600)
def test_serve_mix_equals_alone_and_oracle():
    from paper_2306_08623_amd import nucleus
    reqs = _requests()
    _say(f"[serve] {len(reqs)} requests submitted at once to 2 pipelines")
    with nucleus.Server(device=0, workers=2) as srv:
        tickets = [srv.submit(g, r, s) for g, r, s in reqs]
        mix = []
        for t, (g, r, s) in zip(tickets, reqs):
            res = srv.get(t, r)
            assert res.info["status"] == nucleus.ND_OK
            srv.release(t)
            mix.append(res)
        st = srv.stats()
    _say(f"[serve] stats {st}")
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["batches"] < len(reqs) and st["max_batch_seen"] > 1
    assert st["result_bytes"] == 0
    _say("[serve] the same requests one at a time")
    with nucleus.Server(device=0, workers=1, max_batch=1) as srv:
        for i, (g, r, s) in enumerate(reqs):
            t = srv.submit(g, r, s)
            alone = srv.get(t, r)
            assert alone.info["batch_size"] == 1
            srv.release(t)
            _same(alone, mix[i], ("alone vs mix", i))
    _say("[serve] against the oracle")
    for i, (g, r, s) in enumerate(reqs):
        _vs_oracle(mix[i], g, r, s, ("oracle", i, g.n, g.m, r, s))


@pytest.mark.timeout(300)
def test_serve_device_inputs_admission_and_cancel():
    import torch
    from paper_2306_08623_amd import nucleus
    reqs = _requests(count=24)
    solo = []
    with nucleus.Context(device=0) as ctx:
        for g, r, s in reqs:
            solo.append(ctx.decompose(g, r, s))
    # a budget that admits only a few requests at a time
    ws = [nucleus.estimate_footprint(g, r, s) for g, r, s in reqs]
    big_ws = max(w for w, _ in ws)
    big_res = max(x for _, x in ws)
    budget = 4 * (3 * big_ws + (8 << 20))          # workspace share: ~3 of the largest
    budget = max(budget, 4 * 3 * big_res)
    _say(f"[serve] small budget {budget} bytes, device inputs")
    with nucleus.Server(device=0, workers=2, mem_budget=budget) as srv:
        dev = []
        for g, r, s in reqs:
            rp = torch.from_numpy(g.row_ptr.astype(np.int64)).cuda()
            col = torch.from_numpy(g.col.astype(np.int32)).cuda() if g.col.size else \
                torch.zeros(1, dtype=torch.int32, device="cuda")
            dev.append((g.n, rp, col, r, s, g.nnz))
        torch.cuda.synchronize()
        tickets = [srv.submit_device(*d) for d in dev]
        # cancel two of the last ones (still waiting or already done: both fine)
        cancelled = set(tickets[-2:])
        for t in cancelled:
            srv.cancel(t)
        for i, t in enumerate(tickets):
            info = srv.wait(t)
            if t in cancelled and info["status"] == nucleus.ND_E_CANCELLED:
                srv.release(t)
                continue
            assert info["status"] == nucleus.ND_OK, (i, info)
            res = srv.get(t, reqs[i][1])
            srv.release(t)
            _same(res, solo[i], ("device input", i))
        st = srv.stats()
        assert st["completed"] + st["cancelled"] == len(reqs)
        # a request beyond the shares is refused at submission
        huge = I.rmat(16, 16, 9)
        with pytest.raises(nucleus.NucleusError) as e:
            srv.submit(huge, 3, 4)
        assert e.value.code == nucleus.ND_E_OOM


def test_serve_errors():
    from paper_2306_08623_amd import nucleus
    with nucleus.Server(device=0) as srv:
        with pytest.raises(nucleus.NucleusError) as e:
            srv.submit(I.complete(5), 2, 8)
        assert e.value.code == nucleus.ND_E_UNSUPPORTED
        bad = I.CSR(n=3, row_ptr=np.array([0, 1, 2, 2], np.uint64),
                    col=np.array([1, 3], np.uint32))
        t = srv.submit(bad, 2, 3)
        info = srv.wait(t)
        assert info["done"] == 1 and info["status"] == nucleus.ND_E_BAD_GRAPH
        with pytest.raises(nucleus.NucleusError) as e:
            srv.get(t, 2)
        assert e.value.code == nucleus.ND_E_STATE
        srv.release(t)
        with pytest.raises(nucleus.NucleusError):
            srv.poll(t)


def test_footprint_estimate_bounds_workspace():
    """The admission estimate is an upper bound of what a context holds."""
    from paper_2306_08623_amd import nucleus
    for i, (g, r, s) in enumerate(_requests(count=12) + [(I.workload_er2k(), 3, 4),
                                                         (I.rmat(14, 16, 2), 3, 4)]):
        with nucleus.Context(device=0) as ctx:
            res = ctx.decompose(g, r, s)
            held = res.info["device_bytes"]
        ws, rb = nucleus.estimate_footprint(g, r, s)
        assert held <= ws + (4 << 20), (i, g.n, g.m, r, s, held, ws)
        n_int = res.level.size
        assert rb >= res.counts.size * (4 * r + 16) + n_int * 12, (i, rb)


@pytest.mark.timeout(600)
def test_serve_batches_overlap_on_device():
    """Two pipelines with small batches: their batches run on the GPU at the
    same time (device intervals from HIP events overlap), and every result
    is still exactly the graph's solo result and the oracle's."""
    from paper_2306_08623_amd import nucleus
    reqs = [I.serve_graph(100 + i, m_hi=150_000) for i in range(32)]
    with nucleus.Context(device=0) as ctx:
        solo = [ctx.decompose(g, r, s) for g, r, s in reqs]
    _say(f"[serve] {len(reqs)} requests, 2 pipelines, batches of at most 4")
    with nucleus.Server(device=0, workers=2, max_batch=4) as srv:
        tickets = [srv.submit(g, r, s) for g, r, s in reqs]
        mix = []
        for t, (g, r, s) in zip(tickets, reqs):
            res = srv.get(t, r)
            assert res.info["status"] == nucleus.ND_OK
            srv.release(t)
            mix.append(res)
        st = srv.stats()
    _say(f"[serve] device batch {st['device_batch_ms']:.1f} ms, busy {st['device_busy_ms']:.1f} "
         f"ms, overlapped {st['device_overlap_ms']:.1f} ms over {st['batches']} batches")
    assert st["completed"] == len(reqs) and st["batches"] >= 8
    assert st["device_overlap_ms"] > 0.0
    assert st["device_batch_ms"] >= st["device_busy_ms"] >= st["device_overlap_ms"]
    for i, (g, r, s) in enumerate(reqs):
        _same(mix[i], solo[i], ("overlapped mix vs solo", i))
    for i in range(0, len(reqs), 4):
        g, r, s = reqs[i]
        _vs_oracle(mix[i], g, r, s, ("oracle", i, g.n, g.m, r, s))
