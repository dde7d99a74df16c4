"""nd_decompose_noalloc (the entry point that allocates no device memory)
against the allocating entry point it stands for (nd_load_csr + nd_set_rs +
nd_decompose + nd_get_coreness / nd_get_tree), bit-exact, on two calls in a
row with the second graph smaller than the first, so the shared scratch
holds the first call's contents when the second starts; plus the oracle on
the same graphs, and the size checks."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2306_08623_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    from conftest import progress
    progress(msg)
    sys.stdout.flush()


def _device_csr(g):
    import torch
    rp = torch.from_numpy(g.row_ptr.astype(np.int64)).cuda()
    col = torch.from_numpy(g.col.astype(np.int32)).cuda() if g.col.size else \
        torch.zeros(1, dtype=torch.int32, device="cuda")
    return rp, col


def _noalloc(g, r, s, cap):
    import torch

    from paper_2306_08623_amd import nucleus
    rp, col = _device_csr(g)
    if g.col.size == 0:
        col = col[:0]
    core = torch.full((cap,), 0xABCD, dtype=torch.int32, device="cuda")
    parent = torch.full((2 * cap,), -7, dtype=torch.int64, device="cuda")
    level = torch.full((cap,), 0xABCD, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    info = nucleus.decompose_noalloc(g.n, rp, col, r, s, core, parent, level)
    n_r, n_int = info["n_r"], info["n_int"]
    return (info, core[:n_r].cpu().numpy().view(np.uint32),
            parent[:n_r + n_int].cpu().numpy().view(np.uint64),
            level[:n_int].cpu().numpy().view(np.uint32))


def _check_pair(ctx, g, r, s, tag):
    _say(f"[noalloc] {tag} n={g.n} m={g.m} (r,s)=({r},{s})")
    ref = ctx.decompose(g, r, s)
    n_r = ref.info["n_r"]
    info, core, parent, level = _noalloc(g, r, s, max(n_r, 1) + 17)
    assert info["n_r"] == n_r and info["n_s"] == ref.info["n_s"], tag
    assert info["n_int"] == ref.info["n_int"] and info["k"] == ref.info["k"], tag
    assert np.array_equal(core, ref.coreness), tag
    assert np.array_equal(parent, ref.parent), tag
    assert np.array_equal(level, ref.level), tag
    d = oracle.decompose(g, r, s)
    assert np.array_equal(core.astype(np.uint64), d.coreness), tag
    assert np.array_equal(parent, d.parent), tag
    assert np.array_equal(level.astype(np.uint64), d.level), tag


@pytest.mark.parametrize("r,s", [(2, 3), (3, 4), (1, 2), (2, 4)])
def test_noalloc_equals_allocating_path_twice(r, s):
    from paper_2306_08623_amd import nucleus
    big = I.er_planted(900, 0.02, 8, 5, 16, seed=31)
    small = I.er_planted(150, 0.05, 3, 4, 9, seed=32)
    with nucleus.Context(device=0) as ctx:
        _check_pair(ctx, big, r, s, "first, larger")
        _check_pair(ctx, small, r, s, "second, smaller")


def test_noalloc_edge_cases():
    from paper_2306_08623_amd import nucleus
    with nucleus.Context(device=0) as ctx:
        _check_pair(ctx, I.complete(6), 3, 4, "K6")
        _check_pair(ctx, I.two_k5_bridge(), 2, 3, "two-K5")
        _check_pair(ctx, I.empty(4), 2, 3, "edgeless")


def test_noalloc_rejects_what_does_not_fit():
    import torch

    from paper_2306_08623_amd import nucleus
    g = I.er_planted(300, 0.05, 3, 5, 10, seed=33)
    # outputs too small: the run itself succeeds, the copy-out is refused
    with pytest.raises(nucleus.NucleusError) as e:
        _noalloc(g, 2, 3, 10)
    assert e.value.code == nucleus.ND_E_INVALID_ARG and "r-cliques" in str(e.value)
    # a graph whose CSR alone exceeds the scratch is refused before any work
    n = 1000
    nnz = nucleus.ND_NOALLOC_SCRATCH_BYTES // 12 + 2
    rp = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    col = torch.zeros(nnz, dtype=torch.int32, device="cuda")
    out = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(nucleus.NucleusError) as e:
        nucleus.decompose_noalloc(n, rp, col, 2, 3, out, torch.zeros(8, dtype=torch.int64,
                                                                      device="cuda"), out)
    assert e.value.code == nucleus.ND_E_OOM and "scratch" in str(e.value)
    # and the entry point still works afterwards
    with nucleus.Context(device=0) as ctx:
        _check_pair(ctx, g, 2, 3, "after refusals")
