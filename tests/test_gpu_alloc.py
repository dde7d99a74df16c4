"""The context's device workspace through caller-supplied allocator
callbacks (nd_options.alloc / free): here PyTorch's caching allocator, so
torch accounts for the memory while a context holds it and gets it back when
the context is destroyed; results stay bit-exact with the oracle. Also the
run counters that come with every decomposition."""
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


@pytest.mark.parametrize("r,s", [(2, 3), (3, 4), (2, 4)])
def test_torch_allocator_holds_and_returns_the_workspace(r, s):
    import torch

    from paper_2306_08623_amd import nucleus
    g = I.workload_er2k()
    _say(f"[alloc] er2k (r,s)=({r},{s}) through torch's caching allocator")
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(0)
    ctx = nucleus.Context(device=0, allocator="torch")
    res = ctx.decompose(g, r, s)
    held = torch.cuda.memory_allocated(0) - before
    info = res.info
    assert info["device_bytes"] > 0
    assert held >= info["device_bytes"], (held, info["device_bytes"])
    assert info["device_peak"] >= info["device_bytes"]
    d = oracle.decompose(g, r, s)
    assert np.array_equal(res.coreness.astype(np.uint64), d.coreness)
    assert np.array_equal(res.parent, d.parent)
    assert np.array_equal(res.level.astype(np.uint64), d.level)
    # a second, larger graph grows buffers through the callbacks
    g2 = I.er_planted(3000, 0.01, 25, 5, 30, seed=7)
    res2 = ctx.decompose(g2, r, s)
    d2 = oracle.decompose(g2, r, s)
    assert np.array_equal(res2.coreness.astype(np.uint64), d2.coreness)
    assert np.array_equal(res2.parent, d2.parent)
    ctx.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(0) == before


def test_allocator_and_default_agree_and_counters():
    from paper_2306_08623_amd import nucleus
    g = I.er_planted(800, 0.03, 10, 6, 20, seed=5)
    a = nucleus.decompose(g, 3, 4, allocator="torch")
    b = nucleus.decompose(g, 3, 4)
    assert np.array_equal(a.coreness, b.coreness)
    assert np.array_equal(a.parent, b.parent)
    for res in (a, b):
        i = res.info
        # EL on (3,4): every link step is a top-level call or a cascade
        assert i["hier_te"] == 0
        assert i["links"] == i["link_calls"] + i["cascades"]
        assert i["cas_retries"] >= 0 and i["grid_retries"] == 0


def test_mismatched_callbacks_are_refused():
    import ctypes as C

    from paper_2306_08623_amd import nucleus
    lib = nucleus.load_library()
    alloc, _free = nucleus.torch_allocator(0)
    opt = nucleus.Options()
    opt.device = 0
    opt.validate = 1
    opt.alloc = C.cast(alloc, C.c_void_p)     # free left NULL
    h = C.c_void_p()
    assert lib.nd_create(C.byref(h), C.byref(opt)) == nucleus.ND_E_INVALID_ARG
    assert b"together" in lib.nd_last_error(None)
