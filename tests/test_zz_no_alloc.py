"""The no-allocation entry point (geomst_emst_dev_noalloc) against the plain
device call (geomst_emst_dev) and the CPU checker, called through the C ABI:
two calls in a row on the same device, the second with a smaller input, so
the second one runs over the first one's leftovers in the fixed scratch."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_2104_01126_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def G():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2104_01126_amd import geomst as g
    g.load()
    return g


def _abi(G, fn, p):
    """Call an EMST device entry point through ctypes -> (edges, w, w2)."""
    import torch
    n, d = p.shape
    m = max(n - 1, 0)
    e = torch.full((m, 2), -1, dtype=torch.int64, device=p.device)
    w = torch.full((m,), -1.0, dtype=torch.float64, device=p.device)
    w2 = torch.full((m,), -1.0, dtype=torch.float64, device=p.device)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(G.load(), fn)(p.data_ptr(), n, d, e.data_ptr(), w.data_ptr(), w2.data_ptr(), s)
    assert rc == G.OK, (fn, rc, G.last_error())
    return e.cpu().numpy(), w.cpu().numpy(), w2.cpu().numpy()


def _same(a, b):
    return a.shape == b.shape and np.array_equal(a.view(np.uint8), b.view(np.uint8))


@pytest.mark.parametrize("order", ["large_then_small", "repeat"])
def test_noalloc_matches_plain_call(G, order):
    import torch
    cases = [W.mixture(20000, 3, seed=41, k=8, noise_frac=0.05), W.uniform(3001, 2, seed=42)]
    if order == "repeat":
        cases = [W.uniform(12000, 5, seed=43), W.uniform(257, 7, seed=44)]
    for x in cases:
        say("noalloc", order, x.shape)
        p = torch.from_numpy(x).to("cuda")
        got = _abi(G, "geomst_emst_dev_noalloc", p)
        ref = _abi(G, "geomst_emst_dev", p)
        for a, b in zip(got, ref):
            assert _same(a, b)
        eo, w2o, wo = oracle.emst(x)
        assert np.array_equal(got[0], eo) and _same(got[2], w2o) and _same(got[1], wo)


def test_noalloc_small_and_single_point(G):
    import torch
    for x in (np.array([[0.5, 0.25]]), np.array([[0.0, 0.0], [1.0, 2.0]]), W.grid(9, 2, seed=5)):
        say("noalloc small", x.shape)
        p = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
        got = _abi(G, "geomst_emst_dev_noalloc", p)
        eo, w2o, wo = oracle.emst(x)
        assert np.array_equal(got[0], eo) and _same(got[2], w2o)


def test_noalloc_rejects_too_many_points(G):
    import torch
    nmax = G.header_constant("GEOMST_NOALLOC_MAX_POINTS")
    p = torch.zeros((nmax + 1, 2), dtype=torch.float64, device="cuda")
    e = torch.empty((nmax, 2), dtype=torch.int64, device="cuda")
    rc = G.load().geomst_emst_dev_noalloc(p.data_ptr(), nmax + 1, 2, e.data_ptr(), None, None, None)
    assert rc == G.EINVAL and "GEOMST_NOALLOC_MAX_POINTS" in G.last_error()
