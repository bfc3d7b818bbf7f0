"""GPU parity of the ordered dendrogram and reachability plot
(geomst_dendrogram_dev / geomst_dendrogram) against the checker
(oracle.dendrogram): children, sizes, order and heights byte for byte, on
EMST and HDBSCAN* trees from small sizes to the full workloads, for several
start points, plus the error paths."""
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


def same(a, b):
    a, b = np.ascontiguousarray(a), np.ascontiguousarray(b)
    return a.shape == b.shape and a.dtype == b.dtype and np.array_equal(a.view(np.uint8), b.view(np.uint8))


def run_dev(G, e, w, s):
    import torch
    out = G.dendrogram(torch.from_numpy(e).to("cuda"), torch.from_numpy(w).to("cuda"), s)
    return tuple(x.cpu().numpy() for x in out)


def check(G, e, w, s, tag):
    say("dendrogram", tag, len(e) + 1, "start", s)
    ref = oracle.dendrogram(e, w, s)
    got = run_dev(G, e, w, s)
    for name, a, b in zip(("children", "size", "order", "reach"), got, ref):
        assert same(a, b), f"{tag} start={s}: {name} differs"


@pytest.mark.parametrize("n", [2, 3, 4, 5, 17, 64, 65, 1000, 4097])
def test_emst_trees(G, n):
    p = W.uniform(n, 2, seed=n)
    e, w2, w = oracle.emst(p)
    for s in sorted({0, n // 2, n - 1}):
        check(G, e, w, s, f"uniform2 n={n}")


@pytest.mark.parametrize("case", ["chain", "grid", "mixture3", "dups", "hdb_mixture5", "hdb_grid"])
def test_structured_trees(G, case):
    if case == "chain":
        p, _ = W.collinear(5000, 2, seed=3)
        e, _, w = oracle.emst(p)
    elif case == "grid":
        e, _, w = oracle.emst(W.grid(40, 2, seed=4))
    elif case == "mixture3":
        e, _, w = oracle.emst(W.mixture(8000, 3, seed=5, k=7, noise_frac=0.05))
    elif case == "dups":
        e, _, w = oracle.emst(W.with_duplicates(3000, 3, seed=6, n_unique=300))
    elif case == "hdb_mixture5":
        _, _, e, _, _, w = oracle.hdbscan(W.mixture(6000, 5, seed=7, k=6, noise_frac=0.05), 10)
    else:
        _, _, e, _, _, w = oracle.hdbscan(W.grid(30, 2, seed=8), 4)
    n = len(e) + 1
    for s in (0, n // 3, n - 1):
        check(G, e, w, s, case)


def test_host_api_and_single_point(G):
    p = W.mixture(3000, 2, seed=9, k=4)
    e, _, w = oracle.emst(p)
    ref = oracle.dendrogram(e, w, 11)
    got = G.dendrogram(e, w, 11)
    assert all(same(a, b) for a, b in zip(got, ref))
    ch, sz, order, reach = G.dendrogram(np.zeros((0, 2), np.int64), np.zeros(0), 0)
    assert order.tolist() == [0] and np.isinf(reach[0]) and ch.shape == (0, 2)


def test_rejects_non_trees(G):
    e = np.array([[0, 1], [1, 2], [2, 0]], np.int64)  # a cycle and an isolated point
    with pytest.raises(G.GeomstError) as ei:
        G.dendrogram(e, np.array([1.0, 2.0, 3.0]), 0)
    assert ei.value.code == G.EINVAL
    with pytest.raises(G.GeomstError):
        G.dendrogram(np.array([[0, 4]], np.int64), np.array([1.0]), 0)   # id out of range
    with pytest.raises(G.GeomstError):
        G.dendrogram(np.array([[1, 1]], np.int64), np.array([1.0]), 0)   # self-loop
    with pytest.raises(G.GeomstError):
        G.dendrogram(np.array([[0, 1]], np.int64), np.array([1.0]), 2)   # bad start
    # a valid tree still works after the errors
    e, _, w = oracle.emst(W.uniform(500, 3, seed=10))
    check(G, e, w, 7, "after errors")


def test_pipeline_on_gpu_trees(G):
    """The device pipeline: MST on the GPU, dendrogram on the GPU, both
    against the checker (HDBSCAN* and EMST, 20k points)."""
    import torch
    p = W.hdbscan_2m(20_000)
    cd, e, w = G.hdbscan(torch.from_numpy(p).to("cuda"), 10)
    _, _, eo, _, _, wo = oracle.hdbscan(p, 10)
    assert same(e.cpu().numpy(), eo)
    got = [x.cpu().numpy() for x in G.dendrogram(e, w, 0)]
    ref = oracle.dendrogram(eo, wo, 0)
    assert all(same(a, b) for a, b in zip(got, ref))


@pytest.mark.parametrize("which", ["emst_1m", "hdbscan_2m"])
def test_full_size(G, which):
    """The full workloads: the GPU's MST (byte-identical to the checker's
    dense Prim by the digests tested in test_parity_gpu) is fed to the
    checker's dendrogram and to the kernel."""
    import hashlib
    import json
    import os
    import torch
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"digest_{which}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} has not been generated")
    g = json.load(open(path))
    p = W.emst_1m() if which == "emst_1m" else W.hdbscan_2m()
    say(which, p.shape)
    x = torch.from_numpy(p).to("cuda")
    if which == "emst_1m":
        e, w, w2 = G.emst(x, want_sq=True)
    else:
        cd, e, w, cd2, w2 = G.hdbscan(x, 10, want_sq=True)
    en, w2n = e.cpu().numpy(), w2.cpu().numpy()
    assert hashlib.sha256(en.tobytes()).hexdigest() == g["edges"]
    assert hashlib.sha256(w2n.tobytes()).hexdigest() == g["w2"]
    wn = w.cpu().numpy()
    assert same(wn, np.sqrt(w2n))
    for s in (0, len(p) - 1):
        say(which, "start", s)
        got = [y.cpu().numpy() for y in G.dendrogram(e, w, s)]
        ref = oracle.dendrogram(en, wn, s)
        for name, a, b in zip(("children", "size", "order", "reach"), got, ref):
            assert same(a, b), f"{which} start={s}: {name} differs"
