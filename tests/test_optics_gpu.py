"""GPU parity of approximate OPTICS (paper Appendix, "Parallel Approximate
OPTICS"): the HIP library against the CPU checker's oracle.optics_approx.

Both sides build the same spatial tree and decomposition from the same
definition, so the bar is bit-exact: edge ids and order, squared weights,
weights, core distances, and the decomposition's own counts (well-separated
pairs, evaluated point pairs, examined pairs).  The approximate tree's
reachability plot (geomst_dendrogram) is compared with the checker's too.
"""
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


def dev(p):
    import torch
    return torch.from_numpy(np.ascontiguousarray(p)).to("cuda")


def same(a, b):
    return a.shape == b.shape and np.array_equal(a.view(np.uint8), b.view(np.uint8))


def run(G, p, mp, rho):
    cd, e, w, cd2, w2 = G.optics_approx(dev(p), mp, rho, want_sq=True)
    st = G.stats()
    return (cd.cpu().numpy(), e.cpu().numpy(), w.cpu().numpy(), cd2.cpu().numpy(), w2.cpu().numpy()), st


def check(G, p, mp, rho):
    n = len(p)
    (cd, e, w, cd2, w2), st = run(G, p, mp, rho)
    ocd2, oe, ow2, oe2, ost = oracle.optics_approx(p, mp, rho)
    assert same(cd2, ocd2), "core distances"
    assert same(e, oe), "edges"
    assert same(w2, ow2), "squared weights"
    assert same(w, np.sqrt(ow2)), "weights"
    assert same(cd, np.sqrt(ocd2))
    assert (st.bccp_pairs, st.bccp_evals, st.pair_visits) == ost, (st.bccp_pairs, st.bccp_evals, st.pair_visits, ost)
    return e, w


CASES = [
    ("uniform", 300, 1, 4, 0.125),
    ("uniform", 2000, 2, 10, 0.125),
    ("uniform", 3000, 3, 5, 0.5),
    ("mixture", 5000, 3, 10, 0.125),
    ("mixture", 1500, 5, 16, 1.0),
    ("mixture", 800, 7, 8, 2.0),
    ("uniform", 4000, 2, 1, 0.25),
    ("mixture", 3000, 2, 64, 0.125),
    ("dups", 3000, 3, 6, 0.125),
    ("grid", 0, 2, 4, 0.125),
]


@pytest.mark.parametrize("kind,n,d,mp,rho", CASES)
def test_exact_small(G, kind, n, d, mp, rho):
    say("optics_approx", kind, n, d, mp, rho)
    if kind == "uniform":
        p = W.uniform(n, d, 100 + n + d)
    elif kind == "mixture":
        p = W.mixture(n, d, 200 + n + d, k=6, noise_frac=0.05)
    elif kind == "dups":
        p = W.with_duplicates(n, d, 7, 300)
    else:
        p = W.grid(40, 2, seed=3)
    check(G, p, min(mp, len(p)), rho)


@pytest.mark.parametrize("n", [2, 3, 5, 17])
def test_tiny(G, n):
    say("optics_approx tiny", n)
    p = W.uniform(n, 3, n)
    check(G, p, min(3, n), 0.125)


def test_one_point(G):
    cd, e, w = G.optics_approx(dev(np.zeros((1, 2))), 1, 0.5)
    assert e.shape == (0, 2) and float(cd[0]) == 0.0


def test_20k_workload_and_plot(G):
    p = W.optics_500k(20000)
    say("optics_approx 20k workload prefix")
    e, w = check(G, p, 10, 0.125)
    # the approximate OPTICS reachability plot of this tree
    import torch
    ch, sz, order, reach = G.dendrogram(torch.from_numpy(e).cuda(), torch.from_numpy(w).cuda(), 0)
    och, osz, oorder, oreach = oracle.dendrogram(e, w, 0)
    assert same(order.cpu().numpy(), oorder) and same(reach.cpu().numpy(), oreach)
    assert same(ch.cpu().numpy(), och) and same(sz.cpu().numpy(), osz)


def test_host_api_matches(G):
    p = W.mixture(4000, 3, 5, k=5)
    cd_h, e_h, w_h = G.optics_approx(p, 8, 0.25)
    (cd, e, w, _, _), _ = run(G, p, 8, 0.25)
    assert same(e_h, e) and same(w_h, w) and same(cd_h, cd)


def test_repeatable(G):
    p = W.optics_500k(30000)
    a, _ = run(G, p, 10, 0.125)
    b, _ = run(G, p, 10, 0.125)
    for x, y in zip(a, b):
        assert same(x, y)


def test_errors(G):
    p = dev(W.uniform(100, 2, 1))
    for mp, rho in [(0, 0.5), (65, 0.5), (5, 0.0), (5, -1.0), (5, float("nan")), (5, float("inf"))]:
        with pytest.raises(G.GeomstError) as ei:
            G.optics_approx(p, mp, rho)
        assert ei.value.code == G.EINVAL


def test_full_size_digest(G):
    """The 500,000-point workload, byte for byte against the checker's digest
    (tests/golden/make_digests.py optics_500k), with the decomposition's
    counts; diagnostics first, so that a missing digest still checks the
    tree's weights and shape."""
    import hashlib
    import json
    import os
    p = W.optics_500k()
    n = len(p)
    say("optics_approx full size", n)
    (cd, e, w, cd2, w2), st = run(G, p, 10, 0.125)
    assert e.shape == (n - 1, 2) and (e[:, 0] < e[:, 1]).all()
    # every weight is the approximate weight of its own edge (checker's
    # core distances of a sample, its keys of a sample of edges)
    rng = np.random.default_rng(5)
    idx = rng.choice(n, 64, replace=False)
    assert same(cd2[idx], oracle.core_dist2(p, 10, idx))
    ks = rng.choice(n - 1, 2000, replace=False)
    _, e2s = oracle.edge_keys(p, e[ks, 0], e[ks, 1])
    q = (1.0 + 0.125) * (1.0 + 0.125)
    assert same(w2[ks], np.maximum(np.maximum(cd2[e[ks, 0]], cd2[e[ks, 1]]), e2s / q))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "digest_optics_500k.json")
    if not os.path.exists(path):
        pytest.skip("tests/golden/digest_optics_500k.json has not been generated")
    g = json.load(open(path))

    def sha(a):
        return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
    assert g["n"] == n and g["min_pts"] == 10 and g["rho"] == 0.125
    assert (st.bccp_pairs, st.bccp_evals, st.pair_visits) == (g["wspd_pairs"], g["evals"], g["visits"])
    assert sha(cd2) == g["cd2"], "core distances differ from the checker's"
    assert sha(e) == g["edges"], "edge list differs from the checker's"
    assert sha(w2) == g["w2"], "squared weights differ from the checker's"
