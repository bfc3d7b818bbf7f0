"""GPU parity of batched (forest) solves: every instance's result must be
byte-identical to the checker's, and to the same instance solved alone."""
import hashlib
import json
import os
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
    assert torch.cuda.is_available()
    from paper_2104_01126_amd import geomst as g
    g.load()
    return g


def same(a, b):
    return a.shape == b.shape and np.array_equal(np.ascontiguousarray(a).view(np.uint8),
                                                 np.ascontiguousarray(b).view(np.uint8))


def run_batch(G, inst, mps):
    import torch
    arena, items, stride = G.pack(inst, mps)
    out = G.batch_dev(torch.from_numpy(arena).to("cuda"), items, stride, want_sq=True)
    return G.unpack(out, items)


def mixed_instances(seed, count, nmax, dims=(2, 3)):
    rng = np.random.default_rng(seed)
    inst = []
    for i in range(count):
        n = int(np.exp(rng.uniform(0, np.log(nmax))))
        d = int(rng.choice(dims))
        if i % 3 == 0:
            x = rng.random((n, d))
        elif i % 3 == 1:
            x = W.mixture(n, d, seed=seed * 1000 + i, k=3, noise_frac=0.1) if n >= 3 else rng.random((n, d))
        else:
            x = W.with_duplicates(n, d, seed=seed * 1000 + i, n_unique=max(1, n // 3))
        inst.append(np.ascontiguousarray(x))
    inst[0] = np.zeros((1, 2))          # a single point
    inst[1] = np.full((5, 3), 0.5)      # coincident points
    return inst


def check(inst, res, mps):
    for i, (x, r, mp) in enumerate(zip(inst, res, mps)):
        if mp:
            cd2o, cdo, eo, w2o, _, wo = oracle.hdbscan(x, mp)
            assert same(r["core_dist_sq"], cd2o) and same(r["core_dist"], cdo), i
        else:
            eo, w2o, wo = oracle.emst(x)
        assert np.array_equal(r["edges"], eo), f"instance {i} (n={len(x)}, d={x.shape[1]}, minPts={mp})"
        assert same(r["weights_sq"], w2o) and same(r["weights"], wo), i


def test_batch_emst_mixed_sizes_and_dims(G):
    inst = mixed_instances(1, 160, 3000)
    say("batch emst", len(inst), sum(len(x) for x in inst))
    check(inst, run_batch(G, inst, [0] * len(inst)), [0] * len(inst))


def test_batch_mixed_emst_hdbscan(G):
    inst = mixed_instances(2, 90, 2000, dims=(2, 3, 5))
    rng = np.random.default_rng(5)
    mps = [0 if i % 2 == 0 else int(min(len(x), rng.choice([1, 3, 5, 10, 16]))) for i, x in enumerate(inst)]
    say("batch mixed", len(inst), sum(len(x) for x in inst))
    check(inst, run_batch(G, inst, mps), mps)


def test_batch_equals_single_calls(G):
    inst = mixed_instances(3, 40, 4000)
    res = run_batch(G, inst, [0] * len(inst))
    import torch
    for x, r in zip(inst, res):
        e, w, w2 = G.emst(torch.from_numpy(x).to("cuda"), want_sq=True)
        assert np.array_equal(e.cpu().numpy(), r["edges"]) and same(w2.cpu().numpy(), r["weights_sq"])


def test_batch_host_api(G):
    inst = mixed_instances(4, 30, 1500)
    mps = [0 if i % 3 else min(len(x), 4) for i, x in enumerate(inst)]
    out = G.batch(inst, mps)
    for x, (e, w, cd), mp in zip(inst, out, mps):
        if mp:
            _, cdo, eo, _, _, wo = oracle.hdbscan(x, mp)
            assert same(cd, cdo)
        else:
            eo, _, wo = oracle.emst(x)
        assert np.array_equal(e, eo) and same(w, wo)


def test_tuning_cache_keeps_bytes(G, tmp_path):
    """A tuning cache with unusual knob values (small BCCP tiles, small level
    buckets, fast threshold growth) applies to matching solves and changes
    no byte of any result."""
    inst = mixed_instances(5, 60, 4000)
    mps = [0] * len(inst)
    ref = run_batch(G, inst, mps)
    stride = max(x.shape[1] for x in inst)
    N = sum(len(x) for x in inst)
    nl = int(np.floor(np.log2(N)))
    p = W.mixture(20000, 3, seed=91, k=5, noise_frac=0.02)
    e0, w0 = G.emst(p)
    cache = tmp_path / "tune.jsonl"
    cache.write_text(
        f'{{"kind": "emst", "d": {stride}, "nlog2": {nl}, "bccp_chunk": 64, "small_level_switch": 512, '
        f'"small_level_max": 1024, "beta_growth": 4.0}}\n'
        '{"kind": "emst", "d": 3, "nlog2": 14, "bccp_chunk": 128, "small_level_switch": 256, '
        '"small_level_max": 512, "beta_growth": 1.5, "refresh_divisor": 64}\n')
    try:
        G.load_tuning(str(cache))
        got = run_batch(G, inst, mps)
        assert G.stats().tuning_applied == 1
        e1, w1 = G.emst(p)
        assert G.stats().tuning_applied == 1
    finally:
        G.load_tuning(None)
    for a, b in zip(ref, got):
        assert all(same(a[k], b[k]) for k in a)
    assert same(e0, e1) and same(w0, w1)
    G.emst(p)
    assert G.stats().tuning_applied == 0


def test_batch_all_single_points(G):
    inst = [np.array([[float(i), 0.0]]) for i in range(7)]
    res = run_batch(G, inst, [0] * 7)
    assert all(r["edges"].shape == (0, 2) for r in res)


def _digests(name):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"digest_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_batch_4096_workload(G):
    """The 4,096-instance workload (n log-uniform in [100, 50000], d in {2,3},
    half uniform, half 8-Gaussian mixtures), solved as one forest:
    - every instance with n <= 3000 is compared with the checker directly;
    - every instance, byte for byte, with the digests of the checker's own
      run over all 4,096 (tests/golden/make_digests.py);
    - 100 of the larger instances are solved alone by the plain call and must
      give the same bytes, and pass 20 single-vertex cuts each;
    - every other instance returns one spanning tree whose squared weights
      the checker recomputes."""
    inst = W.batch_4096()
    say("batch_4096", len(inst), sum(len(x) for x in inst))
    res = run_batch(G, inst, [0] * len(inst))
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    for i, (x, r) in enumerate(zip(inst, res)):
        if len(x) <= 3000:
            eo, w2o, _ = oracle.emst(x)
            assert np.array_equal(r["edges"], eo), i
            assert same(r["weights_sq"], w2o), i
        else:
            e = r["edges"]
            n = len(x)
            a = sp.coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n))
            assert connected_components(a, directed=False)[0] == 1, i
            ow2, _ = oracle.edge_keys(x, e[:, 0], e[:, 1])
            assert same(r["weights_sq"], ow2), i
            key = np.lexsort((e[:, 1], e[:, 0], r["weights_sq"]))
            assert np.array_equal(key, np.arange(n - 1)), i
    rng = np.random.default_rng(11)
    big = [i for i, x in enumerate(inst) if len(x) > 3000]
    for i in sorted(rng.choice(big, size=min(100, len(big)), replace=False)):
        x, r = inst[i], res[i]
        import torch
        e1, w1, w21 = G.emst(torch.from_numpy(x).to("cuda"), want_sq=True)
        assert np.array_equal(r["edges"], e1.cpu().numpy()), i
        assert same(r["weights_sq"], w21.cpu().numpy()), i
        tree = {tuple(t) for t in r["edges"].tolist()}
        for v in rng.choice(len(x), 20, replace=False):
            side = np.zeros(len(x), np.uint8)
            side[v] = 1
            lo, hi, _, _ = oracle.lightest_cut_edge(x, side)
            assert (lo, hi) in tree, (i, v)
    g = _digests("batch_4096")
    if g is None:
        pytest.skip("tests/golden/digest_batch_4096.json has not been generated")
    assert g["count"] == len(inst)
    for i, (x, r, gi) in enumerate(zip(inst, res, g["instances"])):
        assert gi["n"] == len(x) and gi["d"] == x.shape[1], i
        assert _sha(r["edges"]) == gi["edges"], f"instance {i}: edges differ from the checker's"
        assert _sha(r["weights_sq"]) == gi["w2"], f"instance {i}: squared weights differ"
