"""Pins for the CPU checker (oracle/), independent of the checker's own code.

Each test checks the dense-Prim oracle against something other than itself:
brute-force Kruskal written here with numpy, closed forms (collinear chains,
integer grids), theorems of the paper (minPts = 1 and minPts <= 3 relations,
appendix "Relationship between EMST and HDBSCAN* MST"), the cut and cycle
properties, the Figure 1 worked example, and hand-derived tie cases.  None of
these needs a GPU.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2104_01126_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ brute force
def all_pair_keys(p, cd2=None):
    """Every edge i<j with (w2, e2) computed directly: d2 summed in dimension
    order with separate multiply and add (numpy ufuncs never fuse)."""
    n, d = p.shape
    i, j = np.triu_indices(n, 1)
    s = np.zeros(len(i))
    for k in range(d):
        t = p[i, k] - p[j, k]
        s = s + t * t
    w2 = s.copy()
    if cd2 is not None:
        w2 = np.maximum(np.maximum(cd2[i], cd2[j]), s)
    return i.astype(np.int64), j.astype(np.int64), w2, s


def kruskal_bruteforce(p, cd2=None):
    n = len(p)
    i, j, w2, e2 = all_pair_keys(p, cd2)
    order = np.lexsort((j, i, e2, w2))  # last key is primary
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    out = []
    for o in order:
        a, b = find(int(i[o])), find(int(j[o]))
        if a != b:
            parent[a] = b
            out.append((int(i[o]), int(j[o]), w2[o], e2[o]))
            if len(out) == n - 1:
                break
    e = np.array([(a, b) for a, b, _, _ in out], dtype=np.int64).reshape(-1, 2)
    return e, np.array([x[2] for x in out]), np.array([x[3] for x in out])


def cd2_bruteforce(p, k):
    n, d = p.shape
    full = np.zeros((n, n))
    for kk in range(d):
        t = p[:, None, kk] - p[None, :, kk]
        full = full + t * t
    return np.partition(full, k - 1, axis=1)[:, k - 1], full


def tree_adj(n, edges):
    adj = [[] for _ in range(n)]
    for k, (a, b) in enumerate(edges):
        adj[a].append((b, k))
        adj[b].append((a, k))
    return adj


def key_tuple(w2, e2, a, b):
    return (w2, e2, min(a, b), max(a, b))


CASES = [
    ("uniform", 120, 2, 11), ("uniform", 200, 3, 12), ("uniform", 90, 5, 13),
    ("uniform", 80, 7, 14), ("mixture", 220, 2, 15), ("mixture", 150, 4, 16),
    ("mixture", 100, 6, 17), ("dups", 160, 2, 18), ("dups", 120, 3, 19),
]


def make_case(kind, n, d, seed):
    if kind == "uniform":
        return W.uniform(n, d, seed)
    if kind == "mixture":
        return W.mixture(n, d, seed, k=4, sig_lo=0.005, sig_hi=0.05, noise_frac=0.1)
    return W.with_duplicates(n, d, seed, n_unique=n // 3)


# ------------------------------------------------------------------ tests
@pytest.mark.parametrize("kind,n,d,seed", CASES)
def test_emst_equals_bruteforce_kruskal(kind, n, d, seed):
    p = make_case(kind, n, d, seed)
    e, w2, w = oracle.emst(p)
    eb, wb, _ = kruskal_bruteforce(p)
    eb_sorted = eb  # Kruskal emits in K order already
    assert np.array_equal(e, eb_sorted)
    assert np.array_equal(w2, wb)
    assert np.array_equal(w, np.sqrt(wb))


@pytest.mark.parametrize("kind,n,d,seed", CASES[::2])
@pytest.mark.parametrize("min_pts", [1, 2, 3, 5, 10])
def test_hdbscan_equals_bruteforce_kruskal(kind, n, d, seed, min_pts):
    p = make_case(kind, n, d, seed)
    cd2, cd, e, w2, e2, w = oracle.hdbscan(p, min_pts)
    cb, _ = cd2_bruteforce(p, min_pts)
    assert np.array_equal(cd2, cb)
    assert np.array_equal(cd, np.sqrt(cb))
    eb, wb, e2b = kruskal_bruteforce(p, cb)
    assert np.array_equal(e, eb)
    assert np.array_equal(w2, wb)
    assert np.array_equal(e2, e2b)


@pytest.mark.parametrize("d,axis", [(2, 0), (3, 2), (5, 1), (7, 6)])
def test_collinear_chain(d, axis):
    """Distinct positions on a line: the EMST is the chain of neighbours in
    sorted order, each edge weighing the gap between them."""
    p, t = W.collinear(400, d, seed=d, axis=axis)
    e, w2, w = oracle.emst(p)
    order = np.argsort(t)
    chain = {(min(a, b), max(a, b)) for a, b in zip(order[:-1], order[1:])}
    assert {tuple(x) for x in e.tolist()} == chain
    gaps = np.sort(np.diff(np.sort(t)))
    assert np.array_equal(np.sort(w), gaps)


@pytest.mark.parametrize("k", [2, 5, 12, 20])
def test_unit_grid_total_weight(k):
    """k x k integer grid: every MST edge has length exactly 1 and the tree
    weighs k^2 - 1; the tie-heavy edge choice is pinned by brute force."""
    p = W.grid(k, 2, seed=k)
    e, w2, w = oracle.emst(p)
    assert np.all(w == 1.0)
    assert w.sum() == k * k - 1
    if k <= 12:
        eb, _, _ = kruskal_bruteforce(p)
        assert np.array_equal(e, eb)


def test_grid_3d_ties():
    p = W.grid(5, 3, seed=1)
    e, w2, w = oracle.emst(p)
    assert np.all(w2 == 1.0) and len(e) == 124
    eb, _, _ = kruskal_bruteforce(p)
    assert np.array_equal(e, eb)


@pytest.mark.parametrize("seed,d", [(1, 2), (2, 3), (3, 5)])
def test_minpts_1_and_2_equal_emst(seed, d):
    """Sec. 2.1: with minPts = 1 the mutual reachability distance is the
    Euclidean distance, so the HDBSCAN* MST is the EMST.  With minPts = 2 the
    core distance of p is its nearest-neighbour distance, never more than
    d(p,q), so the weights are again Euclidean (appendix, minPts <= 2)."""
    p = W.mixture(300, d, seed, k=5, noise_frac=0.2)
    e, w2, _ = oracle.emst(p)
    for mp in (1, 2):
        cd2, cd, eh, w2h, e2h, _ = oracle.hdbscan(p, mp)
        assert np.array_equal(eh, e) and np.array_equal(w2h, w2) and np.array_equal(e2h, w2)
        if mp == 1:
            assert np.all(cd2 == 0.0)


@pytest.mark.parametrize("seed,d", [(4, 2), (5, 3), (6, 4), (7, 2)])
def test_minpts3_emst_is_an_mst_of_mutual_reachability(seed, d):
    """Appendix theorem: for minPts <= 3 an EMST is an MST of the mutual
    reachability graph, so the sorted weights of the HDBSCAN* MST equal the
    sorted mutual reachability weights of the EMST's edges."""
    p = W.mixture(260, d, seed, k=6, noise_frac=0.15)
    e, _, _ = oracle.emst(p)
    cd2, _, eh, w2h, _, _ = oracle.hdbscan(p, 3)
    wm, _ = oracle.edge_keys(p, e[:, 0], e[:, 1], cd2=cd2)
    assert np.array_equal(np.sort(wm), np.sort(w2h))


def test_minpts4_can_differ_from_emst():
    """The same appendix shows the relation fails for minPts = 4; on clustered
    data the HDBSCAN* edge set differs from the EMST's."""
    p = W.mixture(300, 2, 9, k=6, noise_frac=0.2)
    e, _, _ = oracle.emst(p)
    _, _, eh, _, _, _ = oracle.hdbscan(p, 4)
    assert not np.array_equal(np.sort(e, axis=0), np.sort(eh, axis=0))


@pytest.mark.parametrize("mp", [None, 4])
def test_cut_property(mp):
    """Every tree edge is the K-lightest edge across the cut it induces."""
    p = W.mixture(140, 3, 21, k=4, noise_frac=0.2)
    if mp is None:
        e, w2, _ = oracle.emst(p)
        cd2 = None
        e2 = w2
    else:
        cd2, _, e, w2, e2, _ = oracle.hdbscan(p, mp)
    n = len(p)
    i, j, W2, E2 = all_pair_keys(p, cd2)
    adj = tree_adj(n, e)
    for k, (a, b) in enumerate(e):
        side = np.zeros(n, bool)
        stack, seen = [a], {a}
        while stack:
            x = stack.pop()
            side[x] = True
            for y, kk in adj[x]:
                if kk != k and y not in seen:
                    seen.add(y)
                    stack.append(y)
        cross = side[i] != side[j]
        keys = sorted(zip(W2[cross], E2[cross], i[cross], j[cross]))
        assert keys[0] == key_tuple(w2[k], e2[k], a, b)


def test_cycle_property():
    """Every non-tree edge is K-heavier than every edge on the tree path
    joining its endpoints."""
    p = W.uniform(150, 2, 22)
    e, w2, _ = oracle.emst(p)
    n = len(p)
    adj = tree_adj(n, e)
    # path maximum from each root by DFS
    for r in range(0, n, 7):
        best = {r: None}
        stack = [r]
        while stack:
            x = stack.pop()
            for y, k in adj[x]:
                if y not in best:
                    kt = key_tuple(w2[k], w2[k], *e[k])
                    best[y] = kt if best[x] is None or kt > best[x] else best[x]
                    stack.append(y)
        wr, er = oracle.edge_keys(p, np.full(n, r), np.arange(n))
        for v in range(n):
            if v == r:
                continue
            on_tree = any(y == v for y, _ in adj[r])
            kv = key_tuple(wr[v], er[v], r, v)
            if on_tree:
                assert kv == best[v]
            else:
                assert kv > best[v]


def test_relative_neighbourhood():
    """An EMST edge (p,q) has no third point r with max(d(p,r), d(q,r)) < d(p,q)."""
    p = W.uniform(600, 3, 23)
    e, w2, _ = oracle.emst(p)
    _, full = cd2_bruteforce(p, 1)
    for (a, b), x in zip(e, w2):
        m = np.maximum(full[a], full[b])
        m[[a, b]] = np.inf
        assert np.all(m >= x)


@pytest.mark.parametrize("k", [1, 2, 5, 10, 17])
def test_core_distance_properties(k):
    """cd2(i) is one of the values d2(i,.) and exactly fewer than k of them
    are smaller while at least k are smaller or equal (p itself counts)."""
    p = W.with_duplicates(300, 3, 24, n_unique=150)
    cd2 = oracle.core_dist2(p, k)
    _, full = cd2_bruteforce(p, 1)
    for i in range(len(p)):
        assert cd2[i] in full[i]
        assert np.sum(full[i] < cd2[i]) < k <= np.sum(full[i] <= cd2[i])
    idx = np.array([0, 7, 299, 150])
    assert np.array_equal(oracle.core_dist2(p, k, idx), cd2[idx])


def test_hdbscan_edges_dominate_core_distances():
    p = W.mixture(250, 3, 25, k=5, noise_frac=0.1)
    cd2, _, e, w2, e2, _ = oracle.hdbscan(p, 7)
    assert np.all(w2 >= np.maximum(cd2[e[:, 0]], cd2[e[:, 1]]))
    assert np.all(w2 >= e2)


def _read_fig1():
    pts, cd, dist, weight, mp = {}, {}, {}, {}, None
    for line in open(os.path.join(GOLDEN, "fig1_fragment.txt")):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue

        def val(s):
            return math.sqrt(float(s[4:])) if s.startswith("sqrt") else float(s)
        if f[0] == "min_pts":
            mp = int(f[1])
        elif f[0] == "point":
            pts[f[1]] = (float(f[2]), float(f[3]))
        elif f[0] == "cd":
            cd[f[1]] = val(f[2])
        elif f[0] == "dist":
            dist[(f[1], f[2])] = val(f[3])
        elif f[0] == "weight":
            weight[(f[1], f[2])] = val(f[3])
    return pts, cd, dist, weight, mp


def test_figure1_worked_example():
    pts, cd, dist, weight, mp = _read_fig1()
    names = list(pts)
    p = np.array([pts[k] for k in names])
    cd2, cdv, e, w2, e2, w = oracle.hdbscan(p, mp)
    ix = {k: i for i, k in enumerate(names)}
    for k, v in cd.items():
        assert cdv[ix[k]] == v
    for (a, b), v in dist.items():
        _, e2ab = oracle.edge_keys(p, [ix[a]], [ix[b]])
        assert math.sqrt(e2ab[0]) == v
    for (a, b), v in weight.items():
        w2ab, _ = oracle.edge_keys(p, [ix[a]], [ix[b]], cd2=cd2)
        assert math.sqrt(w2ab[0]) == v
        # the caption's edge (a,d) is in the MST it draws
        assert (min(ix[a], ix[b]), max(ix[a], ix[b])) in {tuple(x) for x in e.tolist()}


def test_tie_order_rectangle():
    """Four points b1=(D,0), a1=(0,0), a2=(0,eps), b2=(D,eps), minPts = 4:
    every mutual reachability weight is the diagonal, so the order falls to
    the Euclidean length and then the ids; the tree is {(0,3),(1,2),(0,1)}."""
    D, eps = 10.0, 0.5
    p = np.array([[D, 0.0], [0.0, 0.0], [0.0, eps], [D, eps]])
    cd2, _, e, w2, e2, _ = oracle.hdbscan(p, 4)
    assert np.all(cd2 == D * D + eps * eps) and np.all(w2 == D * D + eps * eps)
    assert e.tolist() == [[0, 3], [1, 2], [0, 1]]


def test_tie_order_unit_square():
    """Unit square 0=(0,0),1=(0,1),2=(1,1),3=(1,0), minPts = 4: all weights
    are sqrt 2; the sides win on Euclidean length and then on ids."""
    p = np.array([[0.0, 0.0], [0.0, 1.0], [1.0, 1.0], [1.0, 0.0]])
    cd2, _, e, w2, e2, _ = oracle.hdbscan(p, 4)
    assert np.all(w2 == 2.0)
    assert e.tolist() == [[0, 1], [0, 3], [1, 2]]
    e_emst, w2e, _ = oracle.emst(p)
    assert e_emst.tolist() == [[0, 1], [0, 3], [1, 2]] and np.all(w2e == 1.0)


def test_lightest_cut_edge_matches_bruteforce():
    p = W.uniform(90, 4, 26)
    rng = np.random.default_rng(0)
    i, j, W2, E2 = all_pair_keys(p)
    for _ in range(5):
        s = rng.random(90) < 0.3
        cross = s[i] != s[j]
        want = sorted(zip(W2[cross], E2[cross], i[cross], j[cross]))[0]
        lo, hi, w2, e2 = oracle.lightest_cut_edge(p, s)
        assert (w2, e2, lo, hi) == want


def test_small_and_invalid_inputs():
    e, w2, w = oracle.emst(np.zeros((1, 3)))
    assert e.shape == (0, 2)
    e, w2, w = oracle.emst(np.array([[0.0, 0.0], [3.0, 4.0]]))
    assert e.tolist() == [[0, 1]] and w.tolist() == [5.0]
    with pytest.raises(ValueError):
        oracle.emst(np.array([[0.0, np.nan], [1.0, 1.0]]))
    with pytest.raises(ValueError):
        oracle.hdbscan(np.zeros((3, 2)), 4)
    with pytest.raises(ValueError):
        oracle.hdbscan(np.zeros((3, 2)), 0)


def test_all_coincident_points():
    p = np.ones((50, 3))
    e, w2, w = oracle.emst(p)
    assert np.all(w2 == 0.0)
    # all keys tie on weight: the tree is the star on vertex 0 ordered by id
    assert e.tolist() == [[0, k] for k in range(1, 50)]
