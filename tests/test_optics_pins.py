"""Pins of the checker's approximate OPTICS (oracle.optics_approx, the paper's
Appendix "Parallel Approximate OPTICS") against facts that do not come from
its own code, on the CPU:

* the decomposition is a WSPD: every pair of distinct points lies in exactly
  one pair (A, B), and A and B are s-separated, s = sqrt(8 / rho), by the
  definition of Sec. 2.3 (two balls of a common radius r holding A and B at
  distance >= s r), checked here with boxes recomputed from the points;
* with rho tiny, s is so large that only single points are separated: every
  point pair is its own base-graph edge, and the result is the MST of the
  complete graph under w = max{cd, cd, d / (1 + rho)} (a brute-force Prim
  written here), which has the exact HDBSCAN* tree's edges;
* every base-graph weight lies between d_m / (1 + rho) and d_m, so the sorted
  tree weights are bounded below by the exact HDBSCAN* MST's divided by
  (1 + rho) (the MST's sorted weights are the smallest of any spanning tree),
  and every tree edge is at most its own d_m;
* the four edge cases: with minPts = 1 every node is large and only
  representatives are joined; with minPts = n no node is, every point pair is
  evaluated exactly once and each tree edge is the lightest point pair of its
  WSPD pair; the evaluation count follows the case rule for any minPts;
* doubling every coordinate (exact in binary floating point) leaves the tree
  and the decomposition unchanged and multiplies every w2 by 4.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2104_01126_amd import workloads as W


def d2_all(p):
    n, d = p.shape
    s = np.zeros((n, n))
    for k in range(d):
        t = p[:, None, k] - p[None, :, k]
        s = s + t * t
    return s


def sets_of(row, pair):
    fa, ca, fb, cb = (int(v) for v in pair)
    return row[fa:fa + ca], row[fb:fb + cb]


def ball_gap_ok(p, A, B, s):
    """Sec. 2.3 separation with balls around the tight boxes' midpoints."""
    def ball(S):
        lo, hi = p[S].min(axis=0), p[S].max(axis=0)
        return 0.5 * (lo + hi), 0.5 * math.sqrt(float(((hi - lo) ** 2).sum()))
    ca, ra = ball(A)
    cb, rb = ball(B)
    r = max(ra, rb)
    dist = math.sqrt(float(((ca - cb) ** 2).sum()))
    scale = max(1.0, float(np.abs(p).max()))
    return dist - 2 * r >= s * r - 1e-6 * scale


@pytest.mark.parametrize("n,d,rho,seed", [(60, 2, 0.125, 1), (60, 3, 0.5, 2), (50, 3, 2.0, 3), (40, 5, 0.125, 4),
                                          (40, 7, 1.0, 5)])
def test_decomposition_is_a_wspd(n, d, rho, seed):
    p = W.mixture(n, d, seed, k=3, sig_lo=0.02, sig_hi=0.2)
    row, pairs = oracle.optics_wspd(p, rho)
    assert sorted(row.tolist()) == list(range(n))
    cover = np.zeros((n, n), np.int64)
    s = math.sqrt(8.0 / rho)
    for pr in pairs:
        A, B = sets_of(row, pr)
        assert len(A) and len(B)
        cover[np.ix_(A, B)] += 1
        cover[np.ix_(B, A)] += 1
        assert ball_gap_ok(p, A, B, s), (pr, A, B)
    off = ~np.eye(n, dtype=bool)
    assert (cover[off] == 1).all()
    assert (np.diag(cover) == 0).all()


def brute_prim_w2(p, cd2, q):
    """Dense Prim under K = (w2, d2, lo, hi) with w2 = max(cd2, cd2, d2 / q)."""
    n = len(p)
    e2 = d2_all(p)
    w2 = np.maximum(np.maximum(cd2[:, None], cd2[None, :]), e2 / q)
    inside = np.zeros(n, bool)
    inside[0] = True
    out = []
    for _ in range(n - 1):
        best = None
        for i in np.flatnonzero(inside):
            for j in np.flatnonzero(~inside):
                k = (w2[i, j], e2[i, j], min(i, j), max(i, j))
                if best is None or k < best:
                    best = k
        out.append(best)
        inside[best[3] if inside[best[2]] else best[2]] = True
    out.sort()
    return np.array([(a, b) for _, _, a, b in out]), np.array([w for w, _, _, _ in out])


@pytest.mark.parametrize("seed,mp", [(1, 1), (2, 3), (3, 5)])
def test_tiny_rho_is_the_complete_graph(seed, mp):
    p = W.uniform(12, 2, seed)
    rho = 1e-9
    row, pairs = oracle.optics_wspd(p, rho)
    assert len(pairs) == 12 * 11 // 2 and (pairs[:, 1] == 1).all() and (pairs[:, 3] == 1).all()
    cd2, e, w2, e2, st = oracle.optics_approx(p, mp, rho)
    q = (1.0 + rho) * (1.0 + rho)
    eb, wb = brute_prim_w2(p, cd2, q)
    assert np.array_equal(e, eb)
    assert np.array_equal(w2, wb)
    # the same tree as exact HDBSCAN* (no near ties at this size), weights
    # within the factor (1 + rho)^2 below
    cdx, _, ex, w2x, _, _ = oracle.hdbscan(p, mp)
    assert np.array_equal(cd2, cdx)
    assert set(map(tuple, e.tolist())) == set(map(tuple, ex.tolist()))
    assert (np.sort(w2) <= np.sort(w2x)).all() and (np.sort(w2) * q >= np.sort(w2x) * (1 - 1e-15)).all()


def is_spanning_tree(e, n):
    par = list(range(n))

    def find(x):
        while par[x] != x:
            par[x] = par[par[x]]
            x = par[x]
        return x
    for a, b in e:
        ra, rb = find(int(a)), find(int(b))
        if ra == rb:
            return False
        par[ra] = rb
    return len(e) == n - 1


@pytest.mark.parametrize("n,d,mp,rho,seed", [(1500, 3, 10, 0.125, 1), (800, 2, 5, 0.5, 2), (400, 5, 16, 1.0, 3)])
def test_weights_bounded_by_exact_hdbscan(n, d, mp, rho, seed):
    p = W.mixture(n, d, seed, k=6, noise_frac=0.05)
    cd2, e, w2, e2, st = oracle.optics_approx(p, mp, rho)
    assert is_spanning_tree(e, n)
    assert (e[:, 0] < e[:, 1]).all()
    q = (1.0 + rho) * (1.0 + rho)
    dd = d2_all(p)
    eu, ev = e[:, 0], e[:, 1]
    assert np.array_equal(e2, dd[eu, ev])
    assert np.array_equal(w2, np.maximum(np.maximum(cd2[eu], cd2[ev]), e2 / q))
    # sorted by K
    keys = list(zip(w2, e2, eu, ev))
    assert keys == sorted(keys)
    cdx, _, ex, w2x, _, _ = oracle.hdbscan(p, mp)
    assert np.array_equal(cd2, cdx)
    dm2 = np.maximum(np.maximum(cd2[eu], cd2[ev]), e2)
    assert (w2 <= dm2).all()
    assert (np.sort(w2) * q >= np.sort(w2x) * (1 - 1e-15)).all()


def test_case_rules():
    p = W.mixture(300, 2, 7, k=4, noise_frac=0.1)
    n = len(p)
    rho = 0.25
    row, pairs = oracle.optics_wspd(p, rho)
    # minPts = 1: every node is large; one evaluation per pair, and every
    # tree edge joins the representatives (first tree positions) of a pair
    cd2, e, w2, e2, st = oracle.optics_approx(p, 1, rho)
    assert st[0] == len(pairs) and st[1] == len(pairs)
    reps = {tuple(sorted((int(row[a]), int(row[b])))) for a, _, b, _ in pairs}
    assert set(map(tuple, e.tolist())) <= reps
    # minPts = n: no node is large; every point pair is evaluated once, and
    # each tree edge is the lightest point pair of the pair that holds it
    cd2, e, w2, e2, st = oracle.optics_approx(p, n, rho)
    assert st[1] == n * (n - 1) // 2
    q = (1.0 + rho) * (1.0 + rho)
    dd = d2_all(p)
    where = {}
    for k, pr in enumerate(pairs):
        A, B = sets_of(row, pr)
        for a in A:
            for b in B:
                where[(min(a, b), max(a, b))] = k
    for (a, b), wv in zip(e.tolist(), w2):
        A, B = sets_of(row, pairs[where[(a, b)]])
        ww = np.maximum(np.maximum(cd2[A][:, None], cd2[B][None, :]), dd[np.ix_(A, B)] / q)
        cand = min((ww[i, j], dd[A[i], B[j]], min(A[i], B[j]), max(A[i], B[j]))
                   for i in range(len(A)) for j in range(len(B)))
        assert (cand[2], cand[3]) == (a, b) and cand[0] == wv
    # any minPts: evaluations follow the case rule
    for mp in (2, 5, 12):
        st = oracle.optics_approx(p, mp, rho)[4]
        exp = sum((1 if ca >= mp else ca) * (1 if cb >= mp else cb) for _, ca, _, cb in pairs)
        assert st[1] == exp


def test_scale_by_two():
    p = W.mixture(500, 3, 9, k=5)
    a = oracle.optics_approx(p, 8, 0.125)
    b = oracle.optics_approx(2.0 * p, 8, 0.125)
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(4.0 * a[2], b[2])
    assert a[4] == b[4]


def test_duplicates_and_tiny_inputs():
    p = W.with_duplicates(200, 3, 11, 40)
    cd2, e, w2, e2, st = oracle.optics_approx(p, 4, 0.125)
    assert is_spanning_tree(e, len(p))
    row, pairs = oracle.optics_wspd(p, 0.125)
    cover = np.zeros((200, 200), np.int64)
    for pr in pairs:
        A, B = sets_of(row, pr)
        cover[np.ix_(A, B)] += 1
        cover[np.ix_(B, A)] += 1
    assert (cover[~np.eye(200, dtype=bool)] == 1).all()
    for n in (1, 2, 3):
        q = W.uniform(n, 2, n)
        cd2, e, w2, e2, st = oracle.optics_approx(q, 1, 0.5)
        assert len(e) == n - 1 and is_spanning_tree(e, n)
        assert st[0] == len(oracle.optics_wspd(q, 0.5)[1]) and (n < 3 or st[0] >= 2)
