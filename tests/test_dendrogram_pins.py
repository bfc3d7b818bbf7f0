"""Pins of the checker's ordered dendrogram and reachability plot
(oracle.dendrogram) against facts the paper and the mathematics fix, on the
CPU:

* single linkage: the dendrogram of the EMST is the single-linkage hierarchy
  (Sec. 4, "single-linkage clustering ... by passing the EMST"); scipy's
  library single linkage must give the same merges, sizes and heights;
* the reachability plot is defined on the complete graph (Sec. 2.1: point p_i
  has height min over earlier points p_j of d_m(p_i, p_j), in the order of
  Prim's algorithm): a brute-force Prim over all point pairs, written here
  without the tree, must give the checker's order and heights;
* Sec. 4.1: the in-order traversal of the ordered dendrogram's leaves is the
  reachability plot, and the node between two neighbouring leaves has the
  second leaf's reachability height (the dendrogram is the plot's Cartesian
  tree);
* cutting the dendrogram at eps leaves the connected components of the MST
  edges of weight <= eps (Sec. 2.1);
* collinear points: Prim from an end visits the chain in order.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.cluster.hierarchy import linkage
from scipy.sparse.csgraph import connected_components

import oracle
from paper_2104_01126_amd import workloads as W


def emst_tree(p):
    e, w2, w = oracle.emst(p)
    return e, w2, w


def brute_prim(p, start, cd2=None):
    """Prim's algorithm on the complete graph under K = (w2, d2, lo, hi),
    plain loops; -> (order, reach) with reach = sqrt(w2) of the edge that
    reached each point (inf for the start)."""
    n = len(p)
    def key(i, j):
        t = p[i] - p[j]
        s = 0.0
        for x in t:
            s = s + x * x
        w2 = s if cd2 is None else max(cd2[i], cd2[j], s)
        return (w2, s, min(i, j), max(i, j))
    best = {v: key(start, v) for v in range(n) if v != start}
    order, reach = [start], [math.inf]
    while best:
        v = min(best, key=lambda u: best[u])
        order.append(v)
        reach.append(math.sqrt(best[v][0]))
        del best[v]
        for u in best:
            k = key(v, u)
            if k < best[u]:
                best[u] = k
    return np.array(order), np.array(reach)


def brute_cd2(p, k):
    d2 = ((p[:, None, :] - p[None, :, :]) ** 2).sum(-1)
    return np.sort(d2, axis=1)[:, k - 1]


def inorder(children, n):
    """In-order sequence of the ordered dendrogram: leaves and internal nodes
    alternate (iterative; the tree can be as deep as n)."""
    root = n + len(children) - 1
    out, stack, node = [], [], root
    while stack or node is not None:
        while node is not None:
            stack.append(node)
            node = children[node - n][0] if node >= n else None
        node = stack.pop()
        out.append(node)
        node = children[node - n][1] if node >= n else None
    return out


@pytest.mark.parametrize("d,seed", [(2, 1), (3, 2), (5, 3)])
def test_single_linkage_matches_scipy(d, seed):
    p = W.uniform(300, d, seed=seed)
    e, w2, w = emst_tree(p)
    ch, sz, order, reach = oracle.dendrogram(e, w, start=0)
    Z = linkage(p, method="single")
    for k in range(len(e)):
        assert {int(Z[k, 0]), int(Z[k, 1])} == set(ch[k].tolist()), k
        assert int(Z[k, 3]) == sz[k], k
    assert np.allclose(Z[:, 2], w, rtol=1e-12, atol=0)


@pytest.mark.parametrize("start", [0, 17, 149])
def test_reachability_plot_is_prim_on_complete_graph(start):
    p = W.mixture(150, 2, seed=5, k=4, noise_frac=0.1)
    e, w2, w = emst_tree(p)
    _, _, order, reach = oracle.dendrogram(e, w, start=start)
    bo, br = brute_prim(p, start)
    assert np.array_equal(order, bo)
    assert np.array_equal(reach, br)


@pytest.mark.parametrize("mp", [3, 5])
def test_hdbscan_reachability_plot(mp):
    """With core distances the weights tie often; the plot still follows
    Prim's order on the complete mutual-reachability graph under K."""
    p = W.mixture(120, 3, seed=7, k=3, noise_frac=0.1)
    cd2, cd, e, w2, e2, w = oracle.hdbscan(p, mp)
    bcd2 = brute_cd2(p, mp)
    assert np.array_equal(cd2, bcd2)
    _, _, order, reach = oracle.dendrogram(e, w, start=3)
    bo, br = brute_prim(p, 3, cd2=bcd2)
    assert np.array_equal(order, bo)
    assert np.array_equal(reach, br)


@pytest.mark.parametrize("start", [0, 250, 599])
def test_inorder_is_the_plot_and_cartesian_tree(start):
    p = W.uniform(600, 3, seed=11)
    e, w2, w = emst_tree(p)
    n = len(p)
    ch, sz, order, reach = oracle.dendrogram(e, w, start=start)
    seq = inorder(ch, n)
    leaves = [x for x in seq if x < n]
    inner = [x for x in seq if x >= n]
    assert leaves == order.tolist()
    assert all(seq[2 * i] < n for i in range(n)) and all(seq[2 * i + 1] >= n for i in range(n - 1))
    assert np.array_equal(np.array([w[x - n] for x in inner]), reach[1:])
    # sizes are leaf counts of each node
    cnt = np.ones(2 * n - 1, np.int64)
    for k in range(n - 1):
        cnt[n + k] = cnt[ch[k, 0]] + cnt[ch[k, 1]]
    assert np.array_equal(cnt[n:], sz)


def test_start_changes_only_the_orientation():
    p = W.mixture(400, 2, seed=13, k=5)
    e, w2, w = emst_tree(p)
    a = oracle.dendrogram(e, w, start=0)
    b = oracle.dendrogram(e, w, start=399)
    assert np.array_equal(np.sort(a[0], axis=1), np.sort(b[0], axis=1))
    assert np.array_equal(a[1], b[1])
    assert not np.array_equal(a[2], b[2])


@pytest.mark.parametrize("eps_q", [0.2, 0.5, 0.9, 0.99])
def test_cut_gives_components_of_light_edges(eps_q):
    p = W.mixture(500, 3, seed=17, k=6, noise_frac=0.05)
    e, w2, w = emst_tree(p)
    n = len(p)
    ch, sz, order, reach = oracle.dendrogram(e, w, start=0)
    eps = np.quantile(w, eps_q)
    keep = w <= eps
    a = sp.coo_matrix((np.ones(keep.sum()), (e[keep, 0], e[keep, 1])), shape=(n, n))
    ncomp, lab = connected_components(a, directed=False)
    # dendrogram cut: nodes of height <= eps whose parent is above eps
    parent = np.full(2 * n - 1, -1)
    for k in range(n - 1):
        parent[ch[k]] = n + k
    height = np.concatenate([np.full(n, -np.inf), w])
    top = np.arange(2 * n - 1)
    tops = [x for x in range(2 * n - 1) if height[x] <= eps and (parent[x] < 0 or height[parent[x]] > eps)]
    assert len(tops) == ncomp
    # every leaf's cut ancestor labels the same partition as the components
    anc = np.arange(n)
    for x in range(n):
        y = x
        while parent[y] >= 0 and height[parent[y]] <= eps:
            y = parent[y]
        anc[x] = y
    pairs = {(int(l), int(a_)) for l, a_ in zip(lab, anc)}
    assert len(pairs) == ncomp
    del top


def test_chain_from_an_end_visits_in_order():
    p, t = W.collinear(200, 3, seed=19, axis=2)
    e, w2, w = emst_tree(p)
    first = int(np.argmin(t))
    _, _, order, reach = oracle.dendrogram(e, w, start=first)
    assert np.array_equal(order, np.argsort(t))
    ts = np.sort(t)
    assert np.array_equal(reach[1:], np.diff(ts))


def test_single_point_and_bad_trees():
    ch, sz, order, reach = oracle.dendrogram(np.zeros((0, 2), np.int64), np.zeros(0), 0)
    assert order.tolist() == [0] and math.isinf(reach[0])
    with pytest.raises(ValueError):   # a cycle plus an isolated vertex
        oracle.dendrogram(np.array([[0, 1], [1, 2], [2, 0]]), np.array([1.0, 2.0, 3.0]), 0)
    with pytest.raises(ValueError):   # an id out of range
        oracle.dendrogram(np.array([[0, 5]]), np.array([1.0]), 0)
    with pytest.raises(ValueError):   # a bad start
        oracle.dendrogram(np.array([[0, 1]]), np.array([1.0]), 2)
