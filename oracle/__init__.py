"""CPU checker (test infrastructure only).

Plain dense-Prim EMST / HDBSCAN* and brute-force core distances, written from
the problem definitions of the paper (Sec. 2.1).  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import this package; the GPU
library never does and shares no code with it.  See ``oracle.c`` for the exact
arithmetic and the total edge order K = (w2, d2, min id, max id).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# -ffp-contract=off and no fast-math: d2 is summed exactly as written, with
# no fused multiply-add (the recipe the GPU library must match bit for bit).
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared", "-Wall"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (always, when force)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        lib.oracle_emst.argtypes = [P, i64, i32, P, P, P]
        lib.oracle_hdbscan.argtypes = [P, i64, i32, i32, P, P, P, P, P, P]
        lib.oracle_core_dist2.argtypes = [P, i64, i32, i32, P, i64, P]
        lib.oracle_edge_keys.argtypes = [P, i64, i32, P, P, P, i64, P, P]
        lib.oracle_lightest_cut_edge.argtypes = [P, i64, i32, P, P, P, P, P, P]
        lib.oracle_dendrogram.argtypes = [P, P, i64, i64, P, P, P, P]
        lib.oracle_optics_approx.argtypes = [P, i64, i32, i32, ctypes.c_double, P, P, P, P, P]
        lib.oracle_optics_wspd.argtypes = [P, i64, i32, ctypes.c_double, P, P, i64, P]
        for f in (lib.oracle_emst, lib.oracle_hdbscan, lib.oracle_core_dist2,
                  lib.oracle_edge_keys, lib.oracle_lightest_cut_edge, lib.oracle_dendrogram,
                  lib.oracle_optics_approx, lib.oracle_optics_wspd):
            f.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _pts(points) -> np.ndarray:
    p = np.ascontiguousarray(points, dtype=np.float64)
    if p.ndim != 2:
        raise ValueError("points must be [n][d]")
    return p


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"{what} failed with status {rc}")


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def emst(points) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """-> (edges int64[n-1][2] sorted by K, w2 float64[n-1], w float64[n-1])"""
    p = _pts(points)
    n, d = p.shape
    e = np.zeros((max(n - 1, 0), 2), np.int64)
    w2 = np.zeros(max(n - 1, 0))
    w = np.zeros(max(n - 1, 0))
    _check(_load().oracle_emst(_ptr(p), n, d, _ptr(e), _ptr(w2), _ptr(w)), "oracle_emst")
    return e, w2, w


def hdbscan(points, min_pts: int):
    """-> (cd2, cd, edges, w2, e2, w), edges sorted by K = (w2, e2, min, max)."""
    p = _pts(points)
    n, d = p.shape
    m = max(n - 1, 0)
    cd2, cd = np.zeros(n), np.zeros(n)
    e = np.zeros((m, 2), np.int64)
    w2, e2, w = np.zeros(m), np.zeros(m), np.zeros(m)
    _check(_load().oracle_hdbscan(_ptr(p), n, d, int(min_pts), _ptr(cd2), _ptr(cd), _ptr(e),
                                  _ptr(w2), _ptr(e2), _ptr(w)), "oracle_hdbscan")
    return cd2, cd, e, w2, e2, w


def core_dist2(points, min_pts: int, idx=None) -> np.ndarray:
    """cd2 of the rows idx (all rows when None), by exhaustive scan."""
    p = _pts(points)
    n, d = p.shape
    if idx is None:
        out = np.zeros(n)
        rc = _load().oracle_core_dist2(_ptr(p), n, d, int(min_pts), None, n, _ptr(out))
    else:
        ix = np.ascontiguousarray(idx, dtype=np.int64)
        out = np.zeros(len(ix))
        rc = _load().oracle_core_dist2(_ptr(p), n, d, int(min_pts), _ptr(ix), len(ix), _ptr(out))
    _check(rc, "oracle_core_dist2")
    return out


def edge_keys(points, a, b, cd2=None) -> Tuple[np.ndarray, np.ndarray]:
    """(w2, e2) of the given vertex pairs; cd2=None means Euclidean (EMST)."""
    p = _pts(points)
    n, d = p.shape
    a = np.ascontiguousarray(a, dtype=np.int64)
    b = np.ascontiguousarray(b, dtype=np.int64)
    c = None if cd2 is None else np.ascontiguousarray(cd2, dtype=np.float64)
    w2, e2 = np.zeros(len(a)), np.zeros(len(a))
    _check(_load().oracle_edge_keys(_ptr(p), n, d, _ptr(c), _ptr(a), _ptr(b), len(a),
                                    _ptr(w2), _ptr(e2)), "oracle_edge_keys")
    return w2, e2


def lightest_cut_edge(points, in_s, cd2=None):
    """K-lightest edge between the vertex set in_s and its complement:
    -> (lo, hi, w2, e2)."""
    p = _pts(points)
    n, d = p.shape
    s = np.ascontiguousarray(in_s, dtype=np.uint8)
    c = None if cd2 is None else np.ascontiguousarray(cd2, dtype=np.float64)
    lo, hi = ctypes.c_int64(), ctypes.c_int64()
    w2, e2 = ctypes.c_double(), ctypes.c_double()
    _check(_load().oracle_lightest_cut_edge(_ptr(p), n, d, _ptr(c), _ptr(s), ctypes.byref(lo),
                                            ctypes.byref(hi), ctypes.byref(w2), ctypes.byref(e2)),
           "oracle_lightest_cut_edge")
    return lo.value, hi.value, w2.value, e2.value


def dendrogram(edges, weights, start: int = 0):
    """Ordered dendrogram and reachability plot of a spanning tree whose edges
    are given in their total order (Sec. 2.1; Sec. 4.1):
    -> (children int64[n-1][2], size int64[n-1], order int64[n], reach float64[n]).
    Internal node n+k is edge k (height weights[k]); its left child holds the
    endpoint nearer to ``start``; order/reach are Prim's visiting order from
    ``start`` on the tree and the weight of the edge that reached each point."""
    e = np.ascontiguousarray(edges, dtype=np.int64).reshape(-1, 2)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    n = len(e) + 1
    ch = np.zeros((n - 1, 2), np.int64)
    sz = np.zeros(n - 1, np.int64)
    order = np.zeros(n, np.int64)
    reach = np.zeros(n)
    _check(_load().oracle_dendrogram(_ptr(e), _ptr(w), n, int(start), _ptr(ch), _ptr(sz), _ptr(order),
                                     _ptr(reach)), "oracle_dendrogram")
    return ch, sz, order, reach


def optics_approx(points, min_pts: int, rho: float):
    """Approximate OPTICS MST (OPTICS-GanTaoApprox, paper Appendix) on the
    spatial-median k-d tree of quantisation cells; readings T1-M in
    ``oracle.c``.  -> (cd2, edges int64[n-1][2] sorted by K, w2, e2,
    stats = (well-separated pairs, evaluated point pairs, examined pairs))."""
    p = _pts(points)
    n, d = p.shape
    m = max(n - 1, 0)
    cd2 = np.zeros(n)
    e = np.zeros((m, 2), np.int64)
    w2, e2 = np.zeros(m), np.zeros(m)
    st = np.zeros(3, np.int64)
    _check(_load().oracle_optics_approx(_ptr(p), n, d, int(min_pts), float(rho), _ptr(cd2), _ptr(e), _ptr(w2),
                                        _ptr(e2), _ptr(st)), "oracle_optics_approx")
    return cd2, e, w2, e2, tuple(int(x) for x in st)


def optics_wspd(points, rho: float, cap: int = 1 << 22):
    """The decomposition of ``optics_approx`` alone: -> (row_of_pos int64[n],
    pairs int64[m][4] = (first A, count A, first B, count B) in tree positions)."""
    p = _pts(points)
    n, d = p.shape
    row = np.zeros(n, np.int64)
    pairs = np.zeros((cap, 4), np.int64)
    m = ctypes.c_int64()
    _check(_load().oracle_optics_wspd(_ptr(p), n, d, float(rho), _ptr(row), _ptr(pairs), cap, ctypes.byref(m)),
           "oracle_optics_wspd")
    if m.value > cap:
        raise ValueError(f"{m.value} pairs exceed cap {cap}")
    return row, pairs[:m.value].copy()
