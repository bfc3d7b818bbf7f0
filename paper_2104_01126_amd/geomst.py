"""Thin ctypes binding of libgeomst (argument marshalling only).

Every step of a solve runs inside the HIP library; this module converts
arguments and raises on error.  There is no CPU fallback: if the library is
missing or no GPU is present, the calls fail.

* ``emst(points)`` / ``hdbscan(points, min_pts)`` take a numpy array (host
  path: the library copies in and out) or a float64 CUDA tensor (device path,
  queued on torch's current stream, outputs returned as CUDA tensors).
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgeomst.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "geomst.h")

OK, EINVAL, EDOM, ENOMEM, EDEVICE, EBUSY, ETIMEDOUT, ECANCELED, EINTERNAL, ENOENT = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
_NAMES = {EINVAL: "EINVAL", EDOM: "EDOM", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", EBUSY: "EBUSY",
          ETIMEDOUT: "ETIMEDOUT", ECANCELED: "ECANCELED", EINTERNAL: "EINTERNAL", ENOENT: "ENOENT"}


class GeomstError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"geomst error {_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("d", ctypes.c_int32), ("min_pts", ctypes.c_int32),
        ("rounds", ctypes.c_int64), ("pair_visits", ctypes.c_int64), ("bccp_pairs", ctypes.c_int64),
        ("bccp_evals", ctypes.c_int64), ("big_pairs", ctypes.c_int64), ("committed_edges", ctypes.c_int64),
        ("max_frontier", ctypes.c_int64), ("ms_total", ctypes.c_double), ("ms_tree", ctypes.c_double),
        ("ms_core", ctypes.c_double), ("ms_rounds", ctypes.c_double), ("ms_final", ctypes.c_double),
        ("big_evals", ctypes.c_int64), ("sort_elems", ctypes.c_int64),
        ("kernel_ms", ctypes.c_double * 16), ("kernel_launches", ctypes.c_int64 * 16),
        ("bccp_evals_done", ctypes.c_int64), ("tuning_applied", ctypes.c_int64),
        ("level_launches", ctypes.c_int64 * 3),
    ]


class BatchItem(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("n", ctypes.c_int64), ("d", ctypes.c_int32),
                ("min_pts", ctypes.c_int32)]


class Instance(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32),
                ("min_pts", ctypes.c_int32), ("core_dist", ctypes.c_void_p), ("edges", ctypes.c_void_p),
                ("weights", ctypes.c_void_p), ("status", ctypes.c_int32)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("workers", ctypes.c_int32), ("device", ctypes.c_int32),
                ("max_batch_requests", ctypes.c_int32), ("small_max_points", ctypes.c_int32),
                ("max_batch_points", ctypes.c_int64), ("tuning_cache", ctypes.c_char_p)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("batch_requests", ctypes.c_int32), ("batch_points", ctypes.c_int64),
                ("queue_ms", ctypes.c_double), ("service_ms", ctypes.c_double), ("latency_ms", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "queued", "running", "completed", "batches",
                                              "reserved_bytes", "peak_reserved_bytes", "max_batch_requests",
                                              "max_batch_points", "enomem_batches", "workspace_bytes")]


_lib = None


def load(path: str = LIB_PATH):
    """Load libgeomst.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2104_01126_amd/build.py")
    lib = ctypes.CDLL(path)
    P, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.geomst_emst.argtypes = [P, i64, i32, P, P]
    lib.geomst_hdbscan.argtypes = [P, i64, i32, i32, P, P, P]
    lib.geomst_emst_dev.argtypes = [P, i64, i32, P, P, P, P]
    lib.geomst_hdbscan_dev.argtypes = [P, i64, i32, i32, P, P, P, P, P, P]
    lib.geomst_emst_dev_noalloc.argtypes = [P, i64, i32, P, P, P, P]
    lib.geomst_optics_approx_dev.argtypes = [P, i64, i32, i32, dbl, P, P, P, P, P, P]
    lib.geomst_optics_approx.argtypes = [P, i64, i32, i32, dbl, P, P, P]
    lib.geomst_optics_approx_dev.restype = ctypes.c_int
    lib.geomst_optics_approx.restype = ctypes.c_int
    lib.geomst_dendrogram_dev.argtypes = [P, P, i64, i64, P, P, P, P, P]
    lib.geomst_dendrogram.argtypes = [P, P, i64, i64, P, P, P, P]
    lib.geomst_load_tuning.argtypes = [ctypes.c_char_p]
    lib.geomst_load_tuning.restype = ctypes.c_int
    lib.geomst_dendrogram_dev.restype = ctypes.c_int
    lib.geomst_dendrogram.restype = ctypes.c_int
    lib.geomst_emst_dev_noalloc.restype = ctypes.c_int
    lib.geomst_batch_dev.argtypes = [P, i32, ctypes.POINTER(BatchItem), i64, P, P, P, P, P, P]
    lib.geomst_batch.argtypes = [ctypes.POINTER(Instance), i64]
    lib.geomst_batch_dev.restype = ctypes.c_int
    lib.geomst_batch.restype = ctypes.c_int
    lib.geomst_server_create.argtypes = [ctypes.POINTER(ServerCfg), ctypes.POINTER(P)]
    lib.geomst_submit.argtypes = [P, ctypes.POINTER(Instance), ctypes.POINTER(ctypes.c_uint64)]
    lib.geomst_wait.argtypes = [P, ctypes.c_uint64, i64, ctypes.POINTER(RequestInfo)]
    lib.geomst_cancel.argtypes = [P, ctypes.c_uint64]
    lib.geomst_server_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
    lib.geomst_server_destroy.argtypes = [P]
    lib.geomst_server_destroy.restype = None
    for f in (lib.geomst_server_create, lib.geomst_submit, lib.geomst_wait, lib.geomst_cancel,
              lib.geomst_server_stats):
        f.restype = ctypes.c_int
    lib.geomst_get_stats.argtypes = [ctypes.POINTER(_Stats)]
    lib.geomst_set_option.argtypes = [ctypes.c_char_p, dbl]
    lib.geomst_last_error.restype = ctypes.c_char_p
    for f in (lib.geomst_emst, lib.geomst_hdbscan, lib.geomst_emst_dev, lib.geomst_hdbscan_dev,
              lib.geomst_get_stats, lib.geomst_set_option, lib.geomst_version):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def declared_symbols(header: str = HEADER):
    """Function names declared in include/geomst.h."""
    txt = open(header).read()
    return sorted(set(re.findall(r"\b(geomst_\w+)\s*\(", txt)))


def _check(rc: int):
    if rc != OK:
        raise GeomstError(rc, load().geomst_last_error().decode())


def last_error() -> str:
    return load().geomst_last_error().decode()


def version() -> int:
    return int(load().geomst_version())


def set_option(name: str, value: float):
    _check(load().geomst_set_option(name.encode(), float(value)))


def load_tuning(path):
    """Load a tuning cache (JSON lines written by tune.py); None clears it."""
    _check(load().geomst_load_tuning(None if path is None else os.fsencode(path)))


@dataclass
class Stats:
    n: int
    d: int
    min_pts: int
    rounds: int
    pair_visits: int
    bccp_pairs: int
    bccp_evals: int
    big_pairs: int
    committed_edges: int
    max_frontier: int
    ms_total: float
    ms_tree: float
    ms_core: float
    ms_rounds: float
    ms_final: float
    big_evals: int
    sort_elems: int
    kernel_ms: list
    kernel_launches: list
    bccp_evals_done: int
    tuning_applied: int
    level_launches: list


# kernel families (GEOMST_K_* in include/geomst.h)
KERNEL_FAMILIES = ["tree", "sort", "core", "split", "expand", "bccp", "kruskal", "refresh", "output", "dendro",
                   "bccp_large"]


def stats() -> Stats:
    s = _Stats()
    _check(load().geomst_get_stats(ctypes.byref(s)))
    vals = {}
    for f, _ in _Stats._fields_:
        v = getattr(s, f)
        vals[f] = list(v) if f in ("kernel_ms", "kernel_launches", "level_launches") else v
    return Stats(**vals)


def _is_cuda_tensor(x) -> bool:
    return type(x).__module__.startswith("torch") and getattr(x, "is_cuda", False)


def _stream_ptr():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def emst(points, want_sq: bool = False):
    """EMST -> (edges int64 [n-1,2], weights float64 [n-1][, weights_sq]).

    numpy in -> numpy out (host path); CUDA tensor in -> CUDA tensors out."""
    lib = load()
    if _is_cuda_tensor(points):
        import torch
        p = points.contiguous()
        if p.dtype != torch.float64 or p.dim() != 2:
            raise ValueError("points must be a float64 [n, d] tensor")
        n, d = p.shape
        m = max(n - 1, 0)
        e = torch.empty((m, 2), dtype=torch.int64, device=p.device)
        w = torch.empty(m, dtype=torch.float64, device=p.device)
        w2 = torch.empty(m, dtype=torch.float64, device=p.device) if want_sq else None
        _check(lib.geomst_emst_dev(p.data_ptr(), n, d, e.data_ptr(), w.data_ptr(),
                                   w2.data_ptr() if w2 is not None else None, _stream_ptr()))
        return (e, w, w2) if want_sq else (e, w)
    p = np.ascontiguousarray(points, dtype=np.float64)
    if p.ndim != 2:
        raise ValueError("points must be [n, d]")
    n, d = p.shape
    m = max(n - 1, 0)
    e = np.zeros((m, 2), np.int64)
    w = np.zeros(m)
    _check(lib.geomst_emst(p.ctypes.data, n, d, e.ctypes.data, w.ctypes.data))
    return e, w


def header_constant(name: str, header: str = HEADER) -> int:
    """Integer value of a #define in include/geomst.h."""
    m = re.search(r"#define\s+" + re.escape(name) + r"\s+\(?(-?\d+)\)?", open(header).read())
    if not m:
        raise KeyError(name)
    return int(m.group(1))


def emst_noalloc(points, want_sq: bool = False):
    """EMST through geomst_emst_dev_noalloc (fixed device scratch, no
    allocation inside the call): CUDA tensor in -> CUDA tensors out, like
    ``emst``.  The output tensors are allocated here, by the caller."""
    import torch
    if not _is_cuda_tensor(points):
        raise ValueError("emst_noalloc takes a float64 CUDA tensor")
    p = points.contiguous()
    if p.dtype != torch.float64 or p.dim() != 2:
        raise ValueError("points must be a float64 [n, d] tensor")
    n, d = p.shape
    m = max(n - 1, 0)
    e = torch.empty((m, 2), dtype=torch.int64, device=p.device)
    w = torch.empty(m, dtype=torch.float64, device=p.device)
    w2 = torch.empty(m, dtype=torch.float64, device=p.device) if want_sq else None
    _check(load().geomst_emst_dev_noalloc(p.data_ptr(), n, d, e.data_ptr(), w.data_ptr(),
                                          w2.data_ptr() if w2 is not None else None, _stream_ptr()))
    return (e, w, w2) if want_sq else (e, w)


def hdbscan(points, min_pts: int, want_sq: bool = False):
    """HDBSCAN* -> (core_dist [n], edges [n-1,2], weights [n-1]
    [, core_dist_sq, weights_sq])."""
    lib = load()
    if _is_cuda_tensor(points):
        import torch
        p = points.contiguous()
        if p.dtype != torch.float64 or p.dim() != 2:
            raise ValueError("points must be a float64 [n, d] tensor")
        n, d = p.shape
        m = max(n - 1, 0)
        dev = p.device
        cd = torch.empty(n, dtype=torch.float64, device=dev)
        e = torch.empty((m, 2), dtype=torch.int64, device=dev)
        w = torch.empty(m, dtype=torch.float64, device=dev)
        cd2 = torch.empty(n, dtype=torch.float64, device=dev) if want_sq else None
        w2 = torch.empty(m, dtype=torch.float64, device=dev) if want_sq else None
        _check(lib.geomst_hdbscan_dev(p.data_ptr(), n, d, int(min_pts), cd.data_ptr(),
                                      cd2.data_ptr() if cd2 is not None else None, e.data_ptr(),
                                      w.data_ptr(), w2.data_ptr() if w2 is not None else None,
                                      _stream_ptr()))
        return (cd, e, w, cd2, w2) if want_sq else (cd, e, w)
    p = np.ascontiguousarray(points, dtype=np.float64)
    if p.ndim != 2:
        raise ValueError("points must be [n, d]")
    n, d = p.shape
    m = max(n - 1, 0)
    cd = np.zeros(n)
    e = np.zeros((m, 2), np.int64)
    w = np.zeros(m)
    _check(lib.geomst_hdbscan(p.ctypes.data, n, d, int(min_pts), cd.ctypes.data, e.ctypes.data,
                              w.ctypes.data))
    return cd, e, w


def optics_approx(points, min_pts: int, rho: float, want_sq: bool = False):
    """Approximate OPTICS MST (Gan-Tao base graph on the WSPD, s = sqrt(8/rho))
    -> (core_dist [n], edges [n-1,2], weights [n-1][, core_dist_sq, weights_sq]).
    numpy in -> numpy out (host path); CUDA tensor in -> CUDA tensors out."""
    lib = load()
    if _is_cuda_tensor(points):
        import torch
        p = points.contiguous()
        if p.dtype != torch.float64 or p.dim() != 2:
            raise ValueError("points must be a float64 [n, d] tensor")
        n, d = p.shape
        m = max(n - 1, 0)
        dev = p.device
        cd = torch.empty(n, dtype=torch.float64, device=dev)
        e = torch.empty((m, 2), dtype=torch.int64, device=dev)
        w = torch.empty(m, dtype=torch.float64, device=dev)
        cd2 = torch.empty(n, dtype=torch.float64, device=dev) if want_sq else None
        w2 = torch.empty(m, dtype=torch.float64, device=dev) if want_sq else None
        _check(lib.geomst_optics_approx_dev(p.data_ptr(), n, d, int(min_pts), float(rho), cd.data_ptr(),
                                            cd2.data_ptr() if cd2 is not None else None, e.data_ptr(),
                                            w.data_ptr(), w2.data_ptr() if w2 is not None else None,
                                            _stream_ptr()))
        return (cd, e, w, cd2, w2) if want_sq else (cd, e, w)
    p = np.ascontiguousarray(points, dtype=np.float64)
    if p.ndim != 2:
        raise ValueError("points must be [n, d]")
    n, d = p.shape
    m = max(n - 1, 0)
    cd = np.zeros(n)
    e = np.zeros((m, 2), np.int64)
    w = np.zeros(m)
    _check(lib.geomst_optics_approx(p.ctypes.data, n, d, int(min_pts), float(rho), cd.ctypes.data,
                                    e.ctypes.data, w.ctypes.data))
    return cd, e, w


def dendrogram(edges, weights, start: int = 0):
    """Ordered dendrogram and reachability plot of a spanning tree given by
    its edges in their total order (as ``emst``/``hdbscan`` return them) ->
    (children int64 [n-1,2], size int64 [n-1], order int64 [n], reach
    float64 [n]).  numpy in -> numpy out; CUDA tensors in -> CUDA tensors
    out (queued on torch's current stream)."""
    lib = load()
    if _is_cuda_tensor(edges):
        import torch
        e = edges.contiguous()
        w = weights.contiguous()
        if e.dtype != torch.int64 or w.dtype != torch.float64:
            raise ValueError("edges must be int64 and weights float64")
        n = e.shape[0] + 1
        dev = e.device
        ch = torch.empty((n - 1, 2), dtype=torch.int64, device=dev)
        sz = torch.empty(n - 1, dtype=torch.int64, device=dev)
        order = torch.empty(n, dtype=torch.int64, device=dev)
        reach = torch.empty(n, dtype=torch.float64, device=dev)
        _check(lib.geomst_dendrogram_dev(e.data_ptr(), w.data_ptr(), n, int(start), ch.data_ptr(), sz.data_ptr(),
                                         order.data_ptr(), reach.data_ptr(), _stream_ptr()))
        return ch, sz, order, reach
    e = np.ascontiguousarray(edges, dtype=np.int64).reshape(-1, 2)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    n = len(e) + 1
    ch = np.zeros((n - 1, 2), np.int64)
    sz = np.zeros(n - 1, np.int64)
    order = np.zeros(n, np.int64)
    reach = np.zeros(n)
    _check(lib.geomst_dendrogram(e.ctypes.data, w.ctypes.data, n, int(start), ch.ctypes.data, sz.ctypes.data,
                                 order.ctypes.data, reach.ctypes.data))
    return ch, sz, order, reach


# ------------------------------------------------------------------ batches
def pack(instances, min_pts=0):
    """Pack a list of [n_i][d_i] arrays into one zero-padded [N][stride]
    arena (instances in order) -> (arena, items, stride).  min_pts: one int
    for all instances or a list (0 = EMST)."""
    mps = list(min_pts) if hasattr(min_pts, "__len__") else [int(min_pts)] * len(instances)
    stride = max(int(np.asarray(x).shape[1]) for x in instances)
    N = sum(len(x) for x in instances)
    arena = np.zeros((N, stride))
    items = (BatchItem * len(instances))()
    off = 0
    for i, x in enumerate(instances):
        x = np.asarray(x, dtype=np.float64)
        arena[off:off + len(x), :x.shape[1]] = x
        items[i].offset, items[i].n, items[i].d, items[i].min_pts = off, len(x), x.shape[1], mps[i]
        off += len(x)
    return arena, items, stride


def batch_dev(arena, items, stride, want_sq=False):
    """Batched solve of a packed arena already on the GPU (float64 CUDA
    tensor [N][stride]) -> dict of CUDA tensors: edges [N-count,2] (instance-
    local ids, instance i's edges start at row offset_i - i), weights,
    core_dist [N] (and weights_sq, core_dist_sq)."""
    import torch
    lib = load()
    a = arena.contiguous()
    N, count = a.shape[0], len(items)
    dev = a.device
    m = N - count
    out = {"edges": torch.empty((m, 2), dtype=torch.int64, device=dev),
           "weights": torch.empty(m, dtype=torch.float64, device=dev),
           "core_dist": torch.empty(N, dtype=torch.float64, device=dev)}
    if want_sq:
        out["weights_sq"] = torch.empty(m, dtype=torch.float64, device=dev)
        out["core_dist_sq"] = torch.empty(N, dtype=torch.float64, device=dev)
    ptr = lambda k: out[k].data_ptr() if k in out else None
    _check(lib.geomst_batch_dev(a.data_ptr(), int(stride), items, count, ptr("edges"), ptr("weights"),
                                ptr("weights_sq"), ptr("core_dist"), ptr("core_dist_sq"), _stream_ptr()))
    return out


def unpack(out, items):
    """Split batch_dev outputs per instance -> list of dicts (numpy)."""
    res = []
    e = out["edges"].cpu().numpy()
    w = out["weights"].cpu().numpy()
    cd = out["core_dist"].cpu().numpy()
    w2 = out["weights_sq"].cpu().numpy() if "weights_sq" in out else None
    cd2 = out["core_dist_sq"].cpu().numpy() if "core_dist_sq" in out else None
    for i, it in enumerate(items):
        eo, n, off = it.offset - i, it.n, it.offset
        r = {"edges": e[eo:eo + n - 1], "weights": w[eo:eo + n - 1], "core_dist": cd[off:off + n]}
        if w2 is not None:
            r["weights_sq"] = w2[eo:eo + n - 1]
            r["core_dist_sq"] = cd2[off:off + n]
        res.append(r)
    return res


def batch(instances, min_pts=0):
    """Host-pointer batch (geomst_batch): list of numpy arrays -> list of
    (edges, weights, core_dist)."""
    lib = load()
    mps = list(min_pts) if hasattr(min_pts, "__len__") else [int(min_pts)] * len(instances)
    arr = (Instance * len(instances))()
    keep = []
    for i, x in enumerate(instances):
        x = np.ascontiguousarray(x, dtype=np.float64)
        n, d = x.shape
        e = np.zeros((max(n - 1, 0), 2), np.int64)
        w = np.zeros(max(n - 1, 0))
        cd = np.zeros(n)
        keep.append((x, e, w, cd))
        arr[i].points, arr[i].n, arr[i].d, arr[i].min_pts = x.ctypes.data, n, d, mps[i]
        arr[i].core_dist, arr[i].edges, arr[i].weights = cd.ctypes.data, e.ctypes.data, w.ctypes.data
    _check(lib.geomst_batch(arr, len(instances)))
    return [(k[1], k[2], k[3]) for k in keep]


# ------------------------------------------------------------------ serving
class Server:
    """Request loop with continuous batching (geomst_server_*).

    ``submit(points, min_pts)`` copies the points and returns a ticket;
    ``wait(ticket)`` returns (edges, weights, core_dist, info) once the
    request's batch is done.  The output arrays are allocated here and kept
    alive until the ticket is released."""

    def __init__(self, hbm_budget_bytes=0, workers=0, device=-1, max_batch_requests=0, max_batch_points=0,
                 small_max_points=0, tuning_cache=None):
        lib = load()
        cfg = ServerCfg(int(hbm_budget_bytes), int(workers), int(device), int(max_batch_requests),
                        int(small_max_points), int(max_batch_points),
                        None if tuning_cache is None else os.fsencode(tuning_cache))
        h = ctypes.c_void_p()
        _check(lib.geomst_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._out = {}

    def submit(self, points, min_pts=0) -> int:
        lib = load()
        x = np.ascontiguousarray(points, dtype=np.float64)
        n, d = x.shape
        e = np.zeros((max(n - 1, 0), 2), np.int64)
        w = np.zeros(max(n - 1, 0))
        cd = np.zeros(n)
        req = Instance(x.ctypes.data, n, d, int(min_pts), cd.ctypes.data, e.ctypes.data, w.ctypes.data, 0)
        t = ctypes.c_uint64()
        _check(lib.geomst_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._out[t.value] = (e, w, cd)
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1):
        """-> (edges, weights, core_dist, info dict); raises GeomstError
        (ETIMEDOUT if not done within timeout_us)."""
        info = RequestInfo()
        rc = load().geomst_wait(self._h, ticket, int(timeout_us), ctypes.byref(info))
        if rc == ETIMEDOUT:
            raise GeomstError(rc, "not done yet")
        out = self._out.pop(ticket, None)
        _check(rc)
        d = {k: getattr(info, k) for k, _ in RequestInfo._fields_}
        return out[0], out[1], out[2], d

    def cancel(self, ticket: int):
        rc = load().geomst_cancel(self._h, ticket)
        self._out.pop(ticket, None)
        _check(rc)

    def stats(self) -> dict:
        s = ServerStats()
        _check(load().geomst_server_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            load().geomst_server_destroy(self._h)
            self._h = None
            self._out.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
