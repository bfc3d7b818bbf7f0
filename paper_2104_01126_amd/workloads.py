"""Seeded synthetic point sets shared by the tests, the benchmark and the checker.

This module only draws numbers: it holds none of the method's arithmetic (no
distances, no trees, no spanning trees), so that the HIP path and the CPU
checker can be fed the very same arrays without sharing any computation.

Every generator uses numpy's ``default_rng(seed)`` (PCG64) and the draw order
written below is part of the contract: changing it changes every stored
expectation.

Workloads (the paper measures on uniformly filled hypercubes and on
varying-density seed-spreader sets of 10M points, Sec. 5 "Data Sets"; those
sets are not available here, so uniform cubes stand in for the former and
Gaussian mixtures with log-uniform widths for the latter):

* ``emst_small``   EMST, 2,000 points in [0,1)^2, seed 0.
* ``emst_1m``      EMST, 1,000,000 points uniform in [0,1000)^3, seed 1.
* ``hdbscan_2m``   HDBSCAN*, minPts=10, 2,000,000 points in 5-D: 95% from 64
                   isotropic Gaussians (centres uniform in [0,1e4)^5, sigma
                   log-uniform in [0.5,20]) and 5% uniform noise, seed 2.
* ``batch_4096``   4,096 EMST instances, n log-uniform in [100,50000], d in
                   {2,3}, half uniform, half 8-Gaussian mixtures, seed 3.
* ``optics_500k``  approximate OPTICS, minPts=10, rho=0.125 (s = 8, the
                   setting of the paper's approximate-OPTICS runs): 500,000
                   points in 3-D drawn like ``hdbscan_2m`` (64 Gaussians,
                   centres uniform in [0,1e4)^3, sigma log-uniform in
                   [0.5,20], plus 5% uniform noise), seed 5.
* ``serving_trace`` a Poisson request stream at 2,000 requests/s for 60 s
                   (seed 4): 70% EMST, 30% HDBSCAN* with minPts in {5,10,16},
                   n log-uniform in [1e3,1e6], d in {2..7}, half uniform and
                   half 8-Gaussian mixtures; request i's points come from
                   seed (4, i) so any request can be drawn alone.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Tuple

import numpy as np

__all__ = [
    "emst_small", "emst_1m", "hdbscan_2m", "batch_4096", "batch_instance",
    "uniform", "mixture", "grid", "collinear", "with_duplicates", "subsample",
    "ServingRequest", "serving_trace", "serving_points",
]


def _c(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- workloads
def emst_small() -> np.ndarray:
    rng = np.random.default_rng(0)
    return _c(rng.random((2000, 2)))


def emst_1m(n: int = 1_000_000) -> np.ndarray:
    """Uniform in [0,1000)^3; ``n`` < 1e6 gives the first rows of the same draw
    order only when drawn with the same n, so a prefix is taken instead."""
    rng = np.random.default_rng(1)
    p = rng.uniform(0.0, 1000.0, (1_000_000, 3))
    return _c(p[:n])


def hdbscan_2m(n_total: int = 2_000_000) -> np.ndarray:
    """64-Gaussian mixture plus 5% uniform noise in [0,1e4)^5 (seed 2).

    ``n_total`` scales the cluster/noise counts proportionally (95% / 5%) for
    reduced test sizes; the full workload is ``n_total=2_000_000``."""
    rng = np.random.default_rng(2)
    d, k = 5, 64
    centres = rng.uniform(0.0, 1e4, (k, d))
    sig = np.exp(rng.uniform(math.log(0.5), math.log(20.0), k))
    nc = (n_total * 95) // 100
    nn = n_total - nc
    lab = rng.integers(0, k, nc)
    x = centres[lab] + sig[lab][:, None] * rng.standard_normal((nc, d))
    noise = rng.uniform(0.0, 1e4, (nn, d))
    p = np.concatenate([x, noise], axis=0)
    p = p[rng.permutation(n_total)]
    return _c(p)


def optics_500k(n_total: int = 500_000) -> np.ndarray:
    """64-Gaussian mixture plus 5% uniform noise in [0,1e4)^3 (seed 5);
    ``n_total`` scales the counts for reduced test sizes."""
    rng = np.random.default_rng(5)
    d, k = 3, 64
    centres = rng.uniform(0.0, 1e4, (k, d))
    sig = np.exp(rng.uniform(math.log(0.5), math.log(20.0), k))
    nc = (n_total * 95) // 100
    nn = n_total - nc
    lab = rng.integers(0, k, nc)
    x = centres[lab] + sig[lab][:, None] * rng.standard_normal((nc, d))
    noise = rng.uniform(0.0, 1e4, (nn, d))
    p = np.concatenate([x, noise], axis=0)
    p = p[rng.permutation(n_total)]
    return _c(p)


def batch_4096(count: int = 4096) -> List[np.ndarray]:
    """Independent EMST instances; ``count`` < 4096 returns a prefix."""
    rng = np.random.default_rng(3)
    out = []
    for i in range(4096):
        n_i = int(round(math.exp(rng.uniform(math.log(100.0), math.log(50000.0)))))
        d_i = int(rng.choice([2, 3]))
        if i % 2 == 0:
            p = rng.random((n_i, d_i))
        else:
            cen = rng.random((8, d_i))
            sg = rng.uniform(0.01, 0.1, 8)
            lab = rng.integers(0, 8, n_i)
            p = cen[lab] + sg[lab][:, None] * rng.standard_normal((n_i, d_i))
        out.append(_c(p))
        if len(out) == count:
            break
    return out


def batch_instance(i: int) -> np.ndarray:
    return batch_4096(i + 1)[i]


@dataclass(frozen=True)
class ServingRequest:
    index: int
    arrival_s: float
    n: int
    d: int
    min_pts: int      # 0 = EMST
    mixture: bool     # False: uniform in [0,1)^d


def serving_trace(duration_s: float = 60.0, rate: float = 2000.0, n_lo: float = 1e3,
                  n_hi: float = 1e6) -> List[ServingRequest]:
    """Arrivals of the serving stream up to ``duration_s`` (a prefix of the
    60 s stream for smaller values; ``n_lo``/``n_hi`` other than the defaults
    give a scaled-down stream of the same shape)."""
    rng = np.random.default_rng(4)
    out: List[ServingRequest] = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s:
            break
        emst = rng.random() < 0.7
        mp = 0 if emst else int(rng.choice([5, 10, 16]))
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        d = int(rng.integers(2, 8))
        mix = bool(rng.random() < 0.5)
        out.append(ServingRequest(len(out), t, n, d, mp, mix))
    return out


def serving_points(req: ServingRequest) -> np.ndarray:
    rng = np.random.default_rng([4, req.index])
    if not req.mixture:
        return _c(rng.random((req.n, req.d)))
    cen = rng.random((8, req.d))
    sg = rng.uniform(0.01, 0.1, 8)
    lab = rng.integers(0, 8, req.n)
    return _c(cen[lab] + sg[lab][:, None] * rng.standard_normal((req.n, req.d)))


# ------------------------------------------------------- small test shapes
def uniform(n: int, d: int, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _c(rng.uniform(lo, hi, (n, d)))


def mixture(n: int, d: int, seed: int, k: int = 8, box: float = 1.0,
            sig_lo: float = 0.01, sig_hi: float = 0.1, noise_frac: float = 0.0) -> np.ndarray:
    """k isotropic Gaussians with log-uniform widths plus optional uniform noise."""
    rng = np.random.default_rng(seed)
    cen = rng.uniform(0.0, box, (k, d))
    sig = np.exp(rng.uniform(math.log(sig_lo * box), math.log(sig_hi * box), k))
    nn = int(n * noise_frac)
    nc = n - nn
    lab = rng.integers(0, k, nc)
    x = cen[lab] + sig[lab][:, None] * rng.standard_normal((nc, d))
    noise = rng.uniform(0.0, box, (nn, d))
    p = np.concatenate([x, noise], axis=0)
    return _c(p[rng.permutation(n)])


def grid(k: int, d: int = 2, seed: int | None = None) -> np.ndarray:
    """The k^d integer lattice points, optionally in a shuffled row order."""
    axes = [np.arange(k, dtype=np.float64)] * d
    g = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, d)
    if seed is not None:
        g = g[np.random.default_rng(seed).permutation(len(g))]
    return _c(g)


def collinear(n: int, d: int, seed: int, axis: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Distinct positions t on one coordinate axis, rows in random order.
    Returns (points, t)."""
    rng = np.random.default_rng(seed)
    t = rng.permutation(np.unique(rng.integers(0, 50 * n, 2 * n)))[:n].astype(np.float64)
    p = np.zeros((len(t), d))
    p[:, axis] = t
    return _c(p), t


def with_duplicates(n: int, d: int, seed: int, n_unique: int) -> np.ndarray:
    """n rows drawn from n_unique distinct uniform locations (many exact repeats)."""
    rng = np.random.default_rng(seed)
    base = rng.random((n_unique, d))
    return _c(base[rng.integers(0, n_unique, n)])


def subsample(p: np.ndarray, m: int) -> np.ndarray:
    return _c(p[:m])
