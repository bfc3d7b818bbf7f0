"""Autotuner of the knobs that never change a result.

For each workload it searches, one knob at a time (coordinate descent), the
settings that make the solve fastest, and writes them as one JSON object per
line to a tuning cache that ``geomst_load_tuning`` (or a server's
``tuning_cache``) applies to solves of the same kind, dimension and size
class:

* ``bccp_chunk``              B points per large-pair BCCP task (the tile's B side);
* ``small_level_switch`` / ``small_level_max``  which expansion levels run in the
  one-workgroup kernel (the bucketing of pair levels by size);
* ``beta_growth``             the factor between round thresholds;
* ``refresh_divisor``         how often node components are refreshed.

Every candidate's output (edges and squared weights, and core distances for
HDBSCAN*) must hash to the same bytes as the default settings' output, or the
tuner stops: a knob that changed a result would be a bug.

    python -m paper_2104_01126_amd.tune --workloads batch_4096 emst_1m hdbscan_2m \\
        --out paper_2104_01126_amd/tuning_cache.jsonl

Only the seeded workload generators and the library are used; timing needs a
GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import sys
import time
from typing import Callable, Dict, List, Tuple

import numpy as np

from . import geomst as G
from . import workloads as W

DEFAULTS = {"bccp_chunk": 2048, "small_level_switch": 2048, "small_level_max": 4096, "beta_growth": 0.0,
            "refresh_divisor": 1048576}

# candidate values per knob (small-level thresholds move together)
CANDIDATES = {
    "bccp_chunk": [512, 1024, 2048, 4096],
    "small_levels": [(1024, 2048), (2048, 4096), (4096, 8192), (8192, 16384)],
    "beta_growth_emst": [1.5, 2.0, 3.0, 4.0],
    "beta_growth_hdbscan": [1.25, 1.4142135623730951, 2.0],
    "refresh_divisor": [1024, 16384, 1048576],
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _apply(settings: Dict[str, float]):
    for k, v in settings.items():
        G.set_option(k, v)


def _reset():
    _apply(DEFAULTS)


class Workload:
    """A solve to tune: run(check) solves once on device-resident data and,
    when check is set, returns a digest of the output bytes."""

    def __init__(self, name: str, kind: str, d: int, npts: int, run: Callable[[], str]):
        self.name, self.kind, self.d, self.npts, self.run = name, kind, d, npts, run

    @property
    def nlog2(self) -> int:
        return int(math.floor(math.log2(max(self.npts, 1))))


def _digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a.cpu().numpy() if hasattr(a, "cpu") else a).tobytes())
    return h.hexdigest()


def make_workload(name: str) -> Workload:
    import torch
    if name == "batch_4096":
        inst = W.batch_4096()
        arena, items, stride = G.pack(inst, 0)
        x = torch.from_numpy(arena).to("cuda")

        def run(check=True):
            out = G.batch_dev(x, items, stride, want_sq=True)
            return _digest(out["edges"], out["weights_sq"]) if check else None
        return Workload(name, "emst", stride, arena.shape[0], run)
    if name in ("emst_1m", "emst_small"):
        p = W.emst_1m() if name == "emst_1m" else W.emst_small()
        x = torch.from_numpy(p).to("cuda")

        def run(check=True):
            e, w, w2 = G.emst(x, want_sq=True)
            return _digest(e, w2) if check else None
        return Workload(name, "emst", p.shape[1], len(p), run)
    if name == "hdbscan_2m":
        p = W.hdbscan_2m()
        x = torch.from_numpy(p).to("cuda")

        def run(check=True):
            cd, e, w, cd2, w2 = G.hdbscan(x, 10, want_sq=True)
            return _digest(cd2, e, w2) if check else None
        return Workload(name, "hdbscan", p.shape[1], len(p), run)
    raise ValueError(f"unknown workload {name}")


def _time(wl: Workload, reps: int) -> Tuple[float, str]:
    import torch
    dig = wl.run(True)  # warm (workspace growth, first touch), and the output digest
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        wl.run(False)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1000.0)
    return float(np.median(ts)), dig


def tune(wl: Workload, reps: int = 3) -> Dict:
    """Coordinate descent from the defaults; returns the cache entry."""
    _reset()
    base_ms, ref = _time(wl, reps)
    log(f"[tune] {wl.name}: default {base_ms:.2f} ms")
    best: Dict[str, float] = {}
    best_ms = base_ms
    gname = "beta_growth_emst" if wl.kind == "emst" else "beta_growth_hdbscan"
    axes: List[Tuple[str, List[Dict[str, float]]]] = [
        ("bccp_chunk", [{"bccp_chunk": v} for v in CANDIDATES["bccp_chunk"]]),
        ("small_levels", [{"small_level_max": b, "small_level_switch": a} for a, b in CANDIDATES["small_levels"]]),
        ("beta_growth", [{"beta_growth": v} for v in CANDIDATES[gname]]),
        ("refresh_divisor", [{"refresh_divisor": v} for v in CANDIDATES["refresh_divisor"]]),
    ]
    for axis, cands in axes:
        for c in cands:
            trial = dict(best)
            trial.update(c)
            _reset()
            _apply(trial)
            ms, dig = _time(wl, reps)
            if dig != ref:
                _reset()
                raise RuntimeError(f"{wl.name}: settings {trial} changed the result")
            log(f"[tune] {wl.name}: {trial} {ms:.2f} ms")
            if ms < best_ms:
                best_ms, best = ms, trial
    _reset()
    entry = {"kind": wl.kind, "d": wl.d, "nlog2": wl.nlog2, "workload": wl.name, "default_ms": round(base_ms, 3),
             "tuned_ms": round(best_ms, 3)}
    full = dict(DEFAULTS)
    full.update(best)
    if full["beta_growth"] == 0.0:
        full.pop("beta_growth")  # the kind's own default
    entry.update(full)
    return entry


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", nargs="+", default=["batch_4096"])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    import torch
    # torch brings up the device first (as the tests and the benchmark do)
    if not torch.cuda.is_available():
        raise SystemExit("the tuner times solves: it needs a GPU")
    G.load()
    G.load_tuning(None)
    lines = []
    for name in a.workloads:
        wl = make_workload(name)
        lines.append(tune(wl, a.reps))
        del wl
    with open(a.out, "w") as fh:
        fh.write("# geomst tuning cache: written by paper_2104_01126_amd/tune.py (coordinate descent; every\n"
                 "# candidate's output was byte-identical to the defaults')\n")
        for e in lines:
            fh.write(json.dumps(e) + "\n")
    print(json.dumps(lines))


if __name__ == "__main__":
    main()
