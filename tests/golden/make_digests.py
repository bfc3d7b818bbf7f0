"""Write SHA-256 digests of the checker's outputs at the full workload sizes.

Runs the dense-Prim checker (``oracle/``) on the seeded workloads and stores
one digest per output array, so that the GPU tests can compare the library's
bytes with the checker's at sizes the checker cannot reach inside a test.
Only ``oracle/`` and the seeded generators are called here; nothing comes
from the HIP library.

Digested bytes (little-endian, C order):
  edges  int64 [n-1][2]   (min id, max id), sorted by K = (w2, d2, min, max)
  w2     float64 [n-1]    squared weights in the same order
  cd2    float64 [n]      squared core distances (HDBSCAN* and approximate OPTICS)
The approximate-OPTICS record also stores the decomposition's counts
(well-separated pairs, evaluated point pairs, examined pairs).

Usage (each workload writes its own JSON file beside this script):
    python tests/golden/make_digests.py emst_small batch_4096 emst_1m hdbscan_2m optics_500k
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2104_01126_amd import workloads as W  # noqa: E402


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _write(name: str, rec: dict):
    path = os.path.join(HERE, f"digest_{name}.json")
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, path)
    print(f"wrote {path}", flush=True)


def _meta(name: str, t0: float) -> dict:
    return {"workload": name, "oracle_seconds": round(time.time() - t0, 1),
            "oracle_threads": oracle.num_threads(), "host_cpus": os.cpu_count(),
            "script": "tests/golden/make_digests.py"}


def emst_digest(name: str, p: np.ndarray):
    t0 = time.time()
    e, w2, _ = oracle.emst(p)
    rec = _meta(name, t0)
    rec.update({"n": int(len(p)), "d": int(p.shape[1]), "edges": sha(e), "w2": sha(w2),
                "total_w2": float(w2.sum())})
    _write(name, rec)


def hdbscan_digest(name: str, p: np.ndarray, min_pts: int):
    t0 = time.time()
    cd2, _, e, w2, _, _ = oracle.hdbscan(p, min_pts)
    rec = _meta(name, t0)
    rec.update({"n": int(len(p)), "d": int(p.shape[1]), "min_pts": min_pts, "edges": sha(e),
                "w2": sha(w2), "cd2": sha(cd2)})
    _write(name, rec)


def batch_digest(name: str):
    t0 = time.time()
    inst = W.batch_4096()
    per = []
    for i, x in enumerate(inst):
        e, w2, _ = oracle.emst(x)
        per.append({"n": int(len(x)), "d": int(x.shape[1]), "edges": sha(e), "w2": sha(w2)})
        if i % 256 == 255:
            print(f"  {name}: {i + 1} instances, {time.time() - t0:.0f} s", flush=True)
    rec = _meta(name, t0)
    rec.update({"count": len(inst), "instances": per})
    _write(name, rec)


def optics_digest(name: str, p: np.ndarray, min_pts: int, rho: float):
    t0 = time.time()
    cd2, e, w2, _, st = oracle.optics_approx(p, min_pts, rho)
    rec = _meta(name, t0)
    rec.update({"n": int(len(p)), "d": int(p.shape[1]), "min_pts": min_pts, "rho": rho, "edges": sha(e),
                "w2": sha(w2), "cd2": sha(cd2), "wspd_pairs": st[0], "evals": st[1], "visits": st[2]})
    _write(name, rec)


JOBS = {
    "emst_small": lambda: emst_digest("emst_small", W.emst_small()),
    "emst_1m": lambda: emst_digest("emst_1m", W.emst_1m()),
    "hdbscan_2m": lambda: hdbscan_digest("hdbscan_2m", W.hdbscan_2m(), 10),
    "batch_4096": lambda: batch_digest("batch_4096"),
    "optics_500k": lambda: optics_digest("optics_500k", W.optics_500k(), 10, 0.125),
}


def main(argv):
    names = argv or list(JOBS)
    for nm in names:
        if nm not in JOBS:
            raise SystemExit(f"unknown workload {nm}; choose from {sorted(JOBS)}")
    oracle.build(force=False)
    for nm in names:
        print(f"[digest] {nm}", flush=True)
        JOBS[nm]()


if __name__ == "__main__":
    main(sys.argv[1:])
