#!/usr/bin/env python3
"""Throughput benchmark of the GPU EMST / HDBSCAN* path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload emst_1m]
                [--no-cpu-baseline] [--no-extras] [--serve-seconds S]

A step is one complete solve (tree build, [core distances,] every
filtered-Kruskal round, output sort and write) of one synthetic workload whose
points are already resident in HBM.  Prints ONE JSON line on stdout; progress
goes to stderr.

The default run times the 1M-point EMST as the headline (`value`, `roofline`,
`cpu_baseline`) and adds, in the same line, the rest of the metric:
`extras.c1_plain_beta` (the same workload with the threshold doubling every
round), `extras.c1_host_api` (host arrays in and out, PCIe copies included),
`extras.c0` (2,000 points), `extras.c2` (2M-point HDBSCAN*, with BCCP
distance evaluations per second as a fraction of FP64 peak and the ordered
dendrogram), `extras.c3` (4,096 instances batched vs one call each) and
`extras.c4` (a prefix of the serving stream, served vs one request per
launch, p50/p99 latency); each of c0-c2 is the median of its timed solves.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "points/s end-to-end + BCCP evals/s (% FP64 peak); batched/served vs plain, p50/p99"
FP64_PEAK_TFLOPS = 78.6   # MI355X vector FP64, an FMA counted as two flops
HBM_PEAK_GBS = 8000.0     # MI355X HBM3E

WORKLOADS = {
    "emst_1m": dict(desc="EMST, 1,000,000 points i.i.d. uniform in [0,1000)^3, seed 1", n=1_000_000, d=3,
                    min_pts=0),
    "hdbscan_2m": dict(desc="HDBSCAN*, minPts=10, 2,000,000 points in 5-D: 95% from 64 Gaussians "
                            "(centres uniform in [0,1e4)^5, sigma log-uniform [0.5,20]) + 5% uniform noise, seed 2",
                       n=2_000_000, d=5, min_pts=10),
    "emst_small": dict(desc="EMST, 2,000 points i.i.d. uniform in [0,1)^2, seed 0", n=2000, d=2, min_pts=0),
    "batch_4096": dict(desc="Batched: 4,096 independent EMST instances, n log-uniform in [100,50000], d in {2,3}, "
                            "half uniform in the unit cube, half 8-Gaussian mixtures (sigma in [0.01,0.1]), seed 3",
                       n=None, d=3, min_pts=0),
    "optics_500k": dict(desc="Approximate OPTICS (Gan-Tao base graph, rho=0.125, s=8), minPts=10, 500,000 points in "
                             "3-D: 95% from 64 Gaussians (centres uniform in [0,1e4)^3, sigma log-uniform [0.5,20]) "
                             "+ 5% uniform noise, seed 5", n=500_000, d=3, min_pts=10),
    "serve_poisson": dict(desc="Serving: Poisson stream at 2,000 requests/s, 70% EMST / 30% HDBSCAN* (minPts in "
                               "{5,10,16}), n log-uniform in [1e3,1e6], d in {2..7}, half uniform, half 8-Gaussian "
                               "mixtures, seed 4; 200 GB admission budget",
                          n=None, d=None, min_pts=None),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gen(name):
    from paper_2104_01126_amd import workloads as W
    return {"emst_1m": W.emst_1m, "hdbscan_2m": W.hdbscan_2m, "emst_small": W.emst_small}[name]()


def solve(G, x, min_pts):
    if min_pts:
        return G.hdbscan(x, min_pts)
    return G.emst(x)


def node_record_bytes(d, hdb=False):
    """Bytes of one tree node the expansion reads: the box (2d binary64 bounds
    for d <= 3, 2d binary32 for d >= 4), first/count/split/component (16 B),
    and for HDBSCAN* the (min, max) core-distance range: 8 B in the record
    where it fits (d = 4, 5, 7), else 16 B from its own array."""
    box = 16 * d if d <= 3 else 8 * d
    cd = 0 if not hdb else (8 if d in (4, 5, 7) else 16)
    return box + 16 + cd


def unit_model(fam, st, d, hdb=False):
    """Algorithmic work of one kernel family over a solve: (amount, unit,
    bound).  Bytes are the data the method itself must move, flops the
    arithmetic it must do; neither counts re-reads or bookkeeping."""
    if fam == "bccp":
        # small-pair BCCP: (3d-1) flops per distance (d sub, d mul, d-1 add),
        # two more for the BCCP* maxima
        return (st.bccp_evals_done - st.big_evals) * (3 * d - 1 + (2 if hdb else 0)), "TFLOP/s", "alu"
    if fam == "bccp_large":
        return st.big_evals * (3 * d - 1 + (2 if hdb else 0)), "TFLOP/s", "alu"
    if fam == "expand":
        # per examined node pair: its 16-byte record and the two nodes'
        # records (box, range, split and component), plus their core-distance
        # ranges for HDBSCAN*
        return st.pair_visits * (16 + 2 * node_record_bytes(d, hdb)), "GB/s", "hbm"
    if fam == "sort":
        # per element and 8-bit pass: 12 bytes read, 12 bytes written
        return st.sort_elems * 24, "GB/s", "hbm"
    if fam == "kruskal":
        # per committed edge and Boruvka step: rank and two endpoint positions
        # read, two root lookups (4 bytes each) and the rank compare
        return st.committed_edges * 24, "GB/s", "hbm"
    return None, None, None


FAMILY_KERNEL = {"expand": "k_level", "bccp": "k_tiny_bccp", "bccp_large": "k_big_bccp", "sort": "k_radix",
                 "kruskal": "k_bor"}
# the library's "expand" timing brackets k_level and k_level_small launches


def source_sha():
    """Hash of the library sources (a traffic figure measured on other sources is stale)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2104_01126_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(family, workload):
    """HBM bytes per solve moved by the family's kernels, and their dispatches
    per solve, from the committed rocprofv3 PMC summary; None when there is
    none or the sources changed since it was taken."""
    k = FAMILY_KERNEL.get(family)
    path = os.path.join(ROOT, "profiles", f"{k}_{workload}_traffic.txt")
    if not k or not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            a, b = line.strip().split("=", 1)
            kv[a] = b
    if kv.get("source_sha") != source_sha():
        return None
    return int(kv["traffic_bytes_per_solve"]), int(kv["dispatches_per_solve"])


def cpu_baseline(name, pts, min_pts, target_s=25.0):
    import oracle
    oracle.build(force=False)
    n = len(pts)
    m0 = min(n, 30000)
    t = time.perf_counter()
    if min_pts:
        oracle.hdbscan(pts[:m0], min_pts)
    else:
        oracle.emst(pts[:m0])
    t0 = time.perf_counter() - t
    m = min(n, max(m0, int(m0 * math.sqrt(target_s / max(t0, 1e-3)))))
    log(f"cpu baseline: calibration {m0} pts in {t0:.2f}s, sample {m} pts")
    t = time.perf_counter()
    if min_pts:
        oracle.hdbscan(pts[:m], min_pts)
    else:
        oracle.emst(pts[:m])
    dt = time.perf_counter() - t
    what = "HDBSCAN* (brute-force core distances + dense Prim)" if min_pts else "EMST (dense Prim)"
    return {"value": m / dt, "unit": "points/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"first {m} of the {n} workload points, {what}, O(m^2), {dt:.1f} s",
            "seconds": dt}


def bench_batch(a, G, torch, np):
    """Batched path (one forest solve of all instances) against the plain
    path (one solve call per instance), both on device-resident points."""
    from paper_2104_01126_amd import workloads as W
    wl = WORKLOADS[a.workload]
    log("workload batch_4096: generating")
    inst = W.batch_4096()
    arena, items, stride = G.pack(inst, 0)
    N = arena.shape[0]
    x = torch.from_numpy(arena).to("cuda:0")
    singles = [torch.from_numpy(np.ascontiguousarray(p)).to("cuda:0") for p in inst]
    torch.cuda.synchronize()
    for i in range(a.warmup):
        G.batch_dev(x, items, stride)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{a.warmup}: {G.stats().ms_total:.1f} ms")
    # device-time breakdown from one extra untimed batch solve; the timed
    # steps run without HIP events
    G.set_option("kernel_timing", 1)
    G.batch_dev(x, items, stride)
    torch.cuda.synchronize()
    kms = np.array(G.stats().kernel_ms)
    G.set_option("kernel_timing", 0)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        G.batch_dev(x, items, stride)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = G.stats()
    value = N * a.steps / dt
    log(f"batched: {dt * 1000 / a.steps:.1f} ms/step, {value / 1e6:.2f} Mpoints/s")
    # plain path: every instance alone, one call each (one pass, after one warm call)
    G.emst(singles[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in singles:
        G.emst(s)
    torch.cuda.synchronize()
    dplain = time.perf_counter() - t0
    plain = N / dplain
    log(f"plain: {dplain:.2f} s for {len(singles)} calls, {plain / 1e6:.2f} Mpoints/s")
    fams = G.KERNEL_FAMILIES
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "points/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(dt * 1000 / a.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["desc"], "instances": len(inst), "total_points": N, "stride": stride,
                   "parallelism": "single GPU"},
        "instances_per_s": round(len(inst) * a.steps / dt, 1),
        "plain_points_per_s": round(plain, 1), "plain_seconds": round(dplain, 3),
        "batched_vs_plain": round(value / plain, 2),
        "kernel_ms_breakdown": {fams[i]: round(float(kms[i]), 3) for i in range(len(fams))},
        "rounds": st.rounds,
    }
    print(json.dumps(out), flush=True)


def replay(G, trace, pts, server_kw, label, dump=None):
    """Open-loop replay of a request trace against a server: a submitter
    thread submits each request at its arrival time; latency = completion -
    scheduled arrival (submission lag included)."""
    import threading
    import numpy as np
    S = G.Server(**server_kw)
    # warm the workspaces on the first requests (not timed)
    for t in [S.submit(pts[i], trace[i].min_pts) for i in range(min(8, len(trace)))]:
        S.wait(t)
    tickets = [None] * len(trace)
    lag = np.zeros(len(trace))
    t0 = time.perf_counter()

    def submitter():
        for i, r in enumerate(trace):
            now = time.perf_counter() - t0
            if r.arrival_s > now:
                time.sleep(r.arrival_s - now)
            lag[i] = max(0.0, time.perf_counter() - t0 - r.arrival_s)
            tickets[i] = S.submit(pts[i], r.min_pts)

    th = threading.Thread(target=submitter)
    th.start()
    lat = np.zeros(len(trace))
    qdepth = 0
    done_at = 0.0
    failed = []
    for i in range(len(trace)):
        while tickets[i] is None:
            time.sleep(0.0005)
        try:
            e, w, cd, info = S.wait(tickets[i])
        except G.GeomstError as err:  # recorded, not fatal: the line must still be printed
            failed.append({"i": trace[i].index, "n": trace[i].n, "d": trace[i].d, "code": err.code})
            lat[i] = np.nan
            continue
        lat[i] = lag[i] * 1000.0 + info["latency_ms"]
        if dump is not None:
            r = trace[i]
            dump.append({"i": r.index, "n": r.n, "d": r.d, "min_pts": r.min_pts, "mixture": r.mixture,
                         "service_ms": round(info["service_ms"], 3), "queue_ms": round(info["queue_ms"], 3),
                         "batch_requests": info["batch_requests"], "batch_points": info["batch_points"]})
        done_at = max(done_at, trace[i].arrival_s + lat[i] / 1000.0)
        if (i + 1) % 100 == 0:
            st = S.stats()
            qdepth = max(qdepth, st["queued"])
            log(f"{label}: {i + 1}/{len(trace)} done, queued {st['queued']}, batches {st['batches']}")
    th.join()
    st = S.stats()
    S.close()
    span = done_at - trace[0].arrival_s
    ok = ~np.isnan(lat)
    npts = sum(r.n for r, good in zip(trace, ok) if good)
    latok = lat[ok] if ok.any() else np.zeros(1)
    return {"solves_per_s": round(int(ok.sum()) / span, 2), "points_per_s": round(npts / span, 1),
            "p50_ms": round(float(np.percentile(latok, 50)), 2), "p99_ms": round(float(np.percentile(latok, 99)), 2),
            "mean_ms": round(float(latok.mean()), 2), "makespan_s": round(span, 3),
            "failed_requests": len(failed), "failures": failed[:8],
            "batches_incl_warmup": st["batches"], "max_batch_requests": st["max_batch_requests"],
            "peak_reserved_gb": round(st["peak_reserved_bytes"] / 1e9, 2), "max_queue_seen": qdepth,
            "enomem_batches": st["enomem_batches"], "workspace_gb": round(st["workspace_bytes"] / 1e9, 2)}


def bench_serve(a, G):
    """Serving: a prefix of the Poisson request stream replayed open-loop
    against the continuous-batching server and against the plain path (one
    instance per launch, FIFO, one worker), measured the same way."""
    from paper_2104_01126_amd import workloads as W
    wl = WORKLOADS[a.workload]
    trace = W.serving_trace(duration_s=a.serve_seconds)
    log(f"serving: {len(trace)} requests in the first {a.serve_seconds} s of the stream, "
        f"{sum(r.n for r in trace) / 1e6:.1f} M points; generating")
    pts = [W.serving_points(r) for r in trace]
    served = plain = None
    dump = [] if a.serve_dump else None
    if a.serve_mode in ("both", "served"):
        served = replay(G, trace, pts, dict(hbm_budget_bytes=200_000_000_000, workers=a.serve_workers,
                                            small_max_points=a.serve_small_max), "served",
                        dump if a.serve_mode == "served" else None)
        log("served:", served)
    if a.serve_mode in ("both", "plain"):
        plain = replay(G, trace, pts, dict(hbm_budget_bytes=200_000_000_000, workers=1, max_batch_requests=1),
                       "plain", dump if a.serve_mode == "plain" else None)
        log("plain:", plain)
    if dump is not None:
        with open(a.serve_dump, "w") as fh:
            for rec in dump:
                fh.write(json.dumps(rec) + "\n")
    if served is None or plain is None:
        one = served or plain
        print(json.dumps({"metric": METRIC, "value": one["points_per_s"], "unit": "points/s", "n_gpus": 1,
                          "mode": a.serve_mode, "requests": len(trace), "result": one}), flush=True)
        return
    out = {
        "metric": METRIC, "value": served["points_per_s"], "unit": "points/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": round(served["makespan_s"] * 1000, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["desc"], "requests": len(trace), "trace_seconds": a.serve_seconds,
                   "offered_req_per_s": 2000, "workers": a.serve_workers, "parallelism": "single GPU"},
        "served": served, "plain": plain,
        "served_vs_plain_solves": round(served["solves_per_s"] / plain["solves_per_s"], 2),
    }
    print(json.dumps(out), flush=True)


def timed_solves(G, torch, x, mp, steps, warmup, label):
    """Per-solve wall times (ms) of `steps` solves after `warmup` ones."""
    for _ in range(warmup):
        solve(G, x, mp)
    torch.cuda.synchronize()
    ts = []
    for i in range(steps):
        t = time.perf_counter()
        solve(G, x, mp)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1000.0)
    log(f"{label}: median {sorted(ts)[len(ts) // 2]:.2f} ms over {steps} solves")
    return ts


def median(v):
    v = sorted(v)
    return v[len(v) // 2] if len(v) % 2 else 0.5 * (v[len(v) // 2 - 1] + v[len(v) // 2])


def bccp_fraction(st, d, hdb):
    """BCCP distance evaluations of one solve (pruned blocks excluded) over
    the device time of the BCCP kernels, as FP64 flops against the vector
    peak: all BCCP kernels together, the small-pair kernel (up to 16 point
    pairs, one pair per thread) and the medium/large-pair kernels apart."""
    ms_s, ms_l = st.kernel_ms[5], st.kernel_ms[10]
    flops = 3 * d - 1 + (2 if hdb else 0)
    if ms_s + ms_l <= 0:
        return None

    def part(evals, ms):
        if ms <= 0:
            return {"evals": evals, "device_ms": 0.0}
        eps = evals / (ms / 1000.0)
        return {"evals": evals, "device_ms": round(ms, 4), "evals_per_s": round(eps, 1),
                "tflops": round(eps * flops / 1e12, 4), "frac_fp64_peak": round(eps * flops / 1e12 / FP64_PEAK_TFLOPS, 5)}
    allp = part(st.bccp_evals_done, ms_s + ms_l)
    return {"flops_per_eval": flops, "all": allp,
            "small_pairs": part(st.bccp_evals_done - st.big_evals, ms_s),
            "large_pairs": part(st.big_evals, ms_l),
            "bccp_evals_per_s": allp.get("evals_per_s"), "bccp_frac_fp64_peak": allp.get("frac_fp64_peak")}


def extra_plain(G, torch, np, name, steps, warmup, dendrogram=False, variants=False):
    from paper_2104_01126_amd import workloads as W
    wl = WORKLOADS[name]
    log(f"{name}: generating")
    pts = {"emst_small": W.emst_small, "emst_1m": W.emst_1m, "hdbscan_2m": W.hdbscan_2m}[name]()
    n, d = pts.shape
    mp = wl["min_pts"]
    x = torch.from_numpy(pts).to("cuda:0")
    ts = timed_solves(G, torch, x, mp, steps, warmup, name)
    st = G.stats()
    G.set_option("kernel_timing", 1)
    solve(G, x, mp)
    torch.cuda.synchronize()
    stk = G.stats()
    G.set_option("kernel_timing", 0)
    fams = G.KERNEL_FAMILIES
    rec = {"workload": wl["desc"], "n": n, "d": d, "min_pts": mp or None,
           "median_ms": round(median(ts), 3), "points_per_s": round(n / (median(ts) / 1000.0), 1),
           "solves": steps, "min_ms": round(min(ts), 3), "max_ms": round(max(ts), 3),
           "kernel_ms_breakdown": {fams[i]: round(float(stk.kernel_ms[i]), 4) for i in range(len(fams))},
           "counts": {k: getattr(st, k) for k in ("rounds", "pair_visits", "bccp_pairs", "bccp_evals",
                                                  "bccp_evals_done", "big_evals", "committed_edges")}}
    rec["bccp"] = bccp_fraction(stk, d, bool(mp))
    if mp and variants:
        # HDBSCAN*-GanTao (geometric separation only, Sec. 3.2.1) beside the
        # default separation (Sec. 3.2.2), and the paper's minPts range
        G.set_option("separation_mode", 1)
        try:
            tg = timed_solves(G, torch, x, mp, 3, 1, f"{name} geometric-only separation")
            sg = G.stats()
        finally:
            G.set_option("separation_mode", 0)
        rec["gantao"] = {"median_ms": round(median(tg), 3), "points_per_s": round(n / (median(tg) / 1000.0), 1),
                         "bccp_pairs": sg.bccp_pairs, "pair_visits": sg.pair_visits,
                         "pairs_vs_default": round(sg.bccp_pairs / max(1, st.bccp_pairs), 3)}
        # WSPD sizes (Naive: every well-separated pair materialised) on the
        # first 200,000 points of the recipe, with and without mutual
        # unreachability
        from paper_2104_01126_amd import workloads as W
        xs = torch.from_numpy(W.hdbscan_2m(200_000)).to("cuda:0")
        wspd = {}
        for sep in (0, 1):
            G.set_option("schedule", 1)
            G.set_option("separation_mode", sep)
            try:
                solve(G, xs, mp)
                torch.cuda.synchronize()
                wspd["geometric_only" if sep else "geometric_or_mutually_unreachable"] = G.stats().bccp_pairs
            finally:
                G.set_option("schedule", 0)
                G.set_option("separation_mode", 0)
        wspd["ratio"] = round(wspd["geometric_only"] / max(1, wspd["geometric_or_mutually_unreachable"]), 4)
        rec["wspd_pairs_first_200k"] = wspd
        del xs
        sweep = {}
        for k in (10, 20, 30, 40, 50):
            tk = timed_solves(G, torch, x, k, 3, 1, f"{name} minPts={k}")
            sk = G.stats()
            sweep[str(k)] = {"median_ms": round(median(tk), 3), "points_per_s": round(n / (median(tk) / 1000.0), 1),
                             "bccp_pairs": sk.bccp_pairs}
        rec["minpts_sweep"] = sweep
    if dendrogram:
        if mp:
            cd, e, w = G.hdbscan(x, mp)
        else:
            e, w = G.emst(x)
        for _ in range(2):
            G.dendrogram(e, w, 0)
        torch.cuda.synchronize()
        dts = []
        for _ in range(5):
            t = time.perf_counter()
            G.dendrogram(e, w, 0)
            torch.cuda.synchronize()
            dts.append((time.perf_counter() - t) * 1000.0)
        rec["dendrogram_median_ms"] = round(median(dts), 3)
        rec["with_dendrogram_points_per_s"] = round(n / ((median(ts) + median(dts)) / 1000.0), 1)
        log(f"{name}: ordered dendrogram + reachability plot median {median(dts):.2f} ms")
    del x
    torch.cuda.empty_cache()
    return rec


def extra_optics(G, torch, np, steps):
    """Approximate OPTICS (paper Appendix) on its own workload: the whole
    decomposition at s = 8, each pair's case candidate, one Kruskal pass."""
    from paper_2104_01126_amd import workloads as W
    wl = WORKLOADS["optics_500k"]
    log("optics_500k: generating")
    pts = W.optics_500k()
    n, d = pts.shape
    mp, rho = wl["min_pts"], 0.125
    x = torch.from_numpy(pts).to("cuda:0")
    G.optics_approx(x, mp, rho)
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        t = time.perf_counter()
        G.optics_approx(x, mp, rho)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1000.0)
    st = G.stats()
    G.set_option("kernel_timing", 1)
    G.optics_approx(x, mp, rho)
    torch.cuda.synchronize()
    stk = G.stats()
    G.set_option("kernel_timing", 0)
    fams = G.KERNEL_FAMILIES
    kms = {fams[i]: round(float(stk.kernel_ms[i]), 4) for i in range(len(fams))}
    log(f"optics_500k: median {median(ts):.2f} ms over {steps} solves")
    rec = {"workload": wl["desc"], "n": n, "d": d, "min_pts": mp, "rho": rho,
           "median_ms": round(median(ts), 3), "points_per_s": round(n / (median(ts) / 1000.0), 1),
           "solves": steps, "kernel_ms_breakdown": kms,
           "counts": {"wspd_pairs": st.bccp_pairs, "point_pairs_evaluated": st.bccp_evals,
                      "pair_visits": st.pair_visits, "levels": st.rounds, "candidates": st.committed_edges}}
    ems = kms.get("expand", 0.0)
    if ems > 0:
        # the decomposition kernel (k_approx_level): per examined pair its
        # record and the two node records
        by = st.pair_visits * (16 + 2 * node_record_bytes(d))
        rec["roofline_decomposition"] = {"kernel": "k_approx_level", "bound": "hbm",
                                         "achieved": round(by / (ems / 1000.0) / 1e9, 3), "peak": HBM_PEAK_GBS,
                                         "unit": "GB/s", "frac": round(by / (ems / 1000.0) / 1e9 / HBM_PEAK_GBS, 5),
                                         "pairs_per_s": round(st.pair_visits / (ems / 1000.0), 1)}
    del x
    torch.cuda.empty_cache()
    return rec


def extra_c1_variants(G, torch, np, x, n, steps):
    """c1 under plain beta doubling, and through the host-array API."""
    out = {}
    G.set_option("beta_schedule", 1)
    try:
        ts = timed_solves(G, torch, x, 0, steps, 2, "c1 plain beta doubling")
        st = G.stats()
    finally:
        G.set_option("beta_schedule", 0)
    out["c1_plain_beta"] = {"schedule": "beta doubles every round from the smallest pair bound",
                            "median_ms": round(median(ts), 3), "points_per_s": round(n / (median(ts) / 1000.0), 1),
                            "rounds": st.rounds, "pair_visits": st.pair_visits}
    # the paper's own schedules (Naive; GFK, Alg. 2; MemoGFK, Alg. 3) as
    # ablations beside the default weight-threshold schedule
    sch = {}
    for code, nm in ((3, "memogfk"), (2, "gfk"), (1, "naive")):
        G.set_option("schedule", code)
        try:
            tsch = timed_solves(G, torch, x, 0, 3, 1, f"c1 schedule {nm}")
            ss = G.stats()
        finally:
            G.set_option("schedule", 0)
        sch[nm] = {"median_ms": round(median(tsch), 3), "rounds": ss.rounds, "bccp_pairs": ss.bccp_pairs,
                   "bccp_evals": ss.bccp_evals_done, "pair_visits": ss.pair_visits}
    out["c1_paper_schedules"] = sch
    ts = timed_solves(G, torch, x, 0, steps, 1, "c1 default schedule, no events")
    out["c1_no_events"] = {"median_ms": round(median(ts), 3), "points_per_s": round(n / (median(ts) / 1000.0), 1)}
    host = x.cpu().numpy()
    G.emst(host)
    hs = []
    for _ in range(steps):
        t = time.perf_counter()
        G.emst(host)
        hs.append((time.perf_counter() - t) * 1000.0)
    out["c1_host_api"] = {"median_ms": round(median(hs), 3), "points_per_s": round(n / (median(hs) / 1000.0), 1),
                          "note": "host arrays in and out (H2D points, D2H edges and weights included)"}
    log(f"c1 host api: median {median(hs):.2f} ms")
    return out


def extra_batch(G, torch, np, steps):
    from paper_2104_01126_amd import workloads as W
    log("c3 batch_4096: generating")
    inst = W.batch_4096()
    arena, items, stride = G.pack(inst, 0)
    N = arena.shape[0]
    x = torch.from_numpy(arena).to("cuda:0")
    singles = [torch.from_numpy(np.ascontiguousarray(p)).to("cuda:0") for p in inst]
    G.batch_dev(x, items, stride)
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        t = time.perf_counter()
        G.batch_dev(x, items, stride)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1000.0)
    log(f"c3 batched: median {median(ts):.1f} ms")
    # device time of one batched solve (HIP events around every kernel
    # family) against its wall time: the share a captured graph could at
    # most remove from host launches and round trips
    G.set_option("kernel_timing", 1)
    t = time.perf_counter()
    G.batch_dev(x, items, stride)
    torch.cuda.synchronize()
    wall_ev = (time.perf_counter() - t) * 1000.0
    stk = G.stats()
    G.set_option("kernel_timing", 0)
    dev_ms = float(sum(stk.kernel_ms))
    launches = int(sum(stk.kernel_launches))
    # the project's tuner's cache, when present: tuned against default
    tuned = None
    cache = os.path.join(ROOT, "paper_2104_01126_amd", "tuning_cache.jsonl")
    if os.path.exists(cache):
        import hashlib
        ref = G.batch_dev(x, items, stride, want_sq=True)
        hd = hashlib.sha256(ref["edges"].cpu().numpy().tobytes() + ref["weights_sq"].cpu().numpy().tobytes()).hexdigest()
        G.load_tuning(cache)
        try:
            out = G.batch_dev(x, items, stride, want_sq=True)
            ht = hashlib.sha256(out["edges"].cpu().numpy().tobytes() + out["weights_sq"].cpu().numpy().tobytes()).hexdigest()
            applied = G.stats().tuning_applied
            tt = []
            for _ in range(steps):
                t = time.perf_counter()
                G.batch_dev(x, items, stride)
                torch.cuda.synchronize()
                tt.append((time.perf_counter() - t) * 1000.0)
        finally:
            G.load_tuning(None)
        tuned = {"cache": "paper_2104_01126_amd/tuning_cache.jsonl", "applied": bool(applied),
                 "median_ms": round(median(tt), 2), "tuned_vs_default": round(median(ts) / median(tt), 3),
                 "same_bytes": hd == ht}
        log(f"c3 batched, tuned: median {median(tt):.1f} ms (same bytes: {hd == ht})")
    G.emst(singles[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, s_ in enumerate(singles):
        G.emst(s_)
        if (i + 1) % 1024 == 0:
            log(f"c3 plain: {i + 1}/{len(singles)} calls")
    torch.cuda.synchronize()
    dplain = time.perf_counter() - t0
    rec = {"workload": WORKLOADS["batch_4096"]["desc"], "instances": len(inst), "total_points": N,
           "batched_median_ms": round(median(ts), 2), "batched_points_per_s": round(N / (median(ts) / 1000.0), 1),
           "batched_instances_per_s": round(len(inst) / (median(ts) / 1000.0), 1),
           "plain_seconds": round(dplain, 3), "plain_points_per_s": round(N / dplain, 1),
           "batched_vs_plain": round(dplain / (median(ts) / 1000.0), 2),
           "device_ms_one_solve": round(dev_ms, 2), "wall_ms_with_events": round(wall_ev, 2),
           "launch_groups_timed": launches, "tuned": tuned}
    del x, singles
    torch.cuda.empty_cache()
    return rec


def extra_serve(G, seconds, workers):
    from paper_2104_01126_amd import workloads as W
    trace = W.serving_trace(duration_s=seconds)
    log(f"c4 serving: {len(trace)} requests in the first {seconds} s of the stream, "
        f"{sum(r.n for r in trace) / 1e6:.1f} M points; generating")
    pts = [W.serving_points(r) for r in trace]
    served = replay(G, trace, pts, dict(hbm_budget_bytes=200_000_000_000, workers=workers), "served")
    log("served:", served)
    plain = replay(G, trace, pts, dict(hbm_budget_bytes=200_000_000_000, workers=1, max_batch_requests=1),
                   "plain")
    log("plain:", plain)
    return {"workload": WORKLOADS["serve_poisson"]["desc"], "trace_seconds": seconds, "requests": len(trace),
            "points": sum(r.n for r in trace), "workers": workers, "served": served, "plain": plain,
            "served_vs_plain_solves": round(served["solves_per_s"] / plain["solves_per_s"], 2),
            "served_vs_plain_points": round(served["points_per_s"] / plain["points_per_s"], 2)}


def oracle_single_thread():
    """The checker on one thread (its own process, OMP_NUM_THREADS=1): the
    2,000-point workload and the first 30,000 points of the 1M workload."""
    import subprocess
    code = ("import time, sys; sys.path.insert(0, %r)\n"
            "import oracle\nfrom paper_2104_01126_amd import workloads as W\n"
            "oracle.build(force=False)\n"
            "p = W.emst_small(); t = time.perf_counter(); oracle.emst(p); a = time.perf_counter() - t\n"
            "q = W.emst_1m()[:30000]; t = time.perf_counter(); oracle.emst(q); b = time.perf_counter() - t\n"
            "print(a, b, oracle.num_threads())\n") % ROOT
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=300)
    a, b, th = r.stdout.split()
    return {"c0_seconds": round(float(a), 4), "c0_points_per_s": round(2000 / float(a), 1),
            "c1_first_30000_seconds": round(float(b), 3), "c1_first_30000_points_per_s": round(30000 / float(b), 1),
            "threads": int(th)}


def oracle_full_size_record():
    """Full-size checker runs behind the parity digests (tests/golden/): run
    on the build host, not on this machine; context for the GPU rates."""
    out = {}
    for name in ("emst_small", "emst_1m", "hdbscan_2m", "batch_4096", "optics_500k"):
        path = os.path.join(ROOT, "tests", "golden", f"digest_{name}.json")
        if os.path.exists(path):
            g = json.load(open(path))
            out[name] = {"oracle_seconds": g["oracle_seconds"], "threads": g["oracle_threads"],
                         "host": "build host (not the GPU box)"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="emst_1m", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=1.0,
                    help="length of the replayed prefix of the 60 s request stream (serving)")
    ap.add_argument("--with-dendrogram", action="store_true",
                    help="single workloads: also time the ordered dendrogram of the solved tree (3 calls)")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline workload only (no c0/c2/c3/c4 sub-records)")
    ap.add_argument("--serve-workers", type=int, default=0, help="server workers (0: the library default)")
    ap.add_argument("--serve-small-max", type=int, default=0,
                    help="server small-lane size limit (0: the library default; 1: no small lane)")
    ap.add_argument("--serve-dump", default=None, help="serve_poisson: write per-request timings (JSON lines)")
    ap.add_argument("--serve-mode", default="both", choices=["both", "served", "plain"],
                    help="serve_poisson: replay against the server, the plain path, or both")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy three times (reference for PMC byte counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2104_01126_amd import geomst as G

    if a.workload == "batch_4096":
        G.load()
        return bench_batch(a, G, torch, np)
    if a.workload == "serve_poisson":
        G.load()
        return bench_serve(a, G)
    if a.workload == "optics_500k":
        G.load()
        for _ in range(a.warmup):
            G.optics_approx(torch.zeros((2, 3), dtype=torch.float64, device="cuda:0"), 1, 0.125)
        rec = extra_optics(G, torch, np, a.steps)
        print(json.dumps({"workload": "optics_500k", "n_gpus": 1, "steps": a.steps, **rec}), flush=True)
        return
    wl = WORKLOADS[a.workload]
    log(f"workload {a.workload}: generating")
    pts = gen(a.workload)
    n, d = pts.shape
    mp = wl["min_pts"]
    G.load()
    x = torch.from_numpy(pts).to("cuda:0")
    torch.cuda.synchronize()
    if a.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 x 1 GiB device-to-device copies done")
    for i in range(a.warmup):
        solve(G, x, mp)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{a.warmup}: {G.stats().ms_total:.2f} ms")
    fams = G.KERNEL_FAMILIES
    # one untimed solve with every kernel family timed: the device-time
    # breakdown, and the dominant family, which alone carries HIP events
    # during the timed steps (fewer events, less overhead in `value`)
    G.set_option("kernel_timing", 1)
    solve(G, x, mp)
    torch.cuda.synchronize()
    st0 = G.stats()
    br = np.array(st0.kernel_ms)
    cand = [i for i in range(len(fams)) if br[i] > 0 and unit_model(fams[i], st0, d, mp)[0] is not None]
    dom = max(cand, key=lambda i: br[i]) if cand else int(np.argmax(br))
    G.set_option("kernel_timing_families", 1 << dom)
    kms = np.zeros(16)
    kl = np.zeros(16)
    agg = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        solve(G, x, mp)
        st = G.stats()
        kms += np.array(st.kernel_ms)
        kl += np.array(st.kernel_launches)
        if agg is None:
            agg = {k: 0 for k in ("pair_visits", "bccp_evals", "big_evals", "sort_elems", "committed_edges",
                                  "bccp_pairs", "rounds", "bccp_evals_done")}
        for k in agg:
            agg[k] += getattr(st, k)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    G.set_option("kernel_timing", 0)
    G.set_option("kernel_timing_families", 0)
    ms_step = dt * 1000.0 / a.steps
    value = n * a.steps / dt
    log(f"timed {a.steps} steps: {ms_step:.2f} ms/step, {value / 1e6:.2f} Mpoints/s")

    class S:
        pass
    s = S()
    for k, v in agg.items():
        setattr(s, k, v)
    per_fam = {fams[i]: round(float(br[i]), 4) for i in range(len(fams))}
    log("device ms by kernel family (untimed breakdown solve):", per_fam)
    evals_per_s = agg["bccp_evals"] / dt
    big_ms = br[fams.index("bccp_large")]
    flops_per_eval = 3 * d - 1 + (2 if mp else 0)
    bccp_tflops = (st0.big_evals * flops_per_eval / (big_ms / 1000.0) / 1e12) if big_ms > 0 else 0.0
    # dominant kernel family and its roofline, from the timed steps
    roof = None
    for i in [dom]:
        amount, unit, bound = unit_model(fams[i], s, d, mp)
        if amount is None or kms[i] <= 0:
            continue
        secs = kms[i] / 1000.0
        if unit == "TFLOP/s":
            ach, peak = amount / secs / 1e12, FP64_PEAK_TFLOPS
        else:
            ach, peak = amount / secs / 1e9, HBM_PEAK_GBS
        mt = measured_traffic(fams[i], a.workload)
        # launches of the family's kernels per step, counted by the library
        # (one timed scope per k_level / k_level_small launch); achieved =
        # algorithmic bytes per launch / average launch duration
        launches = kl[i] / a.steps
        per = launches if launches > 0 else 1
        roof = {"kernel": fams[i], "kernels": FAMILY_KERNEL.get(fams[i]), "bound": bound,
                "achieved": round(ach, 3), "peak": peak, "unit": unit, "frac": round(ach / peak, 5),
                "traffic": round(mt[0] / per) if mt else None,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-scaled)",
                "algorithmic_per_launch": round(amount / a.steps / per, 1),
                "launches_per_step": round(launches, 2),
                "algorithmic_per_step": round(amount / a.steps, 1),
                "traffic_per_step": mt[0] if mt else None,
                "traffic_dispatches_per_step": mt[1] if mt else None,
                "device_ms_per_step": round(kms[i] / a.steps, 4),
                "avg_launch_us": round(kms[i] / a.steps / per * 1000, 3),
                "share_of_device_time": round(float(br[i] / max(br.sum(), 1e-9)), 4)}
        break
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "points/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["desc"], "n": n, "d": d, "min_pts": mp or None, "parallelism": "single GPU"},
        "bccp_evals_per_s": round(evals_per_s, 1),
        "bccp_large_pair_tflops": round(bccp_tflops, 4),
        "bccp_large_pair_frac_fp64_peak": round(bccp_tflops / FP64_PEAK_TFLOPS, 5),
        "bccp": bccp_fraction(st0, d, bool(mp)),
        "roofline": roof,
        "kernel_ms_breakdown": per_fam,
        "counts_per_step": {k: v // a.steps for k, v in agg.items()},
    }
    if a.with_dendrogram:
        if mp:
            cd_, e_, w_ = G.hdbscan(x, mp)
        else:
            e_, w_ = G.emst(x)
        G.dendrogram(e_, w_, 0)
        torch.cuda.synchronize()
        dts = []
        for _ in range(3):
            t = time.perf_counter()
            G.dendrogram(e_, w_, 0)
            torch.cuda.synchronize()
            dts.append((time.perf_counter() - t) * 1000.0)
        out["dendrogram_median_ms"] = round(median(dts), 3)
        log(f"dendrogram: median {median(dts):.2f} ms")
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.workload, pts, mp)
    if a.workload == "emst_1m" and not a.no_extras:
        ex = {}
        ex.update(extra_c1_variants(G, torch, np, x, n, 5))
        del x
        torch.cuda.empty_cache()
        ex["c0"] = extra_plain(G, torch, np, "emst_small", 11, 3)
        ex["c2"] = extra_plain(G, torch, np, "hdbscan_2m", 5, 2, dendrogram=True, variants=True)
        ex["c3"] = extra_batch(G, torch, np, 5)
        ex["c4"] = extra_serve(G, a.serve_seconds, a.serve_workers)
        ex["optics_approx"] = extra_optics(G, torch, np, 5)
        if not a.no_cpu_baseline:
            ex["oracle_single_thread"] = oracle_single_thread()
        ex["oracle_full_size"] = oracle_full_size_record()
        out["extras"] = ex
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
