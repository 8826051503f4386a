#!/usr/bin/env python3
"""SNG-DBSCAN benchmark on one MI355X.

One step is one pass of the whole method over the 5,000,000 x 3 LiDAR-like
scene (s = 0.0005, so 2,500 samples per point and 1.25e10 sample slots;
eps = 0.3, MinPts = 4, seed 5) with X already resident in HBM: draw the
sample (partners sorted by partner block), evaluate it (distances, degrees,
accept bits), then core mask, hook and finalize. This is the largest of the
five workloads that fits one GPU. Prints one JSON line with pair
evaluations per second (whole job), the roofline of the sampled-distance
pass, per-workload entries for the other four workloads (each with its own
roofline and its plain-vs-mixed, plain-vs-sweep and sequential-vs-batched
comparisons at identical labels), and the oracle's CPU rate on a bounded
sample of the same scene.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--schedule tuned|auto|direct]
                    [--configs small,gmm16d,mixed,sweep,batch | --no-configs]
                    [--forms recovery,similarity,simple_graph | --no-forms]
                    [--no-cpu-baseline] [--calibrate-copy]
"""
import argparse
import dataclasses
import hashlib
import json
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "sampled pair-distance evals/sec + end-to-end cluster time (plain vs mixed/batched)"
# The sampled-distance pass of the headline (the partner-block schedule: the
# sample kernel and the LDS evaluate kernel), the sources its kernels are
# built from, and the committed counter summary of its HBM traffic.
PASS = {
    "name": "k_bkt_generate + k_bkt_eval_lds (sample + evaluate: the sampled-distance pass)",
    "traffic": os.path.join(ROOT, "profiles", "pass_lidar3d_traffic.json"),
    "sources": ["paper_2006_06743_amd/csrc/sng_bucket.hip",
                "paper_2006_06743_amd/csrc/sng_bucket_eval.hpp",
                "paper_2006_06743_amd/csrc/sng_bucket_eval_dist.hip",
                "paper_2006_06743_amd/csrc/sng_pass_a.hpp",
                "paper_2006_06743_amd/csrc/sng_device.hpp"],
}


def kernel_source_sha(sources) -> str:
    h = hashlib.sha256()
    for p in sources:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(entry):
    """HBM bytes per pass from the committed rocprofv3 counter runs, or None
    when the kernels changed since."""
    try:
        with open(entry["traffic"]) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_source_sha(entry["sources"]):
        return None
    return float(t["traffic_bytes_per_launch"])


# The paper's own end-to-end numbers (single CPU process; precision not
# stated), for context only. Closest shapes: 949,983 x 3 at s = 0.001 and
# 3,205,431 x 3 at s = 0.01 (Section 5, large datasets).
PAPER_CONTEXT = {
    "system": "paper's SNG-DBSCAN (Cython/C++), one CPU process on a cloud machine, model "
              "unspecified",
    "n949983_d3_s0.001": {"runtime_s": 81, "ram_gb": 1.6, "pairs_per_s_derived": 1.1e7,
                          "vs_sklearn_dbscan": "10.8x faster (14m 37s), 262x less RAM (419 GB)"},
    "n3205431_d3_s0.01": {"runtime_s": 5230, "ram_gb": 8.7, "pairs_per_s_derived": 2.0e7},
    "n1e6_d14_s0.001": {"runtime_s": 96, "ram_gb": 1.5, "pairs_per_s_derived": 1.04e7,
                        "vs_sklearn_dbscan": "227x faster (6h 4m), 188x less RAM (282 GB)"},
}


def summary(xs):
    return {"median": statistics.median(xs), "min": min(xs), "mean": sum(xs) / len(xs)}


def frac(alg_bytes, ms):
    """Algorithmic GB/s and its fraction of the 8 TB/s HBM peak."""
    gbs = alg_bytes / (ms * 1e-3) / 1e9
    return gbs, gbs / HBM_PEAK_GBS


def _cuda_ms(torch, fn, reps):
    """Mean ms per call of fn over reps back-to-back calls (one warm-up)."""
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _each_ms(torch, fn, reps):
    """Per-call ms of fn (events around each call), after one warm-up."""
    fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for k in range(reps):
        fn()
        ev[k + 1].record()
    torch.cuda.synchronize()
    return [ev[k].elapsed_time(ev[k + 1]) for k in range(reps)]


def lscpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return "unknown"


_ORACLE_PROBE = r"""
import json, os, sys, time
sys.path.insert(0, %r)
import numpy as np
import oracle
from paper_2006_06743_amd import workloads as wl
oracle.load()
threads = oracle.set_threads(%d)
W = wl.lidar_3d()
m, budget = %d, %f
k = 1000
for _ in range(3):  # grow the sample until it takes about a tenth of the budget
    t = time.perf_counter(); oracle.degrees(W.X, m, W.eps, W.seed, 0, k)
    dt = time.perf_counter() - t
    if dt > 0.1 * budget or k >= W.n:
        break
    k = int(min(W.n, k * max(2.0, 0.1 * budget / max(dt, 1e-4))))
k = int(min(W.n, max(k, k * budget / max(dt, 1e-4))))
c0 = time.process_time(); t = time.perf_counter()
_, slots, _, _ = oracle.degrees(W.X, m, W.eps, W.seed, 0, k)
dt = time.perf_counter() - t; cpu = time.process_time() - c0
print(json.dumps({"k": k, "slots": slots, "s": dt, "cpu_s": cpu, "threads": threads,
                  "affinity": len(os.sched_getaffinity(0))}))
"""


def cpu_baseline(m, budget_s=12.0):
    """The oracle on the host: its sampling step (Philox partners, binary64
    distances, degree accumulation: the pass the GPU's pair-evaluation rate
    times) for the first k sources of the headline scene, k chosen to take
    about budget_s, with every host thread and with one."""
    threads = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
    runs = {}
    for label, nt in (("all", threads), ("one", 1)):
        r = subprocess.run([sys.executable, "-c", _ORACLE_PROBE % (ROOT, nt, m, budget_s)],
                           capture_output=True, text=True, timeout=600)
        if r.returncode != 0:
            raise RuntimeError("oracle probe failed: %s" % r.stderr[-2000:])
        runs[label] = json.loads(r.stdout.strip().splitlines()[-1])
    a, o = runs["all"], runs["one"]
    return {"value": a["slots"] / a["s"], "unit": "pair evals/s", "cores": a["threads"],
            "kind": "oracle", "cpu_model": lscpu_model(),
            "sample": "sampling step of the oracle (Philox partners, binary64 distance, degree "
                      "accumulation) for sources 0..%d of the LiDAR scene: %d slots in %.1f s "
                      "on %d threads (%.1f s of CPU time; %d CPUs in the affinity mask)"
                      % (a["k"] - 1, a["slots"], a["s"], a["threads"], a["cpu_s"],
                         a["affinity"]),
            "single_thread": {"value": o["slots"] / o["s"], "cores": o["threads"],
                              "sample": "sources 0..%d: %d slots in %.1f s (%.1f s of CPU "
                                        "time)" % (o["k"] - 1, o["slots"], o["s"], o["cpu_s"])}}


# ---------------------------------------------------------------------------
# The sampled-distance pass and the whole method, timed per step with events.
# ---------------------------------------------------------------------------
class SplitRun:
    """sample + evaluate (degrees, reusing the sample) + cluster for one
    workload on one workspace, each call bracketed by events on the stream it
    launches on."""

    def __init__(self, sng, torch, W, cfg, partner):
        self.sng, self.torch, self.W = sng, torch, W
        self.X = torch.from_numpy(W.X).cuda()
        self.m = sng.samples_per_point(W.s, W.n)
        self.slots = W.n * self.m
        self.partner = partner
        self.ws = torch.empty(sng.workspace_size(W.n, W.d, self.m), dtype=torch.uint8,
                              device="cuda")
        if partner:
            sng.sample(W.n, W.d, self.m, W.seed, self.ws)
            self.eval_cfg = dataclasses.replace(cfg, schedule=0, chunks_per_wave=0,
                                                reuse_sample=1)
        else:
            self.eval_cfg = dataclasses.replace(cfg, schedule=1)
        self.deg, _ = sng.degrees(self.X, self.m, W.eps, W.seed, cfg=self.eval_cfg, ws=self.ws)
        self.labels = sng.cluster(self.X, self.m, W.eps, W.seed, W.min_pts, self.deg, self.ws)

    def step(self, ev=None):
        sng, W = self.sng, self.W
        if ev: ev[0].record()
        if self.partner:
            sng.sample(W.n, W.d, self.m, W.seed, self.ws)
        if ev: ev[1].record()
        sng.degrees(self.X, self.m, W.eps, W.seed, cfg=self.eval_cfg, out=self.deg, ws=self.ws)
        if ev: ev[2].record()
        sng.cluster(self.X, self.m, W.eps, W.seed, W.min_pts, self.deg, self.ws,
                    labels=self.labels)
        if ev: ev[3].record()

    def timed(self, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        t0 = time.perf_counter()
        for k in range(steps):
            self.step(evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        span = lambda a: [e[a].elapsed_time(e[a + 1]) for e in evs]
        whole = [e[0].elapsed_time(e[3]) for e in evs]
        st = self.sng.stats(self.ws)
        if st.overflow:
            raise SystemExit("bench.py: the evaluate step reported a missing sample")
        return {"wall_ms_per_step": wall * 1e3 / steps, "step": whole, "sample": span(0),
                "evaluate": span(1), "post": span(2), "stats": st}


def roofline_of(run, t, traffic=None, kernel=None):
    """Roofline of the sampled-distance pass: algorithmic bytes (one
    gathered row of X per sample slot) over the event-timed pass."""
    W = run.W
    alg = run.slots * W.d * 4
    s_ms, e_ms = statistics.mean(t["sample"]), statistics.mean(t["evaluate"])
    pass_ms = s_ms + e_ms
    gbs, fr = frac(alg, pass_ms)
    out = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": fr,
           "traffic": traffic, "kernel": kernel or ("sample + evaluate" if run.partner
                                                    else "k_pass_a (direct gathers)"),
           "algorithmic_bytes": alg, "avg_launch_ms": pass_ms,
           "kernels_ms": {"sample": s_ms, "evaluate": e_ms},
           "evaluate_kernel_frac": frac(alg, e_ms)[1]}
    if traffic:
        out["hbm_moved_gbs"] = traffic / (pass_ms * 1e-3) / 1e9
        out["hbm_moved_frac"] = out["hbm_moved_gbs"] / HBM_PEAK_GBS
    return out


# ---------------------------------------------------------------------------
# The other workloads: each with its roofline and its comparison.
# ---------------------------------------------------------------------------
def cfg_small(sng, torch, wl, reps):
    """10,000 x 2 (1e6 slots), bound by launch latency: the whole call in
    microseconds against a floor of as many empty launches."""
    W = wl.blobs_2d()
    X = torch.from_numpy(W.X).cuda()
    lab, deg, ws = sng.dbscan(X, W.s, W.eps, W.min_pts, W.seed)
    r = max(reps, 50)
    calls = _each_ms(torch, lambda: sng.dbscan(X, W.s, W.eps, W.min_pts, W.seed, labels=lab,
                                               degrees_out=deg, ws=ws), r)
    launches = 5  # kernels the call enqueues (rocprofv3 kernel trace of one call)
    tiny = torch.zeros(1, device="cuda")

    def empty():
        for _ in range(launches):
            tiny.add_(0.0)
    t_floor = _cuda_ms(torch, empty, r)
    g = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=stream):
        sng.dbscan(X, W.s, W.eps, W.min_pts, W.seed, labels=lab, degrees_out=deg, ws=ws)
    t_graph = _cuda_ms(torch, g.replay, r)
    c = summary(calls)
    return {"workload": W.name, "slots": W.n * sng.samples_per_point(W.s, W.n),
            "call_us": {k: v * 1e3 for k, v in c.items()}, "graph_replay_us": t_graph * 1e3,
            "launches": launches, "empty_launches_us": t_floor * 1e3,
            "over_floor": c["median"] / t_floor,
            "roofline": {"bound": "launch latency", "note": "1e6 slots x 8 B = 8 MB: 1 us at "
                         "8 TB/s; the call is priced against its empty-launch floor"}}


def cfg_gmm16d(sng, torch, wl, reps, cfg):
    """1e6 x 16 Gaussian mixture (1e9 slots): the pass and the whole method,
    at sigma = 1 (as specified; almost every point is noise) and at sigma =
    0.25 (50 real clusters, so the hook and finalize have work)."""
    out = {}
    for sigma in (1.0, 0.25):
        W = wl.mixture_16d(sigma=sigma)
        run = SplitRun(sng, torch, W, cfg, partner=True)
        t = run.timed(max(reps, 5), 2)
        key = "sigma1" if sigma == 1.0 else "sigma0.25"
        out[key] = {"workload": W.name, "slots": run.slots,
                    "step_ms": summary(t["step"]), "pass_ms": summary(
                        [a + b for a, b in zip(t["sample"], t["evaluate"])]),
                    "accepted": t["stats"].accepted, "clusters": t["stats"].n_clusters,
                    "roofline": roofline_of(run, t)}
        del run
        torch.cuda.empty_cache()
    return out


def cfg_mixed(sng, torch, wl, reps):
    """70,000 x 784 quantised images: plain binary32 vs the bfloat16 and
    float16 MFMA forms, identical labels and degrees required."""
    import numpy as np
    W = wl.mnistlike_784d()
    X = torch.from_numpy(W.X).cuda()
    m = sng.samples_per_point(W.s, W.n)
    slots = W.n * m
    lab, deg, ws = sng.dbscan(X, W.s, W.eps, W.min_pts, W.seed)
    plain = _each_ms(torch, lambda: sng.dbscan(X, W.s, W.eps, W.min_pts, W.seed, labels=lab,
                                               degrees_out=deg, ws=ws), reps)
    p = summary(plain)
    entry = {"workload": W.name, "slots": slots, "plain_ms": p,
             "roofline_plain_call": {"bound": "hbm", "algorithmic_bytes": slots * W.d * 4,
                                     "frac": frac(slots * W.d * 4, p["median"])[1]}}
    for name, prec, bits in [("bf16", sng.SNG_BF16, W.X_lp), ("fp16", sng.SNG_FP16,
                                                              wl.fp16_bits(W.X))]:
        try:
            Xlp = torch.from_numpy(bits.view(np.int16)).cuda()
            lab2, deg2, ws2 = sng.dbscan_lowp(X, Xlp, W.s, W.eps, W.min_pts, W.seed, prec=prec)
            t = summary(_each_ms(torch, lambda: sng.dbscan_lowp(
                X, Xlp, W.s, W.eps, W.min_pts, W.seed, prec=prec, ws=ws2), reps))
            lab2, deg2, ws2 = sng.dbscan_lowp(X, Xlp, W.s, W.eps, W.min_pts, W.seed, prec=prec,
                                              ws=ws2)
            torch.cuda.synchronize()
            st = sng.stats(ws2)
            entry[name] = {"ms": t, "speedup": p["median"] / t["median"],
                           "labels_identical": bool(torch.equal(lab, lab2)),
                           "degrees_identical": bool(torch.equal(deg, deg2)),
                           "recheck_fraction": st.rechecked / max(1, st.slots),
                           "filter_bound": sng.lowp_bound(ws2),
                           "roofline_call": {"bound": "hbm",
                                             "algorithmic_bytes": slots * W.d * 2,
                                             "frac": frac(slots * W.d * 2, t["median"])[1]}}
            del lab2, deg2, ws2, Xlp
        except sng.SNGError as e:
            entry[name] = "unavailable: %s" % e
    return entry


def cfg_sweep(sng, torch, wl, reps):
    """500k x 32 with a 32 x 4 grid: one sweep call against 128 real plain
    calls (one per grid point), labels compared at every grid point."""
    W = wl.sweep_32d()
    X = torch.from_numpy(W.X).cuda()
    m = sng.samples_per_point(W.s, W.n)
    K, P = len(W.eps_grid), len(W.min_pts_grid)
    sl, sd, sws = sng.sweep(X, W.s, W.eps_grid, W.min_pts_grid, W.seed)
    t_sweep = summary(_each_ms(torch, lambda: sng.sweep(X, W.s, W.eps_grid, W.min_pts_grid,
                                                        W.seed, ws=sws), max(2, reps - 1)))
    sl, sd, sws = sng.sweep(X, W.s, W.eps_grid, W.min_pts_grid, W.seed, ws=sws)
    lab, deg, ws = sng.dbscan(X, W.s, float(W.eps_grid[0]), 2, W.seed)
    labs = [torch.empty_like(lab) for _ in range(K * P)]

    def all_plain():
        for k in range(K):
            for p in range(P):
                sng.dbscan(X, W.s, float(W.eps_grid[k]), int(W.min_pts_grid[p]), W.seed,
                           labels=labs[k * P + p], degrees_out=deg, ws=ws)
    t_all = _cuda_ms(torch, all_plain, 1)
    same = [bool(torch.equal(sl[p, k], labs[k * P + p])) for k in range(K) for p in range(P)]
    single = _cuda_ms(torch, lambda: sng.dbscan(X, W.s, float(W.eps_grid[16]), 4, W.seed,
                                                labels=lab, degrees_out=deg, ws=ws), reps)
    alg = W.n * m * W.d * 4
    return {"workload": W.name, "grid": [K, P], "slots_per_pass": W.n * m,
            "sweep_ms": t_sweep, "plain_128_calls_ms": t_all, "plain_single_ms": single,
            "speedup_vs_128_calls": t_all / t_sweep["median"],
            "labels_identical": all(same), "grid_points_identical": sum(same),
            "roofline_single_plain_call": {"bound": "hbm", "algorithmic_bytes": alg,
                                           "frac": frac(alg, single)[1],
                                           "note": "one 128-byte row per slot over the call's "
                                                   "time; partner blocks serve most rows from "
                                                   "L2, so this can exceed 1"}}


def cfg_batch(sng, torch, wl, reps):
    """64 uneven instances: 64 sequential plain calls vs one captured-graph
    launch, labels compared instance by instance."""
    B = wl.uneven_batch()
    Xs = [torch.from_numpy(b.X).cuda() for b in B]
    slots = sum(b.n * sng.samples_per_point(b.s, b.n) for b in B)
    outs = [sng.dbscan(x, b.s, b.eps, b.min_pts, b.seed) for x, b in zip(Xs, B)]

    def seq():
        for x, b, (l, dg, w) in zip(Xs, B, outs):
            sng.dbscan(x, b.s, b.eps, b.min_pts, b.seed, labels=l, degrees_out=dg, ws=w)
    t_seq = summary(_each_ms(torch, seq, reps))
    entry = {"instances": len(B), "slots": slots, "sequential_ms": t_seq}
    try:
        plan = sng.BatchPlan(Xs, [b.s for b in B], [b.eps for b in B],
                             [b.min_pts for b in B], [b.seed for b in B])
        t_graph = summary(_each_ms(torch, lambda: plan.launch(), reps))
        labels, degs = plan.launch()
        torch.cuda.synchronize()
        same = [bool(torch.equal(labels[k], outs[k][0]) and torch.equal(degs[k], outs[k][1]))
                for k in range(len(B))]
        alg = sum(b.n * sng.samples_per_point(b.s, b.n) * b.d * 4 for b in B)
        entry.update({"graph_batch_ms": t_graph,
                      "speedup": t_seq["median"] / t_graph["median"],
                      "labels_identical": all(same), "instances_identical": sum(same),
                      "roofline_whole_batch": {"bound": "hbm", "algorithmic_bytes": alg,
                                               "frac": frac(alg, t_graph["median"])[1]}})
    except sng.SNGError as e:
        entry["graph_batch"] = "unavailable: %s" % e
    return entry


def form_recovery(sng, torch, wl, reps):
    """The paper's simulated recovery study (three uniform balls in R^3,
    ceil(20 ln n) samples per point): ARI and AMI against the true balls as n
    grows, with the GPU time of each run."""
    from sklearn.metrics import adjusted_mutual_info_score, adjusted_rand_score
    rows = []
    for n in (1000, 10000, 100000, 1000000):
        W, truth = wl.balls_3d(n)
        X = torch.from_numpy(W.X).cuda()
        lab, deg, ws = sng.dbscan(X, W.s, W.eps, W.min_pts, W.seed)
        t = _cuda_ms(torch, lambda: sng.dbscan(X, W.s, W.eps, W.min_pts, W.seed, labels=lab,
                                               degrees_out=deg, ws=ws), reps)
        got = lab.cpu().numpy()
        rows.append({"n": n, "m": W.meta["m"], "ms": t,
                     "ari": float(adjusted_rand_score(truth, got)),
                     "ami": float(adjusted_mutual_info_score(truth, got)),
                     "clusters": int(sng.stats(ws).n_clusters),
                     "noise_fraction": float((got < 0).mean())})
        del X, ws
    return {"workload": "balls3d (eps 0.3, MinPts 3, s = ceil(20 ln n) / n)", "runs": rows}


def form_similarity(sng, torch, wl, reps):
    """Similarity-threshold edges against the distance form on the same
    slots: cosine >= 0.95 and dot product >= 300 on the 1e6 x 16 mixture,
    cosine >= 0.9 on the 70k x 784 images."""
    out = {}
    for W, kind, tau, min_pts in [
            (wl.mixture_16d(), sng.SNG_SIM_COSINE, 0.95, None),
            (wl.mixture_16d(), sng.SNG_SIM_DOT, 300.0, None),
            (wl.mnistlike_784d(), sng.SNG_SIM_COSINE, 0.9, 10)]:
        mp = W.min_pts if min_pts is None else min_pts
        X = torch.from_numpy(W.X).cuda()
        slots = W.n * sng.samples_per_point(W.s, W.n)
        lab, deg, ws = sng.dbscan_similarity(X, W.s, kind, tau, mp, W.seed)
        t_sim = _cuda_ms(torch, lambda: sng.dbscan_similarity(
            X, W.s, kind, tau, mp, W.seed, labels=lab, degrees_out=deg, ws=ws), reps)
        st = sng.stats(ws)
        lab2, deg2, ws2 = sng.dbscan(X, W.s, W.eps, mp, W.seed)
        t_dist = _cuda_ms(torch, lambda: sng.dbscan(X, W.s, W.eps, mp, W.seed, labels=lab2,
                                                    degrees_out=deg2, ws=ws2), reps)
        name = "cosine" if kind == sng.SNG_SIM_COSINE else "dot"
        out["%s_%s" % (W.name, name)] = {
            "query": "%s >= %g" % (name, tau), "slots": slots, "similarity_ms": t_sim,
            "distance_ms": t_dist, "pair_evals_per_s": slots / (t_sim * 1e-3),
            "recheck_fraction": st.rechecked / max(st.slots, 1), "accepted": st.accepted,
            "clusters": st.n_clusters}
        del X, lab, deg, ws, lab2, deg2, ws2
        torch.cuda.empty_cache()
    return out


def form_simple_graph(sng, torch, wl, reps):
    """Simple-graph degrees (distinct accepted neighbours, through the hash
    table of accepted pairs) against the multigraph degrees, on the dense
    1e6 x 16 mixture (sigma = 0.25)."""
    W = wl.mixture_16d(sigma=0.25)
    X = torch.from_numpy(W.X).cuda()
    out = {"workload": W.name, "slots": W.n * sng.samples_per_point(W.s, W.n)}
    for name, cfg in [("multigraph", sng.Config()), ("simple_graph", sng.Config(simple_graph=1))]:
        lab, deg, ws = sng.dbscan(X, W.s, W.eps, W.min_pts, W.seed, cfg=cfg)
        out[name + "_ms"] = _cuda_ms(torch, lambda: sng.dbscan(
            X, W.s, W.eps, W.min_pts, W.seed, cfg=cfg, labels=lab, degrees_out=deg, ws=ws), reps)
        st = sng.stats(ws)
        out[name + "_core"] = st.n_core
        out["accepted"] = st.accepted
        del lab, deg, ws
        torch.cuda.empty_cache()
    return out


CONFIGS = {"small": cfg_small, "gmm16d": None, "mixed": cfg_mixed, "sweep": cfg_sweep,
           "batch": cfg_batch}
FORMS = {"recovery": form_recovery, "similarity": form_similarity,
         "simple_graph": form_simple_graph}


def guarded(torch, fn):
    try:
        return fn()
    except Exception as e:  # the headline line must still print
        return "error: %s: %s" % (type(e).__name__, e)
    finally:
        torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--schedule", choices=["tuned", "auto", "direct"], default="auto",
                    help="auto: the library's rule (partner blocks here); tuned: the "
                         "autotuner's choice (timed first); direct: direct gathers")
    ap.add_argument("--configs", default="small,gmm16d,mixed,sweep,batch")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--forms", default="recovery,similarity,simple_graph")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 256 MiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library runs on one GPU; --gpus %d (WORLD_SIZE=%d) is not "
              "supported" % (args.gpus, world), file=sys.stderr, flush=True)
        sys.exit(2)
    configs = [c for c in args.configs.split(",") if c] if not args.no_configs else []
    forms = [f for f in args.forms.split(",") if f] if not args.no_forms else []
    for c in configs:
        if c not in CONFIGS:
            raise SystemExit("bench.py: unknown config %r" % c)
    for f in forms:
        if f not in FORMS:
            raise SystemExit("bench.py: unknown form %r" % f)

    import torch
    import paper_2006_06743_amd as sng
    from paper_2006_06743_amd import workloads as wl
    sng.load()

    W = wl.lidar_3d()
    m = sng.samples_per_point(W.s, W.n)
    tune = None
    base = sng.Config()
    partner = args.schedule != "direct"
    if args.schedule == "tuned":
        X0 = torch.from_numpy(W.X).cuda()
        ws0 = torch.empty(sng.workspace_size(W.n, W.d, m), dtype=torch.uint8, device="cuda")
        cfg, tuned_ms, tried = sng.autotune(X0, m, W.eps, W.seed, trials=1, ws=ws0)
        tune = {"config": dataclasses.asdict(cfg), "tuned_pass_ms": tuned_ms,
                "candidates": tried}
        partner, base = cfg.schedule == 2, cfg
        del X0, ws0
    run = SplitRun(sng, torch, W, base, partner)
    t = run.timed(args.steps, args.warmup)
    st = t["stats"]
    traffic = measured_traffic(PASS) if partner else None
    roof = roofline_of(run, t, traffic, PASS["name"] if partner else None)
    step = summary(t["step"])
    out = {
        "metric": METRIC,
        "value": run.slots / (t["wall_ms_per_step"] * 1e-3),
        "unit": "pair evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t["wall_ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": W.name + " (LiDAR-like scene: ground plane, 300 ellipsoid "
                   "objects, 1% clutter)", "n": W.n, "d": W.d, "s": W.s, "m": m,
                   "eps": W.eps, "min_pts": W.min_pts, "seed": W.seed,
                   "parallelism": "single GPU"},
        "step_ms": step,
        "end_to_end_ms": step["median"],
        "pass_ms": {"sample": summary(t["sample"]), "evaluate": summary(t["evaluate"]),
                    "core_hook_finalize": summary(t["post"])},
        "sampled_distance_evals_per_s": run.slots / (roof["avg_launch_ms"] * 1e-3),
        "schedule": "partner blocks" if partner else "direct gathers",
        "launch_config": dataclasses.asdict(run.eval_cfg),
        "autotune": tune,
        "stats": {"slots": st.slots, "self_pairs": st.self_pairs, "accepted": st.accepted,
                  "rechecked": st.rechecked, "n_core": st.n_core, "n_clusters": st.n_clusters,
                  "n_noise": st.n_noise},
        "roofline": roof,
        "paper_context": PAPER_CONTEXT,
    }
    if partner:
        direct = dataclasses.replace(base, schedule=1, reuse_sample=0)
        out["direct_gathers_pass_ms"] = _cuda_ms(torch, lambda: sng.degrees(
            run.X, m, W.eps, W.seed, cfg=direct, out=run.deg, ws=run.ws), 1)
    del run
    torch.cuda.empty_cache()
    if args.calibrate_copy:
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel()
        del src, dst
    reps = 5
    if configs:
        out["configs"] = {}
        for c in configs:
            if c == "gmm16d":
                out["configs"][c] = guarded(torch, lambda: cfg_gmm16d(sng, torch, wl, reps, base))
            else:
                out["configs"][c] = guarded(torch, lambda: CONFIGS[c](sng, torch, wl, reps))
    if forms:
        out["forms"] = {f: guarded(torch, lambda: FORMS[f](sng, torch, wl, 3)) for f in forms}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(m)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
