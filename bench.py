"""Benchmark of the min-cut path on one MI355X.

Prints ONE JSON line. The headline `value` is input edges/s of a single
graph solve: one step is one full solve (validation, label propagation,
cluster contraction, Padberg-Rinaldi contraction, bound tracking, exact solve
on the remaining graph, transfer of the side) of one graph already resident
in HBM, with a preallocated workspace. Default workload: the random hyperbolic
graph with n = 2^20, average degree 32, power-law exponent 5, unit weights
(seed 1), n0 = 10,000, two LP iterations, tie-break seed 0.

The same line carries
  * "roofline": the dominant timed tile kernel (largest summed duration among
    the arc-tile LP kernels), its algorithmic bytes per launch over its average
    event-timed duration during the timed steps, against 8 TB/s;
    "traffic": HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE
    counters, scaled by a copy-kernel calibration, read from
    profiles/traffic_<kernel>_<workload>.json when its recorded source hash
    still matches the kernel source (else null);
  * "sweep": round 1's label propagation and cluster contraction (from the
    solve's first launch to the coarse CSR), event-timed, against its
    algorithmic bytes 28A + 4A_x + 8A' + 60n (A input arcs, A_x emitted
    inter-cluster arcs, A' coarse arcs, n vertices);
  * "singles": the other single-graph workloads, median of 5 solves after one
    warm-up: the R-MAT scale-22 10-core (with its own sweep and tile
    rooflines), the same RHG graph with n0 = 64, and the n = 2,000 planted cut;
  * "batched": the batch of 4,096 planted-cut graphs (n U{64..8192}, average
    degree U[8,64], weights U{1..100}, 1-20 cross edges) solved in one batched
    execution (median of 5), against the plain single-graph path on the same
    graphs;
  * "served": 200 warm-up and 2,000 timed requests (n log-uniform in
    [100, 2^20], half RHG, half planted); each request is a distinct weighted
    graph: a topology drawn from a seeded pool with weights U{1..100} drawn for
    that request. Served through a session with a 64 GB budget: the capacity
    with every request queued at once, then Poisson arrivals at 50 % and 80 %
    of it with p50/p99 latency from arrival to result, each against a FIFO
    server running the single-graph path on the same arrivals;
  * "cpu_baseline": the oracle (the plain C++ implementation the tests check
    against) on the host cores, in child processes with a fixed OpenMP thread
    count: all cores and one thread on the headline graph, plus the planted
    cut and a sample of the batch (one graph per core).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "rhg2p20": dict(desc="random hyperbolic graph n=2^20 avg deg 32 gamma 5 unit weights seed 1", n0=10000),
    "rmat22core": dict(desc="R-MAT scale 22 ef 16 (0.57/0.19/0.19) 10-core LCC seed 2", n0=10000),
    "planted2000": dict(desc="planted cut n=2000 d=32 5 cross edges unit weights seed 0", n0=64),
}
TILE_KINDS = ("k_first_tile", "k_first_tile_level0", "k_lp_tile")
SWEEP_KIND = "lp_contract_sweep"


def log(*a):
    print("#", *a, file=sys.stderr, flush=True)


def make_graph(name):
    import graphgen as gg
    if name == "rhg2p20":
        return gg.c2_rhg()
    if name == "rmat22core":
        return gg.c3_rmat()
    if name == "planted2000":
        return gg.c1_planted(0)
    raise SystemExit("unknown workload " + name)


def to_dev(g):
    import numpy as np
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda() for a in (g.row_ptr, g.col, g.w)]


def median(xs):
    s = sorted(xs)
    k = len(s)
    return s[k // 2] if k % 2 else 0.5 * (s[k // 2 - 1] + s[k // 2])


# ------------------------------------------------------------ CPU baseline
def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_child(leg, budget_s, max_runs):
    """Runs in a child process whose OpenMP thread count is fixed by its
    environment; times the oracle (generation excluded) and prints one JSON
    object."""
    import graphgen as gg
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "1"))
    if leg in ("c2", "c1"):
        g = gg.c2_rhg() if leg == "c2" else gg.c1_planted(0)
        n0 = 10000 if leg == "c2" else 64
        oracle.mincut_graph(g, lp_iters=2, n0=n0, seed=0)  # warm-up (page-in, OpenMP pool)
        times = []
        t_start = time.perf_counter()
        while len(times) < max_runs:
            t0 = time.perf_counter()
            oracle.mincut_graph(g, lp_iters=2, n0=n0, seed=0)
            times.append(time.perf_counter() - t0)
            if time.perf_counter() - t_start + times[-1] > budget_s:
                break
        med = median(times)
        print(json.dumps({"value": g.m / med, "unit": "input edges/s", "threads": threads, "runs": len(times),
                          "median_s": med}))
        return
    if leg == "c4":
        from concurrent.futures import ThreadPoolExecutor
        count = max_runs  # graphs in the sample: every 4096/count-th member of the batch
        step = max(1, 4096 // count)
        members = list(range(0, 4096, step))[:count]
        gs = gg.c4_batch(4096, members=members)
        workers = int(os.environ.get("VC_CPU_WORKERS", "1"))
        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(lambda g: oracle.mincut_graph(g, lp_iters=2, n0=64, seed=0), gs))
        dt = time.perf_counter() - t0
        m = sum(g.m for g in gs)
        print(json.dumps({"graphs_per_s": len(gs) / dt, "input_edges_per_s": m / dt, "graphs": len(gs),
                          "workers": workers, "threads_per_graph": threads, "s": dt}))
        return
    raise SystemExit("unknown cpu leg " + leg)


def run_cpu_child(leg, threads, budget_s, max_runs, workers=1):
    env = dict(os.environ)
    env["OMP_NUM_THREADS"] = str(threads)
    env["VC_CPU_WORKERS"] = str(workers)
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-child", leg, "--cpu-budget", str(budget_s),
           "--cpu-runs", str(max_runs)]
    p = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=600)
    if p.returncode != 0:
        raise RuntimeError("cpu leg %s failed: %s" % (leg, p.stderr[-2000:]))
    return json.loads(p.stdout.strip().splitlines()[-1])


def cpu_baseline(m_c2):
    """The oracle as it stands, timed on the host: the headline graph with all
    cores (median of up to 5) and with one thread (median of up to 3), the
    planted n = 2,000 graph, and a 256-graph sample of the batch with one
    graph per core and one thread per graph."""
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    log("cpu baseline: oracle on the RHG graph, %d threads" % cores)
    allc = run_cpu_child("c2", cores, 12.0, 5)
    log("cpu baseline: oracle on the RHG graph, 1 thread")
    one = run_cpu_child("c2", 1, 25.0, 3)
    log("cpu baseline: oracle on the planted n=2000 graph and the batch sample")
    c1 = run_cpu_child("c1", cores, 3.0, 5)
    c4 = run_cpu_child("c4", 1, 0, 256, workers=cores)
    return {"value": allc["value"], "unit": "input edges/s", "cores": allc["threads"], "kind": "oracle",
            "sample": "full solves of the headline RHG graph (m=%d), median of %d, %d OpenMP threads; "
                      "generation excluded" % (m_c2, allc["runs"], allc["threads"]),
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "one_thread": {"value": one["value"], "runs": one["runs"], "median_s": round(one["median_s"], 3)},
            "planted2000": {"value": c1["value"], "runs": c1["runs"], "threads": c1["threads"]},
            "batch_sample": {"graphs_per_s": round(c4["graphs_per_s"], 1),
                             "input_edges_per_s": c4["input_edges_per_s"], "graphs": c4["graphs"],
                             "workers": c4["workers"], "threads_per_graph": 1}}


# ------------------------------------------------------------ roofline
def kernel_source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1708_06127_amd", "csrc", "vc_kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel, workload):
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha") != kernel_source_hash():
        return None  # the kernel changed since the counters were taken
    return rec.get("bytes_per_launch")


COPY_PROBE_BYTES = 256 << 20  # the --copy-probe device copy: 64 Mi int32 read and written
# a timed unit of the library's kernel timer and the device kernels it covers
# (the LP iteration t >= 2 runs the tiles of at most 256 arcs and the larger
# tiles in two launches, timed together)
TIMED_UNITS = {"k_lp_tile": ["k_lp_tile", "k_lp_tile_big"],
               "k_first_tile": ["k_first_tile", "k_first_tile_big", "k_first_tile_each"],
               "k_first_tile_level0": ["k_first_tile", "k_first_tile_big", "k_first_tile_each"]}


def record_traffic(fetch_csv, write_csv, kernel, workload, command):
    """Turn two rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE, in KiB
    per dispatch) of `bench.py --copy-probe` into HBM bytes per launch of
    `kernel`: each counter is scaled by known bytes / reading for the plain
    256 MiB device copy of the same run. Writes
    profiles/traffic_<kernel>_<workload>.json stamped with the kernel source
    hash, which is how the roofline's "traffic" knows it is still current."""
    import csv

    def rows(path):
        """(kernel name, counter name, value in KiB) per dispatch, from the
        counter CSV or from the rocpd database rocprofv3 writes by default"""
        if path.endswith(".db"):
            import sqlite3
            db = sqlite3.connect(path)
            for name, cname, val in db.execute("select kernel_name, counter_name, value from counters_collection"):
                yield name, cname, float(val)
            db.close()
            return
        with open(path) as f:
            for r in csv.DictReader(f):
                yield r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])

    def per_kernel(path, counter):
        copy_best, vals = 0.0, {k: [] for k in TIMED_UNITS.get(kernel, [kernel])}
        for name, cname, kib in rows(path):
            if cname != counter:
                continue
            v = kib * 1024.0
            if "copyBuffer" in name:
                copy_best = max(copy_best, v)
            for k in vals:
                if "::%s(" % k in name or "::%s<" % k in name:
                    vals[k].append(v)
        if not copy_best or not all(vals.values()):
            raise SystemExit("%s: no copy probe or no %s dispatch with %s" % (path, kernel, counter))
        # per timed unit: the sum over its kernels of the mean per dispatch
        return sum(sum(v) / len(v) for v in vals.values()), COPY_PROBE_BYTES / copy_best, \
            [len(v) for v in vals.values()]

    fetch, f_scale, nf = per_kernel(fetch_csv, "FETCH_SIZE")
    write, w_scale, nw = per_kernel(write_csv, "WRITE_SIZE")
    rec = {"kernel": kernel, "workload": workload, "source_sha": kernel_source_hash(),
           "bytes_per_launch": round(fetch * f_scale + write * w_scale),
           "fetch_bytes_per_launch": round(fetch * f_scale), "write_bytes_per_launch": round(write * w_scale),
           "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4), "dispatches": [nf, nw],
           "command": command}
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def roofline(prof, workload):
    """The dominant tile kernel of the timer's totals: algorithmic bytes per
    launch over its mean event-timed duration, against 8 TB/s."""
    timed = {k: v for k, v in prof.items() if k in TILE_KINDS and v["launches"] > 0 and v["total_ms"] > 0}
    if not timed:
        return None
    name = max(timed, key=lambda k: timed[k]["total_ms"])
    v = timed[name]
    per_launch_bytes = v["bytes"] / v["launches"]
    avg_ms = v["total_ms"] / v["launches"]
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_for(name, workload),
            "kernel": name, "launches": v["launches"], "avg_us": round(avg_ms * 1e3, 2),
            "algorithmic_bytes_per_launch": round(per_launch_bytes)}


def sweep_roofline(prof):
    """Round 1's LP + cluster contraction: the event-timed span from the
    solve's first launch to the coarse CSR (host synchronisations inside it
    included) against B_alg = 28A + 4A_x + 8A' + 60n."""
    v = prof.get(SWEEP_KIND)
    if not v or v["launches"] == 0 or v["total_ms"] <= 0:
        return None
    per = v["bytes"] / v["launches"]
    avg_ms = v["total_ms"] / v["launches"]
    achieved = per / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "spans": v["launches"], "avg_us": round(avg_ms * 1e3, 2),
            "algorithmic_bytes": round(per)}


# ------------------------------------------------------------ single graphs
def time_single(vc, dev, g, n0, reps, warmup=1, profile=False):
    """Median of `reps` solves after `warmup`, each bracketed by device
    synchronisation; with profile, the kernel timer's totals over the reps."""
    import torch
    ws = vc.workspace(g.n, g.nnz)
    side = torch.empty((g.n + 63) // 64, dtype=torch.int64, device="cuda")
    kw = dict(lp_iters=2, n0=n0, seed=0, ws=ws, side=side)
    for _ in range(warmup):
        vc.mincut(*dev, **kw)
    torch.cuda.synchronize()
    if profile:
        vc.profile_enable(True)
    times = []
    info = None
    for _ in range(reps):
        t0 = time.perf_counter()
        cut, _, info = vc.mincut(*dev, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    prof = None
    if profile:
        prof = vc.profile_read()
        vc.profile_enable(False)
    del ws
    return median(times), cut, info, prof


def bench_singles(vc, args):
    import graphgen as gg
    out = {}
    if not args.no_c3:
        t0 = time.perf_counter()
        g = gg.c3_rmat()
        log("generated R-MAT 22 10-core: n=%d m=%d in %.1f s" % (g.n, g.m, time.perf_counter() - t0))
        dev = to_dev(g)
        med, cut, info, prof = time_single(vc, dev, g, 10000, 5, profile=True)
        out["rmat22core"] = {"workload": WORKLOADS["rmat22core"]["desc"], "n": g.n, "m": g.m, "n0": 10000,
                             "ms": round(med * 1e3, 3), "input_edges_per_s": g.m / med, "cut": cut,
                             "rounds": info["rounds"], "kernel_n": info["kernel_n"],
                             "sweep": sweep_roofline(prof), "roofline": roofline(prof, "rmat22core")}
        log("single R-MAT:", out["rmat22core"])
        del dev, g
    g = gg.c2_rhg()
    dev = to_dev(g)
    med, cut, info, _ = time_single(vc, dev, g, 64, 5)
    out["rhg2p20_n0_64"] = {"workload": WORKLOADS["rhg2p20"]["desc"] + " n0=64", "n": g.n, "m": g.m, "n0": 64,
                            "ms": round(med * 1e3, 3), "input_edges_per_s": g.m / med, "cut": cut,
                            "rounds": info["rounds"], "kernel_n": info["kernel_n"]}
    log("single RHG n0=64:", out["rhg2p20_n0_64"])
    del dev, g
    g = gg.c1_planted(0)
    dev = to_dev(g)
    med, cut, info, _ = time_single(vc, dev, g, 64, 5)
    out["planted2000"] = {"workload": WORKLOADS["planted2000"]["desc"], "n": g.n, "m": g.m, "n0": 64,
                          "ms": round(med * 1e3, 3), "input_edges_per_s": g.m / med, "cut": cut,
                          "rounds": info["rounds"], "kernel_n": info["kernel_n"]}
    log("single planted:", out["planted2000"])
    return out


# ------------------------------------------------------------ batched
def bench_batched(args):
    import torch
    import graphgen as gg
    import paper_1708_06127_amd as vc
    t0 = time.perf_counter()
    gs = gg.c4_batch(args.batch_count)
    log("generated %d planted graphs in %.1f s" % (len(gs), time.perf_counter() - t0))
    dev = [to_dev(g) for g in gs]
    m_total = sum(g.m for g in gs)
    kw = dict(lp_iters=2, n0=64, seed=0)
    p = vc.params(**kw)
    ws = torch.empty(vc.batch_workspace_bytes(dev, p), dtype=torch.uint8, device="cuda")
    sides = [torch.empty(max((g.n + 63) // 64, 1), dtype=torch.int64, device="cuda") for g in gs]
    log("batch workspace %.1f GB, %d input edges" % (ws.numel() / 1e9, m_total))
    vc.mincut_batch(dev, ws=ws, sides=sides, **kw)  # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(args.batch_reps):
        t0 = time.perf_counter()
        res = vc.mincut_batch(dev, ws=ws, sides=sides, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log("batch call %d: %.1f ms" % (len(times), times[-1] * 1e3))
    tb = median(times)
    del ws
    out = {"workload": "%d planted-cut graphs, n U{64..8192}, avg deg U[8,64], w U{1..100}, 1-20 cross "
                       "edges (seeds 3..), n0=64" % len(gs),
           "graphs": len(gs), "input_edges": m_total, "ms": round(tb * 1e3, 2), "reps": len(times),
           "ms_min": round(min(times) * 1e3, 2), "ms_max": round(max(times) * 1e3, 2),
           "graphs_per_s": round(len(gs) / tb, 1), "input_edges_per_s": m_total / tb}
    if args.no_single_compare:  # e.g. under a kernel tracer: the batch's own dispatches only
        return out
    # the plain single-graph path on the same graphs, one after another
    nmax = max(g.n for g in gs)
    amax = max(g.nnz for g in gs)
    ws1 = vc.workspace(nmax, amax)
    side1 = torch.empty((nmax + 63) // 64, dtype=torch.int64, device="cuda")
    for d in dev[:8]:
        vc.mincut(*d, ws=ws1, side=side1, **kw)
    torch.cuda.synchronize()
    same = 0
    t0 = time.perf_counter()
    for d, r in zip(dev, res):
        cut, _, _ = vc.mincut(*d, ws=ws1, side=side1, **kw)
        same += int(cut == r[0])
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    out.update({"single_path_ms": round(ts * 1e3, 2), "single_path_graphs_per_s": round(len(gs) / ts, 1),
                "speedup_vs_single_path": round(ts / tb, 2), "cuts_equal_single_path": same == len(gs)})
    return out


# ------------------------------------------------------------ served
def _serve_run(vc, reqs, sides, arrival, kw, label):
    """Real-time session run: request j is submitted once the clock passes
    arrival[j]; returns (latencies in s, cuts, wall time, steps)."""
    sess = vc.Session(64 << 30, **kw)
    lat = {}
    cuts = {}
    i = 0
    steps = 0
    nreq = len(reqs)
    next_log = 500
    t_start = time.perf_counter()
    while len(lat) < nreq:
        now = time.perf_counter() - t_start
        while i < nreq and arrival[i] <= now:
            sess.submit(i, *reqs[i], side=sides[i])
            i += 1
        active = sess.step()
        steps += 1
        t_done = time.perf_counter() - t_start
        for rid, cut, _, _ in sess.poll():
            lat[rid] = t_done - arrival[rid]
            cuts[rid] = cut
        if len(lat) >= next_log:
            log("%s: %d of %d requests done after %.1f s" % (label, len(lat), nreq, t_done))
            next_log += 500
        if active == 0 and i < nreq:
            time.sleep(max(0.0, arrival[i] - (time.perf_counter() - t_start)))
    wall = time.perf_counter() - t_start
    sess.close()
    return [lat[j] for j in range(nreq)], [cuts[j] for j in range(nreq)], wall, steps


def bench_served(args):
    import numpy as np
    import torch
    from concurrent.futures import ThreadPoolExecutor
    import graphgen as gg
    import paper_1708_06127_amd as vc
    ps = gg.c5_request_params(args.serve_pool)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        pool = list(ex.map(gg.c5_make, ps))
    log("generated a pool of %d topologies in %.1f s (%d edges)" % (len(pool), time.perf_counter() - t0,
                                                                   sum(g.m for g in pool)))
    topo = []
    for g in pool:
        rp, col, _ = to_dev(g)
        topo.append((rp, col))
    nreq = args.serve_warmup + args.serve_requests
    rng = np.random.default_rng(4)
    pick = rng.integers(0, len(pool), nreq)
    reqs = []
    for j in range(nreq):  # a distinct weighted graph per request: fresh weights on a pool topology
        rp, col = topo[pick[j]]
        reqs.append((rp, col, gg.reweight_device(rp, col, 1000 + j)))
    torch.cuda.synchronize()
    m_req = [pool[k].m for k in pick]
    log("built %d requests (%d distinct topologies, weights per request), %.2f G input edges" %
        (nreq, len(set(pick.tolist())), sum(m_req) / 1e9))
    sides = [torch.empty(max((pool[k].n + 63) // 64, 1), dtype=torch.int64, device="cuda") for k in pick]
    kw = dict(lp_iters=2, n0=64, seed=0)
    # single-path solve time of every request (the FIFO baseline replays them)
    nmax = max(g.n for g in pool)
    amax = max(g.nnz for g in pool)
    ws1 = vc.workspace(nmax, amax)
    side1 = torch.empty((nmax + 63) // 64, dtype=torch.int64, device="cuda")
    for r in reqs[:8]:
        vc.mincut(*r, ws=ws1, side=side1, **kw)
    torch.cuda.synchronize()
    dur, cut1 = [], []
    for j, r in enumerate(reqs):
        t1 = time.perf_counter()
        c, _, _ = vc.mincut(*r, ws=ws1, side=side1, **kw)
        torch.cuda.synchronize()
        dur.append(time.perf_counter() - t1)
        cut1.append(c)
        if (j + 1) % 500 == 0:
            log("single path: %d of %d requests timed" % (j + 1, nreq))
    del ws1
    log("single-path solve times: mean %.3f ms, max %.3f ms" % (1e3 * np.mean(dur), 1e3 * max(dur)))
    # batched capacity: every request queued at time 0
    _serve_run(vc, reqs[:16], sides[:16], np.zeros(16), kw, "session warm-up")
    _, cuts, wall, steps = _serve_run(vc, reqs, sides, np.zeros(nreq), kw, "capacity run")
    capacity = nreq / wall
    single_capacity = nreq / sum(dur)
    log("session capacity %.1f req/s (%d steps); single path %.1f req/s" % (capacity, steps, single_capacity))
    w0 = args.serve_warmup
    out = {"workload": "Poisson stream of %d requests (the first %d are warm-up, not counted): n log-uniform "
                       "[100, 2^20], half RHG (gamma 5, avg deg U[16,64]) half planted (d U[8,64], 1-20 cross "
                       "edges); every request a distinct weighted graph (weights U{1..100} drawn per request "
                       "on one of %d seeded topologies); n0=64, 64 GB budget" % (nreq, w0, len(pool)),
           "requests": nreq, "warmup_requests": w0, "timed_requests": nreq - w0, "topologies": len(pool),
           "input_edges_per_request_mean": float(np.mean(m_req)),
           "capacity_req_per_s": round(capacity, 1), "capacity_steps": steps,
           "single_path_capacity_req_per_s": round(single_capacity, 1),
           "capacity_vs_single_path": round(capacity / single_capacity, 2),
           "cuts_equal_single_path": cuts == cut1, "loads": []}
    for load in (0.5, 0.8):
        rate = load * capacity
        arrival = np.cumsum(np.random.default_rng(11).exponential(1.0 / rate, nreq))
        lat, cuts, wall, steps = _serve_run(vc, reqs, sides, arrival, kw, "load %.1f" % load)
        t = 0.0
        lat_single = []
        for a, d in zip(arrival, dur):  # FIFO server running the single path on the same arrivals
            t = max(t, a) + d
            lat_single.append(t - a)
        ls = np.array(lat[w0:]) * 1e3
        lb = np.array(lat_single[w0:]) * 1e3
        span = arrival[-1] - arrival[w0] if nreq > w0 + 1 else wall
        rec = {"load": load, "rate_per_s": round(rate, 1), "steps": steps,
               "p50_ms": round(float(np.percentile(ls, 50)), 3), "p99_ms": round(float(np.percentile(ls, 99)), 3),
               "throughput_req_per_s": round(nreq / wall, 1), "offered_req_per_s": round((nreq - w0 - 1) / span, 1),
               "single_path_fifo_p50_ms": round(float(np.percentile(lb, 50)), 3),
               "single_path_fifo_p99_ms": round(float(np.percentile(lb, 99)), 3),
               "cuts_equal_single_path": cuts == cut1}
        log("served:", rec)
        out["loads"].append(rec)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rhg2p20", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-singles", action="store_true", help="skip the other single-graph workloads")
    ap.add_argument("--no-c3", action="store_true", help="skip the R-MAT single-graph workload")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--no-single-compare", action="store_true",
                    help="skip the batched leg's single-path comparison (keeps a kernel trace to the batch)")
    ap.add_argument("--serve-pool", type=int, default=300, help="distinct generated topologies")
    ap.add_argument("--serve-requests", type=int, default=2000, help="timed requests in the stream")
    ap.add_argument("--serve-warmup", type=int, default=200, help="warm-up requests ahead of the timed ones")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_<kernel>_<workload>.json from two rocprofv3 --pmc passes "
                         "(FETCH_SIZE, WRITE_SIZE) of this benchmark run with --copy-probe, then exit")
    ap.add_argument("--traffic-kernel", default="k_lp_tile")
    ap.add_argument("--traffic-command", default="", help="the profiled command, stored with the record")
    ap.add_argument("--cpu-child", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-budget", type=float, default=10.0, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-runs", type=int, default=5, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_child:
        cpu_child(args.cpu_child, args.cpu_budget, args.cpu_runs)
        return
    if args.record_traffic:
        record_traffic(args.record_traffic[0], args.record_traffic[1], args.traffic_kernel, args.workload,
                       args.traffic_command)
        return
    if args.gpus != 1:
        print("this benchmark runs on one GPU only: the graphs are solved on a single device "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1708_06127_amd as vc

    wl = WORKLOADS[args.workload]
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t0 = time.perf_counter()
    g = make_graph(args.workload)
    log("generated %s: n=%d m=%d in %.1f s" % (args.workload, g.n, g.m, time.perf_counter() - t0))
    dev = to_dev(g)
    ws = vc.workspace(g.n, g.nnz)
    side = torch.empty((g.n + 63) // 64, dtype=torch.int64, device="cuda")
    kw = dict(lp_iters=2, n0=wl["n0"], seed=0, ws=ws, side=side)
    for _ in range(args.warmup):
        cut, _, info = vc.mincut(*dev, **kw)
    torch.cuda.synchronize()
    vc.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cut, _, info = vc.mincut(*dev, **kw)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    prof = vc.profile_read()
    vc.profile_enable(False)
    log("single: %.3f ms/solve, cut %d" % (dt * 1e3, cut))
    out = {
        "metric": "input edges/s to min cut (single vs batched); graphs/s; p50/p99 served latency",
        "value": g.m / dt,
        "unit": "input edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n": g.n, "m": g.m, "n0": wl["n0"], "lp_iters": 2,
                   "cut": cut, "rounds": info["rounds"], "kernel_n": info["kernel_n"]},
        "roofline": roofline(prof, args.workload),
        "sweep": sweep_roofline(prof),
        # launch-shape table in use (the tuner's file beside the library, or the defaults)
        "tuning": [l for l in vc.tuning_get().splitlines() if l.strip()],
    }
    log("roofline:", out["roofline"])
    log("sweep:", out["sweep"])
    m_c2 = g.m
    del ws, dev, g
    torch.cuda.empty_cache()
    if not args.no_singles:
        out["singles"] = bench_singles(vc, args)
        torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = bench_batched(args)
        log("batched:", out["batched"])
        torch.cuda.empty_cache()
    if not args.no_served:
        out["served"] = bench_served(args)
        log("served:", out["served"])
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(m_c2)
        log("cpu baseline:", out["cpu_baseline"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
