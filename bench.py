"""Benchmark of the min-cut path on one MI355X.

Prints ONE JSON line. The headline `value` is input edges/s of a single
graph solve: one step is one full solve (validation, label propagation,
cluster contraction, Padberg-Rinaldi contraction, bound tracking, exact solve
on the remaining graph, transfer of the side) of one graph already resident
in HBM, with a preallocated workspace. Default workload: the random hyperbolic
graph with n = 2^20, average degree 32, power-law exponent 5, unit weights
(seed 1), n0 = 10,000, two LP iterations, tie-break seed 0.

The same line carries
  * "roofline": the dominant timed kernel (largest summed duration among the
    arc-tile LP kernels), its algorithmic bytes per launch over its average
    event-timed duration during the timed steps, against 8 TB/s;
    "traffic": HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE
    counters, scaled by a copy-kernel calibration, read from
    profiles/traffic_<kernel>_<workload>.json when its recorded source hash
    still matches the kernel source (else null);
  * "cpu_baseline": the oracle (plain C++ implementation used by the tests)
    timed on the host cores on the same graph;
  * "batched": the batch of 4,096 planted-cut graphs (n U{64..8192}, average
    degree U[8,64], weights U{1..100}, 1-20 cross edges) solved in one batched
    execution, against the plain single-graph path on the same graphs;
  * "served": a stream of requests (n log-uniform in [100, 2^20], half RHG,
    half planted, weights U{1..100}, drawn from a generated pool) through a
    session with a 64 GB budget: the capacity with every request queued at
    once, then Poisson arrivals at 50 % and 80 % of it with p50/p99 latency
    from arrival to result, each against a FIFO server running the
    single-graph path on the same arrivals.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
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


def cpu_baseline(g, n0, budget_s=20.0):
    """Time the oracle on the same graph (the whole method, generation and
    I/O excluded), repeating while within the time budget."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        oracle.mincut_graph(g, lp_iters=2, n0=n0, seed=0)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start + times[-1] > budget_s or len(times) >= 5:
            break
    med = sorted(times)[len(times) // 2]
    return {"value": g.m / med, "unit": "input edges/s", "cores": threads, "kind": "oracle",
            "sample": "%d full solve(s) of the same graph, median %.3f s" % (len(times), med)}


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
TIMED_UNITS = {"k_lp_tile": ["k_lp_tile", "k_lp_tile_big"], "k_first_tile": ["k_first_tile"],
               "k_first_tile_level0": ["k_first_tile"]}


def record_traffic(fetch_csv, write_csv, kernel, workload, command):
    """Turn two rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE, in KiB
    per dispatch) of `bench.py --copy-probe` into HBM bytes per launch of
    `kernel`: each counter is scaled by known bytes / reading for the plain
    256 MiB device copy of the same run. Writes
    profiles/traffic_<kernel>_<workload>.json stamped with the kernel source
    hash, which is how the roofline's "traffic" knows it is still current."""
    import csv

    def per_kernel(path, counter):
        copy_best, vals = 0.0, {k: [] for k in TIMED_UNITS.get(kernel, [kernel])}
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"]) * 1024.0
                name = r["Kernel_Name"]
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
    timed = {k: v for k, v in prof.items() if v["launches"] > 0 and v["total_ms"] > 0}
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
    tb = min(times)
    del ws
    out = {"workload": "%d planted-cut graphs, n U{64..8192}, avg deg U[8,64], w U{1..100}, 1-20 cross "
                       "edges (seeds 3..), n0=64" % len(gs),
           "graphs": len(gs), "input_edges": m_total, "ms": round(tb * 1e3, 2),
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
def _serve_run(vc, dev, sides, req, arrival, kw):
    """Real-time session run: request j (graph req[j]) is submitted once the
    clock passes arrival[j]; returns (latencies in s, wall time, steps)."""
    import time as _t
    sess = vc.Session(64 << 30, **kw)
    lat = {}
    i = 0
    steps = 0
    t_start = _t.perf_counter()
    while len(lat) < len(req):
        now = _t.perf_counter() - t_start
        while i < len(req) and arrival[i] <= now:
            sess.submit(i, *dev[req[i]], side=sides[i])
            i += 1
        active = sess.step()
        steps += 1
        t_done = _t.perf_counter() - t_start
        for rid, _, _, _ in sess.poll():
            lat[rid] = t_done - arrival[rid]
        if active == 0 and i < len(req):
            _t.sleep(max(0.0, arrival[i] - (_t.perf_counter() - t_start)))
    wall = _t.perf_counter() - t_start
    sess.close()
    return [lat[j] for j in range(len(req))], wall, steps


def bench_served(args):
    import numpy as np
    import torch
    from concurrent.futures import ThreadPoolExecutor
    import graphgen as gg
    import paper_1708_06127_amd as vc
    ps = gg.c5_request_params(args.serve_pool)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        gs = list(ex.map(gg.c5_make, ps))
    log("generated a pool of %d requests in %.1f s (%d edges)" % (len(gs), time.perf_counter() - t0,
                                                                  sum(g.m for g in gs)))
    dev = [to_dev(g) for g in gs]
    kw = dict(lp_iters=2, n0=64, seed=0)
    rng = np.random.default_rng(4)
    req = rng.integers(0, len(gs), args.serve_requests)
    sides = [torch.empty(max((gs[k].n + 63) // 64, 1), dtype=torch.int64, device="cuda") for k in req]
    # single-path solve time of every pool graph (the FIFO baseline replays them)
    nmax = max(g.n for g in gs)
    amax = max(g.nnz for g in gs)
    ws1 = vc.workspace(nmax, amax)
    side1 = torch.empty((nmax + 63) // 64, dtype=torch.int64, device="cuda")
    dur = []
    for d in dev:
        vc.mincut(*d, ws=ws1, side=side1, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        vc.mincut(*d, ws=ws1, side=side1, **kw)
        torch.cuda.synchronize()
        dur.append(time.perf_counter() - t1)
    del ws1
    log("single-path solve times: mean %.3f ms, max %.3f ms" % (1e3 * np.mean(dur), 1e3 * max(dur)))
    # batched capacity: every request queued at time 0
    _serve_run(vc, dev, sides, req[:16], np.zeros(16), kw)  # warm-up
    _, wall, steps = _serve_run(vc, dev, sides, req, np.zeros(len(req)), kw)
    capacity = len(req) / wall
    single_capacity = len(req) / sum(dur[k] for k in req)
    log("session capacity %.1f req/s (%d steps); single path %.1f req/s" % (capacity, steps, single_capacity))
    out = {"workload": "Poisson stream of %d requests drawn from a pool of %d: n log-uniform [100, 2^20], half "
                       "RHG (gamma 5, avg deg U[16,64]) half planted (d U[8,64], 1-20 cross edges), "
                       "w U{1..100}, n0=64, 64 GB budget" % (len(req), len(gs)),
           "requests": len(req), "capacity_req_per_s": round(capacity, 1),
           "single_path_capacity_req_per_s": round(single_capacity, 1),
           "capacity_vs_single_path": round(capacity / single_capacity, 2), "loads": []}
    for load in (0.5, 0.8):
        rate = load * capacity
        arrival = np.cumsum(np.random.default_rng(11).exponential(1.0 / rate, len(req)))
        lat, wall, steps = _serve_run(vc, dev, sides, req, arrival, kw)
        t = 0.0
        lat_single = []
        for a, k in zip(arrival, req):  # FIFO server running the single path on the same arrivals
            t = max(t, a) + dur[k]
            lat_single.append(t - a)
        ls = np.array(lat) * 1e3
        lb = np.array(lat_single) * 1e3
        rec = {"load": load, "rate_per_s": round(rate, 1), "steps": steps,
               "p50_ms": round(float(np.percentile(ls, 50)), 3), "p99_ms": round(float(np.percentile(ls, 99)), 3),
               "throughput_req_per_s": round(len(req) / wall, 1),
               "single_path_fifo_p50_ms": round(float(np.percentile(lb, 50)), 3),
               "single_path_fifo_p99_ms": round(float(np.percentile(lb, 99)), 3)}
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
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--no-single-compare", action="store_true",
                    help="skip the batched leg's single-path comparison (keeps a kernel trace to the batch)")
    ap.add_argument("--serve-pool", type=int, default=64, help="distinct generated requests")
    ap.add_argument("--serve-requests", type=int, default=256, help="requests in the stream (drawn from the pool)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_<kernel>_<workload>.json from two rocprofv3 --pmc passes "
                         "(FETCH_SIZE, WRITE_SIZE) of this benchmark run with --copy-probe, then exit")
    ap.add_argument("--traffic-kernel", default="k_lp_tile")
    ap.add_argument("--traffic-command", default="", help="the profiled command, stored with the record")
    args = ap.parse_args()
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
    }
    del ws
    if not args.no_batched:
        out["batched"] = bench_batched(args)
        log("batched:", out["batched"])
    if not args.no_served:
        out["served"] = bench_served(args)
        log("served:", out["served"])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, wl["n0"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
