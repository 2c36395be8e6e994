"""Launch-shape tuner of the library (run on the GPU).

Some launch shapes change no result, only speed (see viecut_tuning_set in
include/viecut.h): the radix block size threshold, the compaction variant,
the PR short-row variant on batch unions, the split between the two smaller
long-row label-propagation classes, the long-row emission variant and the
numbers of short-row tiles one label-propagation and one emission workgroup
take, and the launch shape of the first label-propagation iteration. The
library keeps one set per size bucket (arcs of the level being worked on).

This tuner measures, for each bucket, a coordinate descent over those
choices on a workload of that size:
  * up to 2^26 arcs: the random hyperbolic graph n = 2^20, average degree 32
    (single solve, n0 = 10,000);
  * up to 2^28 arcs: the R-MAT scale-22 10-core (single solve);
  * beyond: the batch of 4,096 planted-cut graphs (one batched call).
Every candidate's results (cuts, side bitmaps, loop statistics) must equal
the default schedule's; the median of several timed runs decides. The table
is written in the file format the library reads at load time
(viecut_tuning.txt beside libviecut.so).

    python -m paper_1708_06127_amd.autotune --out paper_1708_06127_amd/viecut_tuning.txt
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CANDIDATES = {
    "radix_large_from": [1 << 18, 1 << 20, 1 << 22, 1 << 24, 1 << 30],
    "compact_direct_max": [1 << 16, 1 << 18, 1 << 20, 1 << 22, 1 << 30],
    "pr_merge_tiles": [1 << 12, 1 << 14, 1 << 16, 1 << 30],
    "long_split": [256, 320, 384, 448, 512, 640, 768],
    "emit_wave": [0, 1],
    "lp_group": [1, 2, 3, 4],
    "emit_group": [1, 2],
    "first_group": [1, 2],
    "huge_part": [0, 1],
}
DEFAULTS = {"radix_large_from": 1 << 22, "compact_direct_max": 1 << 20, "pr_merge_tiles": 16384,
            "long_split": 512, "emit_wave": 1, "lp_group": 2, "emit_group": 2,
            "first_group": 1, "huge_part": 1}


def log(*a):
    print("#", *a, file=sys.stderr, flush=True)


def median(xs):
    s = sorted(xs)
    k = len(s)
    return s[k // 2] if k % 2 else 0.5 * (s[k // 2 - 1] + s[k // 2])


def to_dev(g):
    import numpy as np
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda() for a in (g.row_ptr, g.col, g.w)]


class Single:
    """One graph through the single path: the runner returns its result key."""

    def __init__(self, vc, g, n0, reps):
        import torch
        self.vc, self.reps = vc, reps
        self.dev = to_dev(g)
        self.ws = vc.workspace(g.n, g.nnz)
        self.side = torch.empty((g.n + 63) // 64, dtype=torch.int64, device="cuda")
        self.kw = dict(lp_iters=2, n0=n0, seed=0, ws=self.ws, side=self.side)
        self.m = g.m

    def run(self):
        """(seconds, result key) of one solve; the key is read after the clock stops"""
        import torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cut, side, info = self.vc.mincut(*self.dev, **self.kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt, (cut, bytes(side.cpu().numpy().tobytes()), info["rounds"], info["kernel_n"],
                    info["witness_level"], info["status"])


class Batch:
    def __init__(self, vc, gs, reps):
        import torch
        self.vc, self.reps = vc, reps
        self.dev = [to_dev(g) for g in gs]
        p = vc.params(lp_iters=2, n0=64, seed=0)
        self.ws = torch.empty(vc.batch_workspace_bytes(self.dev, p), dtype=torch.uint8, device="cuda")
        self.sides = [torch.empty(max((g.n + 63) // 64, 1), dtype=torch.int64, device="cuda") for g in gs]
        self.m = sum(g.m for g in gs)

    def run(self):
        import torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = self.vc.mincut_batch(self.dev, lp_iters=2, n0=64, seed=0, ws=self.ws, sides=self.sides)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt, tuple((r[0], r[2]["rounds"], r[2]["kernel_n"], r[2]["witness_level"], r[2]["status"],
                          bytes(s.cpu().numpy().tobytes())) for r, s in zip(res, self.sides))


def timed(w, reps):
    times = []
    key = None
    for _ in range(reps):
        dt, k = w.run()
        times.append(dt)
        if key is None:
            key = k
        elif k != key:
            raise RuntimeError("results changed between runs of one schedule")
    return median(times), key


def tune_bucket(vc, bound, work, reps):
    """Coordinate descent over the choices for one bucket; returns the chosen
    values and the measurements."""
    work.run()  # warm-up
    base_t, base_key = timed(work, reps)
    chosen = dict(DEFAULTS)
    best_t = base_t
    trials = []
    for key, values in CANDIDATES.items():
        for v in values:
            if v == chosen[key]:
                continue
            vc.tuning_set(bound, key, v)
            work.run()
            t, k = timed(work, reps)
            if k != base_key:
                raise RuntimeError("schedule %s=%d changed a result" % (key, v))
            trials.append({"key": key, "value": v, "ms": round(t * 1e3, 3)})
            log("bucket %d: %s=%d -> %.3f ms (best %.3f)" % (bound, key, v, t * 1e3, best_t * 1e3))
            if t < best_t * 0.985:  # a clear gain only
                best_t = t
                chosen[key] = v
        vc.tuning_set(bound, key, chosen[key])
    return chosen, {"default_ms": round(base_t * 1e3, 3), "tuned_ms": round(best_t * 1e3, 3), "trials": trials}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "viecut_tuning.txt"))
    ap.add_argument("--report", default=None, help="also write the measurements as JSON here")
    ap.add_argument("--batch-count", type=int, default=4096)
    args = ap.parse_args()
    import graphgen as gg
    import paper_1708_06127_amd as vc
    vc.tuning_clear()  # start from the defaults, whatever file is installed
    report = {}
    plan = [
        (1 << 26, "random hyperbolic graph n=2^20 avg deg 32 (single)", lambda: Single(vc, gg.c2_rhg(), 10000, 9)),
        (1 << 28, "R-MAT scale 22 10-core (single)", lambda: Single(vc, gg.c3_rmat(), 10000, 7)),
        (-1, "%d planted-cut graphs (batched)" % args.batch_count,
         lambda: Batch(vc, gg.c4_batch(args.batch_count), 3)),
    ]
    for bound, name, make in plan:
        log("bucket %d: %s" % (bound, name))
        work = make()
        for k, v in DEFAULTS.items():
            vc.tuning_set(bound, k, v)
        chosen, meas = tune_bucket(vc, bound, work, work.reps)
        report[str(bound)] = {"workload": name, "chosen": chosen, **meas}
        log("bucket %d: default %.3f ms -> tuned %.3f ms %s" % (bound, meas["default_ms"], meas["tuned_ms"], chosen))
        del work
    text = vc.tuning_get().splitlines()
    with open(args.out, "w") as f:
        f.write("# Launch-shape table written by paper_1708_06127_amd/autotune.py on an MI355X:\n")
        for bound, r in report.items():
            f.write("#   bucket %s (%s): default %.3f ms, tuned %.3f ms\n" % (bound, r["workload"], r["default_ms"],
                                                                            r["tuned_ms"]))
        for line in text:
            if line.startswith("bucket"):
                f.write(line + "\n")
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)
    print(json.dumps({b: {k: r[k] for k in ("workload", "chosen", "default_ms", "tuned_ms")}
                      for b, r in report.items()}))


if __name__ == "__main__":
    main()
