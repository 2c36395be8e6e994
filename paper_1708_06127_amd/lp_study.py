"""Quality study of label-propagation configurations (run on the GPU).

In the style of the paper's configuration study (appendix D, the table of
error rates for different numbers of LP iterations): for every instance the
exact minimum cut is computed first (the library with n0 above n, so the
whole graph goes to the exact solve), then each configuration solves the
instance with n0 = 64, and the table reports how many cuts are not optimal
and their relative distance to the optimum.

Configurations: l = 1, 2, 3, 5, 10 iterations; up to 25 iterations with the
convergence stop; l = 2 with the first-iteration restriction; l = 2 with the
correcting step.

Instances (seeded, synthetic): random hyperbolic graphs with 2^10 and 2^11
vertices and average degree 16 and 32 (gamma 5, weights U{1..10}; smaller
than the paper's 2^15 to 2^19 so that the exact solve stays fast), and
planted-cut graphs of 2,000 vertices (average degree 16 and 32, 2 to 12
cross edges), whose planted cut competes with the minimum degree.

    python -m paper_1708_06127_amd.lp_study --out study.json
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

CONFIGS = [
    ("VieCut1", dict(lp_iters=1)),
    ("VieCut2", dict(lp_iters=2)),
    ("VieCut3", dict(lp_iters=3)),
    ("VieCut5", dict(lp_iters=5)),
    ("VieCut10", dict(lp_iters=10)),
    ("VieCut25 (stop)", dict(lp_iters=25, converge=True)),
    ("VieCut2 restricted", dict(lp_iters=2, restrict=True)),
    ("VieCut2 corrected", dict(lp_iters=2, correct=True)),
]


def log(*a):
    print("#", *a, file=sys.stderr, flush=True)


def instances(per_family):
    import graphgen as gg
    out = []
    for n in (1 << 10, 1 << 11):
        for deg in (16.0, 32.0):
            for s in range(per_family):
                out.append(("rhg n=%d d=%g" % (n, deg), lambda n=n, deg=deg, s=s: gg.rhg(n, deg, 5.0, 100 + s, 1, 10)))
    for deg in (16.0, 32.0):
        for s in range(per_family):
            kx = 2 + (s % 6) * 2
            out.append(("planted n=2000 d=%g" % deg, lambda deg=deg, s=s, kx=kx: gg.planted(2000, deg, kx, 1, 1, 200 + s)))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--per-family", type=int, default=10)
    ap.add_argument("--seeds", type=int, default=3, help="method seeds per instance")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch

    import paper_1708_06127_amd as vc
    rows = {name: {"runs": 0, "non_optimal": 0, "excess": []} for name, _ in CONFIGS}
    fams = {}
    t0 = time.perf_counter()
    insts = instances(args.per_family)
    for i, (fam, make) in enumerate(insts):
        g = make()
        dev = [torch.from_numpy(a).cuda() for a in (g.row_ptr, g.col, g.w)]
        lam, _, _ = vc.mincut(*dev, lp_iters=0, n0=g.n + 1)
        deg_min = int(g.degrees().min())
        fams.setdefault(fam, {"instances": 0, "nontrivial": 0})
        fams[fam]["instances"] += 1
        fams[fam]["nontrivial"] += int(lam < deg_min)
        for name, kw in CONFIGS:
            for s in range(args.seeds):
                cut, _, _ = vc.mincut(*dev, n0=64, seed=s, **kw)
                r = rows[name]
                r["runs"] += 1
                if cut != lam:
                    r["non_optimal"] += 1
                    r["excess"].append((cut - lam) / lam)
        if (i + 1) % 10 == 0:
            log("%d/%d instances, %.0f s" % (i + 1, len(insts), time.perf_counter() - t0))
    table = []
    for name, _ in CONFIGS:
        r = rows[name]
        ex = r["excess"]
        table.append({"config": name, "runs": r["runs"], "non_optimal": r["non_optimal"],
                      "mean_excess_non_optimal": round(100 * sum(ex) / len(ex), 2) if ex else 0.0,
                      "mean_excess_all": round(100 * sum(ex) / r["runs"], 3)})
    res = {"families": fams, "table": table, "seconds": round(time.perf_counter() - t0, 1)}
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
