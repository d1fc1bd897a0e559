"""Variance analysis of the estimators on the GPU (section "How much variance
is reduced?": every estimator's error falls linearly in a log-log plot; the
aggregate sampler sits between per-element importance sampling and plain
Gaussian sampling).

For each sampler and draw count N the estimate is repeated with R seeds; the
standard deviation across seeds of every element is reported, with the
log-log slope of the mean standard deviation against N (about -1/2 for a Monte
Carlo estimator).  Renders per estimate differ between samplers (per-element
IS makes K times more); `per_render` reports the standard deviation at equal
render counts as well.

    python -m paper_2412_03489_amd.variance            # one-disk scene, gradient and Hessian
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np

from . import AIS, FR22, GAUSS, IS, Context, Scene, estimate, n_renders

NAMES = {AIS: "ais", IS: "is", GAUSS: "gauss", FR22: "fr22"}


def analyse(scene, theta, sigma, kinds=("grad", "hess"), samplers=(AIS, IS, GAUSS),
            Ns=(256, 1024, 4096, 16384), R=16, seed0=1000):
    out = []
    for kind in kinds:
        for smp in samplers:
            if kind == "hess" and smp == FR22:
                continue
            rows = []
            for N in Ns:
                xs = np.array([np.ravel(estimate(kind, scene, theta, sigma, N, seed0 + r,
                                                 sampler=smp)) for r in range(R)])
                sd = xs.std(0, ddof=1)
                renders = n_renders(kind, scene.n, N, smp)
                rows.append({"N": N, "renders": renders, "mean": xs.mean(0).tolist(),
                             "std": sd.tolist(), "mean_std": float(sd.mean()),
                             "std_at_equal_renders": float(sd.mean() * math.sqrt(renders))})
            slope = float(np.polyfit(np.log([r["N"] for r in rows]),
                                     np.log([r["mean_std"] for r in rows]), 1)[0])
            out.append({"kind": kind, "sampler": NAMES[smp], "slope": slope, "rows": rows})
    return out


def main():
    import workloads as WL
    import sys
    ap = argparse.ArgumentParser()
    ap.add_argument("--R", type=int, default=16)
    ap.add_argument("--Ns", type=str, default="256,1024,4096,16384")
    args = ap.parse_args()
    w = WL.one_disk()
    ctx = Context(0)
    blank = np.zeros((w.H, w.W, 1), np.float32)
    s0 = Scene.disks(ctx, w.W, w.H, 1, w.colors, blank, radius=w.radius, ppd=2)
    tgt = s0.render(w.theta_star)
    sc = Scene.disks(ctx, w.W, w.H, 1, w.colors, tgt, radius=w.radius, ppd=2)
    res = analyse(sc, w.theta0, w.sigma, samplers=(AIS, IS, GAUSS, FR22),
                  Ns=tuple(int(x) for x in args.Ns.split(",")), R=args.R)
    for r in res:
        print(f"{r['kind']:5s} {r['sampler']:6s} slope {r['slope']:+.3f}  "
              + "  ".join(f"N={x['N']}: sd={x['mean_std']:.4g}" for x in r["rows"]), file=sys.stderr)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
