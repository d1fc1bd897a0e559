"""Writes the full-size expected values of the GPU parity tests with the CPU
FP64 oracle alone (nothing from the GPU library is imported or run).

Each item is one estimator call of a benchmark workload at its full size,
on the same seeded inputs the GPU tests build (``workloads``; targets are the
oracle's own renders at theta*, stored as FP32):

  disks32_grad      gradient, 256x256 RGB, 32 disks (96 parameters),
                    sigma 0.02, N = 65536 aggregate draws, seed 3
  disks32_hvp       HVP along the workload's v, same query
  disks32_hvp_mg    HVP along -g (g = disks32_grad): the first product of
                    the Newton-CG step below
  disks32_hvp_limit the limit-kernel HVP along the workload's v, same query
  disks32_newton    one Newton-CG step (1 gradient + 10 HVPs, Hessian
                    modification inside CG, trust radius 0.05), seed 3
  pt_hess           full 6x6 Hessian of the path-traced spheres scene,
                    128x128, 4 spp, N = 8192, seed 5
  uneven_<i>        eight of the 64 uneven instances at their full sample
                    budgets (gradient, Hessian and HVP; 60x60 to 318x318)

Sections of the paper: "Gradients", "Hessians", "Hessian-vector product",
"Aggregate" (estimators) and "Previous Work" (Newton-CG).

Usage: python tests/golden/make_golden.py [item ...]   (default: all)
Writes tests/golden/full_<item>.npz; takes about 30 minutes on 8 cores.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402
import workloads as WL  # noqa: E402
from scenes import disk_target, oracle_disks, pt_target  # noqa: E402

UNEVEN = (0, 13, 14, 16, 20, 21, 33, 37)
NEWTON = dict(cg_iters=10, trust_radius=0.05, modified=True)


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def save(name, **kw):
    path = os.path.join(HERE, f"full_{name}.npz")
    np.savez(path, **kw)
    print(f"wrote {path}", flush=True)


def disks32_scene():
    w = WL.disks32()
    tgt = disk_target(w)
    return w, tgt, oracle_disks(w, tgt)


def item_disks32_grad():
    w, tgt, sc = disks32_scene()
    t0 = time.time()
    g = O.estimate("grad", sc, w.theta0, w.sigma, w.N, w.seed)
    save("disks32_grad", out=g, N=w.N, seed=w.seed, sigma=w.sigma,
         inputs=digest(w.theta0, tgt), seconds=time.time() - t0)


def item_disks32_hvp():
    w, tgt, sc = disks32_scene()
    t0 = time.time()
    hv = O.estimate("hvp", sc, w.theta0, w.sigma, w.N, w.seed, v=w.v)
    save("disks32_hvp", out=hv, v=w.v, N=w.N, seed=w.seed, sigma=w.sigma,
         inputs=digest(w.theta0, tgt, w.v), seconds=time.time() - t0)


def item_disks32_hvp_mg():
    w, tgt, sc = disks32_scene()
    g = np.load(os.path.join(HERE, "full_disks32_grad.npz"))["out"]
    t0 = time.time()
    hv = O.estimate("hvp", sc, w.theta0, w.sigma, w.N, w.seed, v=-g)
    save("disks32_hvp_mg", out=hv, v=-g, N=w.N, seed=w.seed, sigma=w.sigma,
         inputs=digest(w.theta0, tgt, -g), seconds=time.time() - t0)


def item_disks32_hvp_limit():
    w, tgt, sc = disks32_scene()
    t0 = time.time()
    hv = O.estimate("hvp_limit", sc, w.theta0, w.sigma, w.N, w.seed, v=w.v)
    save("disks32_hvp_limit", out=hv, v=w.v, N=w.N, seed=w.seed, sigma=w.sigma,
         inputs=digest(w.theta0, tgt, w.v), seconds=time.time() - t0)


def item_disks32_newton():
    w, tgt, sc = disks32_scene()
    t0 = time.time()
    th, rep = O.newton_cg_step(sc, w.theta0, w.sigma, w.N, w.seed, **NEWTON)
    save("disks32_newton", theta=th, iters_done=rep["iters_done"], hit_trust=rep["hit_trust"],
         neg_curv=rep["neg_curv"], step_norm=rep["step_norm"], g_norm=rep["g_norm"],
         N=w.N, seed=w.seed, sigma=w.sigma, inputs=digest(w.theta0, tgt),
         seconds=time.time() - t0)


def item_pt_hess():
    w = WL.pt_spheres()
    tgt = pt_target(w)
    sc = O.Scene.pt(w.W, w.H, w.spp, w.desc, tgt)
    t0 = time.time()
    H = O.estimate("hess", sc, w.theta0, w.sigma, w.N, w.seed)
    save("pt_hess", out=H, N=w.N, seed=w.seed, sigma=w.sigma,
         inputs=digest(w.theta0, tgt), seconds=time.time() - t0)


def item_uneven():
    ws = WL.uneven(64)
    for i in UNEVEN:
        w = ws[i]
        tgt = disk_target(w)
        sc = oracle_disks(w, tgt)
        kind = w.kinds[0]
        t0 = time.time()
        out = O.estimate(kind, sc, w.theta0, w.sigma, w.N, w.seed,
                         v=w.v if kind == "hvp" else None)
        save(f"uneven_{i:03d}", out=out, kind=kind, N=w.N, seed=w.seed, sigma=w.sigma,
             inputs=digest(w.theta0, tgt) if kind != "hvp" else digest(w.theta0, tgt, w.v),
             seconds=time.time() - t0)


ITEMS = {"disks32_grad": item_disks32_grad, "disks32_hvp": item_disks32_hvp,
         "disks32_hvp_mg": item_disks32_hvp_mg, "disks32_hvp_limit": item_disks32_hvp_limit,
         "pt_hess": item_pt_hess,
         "uneven": item_uneven, "disks32_newton": item_disks32_newton}

if __name__ == "__main__":
    O.build(force=False)
    for name in sys.argv[1:] or list(ITEMS):
        print(f"golden {name} ...", flush=True)
        ITEMS[name]()
