"""Builds matching oracle and library scenes from the seeded workload
descriptions.  Targets always come from the oracle (FP64 render stored as
FP32), so no input of a parity test is produced by the code under test."""
from __future__ import annotations

import numpy as np

import oracle as O
import workloads as WL


def disk_target(w, theta=None):
    th = w.theta_star if theta is None else theta
    blank = np.zeros((w.H, w.W, w.C), np.float32)
    sc0 = O.Scene.disks(w.W, w.H, w.C, w.colors, blank, radius=w.radius, ppd=w.ppd)
    return O.render(sc0, th, w.H, w.W, w.C).astype(np.float32)


def oracle_disks(w, target):
    return O.Scene.disks(w.W, w.H, w.C, w.colors, target, radius=w.radius, ppd=w.ppd)


def gpu_disks(ctx, w, target):
    import paper_2412_03489_amd as P
    return P.Scene.disks(ctx, w.W, w.H, w.C, w.colors, target, radius=w.radius, ppd=w.ppd)


def pt_target(w, spp=None, W=None, H=None):
    W = W or w.W
    H = H or w.H
    sc0 = O.Scene.pt(W, H, w.spp, w.desc, np.zeros((H, W, 3), np.float32))
    return O.render(sc0, w.theta_star, H, W, 3, seed=w.target_seed, s=0,
                    spp=spp or w.target_spp).astype(np.float32)


def rel_inf(x, ref):
    x = np.asarray(x, float)
    ref = np.asarray(ref, float)
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))


def small_disks(W=50, H=37, D=70, C=3, seed=21):
    """A ragged scene: image sides not multiples of the tile, more disks than a
    wavefront has lanes, some radii that go negative under perturbation."""
    g = np.random.default_rng(seed)
    cxy = g.uniform(0.0, 1.0, size=(D, 2)).astype(np.float32)
    r = g.uniform(0.005, 0.12, size=D).astype(np.float32)
    col = g.uniform(0, 1, size=(D, C)).astype(np.float32)
    ts = np.stack([cxy[:, 0], cxy[:, 1], r], 1).reshape(-1).astype(np.float32)
    t0 = (ts + g.uniform(-0.03, 0.03, size=ts.shape).astype(np.float32)).astype(np.float64)
    return WL.DiskWorkload(name="ragged", W=W, H=H, C=C, ppd=3, colors=col, radius=None,
                           theta_star=ts.astype(np.float64), theta0=t0, sigma=0.02, N=96,
                           seed=17, v=g.standard_normal(D * 3))


def assert_losses_match(lgot, lref, tol=1e-6):
    """The library's per-render losses against the oracle's (same draws).
    Paired HVP renders (half as many outputs, see hvp_pairs) hold the loss
    differences f(+h) - f(-h): they are held to 1e-5 of the largest oracle
    difference (plus 1e-12 of the loss scale), the others to `tol` of the
    largest loss."""
    lgot = np.asarray(lgot, float)
    lref = np.asarray(lref, float)
    if lgot.size * 2 == lref.size:
        dref = lref[0::2] - lref[1::2]
        bound = 1e-5 * np.abs(dref).max() + 1e-12 * np.abs(lref).max()
        err = np.abs(lgot - dref).max()
        assert err <= bound, (err, bound)
    else:
        assert lgot.size == lref.size
        assert np.abs(lgot - lref).max() <= tol * max(np.abs(lref).max(), 1e-30)
