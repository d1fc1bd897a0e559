"""Seeded synthetic inputs shared by the tests, the smoke check and bench.py.

This module holds scene *descriptions* only: parameter vectors, colours,
radii, camera and light placement, drawn from numpy generators with fixed
seeds.  It contains none of the estimator's arithmetic and renders nothing;
targets are produced by whichever side needs them (the oracle for parity
tests, the library under test for its own benchmark input).

Values are drawn as float32 and widened to float64 so that both sides see
exactly representable inputs.

Workloads (shapes of the paper's tasks: the one- and five-square plateau
scenes become disk scenes; the path-traced shadow task becomes a sphere/area
light scene):

* ``one_disk``     -- 64x64, 1 channel, one white disk of radius 0.2, theta = (cx, cy),
                      target at (0.5, 0.5), query at (0.35, 0.6), sigma 0.05, N 4096.
* ``disks32``      -- 256x256 RGB, 32 disks with (cx, cy, r) = 96 parameters,
                      sigma 0.02, aggregate-sampled HVP with N 65536, 10 CG products.
* ``pt_spheres``   -- 128x128 RGB path-traced scene (4 diffuse spheres on a plane, one
                      square light), 4 spp, theta = (light xyz, sphere-0 xyz),
                      sigma 0.05, N 8192, full 6x6 Hessian.
* ``uneven``       -- 64 independent disk scenes of uneven size and sample budget.
* ``serving_clients`` -- Poisson arrivals of Newton optimisations over a 50/50 mix of
                      the ``disks32`` and ``pt_spheres`` scenes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def _f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


@dataclass
class DiskWorkload:
    name: str
    W: int
    H: int
    C: int
    ppd: int                 # parameters per disk: 2 (cx, cy) or 3 (cx, cy, r)
    colors: np.ndarray       # D x C float32
    radius: np.ndarray | None  # D float32 when ppd == 2
    theta_star: np.ndarray   # float64 (float32-exact)
    theta0: np.ndarray
    sigma: float
    N: int
    seed: int
    v: np.ndarray | None = None
    cg_iters: int = 10
    kinds: tuple = ("grad", "hess")

    @property
    def D(self):
        return self.colors.shape[0]

    @property
    def n(self):
        return self.D * self.ppd

    @property
    def pixels(self):
        return self.W * self.H


@dataclass
class PTWorkload:
    name: str
    W: int
    H: int
    spp: int
    desc: np.ndarray         # float64 scene description (see pt_desc_layout)
    theta_star: np.ndarray
    theta0: np.ndarray
    sigma: float
    N: int
    seed: int
    target_spp: int = 1024
    target_seed: int = 7
    nspheres: int = 4
    C: int = 3

    @property
    def n(self):
        return 6

    @property
    def pixels(self):
        return self.W * self.H


PT_DESC_LAYOUT = ("eye[3], look_at[3], vfov_deg, light_side, Le, ground_albedo[3], "
                  "then per sphere centre[3], radius, albedo[3]")


def one_disk(N: int = 4096) -> DiskWorkload:
    return DiskWorkload(
        name="one_disk_64x64", W=64, H=64, C=1, ppd=2,
        colors=np.ones((1, 1), dtype=np.float32),
        radius=np.array([0.2], dtype=np.float32),
        theta_star=_f32([0.5, 0.5]), theta0=_f32([0.35, 0.6]),
        sigma=0.05, N=N, seed=0, kinds=("grad", "hess"))


def disks32(N: int = 65536, W: int = 256, H: int = 256) -> DiskWorkload:
    g = np.random.default_rng(2)
    D = 32
    cxy = g.uniform(0.1, 0.9, size=(D, 2)).astype(np.float32)
    r = g.uniform(0.03, 0.1, size=(D,)).astype(np.float32)
    col = g.uniform(0.0, 1.0, size=(D, 3)).astype(np.float32)
    ts = np.stack([cxy[:, 0], cxy[:, 1], r], axis=1).reshape(-1).astype(np.float32)
    g3 = np.random.default_rng(3)
    t0 = (ts + g3.uniform(-0.05, 0.05, size=ts.shape).astype(np.float32)).reshape(D, 3)
    t0[:, 2] = np.maximum(t0[:, 2], np.float32(0.03))
    t0 = t0.reshape(-1).astype(np.float32)
    g4 = np.random.default_rng(4)
    v = g4.standard_normal(D * 3)
    v = (v / np.linalg.norm(v)).astype(np.float32)
    return DiskWorkload(
        name=f"disks32_{W}x{H}_rgb", W=W, H=H, C=3, ppd=3, colors=col, radius=None,
        theta_star=_f32(ts), theta0=_f32(t0), sigma=0.02, N=N, seed=3, v=_f32(v),
        cg_iters=10, kinds=("hvp",))


def pt_spheres(N: int = 8192, W: int = 128, H: int = 128, spp: int = 4) -> PTWorkload:
    g = np.random.default_rng(5)
    ns = 4
    rad = g.uniform(0.2, 0.35, size=ns).astype(np.float32)
    xz = g.uniform(-1.0, 1.0, size=(ns, 2)).astype(np.float32)
    alb = g.uniform(0.2, 0.8, size=(ns, 3)).astype(np.float32)
    desc = [0.0, 1.6, -3.5, 0.0, 0.3, 0.0, 45.0, 0.5, 8.0, 0.5, 0.5, 0.5]
    for i in range(ns):
        desc += [xz[i, 0], rad[i], xz[i, 1], rad[i], alb[i, 0], alb[i, 1], alb[i, 2]]
    desc = _f32(desc)
    ts = _f32([0.0, 2.0, 0.0, desc[12], desc[13], desc[14]])
    t0 = _f32(ts + g.normal(0.0, 0.2, size=6))
    return PTWorkload(name=f"pt_spheres_{W}x{H}_{spp}spp", W=W, H=H, spp=spp, desc=desc,
                      theta_star=ts, theta0=t0, sigma=0.05, N=N, seed=5)


def quad_paper():
    """The paper's quadratic task a x0^2 + b x1^2 + c x0 x1 with a=b=5, c=7.5,
    written as f = 1/2 x^T A x with A = [[2a, c], [c, 2b]]."""
    return np.array([[10.0, 7.5], [7.5, 10.0]])


def uneven(count: int = 64, base_seed: int = 1000):
    """Batch of uneven disk instances: side log-uniform in [32, 512], 1..32 disks
    with (cx, cy, r), sample budget log-uniform in [2^10, 2^16], sigma 0.02;
    instance 0 is the one-disk workload."""
    out = []
    for i in range(count):
        if i == 0:
            w = one_disk()
            w.name = "uneven_000_one_disk"
            out.append(w)
            continue
        g = np.random.default_rng(base_seed + i)
        side = int(round(2 ** g.uniform(5, 9)))
        D = int(g.integers(1, 33))
        cxy = g.uniform(0.1, 0.9, size=(D, 2)).astype(np.float32)
        r = g.uniform(0.03, 0.1, size=(D,)).astype(np.float32)
        col = g.uniform(0.0, 1.0, size=(D, 3)).astype(np.float32)
        ts = np.stack([cxy[:, 0], cxy[:, 1], r], axis=1).reshape(-1).astype(np.float32)
        t0 = (ts + g.uniform(-0.05, 0.05, size=ts.shape).astype(np.float32)).reshape(D, 3)
        t0[:, 2] = np.maximum(t0[:, 2], np.float32(0.03))
        N = int(round(2 ** g.uniform(10, 16)))
        kind = ("grad", "hess", "hvp")[i % 3]
        v = g.standard_normal(D * 3)
        v = (v / np.linalg.norm(v)).astype(np.float32)
        out.append(DiskWorkload(
            name=f"uneven_{i:03d}", W=side, H=side, C=3, ppd=3, colors=col, radius=None,
            theta_star=_f32(ts), theta0=_f32(t0.reshape(-1)), sigma=0.02, N=N,
            seed=base_seed + i, v=_f32(v), kinds=(kind,)))
    return out


@dataclass
class ServingClient:
    """One Newton optimisation arriving at a server: which scene, where it
    starts, its draws' seed and its arrival time (seconds after the start)."""
    scene: str               # "raster" (disks32, 96 params) or "pt" (pt_spheres, 6 params)
    theta0: np.ndarray
    seed: int
    arrival: float


def serving_clients(count: int = 256, rate: float = 512.0, base_seed: int = 2000):
    """Poisson arrivals (rate per second) of `count` Newton optimisations over a
    50/50 mix of the 96-parameter raster scene and the 6-parameter path-traced
    scene; each starts at a random perturbation of its scene's initial theta."""
    g = np.random.default_rng(base_seed)
    gaps = g.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    r0 = disks32().theta0.astype(np.float64)
    p0 = pt_spheres().theta0.astype(np.float64)
    out = []
    for i in range(count):
        if i % 2 == 0:
            th = r0 + g.uniform(-0.01, 0.01, size=r0.shape)
            th[2::3] = np.maximum(th[2::3], 0.03)
            out.append(ServingClient("raster", th, base_seed + i, float(t[i])))
        else:
            out.append(ServingClient("pt", p0 + g.normal(0.0, 0.05, size=6), base_seed + i,
                                     float(t[i])))
    return out

