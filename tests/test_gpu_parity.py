"""GPU parity: the HIP library (through its C ABI) against the CPU FP64 oracle
on identical seeded inputs and identical Philox draws.

Bar (stated per test): draws within a few ulp; per-render losses within FP32
rendering error (plus rare pixel-centre edge flips); estimates within 1e-4
relative in the infinity norm over the whole output (rel_inf), the parity
tolerance the build targets for FP32 results; FP64 analytic scenes far tighter.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as WL
from scenes import (assert_losses_match, disk_target, gpu_disks, oracle_disks, pt_target, rel_inf,
                    small_disks)

pytestmark = pytest.mark.gpu
TOL = 1e-4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_2412_03489_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def ctx(P):
    c = P.Context(0)
    yield c
    c.close()


# ------------------------------------------------------------------- draws
@pytest.mark.parametrize("kind,sampler,n2", [("grad", 0, False), ("grad", 1, False),
                                             ("grad", 2, False), ("grad", 3, False),
                                             ("hess", 0, False), ("hess", 1, False),
                                             ("hess", 2, False), ("hess", 0, True)])
def test_draws_match_oracle(P, ctx, kind, sampler, n2):
    n = 4
    A = np.eye(n)
    g_sc = P.Scene.quad(ctx, A)
    N = 300
    say(f"draws {kind} sampler={sampler} n2={n2} n={n} N={N}")
    _, taus = P.estimate(kind, g_sc, np.zeros(n), 0.3, N, 99, sampler=sampler, return_draws=True,
                         hess_mix_n2=n2)
    streams = taus.size // (N * n)
    taus = taus.reshape(streams, N, n)
    for st in range(streams):
        for s in range(0, N, 7):
            ref, _ = O.draw_tau(1 if kind == "hess" else 0, n, 0.3, 99, s, sampler, st,
                                mix_n2=n2)
            np.testing.assert_allclose(taus[st, s], ref, rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------- analytic scenes
@pytest.fixture(scope="module")
def quad_pair(P, ctx):
    g = np.random.default_rng(8)
    M = g.standard_normal((3, 3))
    A = M @ M.T + np.eye(3)
    b = g.standard_normal(3)
    return O.Scene.quad(A, b, 0.4), P.Scene.quad(ctx, A, b, 0.4)


# every kind with every sampler it supports (the limit HVP has no per-element
# IS; that combination's error path is tested with the other argument checks)
KIND_SAMPLERS = [(k, s) for k in ("grad", "hess", "hvp", "hvp_limit") for s in (0, 1, 2)
                 if not (k == "hvp_limit" and s == 1)]


@pytest.mark.parametrize("kind,sampler", KIND_SAMPLERS)
@pytest.mark.parametrize("fp64", [False, True])
def test_quadratic_parity(P, quad_pair, kind, sampler, fp64):
    osc, gsc = quad_pair
    th = np.array([0.3, -0.2, 0.5])
    v = np.array([0.5, 1.0, -2.0])
    N = 1000 + 37   # ragged last chunk
    say(f"quad {kind} sampler={sampler} fp64={fp64}")
    ref = O.estimate(kind, osc, th, 0.4, N, 5, v=v, sampler=sampler)
    got = P.estimate(kind, gsc, th, 0.4, N, 5, v=v, sampler=sampler, accum_fp64=fp64)
    # FP64 throughout; compensated FP32 rounds each contribution to FP32 once
    assert rel_inf(got, ref) < (1e-10 if fp64 else 2e-6)


def test_neggauss_parity(P, ctx):
    osc = O.Scene.neggauss(2, 1.0)
    gsc = P.Scene.neggauss(ctx, 2, 1.0)
    th = np.array([1.2, -0.4])
    for kind in ("grad", "hess", "hvp"):
        say(f"neggauss {kind}")
        ref = O.estimate(kind, osc, th, 0.5, 2000, 3, v=[1.0, 0.5])
        got = P.estimate(kind, gsc, th, 0.5, 2000, 3, v=[1.0, 0.5], accum_fp64=True)
        assert rel_inf(got, ref) < 1e-10


# --------------------------------------------------------- one disk (C1)
@pytest.fixture(scope="module")
def one_disk(P, ctx):
    w = WL.one_disk()
    tgt = disk_target(w)
    return w, oracle_disks(w, tgt), gpu_disks(ctx, w, tgt)


@pytest.mark.parametrize("kind,sampler", [("grad", 0), ("hess", 0), ("grad", 1), ("hess", 1),
                                          ("grad", 2), ("hess", 2), ("grad", 3)])
def test_one_disk_full_size_parity(P, one_disk, kind, sampler):
    """64x64 single disk, N = 4096 draws (the full one-disk workload)."""
    w, osc, gsc = one_disk
    say(f"one_disk {kind} sampler={sampler} N={w.N}")
    ref, lref = O.estimate(kind, osc, w.theta0, w.sigma, w.N, w.seed, sampler=sampler,
                           return_losses=True)
    got, lgot = P.estimate(kind, gsc, w.theta0, w.sigma, w.N, w.seed, sampler=sampler,
                           return_losses=True)
    # coverage is decided exactly (FP32 test, FP64 inside its error band), so
    # the per-render losses differ only by FP32 summation of the pixel errors
    assert np.abs(lgot - lref).max() <= 1e-6 * np.abs(lref).max()
    assert rel_inf(got, ref) < TOL
    got64 = P.estimate(kind, gsc, w.theta0, w.sigma, w.N, w.seed, sampler=sampler,
                       accum_fp64=True)
    assert rel_inf(got64, ref) < TOL
    # the compensated-FP32 lobe sums against FP64 sums of the same GPU losses
    assert rel_inf(got, got64) < 1e-6


def test_one_disk_target_render_parity(P, one_disk):
    w, osc, gsc = one_disk
    img = gsc.render(w.theta0)
    ref = O.render(osc, w.theta0, w.H, w.W, 1).astype(np.float32)
    assert np.array_equal(img, ref)


# ------------------------------------------------------- 32 disks (C2)
@pytest.fixture(scope="module")
def disks32(P, ctx):
    w = WL.disks32()
    tgt = disk_target(w)
    return w, oracle_disks(w, tgt), gpu_disks(ctx, w, tgt)


@pytest.mark.parametrize("kind", ["hvp", "grad", "hvp_limit"])
def test_disks32_parity_reduced_n(P, disks32, kind):
    """256x256 RGB, 32 disks, 96 parameters; N = 64 draws (256 renders for the HVP)."""
    w, osc, gsc = disks32
    N = 64
    say(f"disks32 {kind} N={N}")
    ref, lref = O.estimate(kind, osc, w.theta0, w.sigma, N, w.seed, v=w.v, return_losses=True)
    got, lgot = P.estimate(kind, gsc, w.theta0, w.sigma, N, w.seed, v=w.v, return_losses=True)
    assert_losses_match(lgot, lref)
    assert rel_inf(got, ref) < TOL
    if kind == "hvp":
        # the same HVP with every shifted scene rendered and scored separately
        sep, lsep = P.estimate(kind, gsc, w.theta0, w.sigma, N, w.seed, v=w.v,
                               return_losses=True, hvp_per_render=True)
        assert_losses_match(lsep, lref)
        assert rel_inf(sep, ref) < TOL


def test_disks32_full_size_sampled_renders(P, disks32):
    """At the benchmarked size (N = 65536, 262144 renders, bench launch
    configuration) the oracle recomputes a random sample of renders one by one
    from its own draws; the GPU's first renders equal a short run's (prefix)."""
    w, osc, gsc = disks32
    say(f"disks32 full N={w.N}")
    est, lgot = P.estimate("hvp", gsc, w.theta0, w.sigma, w.N, w.seed, v=w.v, return_losses=True)
    assert np.isfinite(est).all()
    # paired renders: one loss difference f(+h) - f(-h) per (draw, sign)
    assert lgot.size == 2 * w.N
    h = 0.1 * w.sigma
    u = w.v / np.linalg.norm(w.v)
    rng = np.random.default_rng(0)
    idx = np.concatenate([[0, 1, 2, 3, lgot.size - 1], rng.integers(0, lgot.size, 40)])
    for p in idx:
        ai, s = p % 2, p // 2
        tau, _ = O.draw_tau(0, w.n, w.sigma, w.seed, int(s), O.AIS)
        a = 1.0 if ai == 0 else -1.0
        fp = O.loss(osc, (w.theta0 + h * u) - a * tau)
        fm = O.loss(osc, (w.theta0 + (-h) * u) - a * tau)
        assert abs(lgot[p] - (fp - fm)) <= 1e-5 * abs(fp - fm) + 1e-12 * fp, (p, lgot[p], fp - fm)
    _, lshort = P.estimate("hvp", gsc, w.theta0, w.sigma, 64, w.seed, v=w.v, return_losses=True)
    assert np.array_equal(lshort, lgot[: lshort.size])


# ---------------------------------------------------------- ragged scene
def test_ragged_scene_parity(P, ctx):
    """50x37 image (partial tiles), 70 disks (two 64-lane groups), radii that
    cross zero under perturbation."""
    w = small_disks()
    tgt = disk_target(w)
    osc, gsc = oracle_disks(w, tgt), gpu_disks(ctx, w, tgt)
    for kind in ("grad", "hess", "hvp"):
        for N in (1, 96):
            say(f"ragged {kind} N={N}")
            ref, lref = O.estimate(kind, osc, w.theta0, w.sigma, N, w.seed, v=w.v,
                                   return_losses=True)
            got, lgot = P.estimate(kind, gsc, w.theta0, w.sigma, N, w.seed, v=w.v,
                                   return_losses=True)
            assert_losses_match(lgot, lref)
            assert rel_inf(got, ref) < TOL


def test_n2_mixture_parity(P, ctx, quad_pair):
    """The aggregate Hessian mixture over all n^2 ordered pairs: the analytic
    quadratic in FP64, the one-disk scene at full size, a ragged 9-parameter
    disk scene (Hessian and limit HVP) and the small path-traced scene."""
    osc, gsc = quad_pair
    th = np.array([0.3, -0.2, 0.5])
    v = np.array([0.5, 1.0, -2.0])
    for kind in ("hess", "hvp_limit"):
        say(f"n2 quad {kind}")
        ref = O.estimate(kind, osc, th, 0.4, 1037, 5, v=v, hess_mix_n2=True)
        got = P.estimate(kind, gsc, th, 0.4, 1037, 5, v=v, hess_mix_n2=True, accum_fp64=True)
        assert rel_inf(got, ref) < 1e-10
        # a different estimator from the unique-element mixture on the same seed
        other = O.estimate(kind, osc, th, 0.4, 1037, 5, v=v)
        assert rel_inf(other, ref) > 1e-3
    w = WL.one_disk()
    tgt = disk_target(w)
    o1, g1 = oracle_disks(w, tgt), gpu_disks(ctx, w, tgt)
    say(f"n2 one_disk hess N={w.N}")
    ref = O.estimate("hess", o1, w.theta0, w.sigma, w.N, w.seed, hess_mix_n2=True)
    got = P.estimate("hess", g1, w.theta0, w.sigma, w.N, w.seed, hess_mix_n2=True)
    assert rel_inf(got, ref) < TOL
    g1.close()
    w = small_disks(W=45, H=33, D=3, seed=12)
    tgt = disk_target(w)
    o3, g3 = oracle_disks(w, tgt), gpu_disks(ctx, w, tgt)
    for kind in ("hess", "hvp_limit"):
        say(f"n2 small disks {kind} n={w.n} N=200")
        ref, lref = O.estimate(kind, o3, w.theta0, w.sigma, 200, w.seed, v=w.v,
                               hess_mix_n2=True, return_losses=True)
        got, lgot = P.estimate(kind, g3, w.theta0, w.sigma, 200, w.seed, v=w.v,
                               hess_mix_n2=True, return_losses=True)
        assert np.abs(lgot - lref).max() <= 1e-6 * np.abs(lref).max()
        assert rel_inf(got, ref) < TOL
    g3.close()


@pytest.mark.parametrize("C_", [1, 2, 4])
def test_channel_counts(P, ctx, C_):
    w = small_disks(W=40, H=40, D=6, C=C_, seed=3 + C_)
    tgt = disk_target(w)
    osc, gsc = oracle_disks(w, tgt), gpu_disks(ctx, w, tgt)
    say(f"channels C={C_}")
    for sampler in (0, 1):
        ref = O.estimate("grad", osc, w.theta0, w.sigma, 200, 4, sampler=sampler)
        got = P.estimate("grad", gsc, w.theta0, w.sigma, 200, 4, sampler=sampler)
        assert rel_inf(got, ref) < TOL


def test_fixed_radius_disks_is_hessian(P, ctx):
    """params_per_disk = 2 (fixed radii), per-element IS over the Hessian."""
    g = np.random.default_rng(4)
    D = 3
    w = WL.DiskWorkload(name="fixed", W=48, H=48, C=1, ppd=2,
                        colors=np.ones((D, 1), np.float32),
                        radius=g.uniform(0.1, 0.2, D).astype(np.float32),
                        theta_star=g.uniform(0.3, 0.7, 2 * D).astype(np.float32).astype(float),
                        theta0=g.uniform(0.3, 0.7, 2 * D).astype(np.float32).astype(float),
                        sigma=0.05, N=256, seed=9)
    tgt = disk_target(w)
    osc, gsc = oracle_disks(w, tgt), gpu_disks(ctx, w, tgt)
    say("fixed-radius IS Hessian")
    ref = O.estimate("hess", osc, w.theta0, w.sigma, w.N, w.seed, sampler=1)
    got = P.estimate("hess", gsc, w.theta0, w.sigma, w.N, w.seed, sampler=1)
    assert rel_inf(got, ref) < TOL


# ---------------------------------------------------------- path tracer (C3)
@pytest.fixture(scope="module")
def pt_small(P, ctx):
    w = WL.pt_spheres()
    W, H = 32, 24
    tgt = pt_target(w, spp=64, W=W, H=H)
    osc = O.Scene.pt(W, H, 2, w.desc, tgt)
    gsc = P.Scene.pt(ctx, W, H, 2, w.desc, tgt)
    return w, osc, gsc


@pytest.mark.parametrize("kind,sampler", [("hess", 0), ("grad", 0), ("hvp", 0), ("hess", 1)])
def test_pt_small_parity(P, pt_small, kind, sampler):
    w, osc, gsc = pt_small
    N = 24 if sampler == 0 else 6
    say(f"pt_small {kind} sampler={sampler} N={N}")
    v = np.array([1.0, 0.2, -0.5, 0.3, 0.0, 0.7])
    ref, lref = O.estimate(kind, osc, w.theta0, w.sigma, N, w.seed, v=v, sampler=sampler,
                           return_losses=True)
    got, lgot = P.estimate(kind, gsc, w.theta0, w.sigma, N, w.seed, v=v, sampler=sampler,
                           return_losses=True)
    # FP32 path tracing of the same paths: per-render losses agree to ~1e-5
    assert np.abs(lgot - lref).max() <= 2e-5 * np.abs(lref).max()
    assert rel_inf(got, ref) < TOL


def test_pt_small_n2_mixture_parity(P, pt_small):
    w, osc, gsc = pt_small
    say("pt_small hess n2 N=24")
    ref = O.estimate("hess", osc, w.theta0, w.sigma, 24, w.seed, hess_mix_n2=True)
    got = P.estimate("hess", gsc, w.theta0, w.sigma, 24, w.seed, hess_mix_n2=True)
    assert rel_inf(got, ref) < TOL


def test_pt_render_parity(P, pt_small):
    w, osc, gsc = pt_small
    img = gsc.render(w.theta0, seed=3, s=2, spp=8)
    ref = O.render(osc, w.theta0, 24, 32, 3, seed=3, s=2, spp=8)
    diff = np.abs(img - ref)
    # same paths in FP32 and FP64: agreement to FP32 rounding except where a
    # grazing ray or shadow test flips (rare)
    assert (diff > 1e-5).mean() < 0.01
    assert np.median(diff) < 1e-6


def test_pt_full_image_parity(P, ctx):
    """128x128, 4 spp, full 6x6 Hessian by AIS at N = 16 draws."""
    w = WL.pt_spheres()
    tgt = pt_target(w, spp=64)
    osc = O.Scene.pt(w.W, w.H, w.spp, w.desc, tgt)
    gsc = P.Scene.pt(ctx, w.W, w.H, w.spp, w.desc, tgt)
    say("pt full image hess N=16")
    ref, lref = O.estimate("hess", osc, w.theta0, w.sigma, 16, w.seed, return_losses=True)
    got, lgot = P.estimate("hess", gsc, w.theta0, w.sigma, 16, w.seed, return_losses=True)
    assert np.abs(lgot - lref).max() <= 2e-5 * np.abs(lref).max()
    assert rel_inf(got, ref) < TOL


# ---------------------------------------------------------- Newton-CG
def test_newton_cg_step_parity_quadratic(P, quad_pair):
    osc, gsc = quad_pair
    th0 = np.array([1.0, -1.0, 0.5])
    say("newton-cg quadratic")
    for kw in (dict(cg_iters=3, trust_radius=5.0), dict(cg_iters=3, trust_radius=0.05),
               dict(use_full_hessian=True, trust_radius=5.0, eig_floor=1e-3)):
        ref, rr = O.newton_cg_step(osc, th0, 0.3, 4000, 2, **kw)
        got, gr = P.newton_cg_step(gsc, th0, 0.3, 4000, 2, accum_fp64=True, **kw)
        assert rel_inf(got - th0, ref - th0) < 1e-8
        assert gr["iters_done"] == rr["iters_done"]
        assert gr["hit_trust"] == rr["hit_trust"] and gr["neg_curv"] == rr["neg_curv"]


def test_newton_cg_step_parity_one_disk(P, one_disk):
    w, osc, gsc = one_disk
    say("newton-cg one disk")
    ref, rr = O.newton_cg_step(osc, w.theta0, w.sigma, 2048, 1, cg_iters=2, trust_radius=0.2)
    got, gr = P.newton_cg_step(gsc, w.theta0, w.sigma, 2048, 1, cg_iters=2, trust_radius=0.2)
    assert gr["iters_done"] == rr["iters_done"]
    err = rel_inf(got - w.theta0, ref - w.theta0)
    say(f"  step error vs FP64 oracle: rel_inf = {err:.3e}")
    assert err < TOL


def test_newton_cg_modified_parity(P, ctx, disks32):
    """Hessian-modification CG (all products used) on the negated Gaussian and
    on the 32-disk scene at reduced N."""
    osc = O.Scene.neggauss(2, 1.0)
    gsc = P.Scene.neggauss(ctx, 2, 1.0)
    th0 = np.array([2.5, 0.1])
    say("newton-cg modified negated gaussian")
    ref, rr = O.newton_cg_step(osc, th0, 0.5, 4000, 5, cg_iters=4, trust_radius=0.2, modified=True)
    got, gr = P.newton_cg_step(gsc, th0, 0.5, 4000, 5, cg_iters=4, trust_radius=0.2, modified=True,
                               accum_fp64=True)
    for key in ("iters_done", "neg_curv", "hit_trust"):
        assert gr[key] == rr[key], key
    assert rel_inf(got - th0, ref - th0) < 1e-8
    w, osc2, gsc2 = disks32
    say("newton-cg modified disks32 N=64")
    ref, rr = O.newton_cg_step(osc2, w.theta0, w.sigma, 64, w.seed, cg_iters=3, trust_radius=0.05,
                               modified=True)
    got, gr = P.newton_cg_step(gsc2, w.theta0, w.sigma, 64, w.seed, cg_iters=3, trust_radius=0.05,
                               modified=True)
    assert gr["iters_done"] == rr["iters_done"] == 3
    err = rel_inf(got - w.theta0, ref - w.theta0)
    say(f"  step error vs FP64 oracle: rel_inf = {err:.3e}")
    assert err < TOL


def test_newton_cg_negative_curvature_parity(P, ctx):
    osc = O.Scene.neggauss(2, 1.0)
    gsc = P.Scene.neggauss(ctx, 2, 1.0)
    th0 = np.array([2.5, 0.1])
    say("newton-cg negated gaussian")
    ref, rr = O.newton_cg_step(osc, th0, 0.5, 4000, 5, cg_iters=5, trust_radius=0.3)
    got, gr = P.newton_cg_step(gsc, th0, 0.5, 4000, 5, cg_iters=5, trust_radius=0.3,
                               accum_fp64=True)
    assert (gr["neg_curv"], gr["hit_trust"]) == (rr["neg_curv"], rr["hit_trust"])
    assert rel_inf(got - th0, ref - th0) < 1e-8


# ---------------------------------------------------------- loss and optimiser
def test_smoothed_loss_parity(P, one_disk, disks32, pt_small):
    for (w, osc, gsc) in (one_disk, disks32, pt_small):
        say(f"loss {w.name}")
        for sg in (0.0, w.sigma):
            ref = O.est_loss(osc, w.theta0, sg, 256, w.seed)
            got = P.est_loss(gsc, w.theta0, sg, 256, w.seed)
            assert abs(got - ref) <= 2e-5 * abs(ref) + 1e-12, (w.name, sg, got, ref)


@pytest.mark.parametrize("method", ["newton_cg", "newton_full", "gd"])
def test_optimiser_parity(P, one_disk, method):
    """Three iterations of the optimiser loop with sigma annealing and line
    search: the trajectory follows the oracle's."""
    w, osc, gsc = one_disk
    kw = dict(iters=3, sigma_start=0.1, sigma_end=0.05, method=method, lr=0.02, ls_iters=3,
              ls_tol=1e-3, recompute=1, N_loss=256, cg_iters=2, trust_radius=0.1, eig_floor=1.0)
    say(f"optimiser {method}")
    ref, tr_r = O.optimize(osc, w.theta0, 1024, 1, **kw)
    got, tr_g = P.optimize(gsc, w.theta0, 1024, 1, **kw)
    assert np.array_equal(tr_g[:, 1], tr_r[:, 1])          # same line-search decisions
    err = rel_inf(got - w.theta0, ref - w.theta0)
    say(f"  trajectory error vs FP64 oracle: rel_inf = {err:.3e}")
    assert err < TOL
    assert np.allclose(tr_g[:, 3], tr_r[:, 3], rtol=2e-5)


# ---------------------------------------------------------- grey-box
@pytest.mark.parametrize("kind", ["grad", "hess", "hvp"])
def test_greybox_parity(P, ctx, one_disk, kind):
    """Composite derivatives through an inner Jacobian (2 scene parameters from
    3 inner ones) on the one-disk scene."""
    w, osc, gsc = one_disk
    J = np.array([[1.0, 0.5, -0.2], [0.3, -1.0, 0.8]])
    vx = np.array([0.4, 1.0, -0.5])
    say(f"greybox {kind}")
    ref = O.estimate_greybox(kind, osc, w.theta0, J, w.sigma, 2048, w.seed, vx=vx)
    got = P.estimate_greybox(kind, gsc, w.theta0, J, w.sigma, 2048, w.seed, vx=vx)
    assert rel_inf(got, ref) < TOL


# ---------------------------------------------------------- device API
def test_device_pointer_api_matches_host_api(P, ctx, disks32):
    w, _, gsc = disks32
    say("device-pointer API")
    th = ctx.alloc(8 * w.n)
    v = ctx.alloc(8 * w.n)
    out = ctx.alloc(8 * w.n)
    th.upload(w.theta0)
    v.upload(w.v)
    P.estimate_dev("hvp", gsc, th.ptr, w.sigma, 256, w.seed, out.ptr, d_v=v.ptr)
    ctx.synchronize()
    host = P.estimate("hvp", gsc, w.theta0, w.sigma, 256, w.seed, v=w.v)
    assert np.array_equal(out.download(w.n), host)
    P.newton_cg_step_dev(gsc, th.ptr, w.sigma, 256, w.seed, cg_iters=2, trust_radius=0.05)
    hth, _ = P.newton_cg_step(gsc, w.theta0, w.sigma, 256, w.seed, cg_iters=2, trust_radius=0.05)
    assert np.array_equal(th.download(w.n), hth)
    for b in (th, v, out):
        b.free()


# ---------------------------------------------------------- errors and edges
def test_errors_and_edge_cases(P, ctx, quad_pair):
    _, gsc = quad_pair
    th = np.zeros(3)
    with pytest.raises(P.HrError, match="EINVAL"):
        P.estimate("grad", gsc, th, 0.0, 10, 1)
    with pytest.raises(P.HrError, match="EINVAL"):
        P.estimate("grad", gsc, th, 0.1, 0, 1)
    with pytest.raises(P.HrError, match="EINVAL"):
        P.estimate("grad", gsc, [np.nan, 0, 0], 0.1, 10, 1)
    with pytest.raises(P.HrError, match="EINVAL"):
        P.estimate("hvp", gsc, th, 0.1, 10, 1, v=[np.inf, 0, 0])
    with pytest.raises(P.HrError, match="EUNSUPPORTED"):
        P.estimate("hvp_limit", gsc, th, 0.1, 10, 1, v=[1.0, 0, 0], sampler=1)
    with pytest.raises(P.HrError, match="EUNSUPPORTED"):
        P.estimate("hess", gsc, th, 0.1, 10, 1, sampler=3)
    assert np.array_equal(P.estimate("hvp", gsc, th, 0.1, 10, 1, v=np.zeros(3)), np.zeros(3))
    # an option outside its documented values is refused at the boundary
    import ctypes as C
    o = P.make_opts()
    o.hess_mix_n2 = 2
    H = np.zeros((3, 3))
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    assert P.lib().hr_est_hessian(gsc.h, dp(th), 0.1, 10, 1, C.byref(o), dp(H)) == -1   # EINVAL
    o.hess_mix_n2 = 0
    o.raster_tile = 7
    assert P.lib().hr_est_hessian(gsc.h, dp(th), 0.1, 10, 1, C.byref(o), dp(H)) == -1
    c2 = P.Context(0)
    try:
        c2.set_memory_budget(1024)
        s2 = P.Scene.quad(c2, np.eye(3))
        with pytest.raises(P.HrError, match="ENOMEM"):
            P.estimate("grad", s2, th, 0.1, 100000, 1)
        s2.close()
    finally:
        c2.close()
    with pytest.raises(P.HrError, match="EINVAL"):
        P.Scene.disks(ctx, 8, 8, 5, np.ones((1, 5)), np.zeros((8, 8, 5)))
    # a scene outliving its context is orphaned: calls fail cleanly, and the
    # next context's launches are unaffected
    c3 = P.Context(0)
    s3 = P.Scene.quad(c3, np.eye(3))
    c3.close()
    with pytest.raises(P.HrError, match="EINVAL"):
        P.estimate("grad", s3, th, 0.1, 10, 1)
    s3.close()
    assert np.isfinite(P.estimate("grad", gsc, th, 0.1, 10, 1)).all()


def test_newton_step_device_resident_and_graph_replays(P, ctx, disks32):
    """The Newton-CG step runs without a host round trip: after the inner
    loop stops on the device (here a trust-region truncation) the remaining
    products' kernels return at once.  Repeating the step with the same
    arguments runs it eagerly, then captured as a hipGraph, then as replays;
    every run (with eager work between the replays) gives the same bits, and
    the step equals the oracle's."""
    w, osc, gsc = disks32
    N, kw = 4096, dict(cg_iters=6, trust_radius=0.02)
    th0, th = ctx.alloc(8 * w.n), ctx.alloc(8 * w.n)
    th0.upload(w.theta0)
    runs = []
    for k in range(5):
        say(f"newton step run {k}")
        th.copy_from(th0)
        rep = P.newton_cg_step_dev(gsc, th.ptr, w.sigma, N, w.seed, **kw)
        runs.append((th.download(w.n), rep))
        if k >= 2:
            P.estimate("grad", gsc, w.theta0, w.sigma, 512, 7)
    for got, rep in runs[1:]:
        assert np.array_equal(got, runs[0][0])
        assert rep == runs[0][1]
    assert runs[0][1]["hit_trust"] == 1 and runs[0][1]["iters_done"] < kw["cg_iters"]
    ref, rr = O.newton_cg_step(osc, w.theta0, w.sigma, N, w.seed, **kw)
    assert rr["iters_done"] == runs[0][1]["iters_done"]
    err = rel_inf(runs[0][0] - w.theta0, ref - w.theta0)
    say(f"  step error vs FP64 oracle: rel_inf = {err:.3e}")
    assert err < TOL
    # other arguments: a fresh eager run, then the new step is captured
    th.copy_from(th0)
    P.newton_cg_step_dev(gsc, th.ptr, w.sigma, N, w.seed + 1, **kw)
    other = th.download(w.n)
    th.copy_from(th0)
    P.newton_cg_step_dev(gsc, th.ptr, w.sigma, N, w.seed + 1, **kw)
    assert np.array_equal(th.download(w.n), other)
    assert not np.array_equal(other, runs[0][0])
    th0.free()
    th.free()
