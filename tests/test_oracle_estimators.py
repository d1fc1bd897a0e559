"""Pins of the oracle's estimators against closed forms, quadrature and invariants.

Statistical pins compare the mean over R independent seeds with the exact
value, within 5 standard errors measured from the same R estimates.
"""
import json
import math
import os

import numpy as np
import pytest

import exact_refs as E
import workloads as WL

HERE = os.path.dirname(os.path.abspath(__file__))
FACTS = json.load(open(os.path.join(HERE, "golden", "paper_facts.json")))


def seeds_mean_se(fn, R):
    xs = np.array([fn(1000 + r) for r in range(R)])
    return xs.mean(0), xs.std(0, ddof=1) / math.sqrt(R)


def assert_within(mean, se, exact, k=5.0, floor=1e-12):
    mean, se, exact = map(np.asarray, (mean, se, exact))
    bad = np.abs(mean - exact) > k * se + floor
    assert not bad.any(), f"mean={mean}\nexact={exact}\nse={se}"


# --------------------------------------------------------------------- Quad
@pytest.fixture(scope="module")
def quad(orc):
    A = np.array(FACTS["quad_task"]["hessian"])
    return orc.Scene.quad(A, np.array([0.3, -0.2]), 0.7), A, np.array([0.3, -0.2])


def test_quad_task_matrix_matches_paper():
    """a x0^2 + b x1^2 + c x0 x1 = 1/2 x^T A x with A = [[2a, c], [c, 2b]]."""
    f = FACTS["quad_task"]
    A = WL.quad_paper()
    x = np.array([0.3, -1.7])
    assert 0.5 * x @ A @ x == pytest.approx(f["a"] * x[0] ** 2 + f["b"] * x[1] ** 2
                                            + f["c"] * x[0] * x[1])
    assert np.array_equal(A, np.array(f["hessian"]))


@pytest.mark.parametrize("sampler", [0, 1, 2])
def test_quad_gradient_unbiased(orc, quad, sampler):
    sc, A, b = quad
    th = np.array([0.4, -0.9])
    g_ex, _ = E.quad_exact(A, b, th)
    m, se = seeds_mean_se(lambda s: orc.estimate("grad", sc, th, 0.5, 2000, s, sampler=sampler), 12)
    assert_within(m, se, g_ex)


@pytest.mark.parametrize("sampler", [0, 1, 2])
def test_quad_hessian_unbiased(orc, quad, sampler):
    sc, A, b = quad
    th = np.array([0.4, -0.9])
    m, se = seeds_mean_se(lambda s: orc.estimate("hess", sc, th, 0.5, 3000, s, sampler=sampler), 12)
    assert_within(m, se, A)


@pytest.mark.parametrize("sampler", [0, 1])
def test_quad_hvp_unbiased(orc, quad, sampler):
    sc, A, b = quad
    th = np.array([0.4, -0.9])
    v = np.array([1.5, 0.5])
    m, se = seeds_mean_se(lambda s: orc.estimate("hvp", sc, th, 0.5, 2000, s, v=v,
                                                 sampler=sampler), 12)
    assert_within(m, se, A @ v)


def test_quad_hessian_n2_mixture_unbiased(orc, quad):
    """The n^2 aggregate mixture (section "Aggregate") is unbiased too: its
    density counts every off-diagonal element twice, matching how often it is
    drawn; the Hessian of a quadratic is A at any sigma."""
    sc, A, b = quad
    th = np.array([0.4, -0.9])
    m, se = seeds_mean_se(lambda s: orc.estimate("hess", sc, th, 0.5, 3000, s,
                                                 hess_mix_n2=True), 12)
    assert_within(m, se, A)
    v = np.array([1.5, 0.5])
    m, se = seeds_mean_se(lambda s: orc.estimate("hvp_limit", sc, th, 0.5, 3000, s, v=v,
                                                 hess_mix_n2=True), 12)
    assert_within(m, se, A @ v)


def test_n2_mixture_reduces_to_unique_mixture_for_one_parameter(orc):
    """n = 1: one element, n^2 = n(n+1)/2 = 1, so both mixtures are the same
    draws and weights."""
    sc = orc.Scene.quad(np.array([[3.0]]), np.array([0.5]), 0.0)
    a = orc.estimate("hess", sc, [0.2], 0.3, 500, 6)
    b = orc.estimate("hess", sc, [0.2], 0.3, 500, 6, hess_mix_n2=True)
    assert np.array_equal(a, b)


def test_quad_hvp_limit_unbiased(orc, quad):
    sc, A, b = quad
    th = np.array([0.4, -0.9])
    v = np.array([1.5, 0.5])
    m, se = seeds_mean_se(lambda s: orc.estimate("hvp_limit", sc, th, 0.5, 3000, s, v=v), 12)
    assert_within(m, se, A @ v)


def test_antithetic_halves_render_cost_contract(orc, quad):
    """Render counts follow the paper's table (x2 antithetic, x2 for the
    central-difference HVP); IS over the Hessian uses the n(n+1)/2 unique
    elements (the symmetry remark in section "Hessians")."""
    sc, _, _ = quad
    n = 2
    for kind, sampler, expect in [("grad", 0, 1), ("grad", 1, n), ("hess", 0, 1),
                                  ("hess", 1, n * (n + 1) // 2), ("hvp", 0, 2), ("hvp", 1, 2 * n),
                                  ("hvp_limit", 0, 1), ("grad", 2, 1)]:
        _, losses = orc.estimate(kind, sc, [0.1, 0.2], 0.3, 16, 5, v=[1.0, 0.0],
                                 sampler=sampler, return_losses=True)
        assert losses.size == expect * 16 * FACTS["antithetic"]["factor"]


def test_constant_function_gives_zero_antithetic_gradient(orc):
    sc = orc.Scene.quad(np.zeros((3, 3)), np.zeros(3), 2.5)
    for sampler in (0, 1, 2):
        g = orc.estimate("grad", sc, [0.1, -0.3, 2.0], 0.2, 500, 3, sampler=sampler)
        assert np.array_equal(g, np.zeros(3))


def test_hessian_symmetric_and_zero_v(orc, quad):
    sc, _, _ = quad
    H = orc.estimate("hess", sc, [0.2, 0.1], 0.4, 300, 9)
    assert np.array_equal(H, H.T)
    hv = orc.estimate("hvp", sc, [0.2, 0.1], 0.4, 300, 9, v=[0.0, 0.0])
    assert np.array_equal(hv, np.zeros(2))


def test_prefix_property(orc, quad):
    """Counter-based draws: the first N' renders of an N-run are the N'-run's."""
    sc, _, _ = quad
    _, l_small = orc.estimate("grad", sc, [0.2, 0.1], 0.4, 64, 9, return_losses=True)
    _, l_big = orc.estimate("grad", sc, [0.2, 0.1], 0.4, 256, 9, return_losses=True)
    assert np.array_equal(l_small, l_big[: l_small.size])
    # a sub-range starting at s0 reproduces the middle of the big run
    _, l_mid = orc.estimate("grad", sc, [0.2, 0.1], 0.4, 64, 9, s0=64, return_losses=True)
    assert np.array_equal(l_mid, l_big[128:256])


def test_thread_count_does_not_change_result(orc, quad):
    sc, _, _ = quad
    a = orc.estimate("hess", sc, [0.2, 0.1], 0.4, 999, 4, nthreads=1)
    b = orc.estimate("hess", sc, [0.2, 0.1], 0.4, 999, 4, nthreads=7)
    assert np.array_equal(a, b)


def test_rmse_shrinks_as_inverse_sqrt_n(orc, quad):
    """Section "How much variance is reduced?": estimators converge linearly in
    log-log; the Monte Carlo slope is -1/2."""
    sc, A, b = quad
    th = np.array([0.4, -0.9])
    g_ex, _ = E.quad_exact(A, b, th)
    Ns = [128, 512, 2048, 8192]
    rmse = []
    for N in Ns:
        errs = [orc.estimate("grad", sc, th, 0.5, N, 500 + s) - g_ex for s in range(24)]
        rmse.append(math.sqrt(np.mean(np.square(errs))))
    slope = np.polyfit(np.log(Ns), np.log(rmse), 1)[0]
    assert slope == pytest.approx(-0.5, abs=0.12)


def test_ais_variance_between_optimal_and_plain(orc):
    """Section "How much variance is reduced?": aggregate sampling is somewhat
    worse than per-element IS and much better than plain Gaussian sampling.
    Checked for the Hessian of a half-plane scene at its edge."""
    W = 64
    tgt = np.zeros((1, W, 1), np.float32)
    sc = orc.Scene.edge(W, 1, 1, tgt)
    th = np.array([0.5])
    var = {}
    for smp in (0, 1, 2):
        xs = [orc.estimate("hess", sc, th, 0.05, 64, 77 + s, sampler=smp)[0, 0] for s in range(200)]
        var[smp] = np.var(xs)
    # n = 1: the aggregate mixture is the single element's density, so AIS and IS
    # have the same variance (different draws); plain sampling is far worse
    assert var[0] == pytest.approx(var[1], rel=0.35)
    assert var[2] > 2.0 * max(var[0], var[1])


# --------------------------------------------------------------- raster pins
def test_halfplane_pixel_closed_form(orc):
    W, sg = 64, 0.05
    ts = 0.5
    xc = (np.arange(W) + 0.5) / W
    tgt = (xc < ts).astype(np.float32).reshape(1, W, 1)
    sc = orc.Scene.edge(W, 1, 1, tgt)
    th = np.array([ts - 0.07])
    F_ex, g_ex, H_ex = E.halfplane_exact(th[0], ts, W, sg)
    m, se = seeds_mean_se(lambda s: orc.estimate("grad", sc, th, sg, 4000, s), 10)
    assert_within(m, se, [g_ex])
    m, se = seeds_mean_se(lambda s: orc.estimate("hess", sc, th, sg, 4000, s, sampler=1), 10)
    assert_within(m, se, [[H_ex]])
    # the smoothed loss itself: Gaussian average of f
    fs = [orc.loss(sc, th - sg * z) for z in np.random.default_rng(0).standard_normal(4000)]
    assert np.mean(fs) == pytest.approx(F_ex, abs=5 * np.std(fs) / math.sqrt(4000))


def test_corner_full_hessian_closed_form(orc):
    W = H_ = 32
    sg = 0.06
    ts = np.array([0.55, 0.45])
    xc = (np.arange(W) + 0.5) / W
    yc = (np.arange(H_) + 0.5) / H_
    tgt = ((xc[None, :] < ts[0]) & (yc[:, None] < ts[1])).astype(np.float32)[..., None]
    sc = orc.Scene.edge(W, H_, 2, tgt)
    th = np.array([0.5, 0.52])
    _, g_ex, H_ex = E.corner_exact(th, ts, W, H_, sg)
    m, se = seeds_mean_se(lambda s: orc.estimate("grad", sc, th, sg, 3000, s), 10)
    assert_within(m, se, g_ex)
    m, se = seeds_mean_se(lambda s: orc.estimate("hess", sc, th, sg, 3000, s, sampler=1), 10)
    assert_within(m, se, H_ex)
    m, se = seeds_mean_se(lambda s: orc.estimate("hess", sc, th, sg, 3000, s, sampler=0), 10)
    assert_within(m, se, H_ex)
    v = np.array([0.6, -0.8])
    m, se = seeds_mean_se(lambda s: orc.estimate("hvp", sc, th, sg, 3000, s, v=v,
                                                 hvp_rel_step=0.05), 10)
    # the central difference carries an O(h^2) bias: h = 0.05 sigma keeps it far below 5 SE
    assert_within(m, se, H_ex @ v)


@pytest.fixture(scope="module")
def one_disk(orc):
    w = WL.one_disk()
    blank = np.zeros((w.H, w.W, 1), np.float32)
    sc0 = orc.Scene.disks(w.W, w.H, 1, w.colors, blank, radius=w.radius, ppd=2)
    tgt = orc.render(sc0, w.theta_star, w.H, w.W, 1).astype(np.float32)
    return w, orc.Scene.disks(w.W, w.H, 1, w.colors, tgt, radius=w.radius, ppd=2), tgt


def test_one_disk_target_is_binary_disk(one_disk):
    w, _, tgt = one_disk
    assert set(np.unique(tgt)) == {0.0, 1.0}
    # area ~ pi r^2
    assert tgt.mean() == pytest.approx(math.pi * 0.2**2, rel=0.02)


def test_one_disk_exact_derivatives(orc, one_disk):
    """Quadrature-exact smoothed derivatives of the one-disk scene (noncentral
    chi-square coverage probabilities, contour integrals) against the oracle."""
    w, sc, _ = one_disk
    F_ex, g_ex, H_ex = E.disk_exact(w.theta0, w.theta_star, 0.2, w.W, w.H, w.sigma)
    m, se = seeds_mean_se(lambda s: orc.estimate("grad", sc, w.theta0, w.sigma, 8192, s), 8)
    assert_within(m, se, g_ex)
    assert np.abs(m - g_ex).max() < 0.01
    m, se = seeds_mean_se(lambda s: orc.estimate("hess", sc, w.theta0, w.sigma, 32768, s,
                                                 sampler=1), 8)
    assert_within(m, se, H_ex)
    m, se = seeds_mean_se(lambda s: orc.estimate("hess", sc, w.theta0, w.sigma, 32768, s,
                                                 sampler=0), 8)
    assert_within(m, se, H_ex)


def test_one_disk_at_target_has_zero_gradient_isotropic_hessian():
    F, g, H = E.disk_exact([0.5, 0.5], [0.5, 0.5], 0.2, 64, 64, 0.05)
    assert np.abs(g).max() < 1e-12
    assert H[0, 0] == pytest.approx(H[1, 1], rel=1e-12)
    assert abs(H[0, 1]) < 1e-12


# --------------------------------------------------------- negated Gaussian
def test_neggauss_closed_form(orc):
    s1, sg = 1.0, 0.5
    sc = orc.Scene.neggauss(2, s1)
    for th in ([0.3, -0.4], [1.5, 1.0]):
        th = np.array(th)
        _, g_ex, H_ex = E.neggauss_exact(th, s1, sg)
        m, se = seeds_mean_se(lambda s: orc.estimate("grad", sc, th, sg, 3000, s), 10)
        assert_within(m, se, g_ex)
        m, se = seeds_mean_se(lambda s: orc.estimate("hess", sc, th, sg, 3000, s), 10)
        assert_within(m, se, H_ex)


# ------------------------------------------------------------------ solvers
def test_jacobi_matches_eigh(orc):
    rng = np.random.default_rng(1)
    for n in (1, 2, 5, 12):
        M = rng.standard_normal((n, n))
        M = M + M.T
        ev, V = orc.jacobi_eig(M)
        ref = np.linalg.eigvalsh(M)
        assert np.sort(ev) == pytest.approx(ref, abs=1e-10)
        assert V @ np.diag(ev) @ V.T == pytest.approx(M, abs=1e-10)
        assert V.T @ V == pytest.approx(np.eye(n), abs=1e-10)


def test_newton_cg_on_quadratic_reaches_minimiser(orc):
    A = WL.quad_paper()
    b = np.array([1.0, -2.0])
    th0 = np.array([1.0, 1.0])
    # the constant only adds variance to the Hessian estimate; zero f(th0)
    sc = orc.Scene.quad(A, b, -(0.5 * th0 @ A @ th0 + b @ th0))
    x_star = -np.linalg.solve(A, b)
    th, rep = orc.newton_cg_step(sc, th0, 0.2, 20000, 3, cg_iters=2, trust_radius=10.0)
    assert rep["iters_done"] == 2 and not rep["hit_trust"] and not rep["neg_curv"]
    assert np.linalg.norm(th - x_star) < 0.05 * np.linalg.norm(th0 - x_star)
    th2, rep2 = orc.newton_cg_step(sc, th0, 0.2, 20000, 3, use_full_hessian=True,
                                   trust_radius=10.0)
    assert np.linalg.norm(th2 - x_star) < 0.05 * np.linalg.norm(th0 - x_star)


def test_newton_cg_trust_region_and_negative_curvature(orc):
    """Appendix on non-PSD Hessians: away from the centre the smoothed negated
    Gaussian has a negative-curvature direction; the step stops on the trust
    boundary instead of diverging."""
    sc = orc.Scene.neggauss(2, 1.0)
    th0 = np.array([2.5, 0.1])
    th, rep = orc.newton_cg_step(sc, th0, 0.5, 20000, 5, cg_iters=5, trust_radius=0.3)
    assert rep["neg_curv"] or rep["hit_trust"]
    assert rep["step_norm"] <= 0.3 + 1e-12
    # the step moves toward the minimum at the origin
    assert np.linalg.norm(th) < np.linalg.norm(th0)
    th2, rep2 = orc.newton_cg_step(sc, th0, 0.5, 20000, 5, use_full_hessian=True,
                                   trust_radius=0.3, eig_floor=1e-3)
    assert rep2["step_norm"] <= 0.3 + 1e-12
    assert np.linalg.norm(th2) < np.linalg.norm(th0)


def test_invalid_arguments_rejected(orc, quad):
    sc, _, _ = quad
    with pytest.raises(ValueError):
        orc.estimate("grad", sc, [0.0, 0.0], 0.0, 10, 1)
    with pytest.raises(ValueError):
        orc.estimate("grad", sc, [0.0, 0.0], 0.1, 0, 1)
    with pytest.raises(ValueError):
        orc.estimate("grad", sc, [np.nan, 0.0], 0.1, 10, 1)
    with pytest.raises(ValueError):
        orc.estimate("hvp_limit", sc, [0.0, 0.0], 0.1, 10, 1, v=[1.0, 0.0], sampler=1)
    # the mixture flag takes 0 or 1 only
    import ctypes as C
    o = orc._opts(0, True, 0.1, 1, 0, None)
    o.hess_mix_n2 = 2
    H = np.zeros((2, 2))
    th = np.zeros(2)
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    assert orc.lib().orc_est_hessian(sc.h, dp(th), 0.1, 10, 1, C.byref(o), dp(H)) == -1


def test_modified_cg_equals_steihaug_on_psd_quadratic(orc):
    """With a positive definite H and no truncation the modification never
    triggers, so both CG variants take the same step."""
    A = WL.quad_paper()
    b = np.array([1.0, -2.0])
    th0 = np.array([1.0, 1.0])
    sc = orc.Scene.quad(A, b, -(0.5 * th0 @ A @ th0 + b @ th0))
    a, ra = orc.newton_cg_step(sc, th0, 0.2, 20000, 3, cg_iters=2, trust_radius=10.0)
    m, rm = orc.newton_cg_step(sc, th0, 0.2, 20000, 3, cg_iters=2, trust_radius=10.0,
                               modified=True)
    assert np.array_equal(a, m)
    assert ra == rm


def test_modified_cg_uses_all_products_and_descends(orc):
    """Negated Gaussian away from its centre: negative curvature is met, the
    modified variant keeps iterating (all products used), each step is at most
    Delta long, and the smoothed loss decreases."""
    s1, sg = 1.0, 0.5
    sc = orc.Scene.neggauss(2, s1)
    th0 = np.array([2.5, 0.1])
    th, rep = orc.newton_cg_step(sc, th0, sg, 20000, 5, cg_iters=4, trust_radius=0.2,
                                 modified=True)
    assert rep["iters_done"] == 4
    assert rep["neg_curv"] == 1
    assert rep["step_norm"] <= 4 * 0.2 + 1e-12
    F0, _, _ = E.neggauss_exact(th0, s1, sg)
    F1, _, _ = E.neggauss_exact(th, s1, sg)
    assert F1 < F0


def test_greybox_linear_inner_map_quadratic(orc):
    """Appendix "Grey-box differentials": for a linear inner map y = J x + c
    the composition is exact, so the composite estimates are unbiased for
    J^T (A y + b), J^T A J and J^T A J v."""
    A = WL.quad_paper()
    b = np.array([0.3, -0.2])
    sc = orc.Scene.quad(A, b, 0.1)
    J = np.array([[1.0, 0.5, -0.2], [0.3, -1.0, 0.8]])
    x = np.array([0.2, -0.4, 0.7])
    y = J @ x + np.array([0.05, -0.1])
    vx = np.array([0.4, 1.0, -0.5])
    m, se = seeds_mean_se(lambda s: orc.estimate_greybox("grad", sc, y, J, 0.4, 2000, s), 12)
    assert_within(m, se, J.T @ (A @ y + b))
    m, se = seeds_mean_se(lambda s: orc.estimate_greybox("hess", sc, y, J, 0.4, 2000, s), 12)
    assert_within(m, se, J.T @ A @ J)
    m, se = seeds_mean_se(lambda s: orc.estimate_greybox("hvp", sc, y, J, 0.4, 2000, s, vx=vx), 12)
    assert_within(m, se, J.T @ A @ J @ vx)
    # composition of the same draws: J^T applied to the plain estimate
    g = orc.estimate("grad", sc, y, 0.4, 500, 3)
    assert np.allclose(orc.estimate_greybox("grad", sc, y, J, 0.4, 500, 3), J.T @ g, rtol=1e-13)


def test_fr22_comparator_pins(orc, quad):
    """FR22 blurs only the differentiated dimension (appendix on the gradient
    derivation).  Quadratic: that smoothing only adds a constant, so the
    gradient is exact in expectation.  One dimension: it is the per-element IS
    estimator, draw for draw.  Corner scene: the closed form of the 1-D-smoothed
    derivative (the other edge stays a step)."""
    sc, A, b = quad
    th = np.array([0.4, -0.9])
    g_ex, _ = E.quad_exact(A, b, th)
    m, se = seeds_mean_se(lambda s: orc.estimate("grad", sc, th, 0.5, 2000, s, sampler=orc.FR22), 12)
    assert_within(m, se, g_ex)
    W = 64
    xc = (np.arange(W) + 0.5) / W
    edge = orc.Scene.edge(W, 1, 1, (xc < 0.5).astype(np.float32).reshape(1, W, 1))
    a = orc.estimate("grad", edge, [0.43], 0.05, 777, 8, sampler=orc.FR22)
    bb = orc.estimate("grad", edge, [0.43], 0.05, 777, 8, sampler=orc.IS)
    assert np.array_equal(a, bb)
    Wc = Hc = 32
    ts = np.array([0.55, 0.45])
    xc = (np.arange(Wc) + 0.5) / Wc
    yc = (np.arange(Hc) + 0.5) / Hc
    tgt = ((xc[None, :] < ts[0]) & (yc[:, None] < ts[1])).astype(np.float32)[..., None]
    corner = orc.Scene.edge(Wc, Hc, 2, tgt)
    thc = np.array([0.5, 0.52])
    m, se = seeds_mean_se(lambda s: orc.estimate("grad", corner, thc, 0.06, 3000, s,
                                                 sampler=orc.FR22), 10)
    assert_within(m, se, E.corner_fr22_grad(thc, ts, Wc, Hc, 0.06))
    with pytest.raises(ValueError):
        orc.estimate("hess", sc, th, 0.5, 10, 1, sampler=orc.FR22)


# ------------------------------------------------------ loss and optimiser
def test_smoothed_loss_closed_forms(orc, quad):
    """F(theta) = E f(theta - tau): quadratic f + sigma^2 tr(A)/2; negated
    Gaussian -N(theta; 0, (s1^2 + sigma^2) I); half-plane erf sum; sigma = 0
    is the plain loss."""
    sc, A, b = quad
    th = np.array([0.4, -0.9])
    f0 = 0.5 * th @ A @ th + b @ th + 0.7
    m, se = seeds_mean_se(lambda s: orc.est_loss(sc, th, 0.5, 4000, s), 10)
    assert_within(m, se, f0 + 0.25 * np.trace(A) / 2)
    assert orc.est_loss(sc, th, 0.0, 1, 0) == pytest.approx(f0, rel=1e-14)
    ng = orc.Scene.neggauss(2, 1.0)
    F, _, _ = E.neggauss_exact(th, 1.0, 0.5)
    m, se = seeds_mean_se(lambda s: orc.est_loss(ng, th, 0.5, 4000, s), 10)
    assert_within(m, se, F)
    W = 64
    xc = (np.arange(W) + 0.5) / W
    edge = orc.Scene.edge(W, 1, 1, (xc < 0.5).astype(np.float32).reshape(1, W, 1))
    F, _, _ = E.halfplane_exact(0.43, 0.5, W, 0.05)
    m, se = seeds_mean_se(lambda s: orc.est_loss(edge, [0.43], 0.05, 4000, s), 10)
    assert_within(m, se, F)


def test_optimiser_schedule_and_second_order_advantage(orc, one_disk):
    """Appendix "Hyperparameters": sigma annealed linearly; the second-order
    methods reach the one-disk target far faster than gradient descent (the
    paper's main claim, on its two-parameter plateau task with a disk)."""
    w, sc, _ = one_disk
    common = dict(iters=8, sigma_start=0.1, sigma_end=0.02, ls_iters=4, ls_tol=1e-3,
                  recompute=1, N_loss=512)
    th_n, tr_n = orc.optimize(sc, w.theta0, 1024, 1, method="newton_cg", cg_iters=2,
                              trust_radius=0.1, **common)
    th_g, tr_g = orc.optimize(sc, w.theta0, 1024, 1, method="gd", lr=0.02, **common)
    assert np.allclose(tr_n[:, 0], np.linspace(0.1, 0.02, 8), rtol=1e-14)
    assert np.linalg.norm(th_n - w.theta_star) < 0.01
    assert np.linalg.norm(th_n - w.theta_star) < 0.2 * np.linalg.norm(th_g - w.theta_star)
    # the line search only moves on a decrease of the smoothed loss: alpha in {0, 2^-k}
    for a in tr_n[:, 1]:
        assert a == 0.0 or np.log2(a) == np.round(np.log2(a))


def test_optimiser_recompute_reuses_alpha(orc, quad):
    sc, A, b = quad
    th, tr = orc.optimize(sc, [2.0, -2.0], 2000, 4, iters=6, sigma_start=0.3, sigma_end=0.3,
                          method="gd", lr=0.05, ls_iters=3, ls_tol=0.0, recompute=3,
                          N_loss=2000)
    assert tr[1, 1] == tr[0, 1] and tr[2, 1] == tr[0, 1]
    assert tr[4, 1] == tr[3, 1] and tr[5, 1] == tr[3, 1]


# ------------------------------------- the exact references, pinned twice
def test_disk_coverage_by_dense_quadrature():
    """The one-disk reference's coverage probabilities (noncentral chi-square)
    against direct 2-D quadrature of the Gaussian over the disk, at pixels
    inside, on and outside the disk's edge."""
    from scipy import integrate
    w = WL.one_disk()
    th, r, sg = w.theta0, 0.2, w.sigma
    q = E.disk_coverage_prob(th, r, w.W, w.H, sg)
    g = np.random.default_rng(4)
    picks = g.choice(w.W * w.H, size=24, replace=False)
    for p in picks:
        y, x = divmod(int(p), w.W)
        c = np.array([th[0] - (x + 0.5) / w.W, th[1] - (y + 0.5) / w.H])
        dens = lambda b, a: np.exp(-((c[0] - a) ** 2 + (c[1] - b) ** 2) / (2 * sg * sg)) / (2 * math.pi * sg * sg)
        val, err = integrate.dblquad(dens, -r, r, lambda a: -math.sqrt(r * r - a * a),
                                     lambda a: math.sqrt(r * r - a * a), epsabs=1e-12, epsrel=1e-10)
        assert abs(val - q[p]) < 1e-8 + 1e-7 * abs(val), (x, y, val, q[p])


@pytest.mark.parametrize("scene", ["disk", "corner"])
def test_exact_derivatives_match_finite_differences(scene):
    """The analytic gradient and Hessian of each 2-parameter reference (contour
    integrals for the disk, Gaussian CDF products for the corner) against
    central finite differences of its smoothed loss F."""
    if scene == "disk":
        w = WL.one_disk()
        th0 = np.array(w.theta0)
        Ff = lambda t: E.disk_exact(t, w.theta_star, 0.2, w.W, w.H, w.sigma)
        d = 1e-4
    else:
        th0 = np.array([0.5, 0.52])
        Ff = lambda t: E.corner_exact(t, np.array([0.55, 0.45]), 32, 32, 0.06)
        d = 1e-4
    F0, g, H = Ff(th0)
    e = np.eye(2)
    gfd = np.array([(Ff(th0 + d * e[i])[0] - Ff(th0 - d * e[i])[0]) / (2 * d) for i in range(2)])
    Hfd = np.zeros((2, 2))
    for i in range(2):
        for j in range(2):
            Hfd[i, j] = (Ff(th0 + d * e[i] + d * e[j])[0] - Ff(th0 + d * e[i] - d * e[j])[0]
                         - Ff(th0 - d * e[i] + d * e[j])[0] + Ff(th0 - d * e[i] - d * e[j])[0]) / (4 * d * d)
    # gradients of the FD of F against the analytic derivatives
    np.testing.assert_allclose(gfd, g, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(Hfd, H, rtol=2e-4, atol=1e-4 * np.abs(H).max())
    # and the gradient's own differences against the Hessian
    Hg = np.array([(Ff(th0 + d * e[i])[1] - Ff(th0 - d * e[i])[1]) / (2 * d) for i in range(2)])
    np.testing.assert_allclose(0.5 * (Hg + Hg.T), H, rtol=1e-5, atol=1e-6 * np.abs(H).max())
