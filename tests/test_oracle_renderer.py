"""Pins of the oracle's disk rasteriser and path tracer against values fixed
by construction, geometry and quadrature (nothing here calls the GPU library).

Rasteriser (the plateau tasks of section "Methods", with disks for squares):
  * hand-built images whose every pixel is known by construction: painter's
    order (a later disk covers an earlier one), per-channel colours (C = 1, 3,
    4), the radius read from theta for (cx, cy, r) disks and from the radius
    array for (cx, cy) disks, radii <= 0 never drawn, a pixel centre exactly
    on an edge not covered;
  * the image loss as the mean over H*W*C of (I - T)^2, by hand;
  * the exact smoothed loss of three overlapping RGB disks whose centres and
    radii are all perturbed (noncentral chi-square coverage integrated over
    the radius offset; painter's order makes disk k the top one with
    probability q_k prod_{j>k} (1 - q_j)), its g and H by central differences,
    against the oracle's aggregate and per-element estimates within 5
    standard errors.  The same reference with the painter's order reversed,
    or with the r > 0 rule dropped, moves g by 14 to 200 standard errors.
Path tracer (section "Background", rendering equation):
  * closest hits along rays against the closed-form ray/sphere, ray/plane and
    ray/square distances;
  * the shadow of a sphere under a small light: zero exactly where the
    segment to the light meets the sphere, Lambert's polygon irradiance
    elsewhere;
  * the one-bounce indirect light at a ground point beside a lit sphere:
    the mean over a jittered grid of bounce uniforms against the
    rendering equation's surface-area form integrated over the sphere.
"""
import math

import numpy as np
import pytest

import exact_refs as E
from test_oracle_pt import polygon_irradiance

# ------------------------------------------------------------- hand-built
# 4x4 image: pixel centres at 1/8, 3/8, 5/8, 7/8 (exact in binary)
BASE_COLORS = np.array([[0.1, 0.2, 0.3, 0.4],     # disk 0: covers every centre
                        [0.9, 0.8, 0.7, 0.6],     # disk 1: one pixel only
                        [1.0, 1.0, 1.0, 1.0],     # disk 2: r < 0
                        [0.5, 0.25, 0.75, 0.05]],  # disk 3: r = 0
                       np.float32)
# (cx, cy, r): disk 1 sits on the centre of pixel (x=1, y=2); its radius is
# exactly the pixel pitch, so the four neighbouring centres lie on its edge
HAND_THETA = np.array([0.5, 0.5, 1.0,
                       0.375, 0.625, 0.25,
                       0.5, 0.5, -0.5,
                       0.125, 0.125, 0.0])


def hand_expected(C, small_on_top=True):
    col = BASE_COLORS[:, :C].astype(np.float64)
    img = np.empty((4, 4, C))
    img[:, :] = col[0]
    if small_on_top:
        img[2, 1] = col[1]
    return img


@pytest.mark.parametrize("C", [1, 3, 4])
def test_hand_built_disks_painter_order_and_colours(orc, C):
    cols = BASE_COLORS[:, :C]
    blank = np.zeros((4, 4, C), np.float32)
    # radius argument ignored for (cx, cy, r) disks: garbage must not matter
    sc = orc.Scene.disks(4, 4, C, cols, blank, radius=np.full(4, 5.0, np.float32), ppd=3)
    img = orc.render(sc, HAND_THETA, 4, 4, C)
    assert np.array_equal(img, hand_expected(C))
    # reversed painter's order: the small disk drawn first is hidden
    order = [1, 0, 2, 3]
    th = HAND_THETA.reshape(4, 3)[order].ravel()
    sc_r = orc.Scene.disks(4, 4, C, cols[order], blank, ppd=3)
    assert np.array_equal(orc.render(sc_r, th, 4, 4, C), hand_expected(C, small_on_top=False))


@pytest.mark.parametrize("C", [1, 3])
def test_hand_built_disks_radius_array(orc, C):
    """(cx, cy) disks read disk k's radius from radius[k]."""
    cols = BASE_COLORS[:, :C]
    blank = np.zeros((4, 4, C), np.float32)
    rad = np.array([1.0, 0.25, -0.5, 0.0], np.float32)
    sc = orc.Scene.disks(4, 4, C, cols, blank, radius=rad, ppd=2)
    th = HAND_THETA.reshape(4, 3)[:, :2].ravel()
    assert np.array_equal(orc.render(sc, th, 4, 4, C), hand_expected(C))


def test_nonpositive_radius_never_drawn_even_on_top(orc):
    """A disk of radius -r is not a disk of radius r: on top of everything,
    with its centre on a pixel centre, it still colours nothing."""
    cols = np.array([[0.3], [1.0]], np.float32)
    sc = orc.Scene.disks(4, 4, 1, cols, np.zeros((4, 4, 1), np.float32), ppd=3)
    for r in (-0.3, -1e-9, 0.0):
        img = orc.render(sc, np.array([0.5, 0.5, 1.0, 0.375, 0.375, r]), 4, 4, 1)
        assert np.array_equal(img, np.full((4, 4, 1), np.float32(0.3), np.float64)), r


def test_loss_is_mean_over_pixels_and_channels(orc):
    C = 3
    cols = BASE_COLORS[:, :C]
    c0 = cols[0].astype(np.float64)
    c1 = cols[1].astype(np.float64)
    sc = orc.Scene.disks(4, 4, C, cols, np.zeros((4, 4, C), np.float32), ppd=3)
    want = (15 * (c0 * c0).sum() + (c1 * c1).sum()) / (16 * 3)
    assert orc.loss(sc, HAND_THETA) == pytest.approx(want, rel=1e-15)
    sc1 = orc.Scene.disks(4, 4, C, cols, np.ones((4, 4, C), np.float32), ppd=3)
    want1 = (15 * ((c0 - 1) ** 2).sum() + ((c1 - 1) ** 2).sum()) / (16 * 3)
    assert orc.loss(sc1, HAND_THETA) == pytest.approx(want1, rel=1e-15)


# ------------------------------------------- exact smoothed loss, 3 disks
W3 = H3 = 24
SIG3 = 0.04
THETA3 = np.array([0.40, 0.50, 0.22, 0.62, 0.45, 0.17, 0.30, 0.35, 0.03])
DSTAR3 = np.array([0.02, -0.01, 0.01, -0.015, 0.02, -0.01, 0.01, 0.015, 0.005])
COLS3 = np.array([[0.9, 0.2, 0.1], [0.1, 0.3, 0.95], [0.2, 0.85, 0.3]], np.float32)


def numpy_raster(theta, colors, W, H):
    """Painter's-order disks at pixel centres (the target image only)."""
    xs = (np.arange(W) + 0.5) / W
    ys = (np.arange(H) + 0.5) / H
    X, Y = np.meshgrid(xs, ys)
    img = np.zeros((H, W, colors.shape[1]))
    for k in range(colors.shape[0]):
        cx, cy, r = theta[3 * k:3 * k + 3]
        img[(r > 0) & ((X - cx) ** 2 + (Y - cy) ** 2 < r * r)] = colors[k]
    return img


@pytest.fixture(scope="module")
def three_disks(orc):
    target = numpy_raster(THETA3 + DSTAR3, COLS3, W3, H3).astype(np.float32)
    F, g, Hm = E.disks_exact_fd(THETA3, COLS3.astype(float), target, W3, H3, SIG3, 1e-3)
    sc = orc.Scene.disks(W3, H3, 3, COLS3, target, ppd=3)
    return sc, target, F, g, Hm


def seeds_mean_se(fn, R):
    xs = np.array([fn(1000 + r) for r in range(R)])
    return xs.mean(0), xs.std(0, ddof=1) / math.sqrt(R)


def test_radius_coverage_reference_by_nested_quadrature():
    """The radius-perturbed coverage probability against direct quadrature:
    the radius offset t outside, the 2-D Gaussian over the disk of radius
    r - t inside."""
    from scipy import integrate
    c, r, sg = (0.3, 0.35), 0.03, SIG3
    q = E.disk_cover_prob_r(c, r, W3, H3, sg)
    for p in (int(8.5 * W3 + 7), 0, 9 * W3 + 9, 5 * W3 + 11):
        y, x = divmod(p, W3)
        dx, dy = c[0] - (x + 0.5) / W3, c[1] - (y + 0.5) / H3

        def inner(t):
            rr = r - t
            if rr <= 0:
                return 0.0
            dens = lambda b, a: math.exp(-((dx - a) ** 2 + (dy - b) ** 2) / (2 * sg * sg)) / (2 * math.pi * sg * sg)
            v, _ = integrate.dblquad(dens, -rr, rr, lambda a: -math.sqrt(max(rr * rr - a * a, 0.0)),
                                     lambda a: math.sqrt(max(rr * rr - a * a, 0.0)),
                                     epsabs=1e-13, epsrel=1e-10)
            return v * math.exp(-t * t / (2 * sg * sg)) / (sg * math.sqrt(2 * math.pi))

        val, _ = integrate.quad(inner, -9 * sg, r, epsabs=1e-12, epsrel=1e-9, limit=200)
        assert abs(val - q[p]) < 1e-8 + 1e-6 * val, (x, y, val, q[p])


def test_three_disks_exact_derivatives(orc, three_disks):
    sc, target, F, g, Hm = three_disks
    # the smoothed loss itself: the oracle's mean over plain Gaussian draws
    m, se = seeds_mean_se(lambda s: orc.est_loss(sc, THETA3, SIG3, 4096, s, nthreads=8), 8)
    assert abs(m - F) < 5 * se
    m, se = seeds_mean_se(lambda s: orc.estimate("grad", sc, THETA3, SIG3, 16384, s), 32)
    assert np.all(np.abs(m - g) < 5 * se), ((m - g) / se)
    m, se = seeds_mean_se(lambda s: orc.estimate("hess", sc, THETA3, SIG3, 32768, s), 12)
    assert np.all(np.abs(m - Hm) < 5 * se), ((m - Hm) / se)
    m, se = seeds_mean_se(lambda s: orc.estimate("hess", sc, THETA3, SIG3, 4096, s, sampler=1), 8)
    assert np.all(np.abs(m - Hm) < 5 * se), ((m - Hm) / se)
    # and the reference has teeth: the reversed painter's order moves g far
    # outside these errors
    rev = np.r_[THETA3[6:], THETA3[3:6], THETA3[:3]]
    _, grev, _ = E.disks_exact_fd(rev, COLS3[::-1].astype(float), target, W3, H3, SIG3, 1e-3)
    grev = np.r_[grev[6:], grev[3:6], grev[:3]]
    assert np.abs(grev - g).max() > 0.05


def test_three_disks_fd_step_converged(three_disks):
    """The finite-difference derivatives do not move with the step."""
    sc, target, F, g, Hm = three_disks
    _, g2, H2 = E.disks_exact_fd(THETA3, COLS3.astype(float), target, W3, H3, SIG3, 5e-4)
    assert np.abs(g2 - g).max() < 1e-5
    assert np.abs(H2 - Hm).max() < 1e-3 * np.abs(Hm).max()


# ------------------------------------------------------------ path tracer
def pt_desc(spheres, light_side, Le, ground=(0.5, 0.5, 0.5)):
    """eye, look-at, vfov, light side, Le, ground albedo, then per sphere
    centre (sphere 0's comes from theta), radius, albedo."""
    d = [0.0, 1.6, -3.5, 0.0, 0.3, 0.0, 45.0, light_side, Le, *ground]
    for c, r, alb in spheres:
        d += [*c, r, *alb]
    return np.array(d)


def test_ray_hits_closed_form(orc):
    """Sphere: hit iff the angle to its centre is below asin(R/D), at
    t = D cos a - sqrt(R^2 - D^2 sin^2 a); ground: t = -o_y / d_y; the light
    square: t = (L_y - o_y) / d_y where the hit lies inside the square."""
    R, cen = 0.4, np.array([0.2, 1.0, 0.5])
    light = np.array([-0.3, 2.5, 0.4])
    desc = pt_desc([(cen, R, (0.5, 0.5, 0.5))], light_side=0.6, Le=8.0)
    sc = orc.Scene.pt(8, 8, 1, desc, np.zeros((8, 8, 3), np.float32), nspheres=1)
    theta = np.r_[light, cen]
    g = np.random.default_rng(3)
    o = np.array([0.1, 0.9, -2.5])
    counts = {0: 0, 1: 0, 2: 0, -1: 0}
    for k in range(4000):
        # a third aimed near the sphere, a third near the light, the rest anywhere
        aim = (cen, light, None)[k % 3]
        d = g.standard_normal(3) if aim is None else (aim - o) + 0.5 * g.standard_normal(3)
        d /= np.linalg.norm(d)
        hit, t = orc.pt_trace(sc, theta, o, d)
        oc = cen - o
        D = np.linalg.norm(oc)
        ca = float(d @ oc) / D
        sa2 = max(0.0, 1 - ca * ca)
        cands = []
        if ca > 0 and D * D * sa2 < R * R:
            if abs(D * D * sa2 - R * R) < 1e-9:
                continue   # grazing: either answer is right
            cands.append((D * ca - math.sqrt(R * R - D * D * sa2), 0))
        if d[1] != 0:
            tg = -o[1] / d[1]
            if tg > 0:
                cands.append((tg, 1))
            tl = (light[1] - o[1]) / d[1]
            p = o + tl * d
            if tl > 0:
                ex = max(abs(p[0] - light[0]), abs(p[2] - light[2])) - 0.3
                if abs(ex) < 1e-9:
                    continue
                if ex <= 0:
                    cands.append((tl, 2))
        want, want_t = (-1, None) if not cands else min(cands)[::-1]
        assert hit == want, (d, hit, want)
        counts[want] += 1
        if want >= 0:
            assert t == pytest.approx(want_t, rel=1e-12, abs=1e-12)
    assert min(counts.values()) > 100, counts


def test_shadow_of_sphere_under_small_light(orc):
    """A sphere resting on the ground under a small light: a ground point's
    path radiance (light sampled at the square's centre, bounce straight up)
    is exactly zero where the segment from the point to the light meets the
    sphere, and the ground albedo times the light's polygon irradiance / pi
    elsewhere.  The umbra's edge sits where that segment grazes the sphere."""
    R, cen = 0.3, np.array([0.0, 0.3, 0.0])
    light, side, Le = np.array([0.0, 2.0, 0.0]), 1e-3, 1e6
    alb_g = 0.5
    desc = pt_desc([(cen, R, (0.6, 0.6, 0.6))], light_side=side, Le=Le, ground=(alb_g,) * 3)
    sc = orc.Scene.pt(8, 8, 1, desc, np.zeros((8, 8, 3), np.float32), nspheres=1)
    theta = np.r_[light, cen]
    u = np.array([0.5, 0.5, 0.5, 0.5, 1e-14, 0.3, 0.5, 0.5])
    half = side / 2
    verts = [light + np.array(v) for v in ([-half, 0, -half], [half, 0, -half],
                                          [half, 0, half], [-half, 0, half])]
    nshadow = nlit = 0
    for rho in np.linspace(0.02, 1.2, 119):
        for phi in (0.0, 1.3, 3.9):
            x = np.array([rho * math.cos(phi), 0.0, rho * math.sin(phi)])
            gap = cen[1] - math.sqrt(max(R * R - rho * rho, 0.0)) if rho < R else 0.5
            o = x + np.array([0.0, 0.5 * gap, 0.0])
            L = orc.pt_path(sc, theta, o, np.array([0.0, -1.0, 0.0]), u)
            # segment from the shading point to the light's centre vs the sphere
            p0 = x + np.array([0.0, 1e-4, 0.0])
            seg = light - p0
            s = np.clip((cen - p0) @ seg / (seg @ seg), 0.0, 1.0)
            dist = np.linalg.norm(p0 + s * seg - cen)
            if abs(dist - R) < 1e-6:
                continue
            if dist < R:
                assert np.all(L == 0.0), (rho, phi, L)
                nshadow += 1
            else:
                want = alb_g / math.pi * polygon_irradiance(p0, np.array([0.0, 1.0, 0.0]), verts, Le)
                np.testing.assert_allclose(L, want, rtol=1e-5)
                nlit += 1
    assert nshadow > 40 and nlit > 200
    # the umbra reaches past the sphere's own footprint (radius R) to where
    # the segment grazes it
    rho_star = light[1] * R / math.sqrt((light[1] - R) ** 2 - R * R)
    assert R < rho_star < 0.37


def test_one_bounce_indirect_light_by_surface_quadrature(orc):
    """Indirect light at a ground point beside a lit sphere.  The path's
    bounce term, averaged over a stratified grid of bounce uniforms (light
    points fixed at the squares' centres), against the rendering equation in
    surface-area form over the sphere:
        alb_g / pi * int L_o(p) cos_x cos_p / |x - p|^2 dA_p,
        L_o(p) = alb_s Le cos_p' cos_l A / (pi d^2)  (lit side, else 0)."""
    R, cen = 0.3, np.array([0.0, 0.3, 0.0])
    light, side, Le = np.array([0.2, 2.0, -0.1]), 1e-3, 1e6
    alb_g, alb_s = 0.5, np.array([0.8, 0.4, 0.2])
    desc = pt_desc([(cen, R, tuple(alb_s))], light_side=side, Le=Le, ground=(alb_g,) * 3)
    sc = orc.Scene.pt(8, 8, 1, desc, np.zeros((8, 8, 3), np.float32), nspheres=1)
    theta = np.r_[light, cen]
    x = np.array([0.75, 0.0, 0.2])
    o = x + np.array([0.0, 0.1, 0.0])
    down = np.array([0.0, -1.0, 0.0])
    # the direct term alone: bounce straight up sees the sky
    L_dir = orc.pt_path(sc, theta, o, down, np.array([0.5, 0.5, 0.5, 0.5, 1e-14, 0.0, 0.5, 0.5]))
    # jittered stratification (the sphere's silhouette cuts the grid)
    n = 512
    jit = np.random.default_rng(5).random((n, n, 2))
    acc = np.zeros(3)
    for i in range(n):
        for j in range(n):
            u = np.array([0.5, 0.5, 0.5, 0.5, (i + jit[i, j, 0]) / n, (j + jit[i, j, 1]) / n,
                          0.5, 0.5])
            acc += orc.pt_path(sc, theta, o, down, u)
    indirect_mc = acc / (n * n) - L_dir
    # surface quadrature over the sphere (midpoint rule in (cos polar, azimuth))
    m = 1200
    ct = -1 + (np.arange(m) + 0.5) * (2.0 / m)
    ph = (np.arange(2 * m) + 0.5) * (math.pi / m)
    CT, PH = np.meshgrid(ct, ph, indexing="ij")
    ST = np.sqrt(1 - CT * CT)
    nrm = np.stack([ST * np.cos(PH), CT, ST * np.sin(PH)], -1)
    p = cen + R * nrm
    dA = R * R * (2.0 / m) * (math.pi / m)
    wx = p - x
    dist2 = (wx * wx).sum(-1)
    cos_x = wx[..., 1] / np.sqrt(dist2)
    cos_p = -(nrm * wx).sum(-1) / np.sqrt(dist2)
    wl = light - p
    dl2 = (wl * wl).sum(-1)
    cos_pl = (nrm * wl).sum(-1) / np.sqrt(dl2)
    cos_l = wl[..., 1] / np.sqrt(dl2)
    lit = (cos_pl > 0) & (cos_l > 0)
    Lo = np.where(lit, Le * cos_pl * cos_l * side * side / (math.pi * dl2), 0.0)
    vis = (cos_p > 0) & (cos_x > 0)
    integral = np.where(vis, Lo * cos_x * cos_p / dist2, 0.0).sum() * dA
    want = alb_g / math.pi * alb_s * integral
    assert want.min() > 1e-3 * L_dir.max()   # the bounce term is not negligible
    np.testing.assert_allclose(indirect_mc, want, rtol=2e-3)
