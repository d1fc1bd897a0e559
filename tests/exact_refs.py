"""Exact smoothed losses and derivatives used to pin the oracle.

Everything here is a closed form or a quadrature derived from the definition
of the smoothed loss F(theta) = E_{tau ~ N(0, sigma^2 I)} f(theta - tau)
(section "Background", convolution with a Gaussian kernel) -- independent of
the Monte Carlo estimators being checked.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import stats


# ---------------------------------------------------------------- quadratic
def quad_exact(A, b, theta):
    """f = 1/2 x^T A x + b^T x: smoothing adds a constant, so grad = A theta + b, H = A."""
    A = np.asarray(A, float)
    return A @ theta + (0 if b is None else b), A.copy()


# ---------------------------------------------------------- negated Gaussian
def neggauss_exact(theta, s1, sigma):
    """f = -N(theta; 0, s1^2 I): the convolution with N(0, sigma^2 I) is
    -N(theta; 0, (s1^2 + sigma^2) I) (appendix on non-PSD Hessians)."""
    theta = np.asarray(theta, float)
    n = theta.size
    s2 = s1 * s1 + sigma * sigma
    G = (2 * math.pi * s2) ** (-n / 2) * math.exp(-theta @ theta / (2 * s2))
    F = -G
    g = theta / s2 * G
    H = -(np.outer(theta, theta) / s2**2 - np.eye(n) / s2) * G
    return F, g, H


# ------------------------------------------------------- half-plane / corner
def halfplane_exact(theta, theta_star, W, sigma):
    """Image 1 where the pixel centre x_c < theta.  With tau ~ N(0, s^2),
    P(x_c < theta - tau) = Phi((theta - x_c)/s); the pixel loss is that
    probability where the target is 0 and its complement where it is 1."""
    xc = (np.arange(W) + 0.5) / W
    a = (theta - xc) / sigma
    T = (xc < theta_star).astype(float)
    Phi, phi = stats.norm.cdf(a), stats.norm.pdf(a)
    sgn = 1 - 2 * T
    F = np.mean(T + sgn * Phi)
    g = np.mean(sgn * phi / sigma)
    H = np.mean(sgn * (-a * phi) / sigma**2)
    return F, g, H


def corner_exact(theta, theta_star, W, H_, sigma):
    """Image 1 where x_c < theta_0 and y_c < theta_1.  Independent tau_0, tau_1
    make the coverage probability Phi(a) Phi(b); binary images give
    (I - T)^2 = I + T - 2 I T, so E = T + (1 - 2T) Phi(a) Phi(b)."""
    xc = (np.arange(W) + 0.5) / W
    yc = (np.arange(H_) + 0.5) / H_
    a = (theta[0] - xc[None, :]) / sigma
    b = (theta[1] - yc[:, None]) / sigma
    T = ((xc[None, :] < theta_star[0]) & (yc[:, None] < theta_star[1])).astype(float)
    sgn = 1 - 2 * T
    Pa, pa = stats.norm.cdf(a), stats.norm.pdf(a)
    Pb, pb = stats.norm.cdf(b), stats.norm.pdf(b)
    F = np.mean(T + sgn * Pa * Pb)
    g = np.array([np.mean(sgn * pa * Pb) / sigma, np.mean(sgn * Pa * pb) / sigma])
    h00 = np.mean(sgn * (-a * pa) * Pb) / sigma**2
    h11 = np.mean(sgn * Pa * (-b * pb)) / sigma**2
    h01 = np.mean(sgn * pa * pb) / sigma**2
    return F, g, np.array([[h00, h01], [h01, h11]])


# ----------------------------------------------------------------- one disk
def disk_coverage_prob(theta, r, W, H_, sigma):
    """q_p = P(|c_p - tau| < r), c_p = theta - x_p, for every pixel centre x_p
    (row-major): a noncentral chi-square CDF with 2 degrees of freedom."""
    theta = np.asarray(theta, float)
    xs = (np.arange(W) + 0.5) / W
    ys = (np.arange(H_) + 0.5) / H_
    X, Y = np.meshgrid(xs, ys)
    cx = (theta[0] - X).ravel()
    cy = (theta[1] - Y).ravel()
    return stats.ncx2.cdf(r * r / sigma**2, 2, (cx * cx + cy * cy) / sigma**2)


def disk_exact(theta, theta_star, r, W, H_, sigma, nodes=2048):
    """One white disk of radius r on black, single channel.  Pixel p is covered
    iff tau lies in the disk B(c_p, r), c_p = theta - x_p, so
    q_p = P(|c_p - tau| < r) is a noncentral chi-square CDF.  Derivatives move
    the disk: grad q_p = contour integral of N_s(c_p + r n) n ds and
    d_j d_i q_p = contour integral of -(c_p + r n)_j / s^2 N_s(c_p + r n) n_i ds
    (divergence theorem), evaluated by the trapezoid rule (periodic, smooth)."""
    theta = np.asarray(theta, float)
    xs = (np.arange(W) + 0.5) / W
    ys = (np.arange(H_) + 0.5) / H_
    X, Y = np.meshgrid(xs, ys)
    T = ((X - theta_star[0]) ** 2 + (Y - theta_star[1]) ** 2 < r * r).astype(float).ravel()
    cx = (theta[0] - X).ravel()
    cy = (theta[1] - Y).ravel()
    q = stats.ncx2.cdf(r * r / sigma**2, 2, (cx * cx + cy * cy) / sigma**2)
    t = np.arange(nodes) * (2 * math.pi / nodes)
    nx, ny = np.cos(t), np.sin(t)
    px = cx[:, None] + r * nx[None, :]
    py = cy[:, None] + r * ny[None, :]
    ph = np.exp(-(px * px + py * py) / (2 * sigma**2)) / (2 * math.pi * sigma**2)
    ds = r * 2 * math.pi / nodes
    gq = np.stack([(ph * nx).sum(1) * ds, (ph * ny).sum(1) * ds], axis=1)
    Hq = np.zeros((cx.size, 2, 2))
    comp = (px, py)
    nrm = (nx, ny)
    for i in range(2):
        for j in range(2):
            Hq[:, i, j] = (-(comp[j]) / sigma**2 * ph * nrm[i][None, :]).sum(1) * ds
    sgn = 1 - 2 * T
    F = np.mean(T + sgn * q)
    g = (sgn[:, None] * gq).mean(0)
    Hm = (sgn[:, None, None] * Hq).mean(0)
    return F, g, 0.5 * (Hm + Hm.T)


def corner_fr22_grad(theta, theta_star, W, H_, sigma):
    """Gradient of the corner scene's loss smoothed along the differentiated
    dimension only (the FR22 comparator): for d/dtheta_0 the y-edge stays a
    step, E = T + (1 - 2T) Phi(a) [y_c < theta_1], and symmetrically."""
    xc = (np.arange(W) + 0.5) / W
    yc = (np.arange(H_) + 0.5) / H_
    a = (theta[0] - xc[None, :]) / sigma
    b = (theta[1] - yc[:, None]) / sigma
    T = ((xc[None, :] < theta_star[0]) & (yc[:, None] < theta_star[1])).astype(float)
    sgn = 1 - 2 * T
    inx = (xc[None, :] < theta[0]).astype(float)
    iny = (yc[:, None] < theta[1]).astype(float)
    g0 = np.mean(sgn * stats.norm.pdf(a) / sigma * iny)
    g1 = np.mean(sgn * inx * stats.norm.pdf(b) / sigma)
    return np.array([g0, g1])


# ------------------------------------------------- disks with radius parameters
def disk_cover_prob_r(c, r, W, H_, sigma, nodes=64):
    """Coverage probability of every pixel centre (row-major) by one disk whose
    centre c and radius r are all perturbed by independent N(0, sigma^2)
    offsets: pixel p is covered iff r - t > 0 and |c - x_p - tau| < r - t, so
        q_p = int phi_sigma(t) ncx2.cdf(((r - t)_+)^2 / sigma^2, 2, |c - x_p|^2 / sigma^2) dt
    (the radius offset t is independent of the centre offset tau).  The t
    integral runs over [-9 sigma, min(r, 9 sigma)] by Gauss-Legendre (above r
    the radius is not positive and nothing is covered)."""
    xs = (np.arange(W) + 0.5) / W
    ys = (np.arange(H_) + 0.5) / H_
    X, Y = np.meshgrid(xs, ys)
    lam = (((c[0] - X) ** 2 + (c[1] - Y) ** 2) / sigma**2).ravel()
    lo, hi = -9.0 * sigma, min(r, 9.0 * sigma)
    if hi <= lo:
        return np.zeros(lam.size)
    z, wz = np.polynomial.legendre.leggauss(nodes)
    t = lo + (hi - lo) * (z + 1) / 2
    wt = wz * (hi - lo) / 2 * np.exp(-t * t / (2 * sigma**2)) / (sigma * math.sqrt(2 * math.pi))
    cdf = stats.ncx2.cdf(((r - t) ** 2 / sigma**2)[None, :], 2, lam[:, None])
    return cdf @ wt


def disks_smoothed_loss(q, colors, target):
    """Exact smoothed MSE of a disk scene in painter's order from per-disk
    coverage probabilities q[k] (P x 1 each) of independently perturbed disks:
    disk k is the top one with probability q_k prod_{j > k} (1 - q_j) and no
    disk covers with probability prod_j (1 - q_j); then
        F = mean over pixels and channels of
            sum_k P(top = k) (c_k - T)^2 + P(none) T^2."""
    T = np.asarray(target, float).reshape(-1, colors.shape[1])
    D = len(q)
    acc = np.zeros(T.shape[0])
    above = np.ones(T.shape[0])   # prod over disks above k of (1 - q_j)
    for k in range(D - 1, -1, -1):
        err = ((colors[k][None, :] - T) ** 2).sum(1)
        acc += q[k] * above * err
        above = above * (1.0 - q[k])
    acc += above * (T * T).sum(1)
    return acc.sum() / T.size


def disks_exact_fd(theta, colors, target, W, H_, sigma, h):
    """F, and g and H by central differences of the exact smoothed loss of a
    scene of disks with (cx, cy, r) parameters (theta interleaved).  A change
    of one disk's parameters changes only that disk's coverage probabilities,
    so each difference recomputes one disk."""
    theta = np.asarray(theta, float)
    D = theta.size // 3
    base = [disk_cover_prob_r(theta[3 * k:3 * k + 2], theta[3 * k + 2], W, H_, sigma)
            for k in range(D)]
    F0 = disks_smoothed_loss(base, colors, target)

    def F_with(changes):
        # changes: {disk: parameter triple}
        q = list(base)
        for k, p in changes.items():
            q[k] = disk_cover_prob_r(p[:2], p[2], W, H_, sigma)
        return disks_smoothed_loss(q, colors, target)

    def shifted(delta):
        ch = {}
        for i, di in delta.items():
            k = i // 3
            p = ch.get(k, theta[3 * k:3 * k + 3].copy())
            p = p.copy()
            p[i % 3] += di
            ch[k] = p
        return F_with(ch)

    n = theta.size
    g = np.array([(shifted({i: h}) - shifted({i: -h})) / (2 * h) for i in range(n)])
    Hm = np.zeros((n, n))
    for i in range(n):
        Hm[i, i] = (shifted({i: h}) - 2 * F0 + shifted({i: -h})) / (h * h)
        for j in range(i + 1, n):
            Hm[i, j] = Hm[j, i] = (shifted({i: h, j: h}) - shifted({i: h, j: -h})
                                   - shifted({i: -h, j: h}) + shifted({i: -h, j: -h})) / (4 * h * h)
    return F0, g, Hm
