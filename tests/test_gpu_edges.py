"""Edge cases of the disk path against the oracle on the same draws: a 1x1
image, the maximum disk count, a 4096x4096 image, the render pairs' largest
images (W + H = 2048) and the first size past them, the rasteriser's disk-count
boundaries (32 / 33: two renders per cull or one; 64 / 65: one wavefront of
disks or several), odd render counts, nothing covered (disks outside the
image or with non-positive radii), and extreme sigma.  Bar as in the parity suite: 1e-4
relative (infinity norm) on estimates, per-render losses to FP32 rounding."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as WL
from scenes import assert_losses_match, disk_target, gpu_disks, oracle_disks, rel_inf

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


def make(W, H, D, C=3, seed=0, centre=(0.0, 1.0), radius=(0.03, 0.3), sigma=0.02, jitter=0.03):
    g = np.random.default_rng(seed)
    cxy = g.uniform(centre[0], centre[1], size=(D, 2)).astype(np.float32)
    r = g.uniform(radius[0], radius[1], size=D).astype(np.float32)
    col = g.uniform(0, 1, size=(D, C)).astype(np.float32)
    ts = np.stack([cxy[:, 0], cxy[:, 1], r], 1).reshape(-1).astype(np.float32)
    t0 = (ts + g.uniform(-jitter, jitter, size=ts.shape).astype(np.float32)).astype(np.float64)
    v = g.standard_normal(D * 3)
    return WL.DiskWorkload(name=f"edge_{W}x{H}_{D}", W=W, H=H, C=C, ppd=3, colors=col,
                           radius=None, theta_star=ts.astype(np.float64), theta0=t0,
                           sigma=sigma, N=64, seed=seed + 100, v=v / np.linalg.norm(v))


def check(P, ctx, w, kinds=("grad", "hess", "hvp"), N=None, sampler=0, loss_tol=1e-6,
          antithetic=True, spbs=()):
    tgt = disk_target(w)
    osc, gsc = oracle_disks(w, tgt), gpu_disks(ctx, w, tgt)
    N = N or w.N
    for kind in kinds:
        say(f"{w.name} {kind} N={N} sigma={w.sigma} antithetic={antithetic}")
        ref, lref = O.estimate(kind, osc, w.theta0, w.sigma, N, w.seed, v=w.v, sampler=sampler,
                               antithetic=antithetic, return_losses=True)
        got, lgot = P.estimate(kind, gsc, w.theta0, w.sigma, N, w.seed, v=w.v, sampler=sampler,
                               antithetic=antithetic, return_losses=True)
        for spb in spbs:
            say(f"  samples_per_block={spb}")
            again = P.estimate(kind, gsc, w.theta0, w.sigma, N, w.seed, v=w.v, sampler=sampler,
                               antithetic=antithetic, samples_per_block=spb)
            assert np.array_equal(again, got)
        assert_losses_match(lgot, lref, loss_tol)
        if np.abs(ref).max() == 0.0:
            assert np.abs(got).max() == 0.0
        else:
            assert rel_inf(got, ref) < TOL, (kind, rel_inf(got, ref))
    gsc.close()


def test_one_pixel_image(P, ctx):
    w = make(1, 1, 2, C=1, seed=1, centre=(0.3, 0.7), radius=(0.2, 0.4), sigma=0.1)
    check(P, ctx, w)


@pytest.mark.parametrize("D", [31, 32, 33, 64, 65])
def test_wavefront_group_boundary(P, ctx, D):
    w = make(40, 24, D, seed=D, radius=(0.02, 0.08))
    check(P, ctx, w, N=48)


def test_odd_render_counts(P, ctx):
    """Single draws (no antithetic pair) and an odd N: the last block's render
    count is odd, so the last cull pass of two renders holds one; the same
    bits for 7 and 256 renders per block."""
    w = make(48, 40, 20, seed=9, radius=(0.05, 0.2))
    check(P, ctx, w, N=37, antithetic=False, spbs=(7, 256))


def test_maximum_disk_count(P, ctx):
    """1024 disks (3072 parameters): gradient and HVP by the aggregate sampler."""
    w = make(32, 32, 1024, seed=7, radius=(0.01, 0.05))
    check(P, ctx, w, kinds=("grad", "hvp"), N=8)


def test_large_image(P, ctx):
    """4096 x 4096, one channel: 16.8 M pixels per render."""
    w = make(4096, 4096, 4, C=1, seed=11, centre=(0.2, 0.8), radius=(0.1, 0.2))
    check(P, ctx, w, kinds=("grad", "hvp"), N=2)


@pytest.mark.parametrize("W,H,D", [(2040, 8, 12), (8, 2040, 40), (1024, 1024, 20), (1025, 1024, 6)])
def test_render_pairs_at_the_image_size_limit(P, ctx, W, H, D):
    """The HVP's render pairs up to W + H = 2048 (pixel coordinates packed in 11
    bits each; 32- and 64-disk layouts), and one pixel beyond it, where the
    per-render path takes over."""
    w = make(W, H, D, C=1, seed=W + 3 * H + D, radius=(0.02, 0.1))
    check(P, ctx, w, kinds=("hvp",), N=4)


def test_nothing_covered(P, ctx):
    """Disks far outside the image, and disks whose radii stay non-positive:
    every render is the background, the antithetic gradient is exactly 0."""
    w = make(40, 40, 5, seed=3, centre=(4.0, 5.0))
    check(P, ctx, w)
    w = make(40, 40, 5, seed=4, radius=(-0.3, -0.2), jitter=0.01)
    check(P, ctx, w)


@pytest.mark.parametrize("sigma", [1e-5, 1.0])
def test_extreme_sigma(P, ctx, sigma):
    w = make(48, 40, 6, seed=5, radius=(0.05, 0.15), sigma=sigma)
    check(P, ctx, w, N=128)


def test_pixel_centres_on_disk_edges(P, ctx):
    """A disk centred on a pixel centre with a 10-pixel radius passes exactly
    through 12 pixel centres ((6, 8)-type offsets); with sigma = 1e-9 every
    render leaves them inside the FP32 test's error band, so their coverage is
    decided by the FP64 path from the unrounded parameters, in every render.
    Per-render losses against the oracle (the estimates, 1/sigma-scaled
    differences of near-equal losses, are covered by the other tests), and
    the batch kernel's bits against the single query's."""
    W = H = 64
    c = 32.5 / 64.0
    ts = np.array([c, c, 10.0 / 64.0, 0.25, 0.7, 0.1], np.float64)
    col = np.array([[0.9, 0.3, 0.2], [0.1, 0.6, 0.8]], np.float32)
    w = WL.DiskWorkload(name="edges_on_centres", W=W, H=H, C=3, ppd=3, colors=col, radius=None,
                        theta_star=np.array([c + 0.01, c - 0.02, 0.15, 0.26, 0.69, 0.11]),
                        theta0=ts, sigma=1e-9, N=256, seed=21,
                        v=np.array([0.5, -0.5, 0.5, 0.0, 0.5, 0.0]))
    tgt = disk_target(w)
    osc, gsc = oracle_disks(w, tgt), gpu_disks(ctx, w, tgt)
    for kind in ("grad", "hvp"):
        say(f"{w.name} {kind}")
        _, lref = O.estimate(kind, osc, w.theta0, w.sigma, w.N, w.seed, v=w.v,
                             return_losses=True)
        single, lgot = P.estimate(kind, gsc, w.theta0, w.sigma, w.N, w.seed, v=w.v,
                                  return_losses=True)
        # the edge pixels flip from render to render, and both sides agree on
        # every flip: a wrong FP64 decision moves a loss by ~1e-4 relative
        # (paired HVP renders: a wrong decision moves a difference off zero)
        assert np.ptp(lref) > 1e-5 * np.abs(lref).max()
        assert_losses_match(lgot, lref)
        if kind == "hvp":
            assert lgot.size * 2 == lref.size
            assert np.abs(lref[0::2] - lref[1::2]).max() > 1e-5 * np.abs(lref).max()
        batched = P.Batch(ctx).run([dict(scene=gsc, kind=kind, theta=w.theta0, sigma=w.sigma,
                                         N=w.N, seed=w.seed, v=w.v)] * 2)
        for got in batched:
            assert np.array_equal(got, single)
    gsc.close()
