"""GPU parity at the benchmarked sizes: the HIP library against expected
values the CPU FP64 oracle wrote (tests/golden/make_golden.py, which calls the
oracle alone), on the same seeded inputs and the same Philox draws.

Each test prints the error of the GPU result against FP64 (rel_inf: the
infinity norm of the difference over that of the oracle's result) and holds
it to 1e-4, the parity bar for FP32 results:
  * disks32 (256x256 RGB, 96 parameters, N = 65536 draws: 2,048 accumulation
    chunks, the strided finalisation): gradient, HVP along v, HVP along -g,
    with compensated-FP32 and FP64 lobe sums;
  * the Newton-CG step the benchmark times (1 gradient + 10 HVPs, Hessian
    modification, trust radius 0.05): the step d = theta_new - theta;
  * the path-traced 6x6 Hessian (128x128, 4 spp, N = 8192: 512 chunks);
  * eight uneven instances at their full budgets (gradient, Hessian, HVP;
    60x60 to 318x318, N up to 63030), alone and in one batch.
"""
import os
import sys

import numpy as np
import pytest

import workloads as WL
from scenes import disk_target, gpu_disks, pt_target, rel_inf

pytestmark = pytest.mark.gpu
TOL = 1e-4
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
UNEVEN = (0, 13, 14, 16, 20, 21, 33, 37)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def golden(name):
    path = os.path.join(GOLDEN, f"full_{name}.npz")
    assert os.path.exists(path), f"{path} missing: run tests/golden/make_golden.py"
    return np.load(path)


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


@pytest.fixture(scope="module")
def disks32(P, ctx):
    w = WL.disks32()
    tgt = disk_target(w)
    sc = gpu_disks(ctx, w, tgt)
    yield w, sc
    sc.close()


@pytest.mark.parametrize("fp64", [False, True])
def test_disks32_gradient_full(P, disks32, fp64):
    w, sc = disks32
    ref = golden("disks32_grad")
    assert int(ref["N"]) == w.N and int(ref["seed"]) == w.seed
    say(f"disks32 gradient N={w.N} fp64={fp64}")
    g = P.estimate("grad", sc, w.theta0, w.sigma, w.N, w.seed, accum_fp64=fp64)
    err = rel_inf(g, ref["out"])
    say(f"  error vs FP64 oracle: rel_inf = {err:.3e}")
    assert err < TOL


@pytest.mark.parametrize("which", ["hvp", "hvp_mg"])
@pytest.mark.parametrize("fp64", [False, True])
def test_disks32_hvp_full(P, disks32, which, fp64):
    w, sc = disks32
    ref = golden(f"disks32_{which}")
    say(f"disks32 HVP ({which}) N={w.N} fp64={fp64}")
    hv = P.estimate("hvp", sc, w.theta0, w.sigma, w.N, w.seed, v=ref["v"], accum_fp64=fp64)
    err = rel_inf(hv, ref["out"])
    say(f"  error vs FP64 oracle: rel_inf = {err:.3e}")
    assert err < TOL


def test_disks32_hvp_limit_full(P, disks32):
    """The limit-kernel HVP (one render per draw and sign, the kernel's
    v-weighted lobe sums) at the full size."""
    w, sc = disks32
    ref = golden("disks32_hvp_limit")
    say(f"disks32 limit-kernel HVP N={w.N}")
    hv = P.estimate("hvp_limit", sc, w.theta0, w.sigma, w.N, w.seed, v=ref["v"])
    err = rel_inf(hv, ref["out"])
    say(f"  error vs FP64 oracle: rel_inf = {err:.3e}")
    assert err < TOL


def test_disks32_hvp_full_rendered_one_by_one(P, disks32):
    """The same HVP with every shifted scene rendered and its loss taken
    separately (hvp_per_render): 262144 renders through the per-render
    rasteriser and the loss pass instead of the render pairs."""
    w, sc = disks32
    ref = golden("disks32_hvp")
    say(f"disks32 HVP rendered one by one N={w.N}")
    hv = P.estimate("hvp", sc, w.theta0, w.sigma, w.N, w.seed, v=ref["v"], hvp_per_render=True)
    err = rel_inf(hv, ref["out"])
    say(f"  error vs FP64 oracle: rel_inf = {err:.3e}")
    assert err < TOL


@pytest.mark.parametrize("fp64", [False, True])
def test_disks32_benchmarked_newton_step(P, disks32, fp64):
    w, sc = disks32
    ref = golden("disks32_newton")
    say(f"disks32 Newton-CG step (bench configuration) fp64={fp64}")
    th, rep = P.newton_cg_step(sc, w.theta0, w.sigma, w.N, w.seed, cg_iters=10,
                               trust_radius=0.05, modified=True, accum_fp64=fp64)
    d_ref = ref["theta"] - w.theta0
    err = rel_inf(th - w.theta0, d_ref)
    say(f"  step error vs FP64 oracle: rel_inf = {err:.3e}; products {rep['iters_done']} "
        f"(oracle {int(ref['iters_done'])}), |g| {rep['g_norm']:.6e} "
        f"(oracle {float(ref['g_norm']):.6e})")
    assert rep["iters_done"] == int(ref["iters_done"])
    assert rep["hit_trust"] == int(ref["hit_trust"]) and rep["neg_curv"] == int(ref["neg_curv"])
    assert err < TOL


def test_pt_hessian_full(P, ctx):
    w = WL.pt_spheres()
    ref = golden("pt_hess")
    tgt = pt_target(w)
    sc = P.Scene.pt(ctx, w.W, w.H, w.spp, w.desc, tgt)
    say(f"path-traced 6x6 Hessian N={w.N}")
    H = P.estimate("hess", sc, w.theta0, w.sigma, w.N, w.seed)
    err = rel_inf(H, ref["out"])
    say(f"  error vs FP64 oracle: rel_inf = {err:.3e}")
    sc.close()
    assert err < TOL


def test_uneven_instances_full_budgets(P, ctx):
    ws = WL.uneven(64)
    scenes, qs, refs = [], [], []
    for i in UNEVEN:
        w = ws[i]
        ref = golden(f"uneven_{i:03d}")
        kind = str(ref["kind"])
        assert int(ref["N"]) == w.N and kind == w.kinds[0]
        sc = gpu_disks(ctx, w, disk_target(w))
        scenes.append(sc)
        q = dict(scene=sc, kind=kind, theta=w.theta0, sigma=w.sigma, N=w.N, seed=w.seed)
        if kind == "hvp":
            q["v"] = w.v
        qs.append(q)
        refs.append(ref["out"])
    say(f"uneven instances {UNEVEN} at full budgets, alone")
    alone = [P.estimate(q["kind"], q["scene"], q["theta"], q["sigma"], q["N"], q["seed"],
                        v=q.get("v")) for q in qs]
    say("uneven instances in one batch")
    b = P.Batch(ctx, use_graph=True)
    got = b.run(qs)
    b.close()
    for i, a, g, r in zip(UNEVEN, alone, got, refs):
        err = rel_inf(a, r)
        say(f"  instance {i} ({ws[i].W}x{ws[i].H}, n={ws[i].n}, N={ws[i].N}, "
            f"{ws[i].kinds[0]}): error vs FP64 oracle rel_inf = {err:.3e}")
        assert err < TOL
        assert np.array_equal(np.ravel(a), np.ravel(g))
    for sc in scenes:
        sc.close()
