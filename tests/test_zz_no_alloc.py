"""The entry point that allocates nothing (hr_est_hvp_dev_noalloc) against
the HVP entry point it is a variant of (hr_est_hvp_dev): same kernels, so the
same result bits, on two calls in a row, the second smaller (fewer draws, a
smaller scene on the per-render path), then a request beyond the fixed
workspace, refused."""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads as WL
from scenes import disk_target, gpu_disks, small_disks

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_no_alloc_hvp_matches_device_entry_point():
    import paper_2412_03489_amd as P
    ctx = P.Context(0)
    L = P.lib()
    w = WL.disks32()
    ws = small_disks()              # 50x37, 70 disks: the per-render HVP path
    cases = [(w, gpu_disks(ctx, w, disk_target(w)), 8192),
             (w, None, 3000),        # same scene, fewer draws
             (ws, gpu_disks(ctx, ws, disk_target(ws)), 50)]
    cases[1] = (w, cases[0][1], 3000)
    for wk, sc, N in cases:
        n = wk.n
        th, v, a, b = (ctx.alloc(8 * n) for _ in range(4))
        th.upload(np.asarray(wk.theta0, np.float64))
        v.upload(np.asarray(wk.v, np.float64))
        say(f"no-alloc HVP: {wk.name} n={n} N={N}")
        o = P.make_opts()
        st = L.hr_est_hvp_dev(sc.h, C.c_void_p(th.ptr), float(wk.sigma), int(N), int(wk.seed),
                              C.c_void_p(v.ptr), C.byref(o), C.c_void_p(a.ptr))
        assert st == 0, P.lib().hr_last_error()
        st = L.hr_est_hvp_dev_noalloc(sc.h, C.c_void_p(th.ptr), float(wk.sigma), int(N),
                                      int(wk.seed), C.c_void_p(v.ptr), C.byref(o),
                                      C.c_void_p(b.ptr))
        assert st == 0, P.lib().hr_last_error()
        ctx.synchronize()
        ref, got = a.download(n), b.download(n)
        assert np.isfinite(ref).all() and np.abs(ref).max() > 0
        assert np.array_equal(got, ref)
        for buf in (th, v, a, b):
            buf.free()
    # beyond the fixed workspace: refused with a message, nothing launched
    sc = cases[0][1]
    th, v, b = (ctx.alloc(8 * w.n) for _ in range(3))
    th.upload(w.theta0)
    v.upload(w.v)
    o = P.make_opts()
    st = L.hr_est_hvp_dev_noalloc(sc.h, C.c_void_p(th.ptr), float(w.sigma), 1 << 20, 1,
                                  C.c_void_p(v.ptr), C.byref(o), C.c_void_p(b.ptr))
    assert st == -2
    assert b"fixed workspace" in P.lib().hr_last_error()
    for buf in (th, v, b):
        buf.free()
    cases[0][1].close()
    cases[2][1].close()
    ctx.close()
