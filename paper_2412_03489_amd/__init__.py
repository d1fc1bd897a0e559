"""MI355X (gfx950) Monte Carlo gradients, Hessians and Hessian-vector products
of Gaussian-smoothed rendering losses, after Wang, Fischer, Ritschel,
"Stochastic Gradient Estimation for Higher-order Differentiable Rendering"
(ICCV 2025).

This package is a thin ctypes binding of ``libhrest.so`` (C ABI in
``include/hrest.h``); it only marshals arguments.  Every step of the estimator
runs in the library's HIP kernels.  There is no CPU fallback: if the library
is missing or no GPU is visible, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhrest.so")

AIS, IS, GAUSS, FR22 = 0, 1, 2, 3
STATUS = {0: "HR_OK", -1: "HR_EINVAL", -2: "HR_ENOMEM", -3: "HR_EDEVICE", -4: "HR_EUNSUPPORTED",
          -5: "HR_EBUSY"}
KIND = {"grad": 0, "hess": 1, "hvp": 2, "hvp_limit": 3, "loss": 4}

EXPORTED = (
    "hr_opts_default", "hr_ncg_opts_default", "hr_ctx_create", "hr_ctx_destroy",
    "hr_ctx_set_stream", "hr_ctx_set_memory_budget", "hr_ctx_synchronize",
    "hr_ctx_enable_timing", "hr_ctx_kernel_stats", "hr_ctx_reset_stats", "hr_last_error",
    "hr_scene_disks", "hr_scene_pt", "hr_scene_quad", "hr_scene_neggauss", "hr_scene_destroy",
    "hr_scene_nparams", "hr_render", "hr_est_grad", "hr_est_hessian", "hr_est_hvp",
    "hr_est_hvp_limit", "hr_est_grad_dev", "hr_est_hessian_dev", "hr_est_hvp_dev",
    "hr_est_hvp_dev_noalloc",
    "hr_newton_cg_step", "hr_newton_cg_step_dev", "hr_dev_alloc", "hr_dev_free", "hr_memcpy",
    "hr_est_grad_greybox", "hr_est_hessian_greybox", "hr_est_hvp_greybox",
    "hr_est_loss", "hr_optim_opts_default", "hr_optimize",
    "hr_batch_opts_default", "hr_batch_create", "hr_batch_destroy", "hr_batch_run",
    "hr_batch_report_get", "hr_batch_tuned",
    "hr_server_opts_default", "hr_server_create", "hr_server_destroy", "hr_submit", "hr_wait",
    "hr_wait_any", "hr_server_stats_get",
)


class HrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Opts(C.Structure):
    _fields_ = [("sampler", C.c_int), ("antithetic", C.c_int), ("hvp_rel_step", C.c_double),
                ("accum_fp64", C.c_int), ("samples_per_block", C.c_int),
                ("raster_tile", C.c_int), ("dbg_loss", C.POINTER(C.c_double)),
                ("dbg_tau", C.POINTER(C.c_double)), ("hess_mix_n2", C.c_int),
                ("hvp_per_render", C.c_int)]


class NcgOpts(C.Structure):
    _fields_ = [("cg_iters", C.c_int), ("trust_radius", C.c_double),
                ("use_full_hessian", C.c_int), ("eig_floor", C.c_double), ("hvp_limit", C.c_int),
                ("modified", C.c_int)]


class OptimOpts(C.Structure):
    _fields_ = [("iters", C.c_int), ("sigma_start", C.c_double), ("sigma_end", C.c_double),
                ("method", C.c_int), ("lr", C.c_double), ("ls_iters", C.c_int),
                ("ls_tol", C.c_double), ("recompute", C.c_int), ("N_loss", C.c_uint64),
                ("ncg", NcgOpts)]


class Query(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("kind", C.c_int), ("sigma", C.c_double),
                ("N", C.c_uint64), ("seed", C.c_uint64), ("theta", C.c_void_p),
                ("v", C.c_void_p), ("opts", C.POINTER(Opts)), ("out", C.c_void_p)]


class BatchOpts(C.Structure):
    _fields_ = [("use_graph", C.c_int), ("autotune", C.c_int)]


class BatchReport(C.Structure):
    _fields_ = [("queries", C.c_uint64), ("raster_items", C.c_uint64), ("pt_items", C.c_uint64),
                ("raster_blocks", C.c_int), ("pt_blocks", C.c_int),
                ("workspace_bytes", C.c_uint64), ("lds_bytes", C.c_uint64), ("graph", C.c_int)]


class ServerOpts(C.Structure):
    _fields_ = [("slots", C.c_int), ("max_batch", C.c_int), ("max_batch_ms", C.c_double),
                ("memory_bytes", C.c_uint64), ("use_graph", C.c_int), ("autotune", C.c_int),
                ("metrics_path", C.c_char_p)]


class QueryStats(C.Structure):
    _fields_ = [("submit_ms", C.c_double), ("start_ms", C.c_double), ("end_ms", C.c_double),
                ("batch_size", C.c_int), ("status", C.c_int)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("batches", C.c_uint64),
                ("mean_batch", C.c_double), ("busy_ms", C.c_double)]


class NcgReport(C.Structure):
    _fields_ = [("iters_done", C.c_int), ("hit_trust", C.c_int), ("neg_curv", C.c_int),
                ("step_norm", C.c_double), ("g_norm", C.c_double)]


_lib = None


def lib():
    """Load libhrest.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2412_03489_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i, d, u64, u32 = C.c_void_p, C.c_int, C.c_double, C.c_uint64, C.c_uint32
    pv = C.POINTER(C.c_void_p)
    L.hr_opts_default.argtypes = [C.POINTER(Opts)]
    L.hr_ncg_opts_default.argtypes = [C.POINTER(NcgOpts)]
    L.hr_last_error.restype = C.c_char_p
    L.hr_ctx_create.argtypes = [i, pv]
    L.hr_ctx_destroy.argtypes = [vp]
    L.hr_ctx_set_stream.argtypes = [vp, vp]
    L.hr_ctx_set_memory_budget.argtypes = [vp, u64]
    L.hr_ctx_synchronize.argtypes = [vp]
    L.hr_ctx_enable_timing.argtypes = [vp, i]
    L.hr_ctx_kernel_stats.argtypes = [vp, C.c_char_p, C.POINTER(u64), C.POINTER(d)]
    L.hr_ctx_reset_stats.argtypes = [vp]
    L.hr_dev_alloc.argtypes = [vp, C.c_size_t, pv]
    L.hr_dev_free.argtypes = [vp, vp]
    L.hr_memcpy.argtypes = [vp, vp, vp, C.c_size_t, i]
    L.hr_scene_disks.argtypes = [vp, i, i, i, i, i, vp, vp, vp, pv]
    L.hr_scene_pt.argtypes = [vp, i, i, i, i, vp, vp, pv]
    L.hr_scene_quad.argtypes = [vp, i, vp, vp, d, pv]
    L.hr_scene_neggauss.argtypes = [vp, i, d, pv]
    L.hr_scene_destroy.argtypes = [vp]
    L.hr_scene_nparams.argtypes = [vp]
    L.hr_render.argtypes = [vp, vp, u64, u32, i, vp]
    for nm in ("hr_est_grad", "hr_est_hessian", "hr_est_grad_dev", "hr_est_hessian_dev"):
        getattr(L, nm).argtypes = [vp, vp, d, u64, u64, C.POINTER(Opts), vp]
    for nm in ("hr_est_hvp", "hr_est_hvp_limit", "hr_est_hvp_dev", "hr_est_hvp_dev_noalloc"):
        getattr(L, nm).argtypes = [vp, vp, d, u64, u64, vp, C.POINTER(Opts), vp]
    for nm in ("hr_newton_cg_step", "hr_newton_cg_step_dev"):
        getattr(L, nm).argtypes = [vp, vp, d, u64, u64, C.POINTER(NcgOpts), C.POINTER(Opts),
                                   C.POINTER(NcgReport)]
    for nm in ("hr_est_grad_greybox", "hr_est_hessian_greybox"):
        getattr(L, nm).argtypes = [vp, vp, vp, i, d, u64, u64, C.POINTER(Opts), vp]
    L.hr_est_hvp_greybox.argtypes = [vp, vp, vp, i, d, u64, u64, vp, C.POINTER(Opts), vp]
    L.hr_est_loss.argtypes = [vp, vp, d, u64, u64, C.POINTER(Opts), vp]
    L.hr_optim_opts_default.argtypes = [C.POINTER(OptimOpts)]
    L.hr_optimize.argtypes = [vp, vp, u64, u64, C.POINTER(OptimOpts), C.POINTER(Opts), vp]
    L.hr_batch_opts_default.argtypes = [C.POINTER(BatchOpts)]
    L.hr_batch_create.argtypes = [vp, C.POINTER(BatchOpts), pv]
    L.hr_batch_destroy.argtypes = [vp]
    L.hr_batch_run.argtypes = [vp, C.POINTER(Query), i]
    L.hr_batch_report_get.argtypes = [vp, C.POINTER(BatchReport)]
    L.hr_batch_tuned.argtypes = [vp, vp, C.POINTER(i), C.POINTER(i)]
    L.hr_server_opts_default.argtypes = [C.POINTER(ServerOpts)]
    L.hr_server_create.argtypes = [vp, C.POINTER(ServerOpts), pv]
    L.hr_server_destroy.argtypes = [vp]
    L.hr_submit.argtypes = [vp, C.POINTER(Query), C.POINTER(u64)]
    L.hr_wait.argtypes = [vp, u64, vp, C.POINTER(QueryStats)]
    L.hr_wait_any.argtypes = [vp, d, C.POINTER(u64)]
    L.hr_server_stats_get.argtypes = [vp, C.POINTER(ServerStats)]
    _lib = L
    return L


def _check(st):
    if st != 0:
        raise HrError(st, lib().hr_last_error().decode())


def _p(a):
    return C.c_void_p(a.ctypes.data)


def make_opts(sampler=AIS, antithetic=True, hvp_rel_step=0.1, accum_fp64=False,
              samples_per_block=0, dbg=None, dbg_tau=None, raster_tile=0, hess_mix_n2=False,
              hvp_per_render=False):
    o = Opts()
    lib().hr_opts_default(C.byref(o))
    o.sampler = sampler
    o.antithetic = 1 if antithetic else 0
    o.hvp_rel_step = hvp_rel_step
    o.accum_fp64 = 1 if accum_fp64 else 0
    o.samples_per_block = samples_per_block
    o.raster_tile = raster_tile
    o.hess_mix_n2 = 1 if hess_mix_n2 else 0
    o.hvp_per_render = 1 if hvp_per_render else 0
    o.dbg_loss = dbg.ctypes.data_as(C.POINTER(C.c_double)) if dbg is not None else None
    o.dbg_tau = dbg_tau.ctypes.data_as(C.POINTER(C.c_double)) if dbg_tau is not None else None
    return o


class Context:
    """One GPU: stream, workspace and kernel timers (hr_ctx)."""

    def __init__(self, device=0):
        h = C.c_void_p()
        _check(lib().hr_ctx_create(int(device), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().hr_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream_handle):
        _check(lib().hr_ctx_set_stream(self.h, C.c_void_p(stream_handle or 0)))

    def set_memory_budget(self, nbytes):
        _check(lib().hr_ctx_set_memory_budget(self.h, int(nbytes)))

    def synchronize(self):
        _check(lib().hr_ctx_synchronize(self.h))

    def enable_timing(self, on=True):
        _check(lib().hr_ctx_enable_timing(self.h, 1 if on else 0))

    def kernel_stats(self, name):
        n = C.c_uint64()
        t = C.c_double()
        _check(lib().hr_ctx_kernel_stats(self.h, name.encode(), C.byref(n), C.byref(t)))
        return n.value, t.value

    def reset_stats(self):
        _check(lib().hr_ctx_reset_stats(self.h))

    def alloc(self, nbytes):
        """Device buffer on this context's GPU (hr_dev_alloc)."""
        return DeviceBuffer(self, nbytes)


class DeviceBuffer:
    """HBM allocation owned by the library's runtime; .ptr is the device address."""

    def __init__(self, ctx, nbytes):
        p = C.c_void_p()
        _check(lib().hr_dev_alloc(ctx.h, int(nbytes), C.byref(p)))
        self.ctx, self.ptr, self.nbytes = ctx, p.value, int(nbytes)

    def upload(self, arr):
        a = np.ascontiguousarray(arr)
        assert a.nbytes <= self.nbytes
        _check(lib().hr_memcpy(self.ctx.h, C.c_void_p(self.ptr), _p(a), a.nbytes, 0))

    def download(self, shape, dtype=np.float64):
        out = np.zeros(shape, dtype=dtype)
        assert out.nbytes <= self.nbytes
        _check(lib().hr_memcpy(self.ctx.h, _p(out), C.c_void_p(self.ptr), out.nbytes, 1))
        return out

    def copy_from(self, other):
        """Device-to-device copy of other's bytes into this buffer."""
        assert other.nbytes <= self.nbytes
        _check(lib().hr_memcpy(self.ctx.h, C.c_void_p(self.ptr), C.c_void_p(other.ptr),
                               other.nbytes, 2))

    def free(self):
        if self.ptr:
            _check(lib().hr_dev_free(self.ctx.h, C.c_void_p(self.ptr)))
            self.ptr = None


class Scene:
    """A device-resident scene (hr_scene)."""

    def __init__(self, ctx, handle, n, shape=None):
        self.ctx = ctx
        self.h = handle
        self.n = n
        self.shape = shape

    def close(self):
        if getattr(self, "h", None):
            lib().hr_scene_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def disks(ctx, W, H, C_, colors, target, radius=None, ppd=3):
        colors = np.ascontiguousarray(colors, dtype=np.float32)
        target = np.ascontiguousarray(target, dtype=np.float32)
        D = colors.shape[0]
        rad = None if radius is None else np.ascontiguousarray(radius, dtype=np.float32)
        h = C.c_void_p()
        _check(lib().hr_scene_disks(ctx.h, W, H, C_, D, ppd, None if rad is None else _p(rad),
                                    _p(colors), _p(target), C.byref(h)))
        sc = Scene(ctx, h, D * ppd, (H, W, C_))
        sc.n_disks, sc.W, sc.H = D, W, H
        return sc

    @staticmethod
    def pt(ctx, W, H, spp, desc, target, nspheres=4):
        desc = np.ascontiguousarray(desc, dtype=np.float64)
        target = np.ascontiguousarray(target, dtype=np.float32)
        h = C.c_void_p()
        _check(lib().hr_scene_pt(ctx.h, W, H, spp, nspheres, _p(desc), _p(target), C.byref(h)))
        return Scene(ctx, h, 6, (H, W, 3))

    @staticmethod
    def quad(ctx, A, b=None, c=0.0):
        A = np.ascontiguousarray(A, dtype=np.float64)
        n = A.shape[0]
        bb = np.zeros(n) if b is None else np.ascontiguousarray(b, dtype=np.float64)
        h = C.c_void_p()
        _check(lib().hr_scene_quad(ctx.h, n, _p(A), _p(bb), float(c), C.byref(h)))
        return Scene(ctx, h, n)

    @staticmethod
    def neggauss(ctx, n, s1):
        h = C.c_void_p()
        _check(lib().hr_scene_neggauss(ctx.h, int(n), float(s1), C.byref(h)))
        return Scene(ctx, h, n)

    def render(self, theta, seed=0, s=0, spp=0):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        out = np.zeros(self.shape, dtype=np.float32)
        _check(lib().hr_render(self.h, _p(th), int(seed), int(s), int(spp), _p(out)))
        return out


def n_renders(kind, n, N, sampler=AIS, antithetic=True):
    A = 2 if antithetic else 1
    K = n * (n + 1) // 2 if kind == "hess" else n
    streams = K if (sampler in (IS, FR22) and kind != "hvp_limit") else 1
    return streams * N * A * (2 if kind == "hvp" else 1)


def n_streams(kind, n, sampler=AIS):
    K = n * (n + 1) // 2 if kind == "hess" else n
    return K if (sampler in (IS, FR22) and kind != "hvp_limit") else 1


def hvp_pairs(kind, scene, hvp_per_render=False):
    """Whether an HVP on this scene takes its +-h scenes as pairs (a disk
    scene of at most 64 disks with W + H <= 2048, hvp_per_render off): then
    the per-render loss output holds one loss difference f(+h) - f(-h) per
    (draw, sign)."""
    return (kind == "hvp" and getattr(scene, "n_disks", 10 ** 9) <= 64
            and getattr(scene, "W", 0) + getattr(scene, "H", 0) <= 2048 and not hvp_per_render)


def estimate(kind, scene, theta, sigma, N, seed, v=None, sampler=AIS, antithetic=True,
             hvp_rel_step=0.1, accum_fp64=False, samples_per_block=0, return_losses=False,
             return_draws=False, raster_tile=0, hess_mix_n2=False, hvp_per_render=False):
    """kind in {'grad', 'hess', 'hvp', 'hvp_limit'} (host-pointer entry points).
    With return_losses / return_draws the per-render losses (for paired HVP
    renders, see hvp_pairs: the loss differences) and the draws are returned
    as well (in that order).  hess_mix_n2: the aggregate Hessian mixture over
    all n^2 ordered pairs.  hvp_per_render: render and score each shifted
    scene of an HVP separately."""
    n = scene.n
    th = np.ascontiguousarray(theta, dtype=np.float64)
    nl = n_renders(kind, n, N, sampler, antithetic)
    if hvp_pairs(kind, scene, hvp_per_render):
        nl //= 2
    dbg = np.zeros(nl) if return_losses else None
    taus = np.zeros(n_streams(kind, n, sampler) * N * n) if return_draws else None
    o = make_opts(sampler, antithetic, hvp_rel_step, accum_fp64, samples_per_block, dbg, taus,
                  raster_tile, hess_mix_n2, hvp_per_render)
    L = lib()
    if kind == "grad":
        out = np.zeros(n)
        st = L.hr_est_grad(scene.h, _p(th), float(sigma), int(N), int(seed), C.byref(o), _p(out))
    elif kind == "hess":
        out = np.zeros((n, n))
        st = L.hr_est_hessian(scene.h, _p(th), float(sigma), int(N), int(seed), C.byref(o), _p(out))
    elif kind in ("hvp", "hvp_limit"):
        vv = np.ascontiguousarray(v, dtype=np.float64)
        out = np.zeros(n)
        fn = L.hr_est_hvp if kind == "hvp" else L.hr_est_hvp_limit
        st = fn(scene.h, _p(th), float(sigma), int(N), int(seed), _p(vv), C.byref(o), _p(out))
    else:
        raise ValueError(kind)
    _check(st)
    extra = ([dbg] if return_losses else []) + ([taus] if return_draws else [])
    return (out, *extra) if extra else out


def estimate_dev(kind, scene, d_theta, sigma, N, seed, d_out, d_v=None, sampler=AIS,
                 antithetic=True, hvp_rel_step=0.1, accum_fp64=False, samples_per_block=0):
    """Device-pointer entry points (asynchronous on the context stream).
    d_theta, d_v, d_out are integer device addresses (e.g. torch tensor data_ptr())."""
    o = make_opts(sampler, antithetic, hvp_rel_step, accum_fp64, samples_per_block)
    L = lib()
    a = (scene.h, C.c_void_p(d_theta), float(sigma), int(N), int(seed))
    if kind == "grad":
        st = L.hr_est_grad_dev(*a, C.byref(o), C.c_void_p(d_out))
    elif kind == "hess":
        st = L.hr_est_hessian_dev(*a, C.byref(o), C.c_void_p(d_out))
    elif kind == "hvp":
        st = L.hr_est_hvp_dev(*a, C.c_void_p(d_v), C.byref(o), C.c_void_p(d_out))
    else:
        raise ValueError(kind)
    _check(st)


def newton_cg_step(scene, theta, sigma, N, seed, cg_iters=10, trust_radius=1.0,
                   use_full_hessian=False, eig_floor=1e-6, hvp_limit=False, sampler=AIS,
                   antithetic=True, hvp_rel_step=0.1, accum_fp64=False, samples_per_block=0,
                   modified=False):
    th = np.array(theta, dtype=np.float64)
    o = make_opts(sampler, antithetic, hvp_rel_step, accum_fp64, samples_per_block)
    no = NcgOpts(int(cg_iters), float(trust_radius), 1 if use_full_hessian else 0,
                 float(eig_floor), 1 if hvp_limit else 0, 1 if modified else 0)
    rep = NcgReport()
    _check(lib().hr_newton_cg_step(scene.h, _p(th), float(sigma), int(N), int(seed),
                                   C.byref(no), C.byref(o), C.byref(rep)))
    return th, {"iters_done": rep.iters_done, "hit_trust": rep.hit_trust,
                "neg_curv": rep.neg_curv, "step_norm": rep.step_norm, "g_norm": rep.g_norm}


def newton_cg_step_dev(scene, d_theta, sigma, N, seed, cg_iters=10, trust_radius=1.0,
                       use_full_hessian=False, eig_floor=1e-6, hvp_limit=False, sampler=AIS,
                       antithetic=True, hvp_rel_step=0.1, accum_fp64=False, samples_per_block=0,
                       modified=False):
    o = make_opts(sampler, antithetic, hvp_rel_step, accum_fp64, samples_per_block)
    no = NcgOpts(int(cg_iters), float(trust_radius), 1 if use_full_hessian else 0,
                 float(eig_floor), 1 if hvp_limit else 0, 1 if modified else 0)
    rep = NcgReport()
    _check(lib().hr_newton_cg_step_dev(scene.h, C.c_void_p(d_theta), float(sigma), int(N),
                                       int(seed), C.byref(no), C.byref(o), C.byref(rep)))
    return {"iters_done": rep.iters_done, "hit_trust": rep.hit_trust, "neg_curv": rep.neg_curv,
            "step_norm": rep.step_norm, "g_norm": rep.g_norm}


def estimate_greybox(kind, scene, y, J, sigma, N, seed, vx=None, sampler=AIS, antithetic=True,
                     hvp_rel_step=0.1, accum_fp64=False, samples_per_block=0):
    """Grey-box composition (hr_est_*_greybox): kind in {'grad', 'hess', 'hvp'};
    J has shape (n, n_in)."""
    yy = np.ascontiguousarray(y, dtype=np.float64)
    JJ = np.ascontiguousarray(J, dtype=np.float64)
    n_in = JJ.shape[1]
    o = make_opts(sampler, antithetic, hvp_rel_step, accum_fp64, samples_per_block)
    L = lib()
    a = (scene.h, _p(yy), _p(JJ), n_in, float(sigma), int(N), int(seed))
    if kind == "grad":
        out = np.zeros(n_in)
        st = L.hr_est_grad_greybox(*a, C.byref(o), _p(out))
    elif kind == "hess":
        out = np.zeros((n_in, n_in))
        st = L.hr_est_hessian_greybox(*a, C.byref(o), _p(out))
    elif kind == "hvp":
        v = np.ascontiguousarray(vx, dtype=np.float64)
        out = np.zeros(n_in)
        st = L.hr_est_hvp_greybox(*a, _p(v), C.byref(o), _p(out))
    else:
        raise ValueError(kind)
    _check(st)
    return out


def est_loss(scene, theta, sigma, N, seed, antithetic=True):
    """Smoothed loss (hr_est_loss); sigma = 0 gives the plain loss."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    o = make_opts(GAUSS, antithetic)
    F = C.c_double()
    _check(lib().hr_est_loss(scene.h, _p(th), float(sigma), int(N), int(seed), C.byref(o),
                             C.byref(F)))
    return F.value


METHODS = {"newton_cg": 0, "newton_full": 1, "gd": 2}


def optimize(scene, theta, N, seed, iters, sigma_start, sigma_end, method="newton_cg", lr=0.1,
             ls_iters=0, ls_tol=1e-3, recompute=1, N_loss=0, cg_iters=10, trust_radius=1.0,
             eig_floor=1e-6, modified=False, hvp_limit=False, sampler=AIS, antithetic=True,
             hvp_rel_step=0.1, accum_fp64=False, samples_per_block=0):
    """Optimiser loop (hr_optimize); returns (theta, trace[iters, 5])."""
    th = np.array(theta, dtype=np.float64)
    o = make_opts(sampler, antithetic, hvp_rel_step, accum_fp64, samples_per_block)
    oo = OptimOpts(int(iters), float(sigma_start), float(sigma_end), METHODS[method], float(lr),
                   int(ls_iters), float(ls_tol), int(recompute), int(N_loss),
                   NcgOpts(int(cg_iters), float(trust_radius), 0, float(eig_floor),
                           1 if hvp_limit else 0, 1 if modified else 0))
    trace = np.zeros((iters, 5))
    _check(lib().hr_optimize(scene.h, _p(th), int(N), int(seed), C.byref(oo), C.byref(o),
                             _p(trace)))
    return th, trace


# ------------------------------------------------------------ batches, serving
def out_shape(kind, n):
    return (n, n) if kind == "hess" else ((1,) if kind == "loss" else (n,))


_OPT_KEYS = ("sampler", "antithetic", "hvp_rel_step", "accum_fp64", "samples_per_block",
             "raster_tile", "hess_mix_n2", "hvp_per_render")


def _query(scene, kind, theta, sigma, N, seed, v=None, out=None, **opt):
    """Builds an hr_query; returns it with the arrays it points at (kept alive)."""
    bad = set(opt) - set(_OPT_KEYS)
    if bad:
        raise TypeError(f"unknown query options {sorted(bad)}")
    th = np.ascontiguousarray(theta, dtype=np.float64)
    vv = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
    o = make_opts(opt.get("sampler", AIS), opt.get("antithetic", True),
                  opt.get("hvp_rel_step", 0.1), opt.get("accum_fp64", False),
                  opt.get("samples_per_block", 0), raster_tile=opt.get("raster_tile", 0),
                  hess_mix_n2=opt.get("hess_mix_n2", False),
                  hvp_per_render=opt.get("hvp_per_render", False))
    q = Query(scene.h, KIND[kind], float(sigma), int(N), int(seed), _p(th),
              None if vv is None else _p(vv), C.pointer(o), None if out is None else _p(out))
    return q, (th, vv, o, out)


class Batch:
    """Batched executor (hr_batch): many uneven queries per launch sequence."""

    def __init__(self, ctx, use_graph=True, autotune=False):
        o = BatchOpts(1 if use_graph else 0, 1 if autotune else 0)
        h = C.c_void_p()
        _check(lib().hr_batch_create(ctx.h, C.byref(o), C.byref(h)))
        self.ctx, self.h = ctx, h

    def run(self, queries):
        """queries: dicts with scene, kind, theta, sigma, N, seed[, v] and
        optional estimator options; returns the results in order."""
        outs, keep = [], []
        arr = (Query * max(1, len(queries)))()
        for k, q in enumerate(queries):
            q = dict(q)
            out = np.zeros(out_shape(q["kind"], q["scene"].n))
            qq, alive = _query(out=out, **q)
            arr[k] = qq
            outs.append(out)
            keep.append(alive)
        _check(lib().hr_batch_run(self.h, arr, len(queries)))
        return outs

    def report(self):
        r = BatchReport()
        _check(lib().hr_batch_report_get(self.h, C.byref(r)))
        return {f: getattr(r, f) for f, _ in BatchReport._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().hr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tuned(ctx, scene):
    """The autotuner's (samples_per_block, raster_tile) for the scene's class."""
    s, t = C.c_int(), C.c_int()
    _check(lib().hr_batch_tuned(ctx.h, scene.h, C.byref(s), C.byref(t)))
    return s.value, t.value


class Server:
    """Continuous-batching server (hr_server)."""

    def __init__(self, ctx, slots=4, max_batch=64, max_batch_ms=2.0, memory_bytes=0,
                 use_graph=True, autotune=False, metrics_path=None):
        """metrics_path: append one JSON line per completed query to this file."""
        o = ServerOpts(int(slots), int(max_batch), float(max_batch_ms), int(memory_bytes),
                       1 if use_graph else 0, 1 if autotune else 0,
                       os.fsencode(metrics_path) if metrics_path else None)
        h = C.c_void_p()
        _check(lib().hr_server_create(ctx.h, C.byref(o), C.byref(h)))
        self.ctx, self.h = ctx, h
        self._kind = {}

    def submit(self, scene, kind, theta, sigma, N, seed, v=None, **opt):
        q, alive = _query(scene, kind, theta, sigma, N, seed, v, **opt)
        t = C.c_uint64()
        _check(lib().hr_submit(self.h, C.byref(q), C.byref(t)))
        self._kind[t.value] = out_shape(kind, scene.n)
        return t.value

    def wait(self, ticket):
        """(result, stats) of a ticket; retires it."""
        out = np.zeros(self._kind.pop(ticket))
        st = QueryStats()
        _check(lib().hr_wait(self.h, int(ticket), _p(out), C.byref(st)))
        return out, {f: getattr(st, f) for f, _ in QueryStats._fields_}

    def wait_any(self, timeout_ms=-1.0):
        """A completed ticket, or None on time-out."""
        t = C.c_uint64()
        st = lib().hr_wait_any(self.h, float(timeout_ms), C.byref(t))
        if st == -5:
            return None
        _check(st)
        return t.value

    def stats(self):
        s = ServerStats()
        _check(lib().hr_server_stats_get(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().hr_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
