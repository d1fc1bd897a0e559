"""Serving load: Newton optimisations, each a loop of dependent estimator
queries, run either through the continuous-batching server (hr_server) or as
plain per-query calls served one at a time in the order they become ready.
Two client models: open loop (clients arrive as a Poisson stream and issue
their queries back to back) and closed loop (all clients start together and
wait an exponential think time before each query, drawn from the client's
own seeded generator).  Both modes issue the same queries (results are the
same bits either way, so every client follows the same trajectory) and report
queries per second over the run with p50 / p99 query latency (from the
moment a query is ready to its result, on the host).

Client step (the Newton step of section "Newton's method"):
  raster (96 params): gradient, then `cg_iters` HVPs of a conjugate-gradient
    solve with the Hessian-modification rule (curvature max(|p^T Hp|,
    floor |p|^2)), step clipped to the trust radius;
  path-traced (6 params): gradient and full Hessian, eigenvalue-clamped
    Newton step clipped to the trust radius.
"""
from __future__ import annotations

import heapq
import time

import numpy as np

from paper_2412_03489_amd import Server, estimate

TRUST = 0.05
EIG_FLOOR = 1e-3


class NewtonClient:
    """Application-side state of one Newton step (numpy, FP64).  With
    full_cg the raster client makes all cg_iters products (the curvature
    rule keeps every step well defined) and clips the final step to the trust
    radius; otherwise CG stops as soon as the step reaches it."""

    def __init__(self, spec, scene, sigma, N, cg_iters, steps=1, full_cg=False):
        self.spec, self.scene, self.sigma, self.N = spec, scene, sigma, N
        self.cg_iters, self.steps, self.full_cg = cg_iters, steps, full_cg
        self.theta = np.array(spec.theta0, dtype=np.float64)
        self.queries = 0
        self.step = 0
        self._think = np.random.default_rng(spec.seed + 7919)
        self._start_step()

    def think_s(self, mean_s):
        """The next exponential think time (seconds) of this client."""
        return float(self._think.exponential(mean_s))

    def _seed(self):
        return self.spec.seed * 1000 + self.step

    def _start_step(self):
        self.g = None
        self.H = None
        self.next = ("grad", None)

    def query(self):
        kind, v = self.next
        q = dict(scene=self.scene, kind=kind, theta=self.theta, sigma=self.sigma, N=self.N,
                 seed=self._seed())
        if v is not None:
            q["v"] = v
        return q

    def on_result(self, out):
        """Consumes a result; returns False when the client is finished."""
        self.queries += 1
        kind, _ = self.next
        if kind == "grad":
            self.g = np.array(out, dtype=np.float64)
            if self.spec.scene == "pt":
                self.next = ("hess", None)
                return True
            # conjugate gradients on H d = -g from d = 0
            self.d = np.zeros_like(self.g)
            self.r = -self.g
            self.p = self.r.copy()
            self.it = 0
            self.next = ("hvp", self.p.copy())
            return True
        if kind == "hess":
            H = 0.5 * (out + out.T)
            lam, V = np.linalg.eigh(H)
            lam = np.maximum(np.abs(lam), EIG_FLOOR)
            d = -V @ ((V.T @ self.g) / lam)
            return self._apply(d)
        # hvp
        Hp = np.array(out, dtype=np.float64)
        pp = float(self.p @ self.p)
        kappa = max(abs(float(self.p @ Hp)), EIG_FLOOR * pp)
        rr = float(self.r @ self.r)
        alpha = rr / kappa
        self.d = self.d + alpha * self.p
        self.r = self.r - alpha * Hp
        self.it += 1
        rr_new = float(self.r @ self.r)
        at_trust = not self.full_cg and np.linalg.norm(self.d) >= TRUST
        if self.it >= self.cg_iters or at_trust or rr_new == 0.0:
            return self._apply(self.d)
        self.p = self.r + (rr_new / rr) * self.p
        self.next = ("hvp", self.p.copy())
        return True

    def _apply(self, d):
        nd = np.linalg.norm(d)
        if nd > TRUST:
            d = d * (TRUST / nd)
        self.theta = self.theta + d
        self.step += 1
        if self.step >= self.steps:
            return False
        self._start_step()
        return True


def _pct(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else float("nan")


def _summary(lat, t_total, extra=None):
    """lat: (query label, latency ms) pairs."""
    ms = [x for _, x in lat]
    out = {"queries": len(lat), "seconds": t_total, "queries_per_s": len(lat) / t_total,
           "p50_ms": _pct(ms, 50), "p99_ms": _pct(ms, 99),
           "mean_ms": float(np.mean(ms)) if ms else float("nan")}
    by = {}
    for label, x in lat:
        by.setdefault(label, []).append(x)
    out["by_kind"] = {k: {"queries": len(v), "p50_ms": round(_pct(v, 50), 3),
                          "p99_ms": round(_pct(v, 99), 3)} for k, v in sorted(by.items())}
    if extra:
        out.update(extra)
    return out


def _label(client, q):
    return f"{client.spec.scene}_{q['kind']}"


def make_clients(specs, scenes, sigma, N, cg_iters, steps=1, full_cg=False):
    return [NewtonClient(s, scenes[s.scene], sigma[s.scene], N[s.scene], cg_iters, steps,
                         full_cg) for s in specs]


def _first_ready(clients, think_ms, window_s=None):
    """(ready time in seconds from the start, order, client) of each first
    query that falls within the window."""
    ev = []
    for k, c in enumerate(sorted(clients, key=lambda c: c.spec.arrival)):
        t = c.spec.arrival if think_ms is None else c.think_s(think_ms / 1e3)
        if window_s is None or t <= window_s:
            ev.append((t, k, c))
    heapq.heapify(ev)
    return ev


def run_served(ctx, clients, slots=4, max_batch=64, max_batch_ms=2.0, memory_bytes=16 << 30,
               use_graph=True, think_ms=None, window_s=None):
    """All clients through one continuous-batching server.  think_ms None: open
    loop (queries back to back after the client's arrival); else closed loop
    with exponential think times of that mean before every query.  window_s:
    no query becomes ready after this time (the clients stop; the ones in
    flight finish)."""
    srv = Server(ctx, slots=slots, max_batch=max_batch, max_batch_ms=max_batch_ms,
                 memory_bytes=memory_bytes, use_graph=use_graph)
    ready = _first_ready(clients, think_ms, window_s)
    order = len(clients)
    live = {}
    lat = []
    t0 = time.perf_counter()

    def submit(c, ts):
        q = c.query()
        label = _label(c, q)
        t = srv.submit(q.pop("scene"), q.pop("kind"), q.pop("theta"), q.pop("sigma"),
                       q.pop("N"), q.pop("seed"), v=q.pop("v", None))
        live[t] = (c, ts, label)

    while ready or live:
        now = time.perf_counter() - t0
        while ready and ready[0][0] <= now:
            tr, _, c = heapq.heappop(ready)
            submit(c, t0 + tr)
        wait = -1.0 if not ready else max(0.0, (ready[0][0] - now) * 1e3)
        if not live:
            time.sleep(wait / 1e3)
            continue
        t = srv.wait_any(timeout_ms=wait)
        if t is None:
            continue
        out, st = srv.wait(t)
        c, ts, label = live.pop(t)
        tn = time.perf_counter()
        lat.append((label, (tn - ts) * 1e3))
        if c.on_result(out):
            nxt = tn - t0 if think_ms is None else tn - t0 + c.think_s(think_ms / 1e3)
            if window_s is None or nxt <= window_s:
                if think_ms is None:
                    submit(c, tn)
                else:
                    heapq.heappush(ready, (nxt, order, c))
                    order += 1
    total = time.perf_counter() - t0
    s = srv.stats()
    srv.close()
    return _summary(lat, total, {"batches": s["batches"],
                                 "mean_batch": s["mean_batch"],
                                 "slots": slots, "max_batch": max_batch,
                                 "max_batch_ms": max_batch_ms})


def run_plain(ctx, clients, think_ms=None, window_s=None):
    """The same clients, each query a plain single-query call, served one at a
    time in the order the queries become ready (think_ms, window_s as in
    run_served)."""
    ready = _first_ready(clients, think_ms, window_s)
    order = len(clients)
    lat = []
    t0 = time.perf_counter()
    while ready:
        now = time.perf_counter() - t0
        tr, _, c = ready[0]
        if tr > now:
            time.sleep(tr - now)
            continue
        heapq.heappop(ready)
        q = c.query()
        label = _label(c, q)
        kind = q.pop("kind")
        out = estimate(kind, q.pop("scene"), q.pop("theta"), q.pop("sigma"), q.pop("N"),
                       q.pop("seed"), v=q.pop("v", None))
        tn = time.perf_counter()
        lat.append((label, (tn - (t0 + tr)) * 1e3))
        if c.on_result(out):
            nxt = tn - t0 if think_ms is None else tn - t0 + c.think_s(think_ms / 1e3)
            if window_s is None or nxt <= window_s:
                heapq.heappush(ready, (nxt, order, c))
                order += 1
    total = time.perf_counter() - t0
    return _summary(lat, total)
