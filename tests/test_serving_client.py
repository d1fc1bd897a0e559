"""Host-side logic of the serving load generator (no GPU): a client's Newton
step is the exact Newton step when fed exact derivatives of a quadratic."""
import numpy as np
import pytest

import workloads as WL
import bench_serving as SV


def _quadratic(n, seed):
    g = np.random.default_rng(seed)
    M = g.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    b = g.standard_normal(n)
    return A, b


def _drive(client, A, b):
    """Answers the client's queries exactly; returns the kinds asked."""
    kinds = []
    while True:
        q = client.query()
        kinds.append(q["kind"])
        th = q["theta"]
        if q["kind"] == "grad":
            out = A @ th + b
        elif q["kind"] == "hess":
            out = A.copy()
        else:
            out = A @ q["v"]
        if not client.on_result(out):
            return kinds


@pytest.mark.parametrize("scene,n", [("raster", 6), ("pt", 6)])
def test_client_takes_the_newton_step(monkeypatch, scene, n):
    monkeypatch.setattr(SV, "TRUST", 1e6)
    A, b = _quadratic(n, 3)
    spec = WL.ServingClient(scene, np.linspace(-0.3, 0.4, n), 11, 0.0)
    c = SV.NewtonClient(spec, scene=None, sigma=0.1, N=64, cg_iters=n)
    kinds = _drive(c, A, b)
    expected = -np.linalg.solve(A, A @ spec.theta0 + b)
    np.testing.assert_allclose(c.theta - spec.theta0, expected, rtol=1e-8, atol=1e-10)
    if scene == "pt":
        assert kinds == ["grad", "hess"]
    else:
        assert kinds[0] == "grad" and set(kinds[1:]) == {"hvp"} and len(kinds) <= n + 1


def test_client_step_is_clipped_to_the_trust_radius():
    A, b = _quadratic(4, 5)
    spec = WL.ServingClient("pt", np.zeros(4), 1, 0.0)
    c = SV.NewtonClient(spec, scene=None, sigma=0.1, N=64, cg_iters=4)
    _drive(c, 1e-3 * A, b)   # a flat quadratic: the Newton step is long
    assert np.linalg.norm(c.theta) == pytest.approx(SV.TRUST, rel=1e-12)


def test_serving_clients_are_seeded_and_mixed():
    a = WL.serving_clients(16, rate=100.0)
    b = WL.serving_clients(16, rate=100.0)
    assert [x.arrival for x in a] == [x.arrival for x in b]
    assert all(np.array_equal(x.theta0, y.theta0) for x, y in zip(a, b))
    assert [x.scene for x in a[:4]] == ["raster", "pt", "raster", "pt"]
    assert np.all(np.diff([x.arrival for x in a]) >= 0) and a[0].arrival == 0.0
    assert len({x.seed for x in a}) == 16


def test_closed_loop_plain_runner_serves_every_query(monkeypatch):
    """Closed loop: every client's queries are served, each after its think
    time; the per-kind counts match the clients' Newton steps."""
    A, b = _quadratic(6, 9)

    def exact(kind, scene, theta, sigma, N, seed, v=None):
        return {"grad": A @ theta + b, "hess": A.copy(), "hvp": None}[kind] if kind != "hvp" \
            else A @ v

    monkeypatch.setattr(SV, "estimate", exact)
    specs = WL.serving_clients(6, rate=1e6)
    for sp in specs:
        sp.theta0 = np.linspace(-0.2, 0.3, 6)
    clients = [SV.NewtonClient(sp, scene=None, sigma=0.1, N=64, cg_iters=4, full_cg=True)
               for sp in specs]
    out = SV.run_plain(None, clients, think_ms=2.0)
    kinds = out["by_kind"]
    assert kinds["raster_grad"]["queries"] == 3 and kinds["raster_hvp"]["queries"] == 12
    assert kinds["pt_grad"]["queries"] == 3 and kinds["pt_hess"]["queries"] == 3
    assert out["queries"] == 21
    # 21 queries, each preceded by a think time of mean 2 ms, on one server
    assert out["seconds"] > 0.005
    # the same think-time draws on a second run: same client trajectories
    clients2 = [SV.NewtonClient(sp, scene=None, sigma=0.1, N=64, cg_iters=4, full_cg=True)
                for sp in specs]
    SV.run_plain(None, clients2, think_ms=2.0)
    for c1, c2 in zip(clients, clients2):
        assert np.array_equal(c1.theta, c2.theta)


def test_closed_loop_window_stops_the_clients(monkeypatch):
    """With a measurement window, clients that would run for ever stop
    scheduling queries once the window has passed."""
    A, b = _quadratic(6, 4)
    monkeypatch.setattr(SV, "estimate", lambda kind, scene, theta, sigma, N, seed, v=None:
                        {"grad": A @ theta + b, "hess": A.copy()}.get(kind) if kind != "hvp"
                        else A @ v)
    specs = WL.serving_clients(4, rate=1e6)
    for sp in specs:
        sp.theta0 = np.zeros(6)
    clients = [SV.NewtonClient(sp, scene=None, sigma=0.1, N=64, cg_iters=3, steps=10 ** 6)
               for sp in specs]
    out = SV.run_plain(None, clients, think_ms=1.0, window_s=0.05)
    assert out["queries"] > 8
    assert out["seconds"] < 1.0
