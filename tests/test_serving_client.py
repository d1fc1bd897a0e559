"""Host-side logic of the serving load generator (no GPU): a client's Newton
step is the exact Newton step when fed exact derivatives of a quadratic."""
import numpy as np
import pytest

import workloads as WL
from paper_2412_03489_amd import serving as SV


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
