"""Pins for the FP64 iPALM oracle and the VarNet constraint projections:
iPALM on a non-negative least-squares problem reaches scipy's NNLS solution,
the inertia schedule, and the projection's feasibility, idempotence and
optimality against random feasible points."""
import numpy as np
import scipy.optimize

from oracle import ipalm


def test_ipalm_solves_nonnegative_least_squares(rng):
    A = rng.standard_normal((30, 12))
    b = rng.standard_normal(30)
    L = 2 * np.linalg.norm(A, 2) ** 2
    grad = lambda y: {"x": 2 * A.T @ (A @ y["x"] - b)}
    prox = lambda d: {"x": np.maximum(d["x"], 0.0)}
    th = {"x": np.zeros(12)}
    prev = th
    for k in range(1, 3001):
        th, prev = ipalm.step(th, prev, k, 1.0 / L, grad, prox)
    ref, _ = scipy.optimize.nnls(A, b)
    assert np.max(np.abs(th["x"] - ref)) < 1e-8
    assert np.any(ref == 0)  # the constraint is active


def test_inertia_schedule_and_first_step_is_proximal_gradient(rng):
    assert ipalm.alpha(1) == 0.0 and abs(ipalm.alpha(4) - 0.5) < 1e-15
    th = {"x": rng.standard_normal(5)}
    g = rng.standard_normal(5)
    new, prev = ipalm.step(th, th, 1, 0.1, lambda y: {"x": g}, lambda d: d)
    assert np.max(np.abs(new["x"] - (th["x"] - 0.1 * g))) < 1e-15 and prev is th
    th2 = {"x": rng.standard_normal(5)}
    new2, _ = ipalm.step(th2, th, 4, 0.0, lambda y: {"x": 0 * y["x"]}, lambda d: d)
    assert np.max(np.abs(new2["x"] - (th2["x"] + 0.5 * (th2["x"] - th["x"])))) < 1e-15


def test_filter_projection_is_the_nearest_feasible_point(rng):
    v = rng.standard_normal((3, 4, 11, 11)) + 1j * rng.standard_normal((3, 4, 11, 11))
    p = ipalm.project_filters(v)
    assert np.max(np.abs(p.mean(axis=(-2, -1)))) < 1e-15
    assert np.max(np.abs(np.sum(np.abs(p) ** 2, axis=(-2, -1)) - 1)) < 1e-12
    assert np.max(np.abs(ipalm.project_filters(p) - p)) < 1e-15
    d0 = np.sum(np.abs(v - p) ** 2, axis=(-2, -1))
    for _ in range(20):
        u = ipalm.project_filters(rng.standard_normal(v.shape) + 1j * rng.standard_normal(v.shape))
        assert np.all(d0 <= np.sum(np.abs(v - u) ** 2, axis=(-2, -1)) + 1e-12)
    z = np.full((1, 1, 11, 11), 2.0 + 1.0j)
    assert np.all(ipalm.project_filters(z) == 0)
    lam = ipalm.project_vn({"k": v, "w": np.ones(3), "lam": np.array([-0.1, 0.0, 0.3])})["lam"]
    assert list(lam) == [0.0, 0.0, 0.3]
