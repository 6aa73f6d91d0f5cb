"""Pins for the FP64 variational-network oracle (oracle/vn.py): the paper's
parameter count, the adjoint pairing of K and K^T, a library
cross-correlation, the RBF knots and finite differences of the stage."""
import json
import os

import numpy as np
import scipy.signal

from oracle import sense, vn

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_parameter_count_matches_paper():
    g = json.load(open(GOLDEN))
    assert vn.n_params(g["vn_T"], g["vn_filters"], g["vn_kernel"], g["vn_rbf"]) == g["vn_real_params"]


def test_filter_matches_scipy(rng):
    x = rand_c(rng, 1, 9, 8)
    k = rand_c(rng, 2, 5, 5)
    s = vn.filt(x, k)
    for i in range(2):
        ref = (scipy.signal.correlate2d(x[0].real, k[i].real, mode="same")
               - scipy.signal.correlate2d(x[0].imag, k[i].imag, mode="same"))
        assert np.max(np.abs(s[0, i] - ref)) < 1e-12


def test_filter_adjoint_pairing(rng):
    x = rand_c(rng, 2, 10, 7)
    k = rand_c(rng, 3, 5, 5)
    u = rng.standard_normal((2, 3, 10, 7))
    lhs = np.sum(vn.filt(x, k) * u)
    rhs = np.real(np.vdot(x, vn.filt_adj(u, k)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_rbf_unit_weight_is_gaussian_at_knot():
    w = np.zeros((1, 31)); w[0, 10] = 1.0
    mu, sig = vn.knots(31)
    s = np.array([mu[10], mu[10] + sig]).reshape(1, 1, 1, 2)
    p1, p2, _ = vn.rbf(s, w)
    assert abs(p1.ravel()[0] - 1.0) < 1e-15
    assert abs(p1.ravel()[1] - np.exp(-0.5)) < 1e-15
    assert abs(p2.ravel()[1] - (-1.0 / sig) * np.exp(-0.5)) < 1e-12


def _problem(rng):
    B, C, H, W = 1, 2, 8, 10
    S = rand_c(rng, B, C, H, W) * 0.5
    m = np.zeros((B, H)); m[0, [0, 2, 5]] = 1
    aHy = sense.sense_adj(sense.sense_fwd(rand_c(rng, B, H, W), S, m), S, m)
    x = rand_c(rng, B, H, W) * 0.3
    k = rand_c(rng, 3, 5, 5) * 0.2
    w = rng.standard_normal((3, 31)) * 0.3
    return S, m, aHy, x, k, w, 0.3


def test_stage_backward_finite_differences(rng):
    S, m, aHy, x, k, w, lam = _problem(rng)
    g = rand_c(rng, *x.shape)
    L = lambda x_, k_, w_, l_: np.real(np.vdot(g, vn.stage(x_, aHy, S, m, k_, w_, l_)))
    gx, gk, gw, gl = vn.stage_backward(g, x, aHy, S, m, k, w, lam)
    eps = 1e-6
    d = rand_c(rng, *x.shape)
    fd = (L(x + eps * d, k, w, lam) - L(x - eps * d, k, w, lam)) / (2 * eps)
    assert abs(fd - np.real(np.vdot(gx, d))) < 1e-7 * max(1, abs(fd))
    dk = rand_c(rng, *k.shape)
    fd = (L(x, k + eps * dk, w, lam) - L(x, k - eps * dk, w, lam)) / (2 * eps)
    assert abs(fd - np.real(np.vdot(gk, dk))) < 1e-7 * max(1, abs(fd))
    dw = rng.standard_normal(w.shape)
    fd = (L(x, k, w + eps * dw, lam) - L(x, k, w - eps * dw, lam)) / (2 * eps)
    assert abs(fd - np.sum(gw * dw)) < 1e-7 * max(1, abs(fd))
    fd = (L(x, k, w, lam + eps) - L(x, k, w, lam - eps)) / (2 * eps)
    assert abs(fd - gl) < 1e-7 * max(1, abs(fd))


def fd_rich(f, eps):
    """Central difference with one Richardson step (error O(eps^4)): the RBF
    activations have large higher derivatives (width 2/30)."""
    d1 = (f(eps) - f(-eps)) / (2 * eps)
    d2 = (f(eps / 2) - f(-eps / 2)) / eps
    return (4 * d2 - d1) / 3


def test_stack_backward_finite_differences(rng):
    S, m, aHy, _, k, w, lam = _problem(rng)
    params = {"k": np.stack([k, 0.5 * k]), "w": np.stack([w, -w]), "lam": np.array([lam, 0.2])}
    g = rand_c(rng, *aHy.shape)
    L = lambda p: np.real(np.vdot(g, vn.forward(aHy, S, m, p)[0]))
    _, states = vn.forward(aHy, S, m, params)
    gk, gw, gl, _ = vn.backward(g, states, aHy, S, m, params)
    eps = 1e-5
    dk = rand_c(rng, *params["k"].shape)
    fd = fd_rich(lambda e: L(dict(params, k=params["k"] + e * dk)), eps)
    assert abs(fd - np.real(np.vdot(gk, dk))) < 1e-7 * max(1, abs(fd))
    dw = rng.standard_normal(params["w"].shape)
    fd = fd_rich(lambda e: L(dict(params, w=params["w"] + e * dw)), eps)
    assert abs(fd - np.sum(gw * dw)) < 1e-7 * max(1, abs(fd))
    fd = fd_rich(lambda e: L(dict(params, lam=params["lam"] + np.array([0, e]))), eps)
    assert abs(fd - gl[1]) < 1e-7 * max(1, abs(fd))


def test_zero_filters_reduce_to_gradient_step(rng):
    S, m, aHy, x, k, w, lam = _problem(rng)
    out = vn.stage(x, aHy, S, m, np.zeros_like(k), w, lam)
    ref = x - lam * (sense.sense_normal(x, S, m, [0.0]) - aHy)
    assert np.max(np.abs(out - ref)) < 1e-14
