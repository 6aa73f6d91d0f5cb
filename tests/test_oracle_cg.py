"""Pins for the FP64 CG oracle (oracle/cg.py): a dense direct solve of the
normal equations, the Krylov-subspace characterisation of the k-th CG
iterate, the monotone decrease of the energy-norm error, and finite
differences of the data-consistency derivative on converged problems."""
import numpy as np
import pytest

from oracle import cg, sense


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def dense_normal(S, m, lam):
    """Explicit matrix of (A^H A + lambda I) for one slice, column by column
    (applying the operator to unit vectors)."""
    _, C, H, W = S.shape
    n = H * W
    M = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros((1, H, W), dtype=np.complex128)
        e.flat[j] = 1.0
        M[:, j] = sense.sense_normal(e, S, m, [lam]).ravel()
    return M


@pytest.fixture
def tiny(rng):
    B, C, H, W = 1, 3, 8, 6
    S = rand_c(rng, B, C, H, W) * 0.5
    m = np.zeros((B, H)); m[0, [0, 2, 3, 4, 7]] = 1
    return S, m, 0.1


def test_cg_converges_to_dense_solve(rng, tiny):
    S, m, lam = tiny
    H, W = S.shape[2:]
    b = rand_c(rng, 1, H, W)
    M = dense_normal(S, m, lam)
    ref = np.linalg.solve(M, b.ravel()).reshape(1, H, W)
    x, hist = cg.cg(cg.normal_op(S, m, [lam]), b, H * W)
    assert np.linalg.norm(x - ref) < 1e-10 * np.linalg.norm(ref)
    # sanity: matrix is Hermitian positive definite
    assert np.max(np.abs(M - M.conj().T)) < 1e-13
    assert np.min(np.linalg.eigvalsh(M)) > 0


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_kth_iterate_is_krylov_minimiser(rng, tiny, k):
    """x_k = argmin over K_k(S, b) of the S-energy error, i.e.
    x_k = Q (Q^H S Q)^{-1} Q^H b with Q an orthonormal basis of
    span{b, Sb, ..., S^{k-1} b}."""
    S, m, lam = tiny
    H, W = S.shape[2:]
    b = rand_c(rng, 1, H, W)
    M = dense_normal(S, m, lam)
    vs = [b.ravel()]
    for _ in range(k - 1):
        vs.append(M @ vs[-1])
    Q, _ = np.linalg.qr(np.stack(vs, axis=1))
    ref = Q @ np.linalg.solve(Q.conj().T @ M @ Q, Q.conj().T @ b.ravel())
    x, _ = cg.cg(cg.normal_op(S, m, [lam]), b, k)
    assert np.linalg.norm(x.ravel() - ref) < 1e-10 * np.linalg.norm(ref)


def test_energy_error_decreases(rng, tiny):
    S, m, lam = tiny
    H, W = S.shape[2:]
    b = rand_c(rng, 1, H, W)
    M = dense_normal(S, m, lam)
    xs = np.linalg.solve(M, b.ravel())
    errs = []
    for k in range(0, 12):
        x, _ = cg.cg(cg.normal_op(S, m, [lam]), b, k)
        e = x.ravel() - xs
        errs.append(np.real(np.vdot(e, M @ e)))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))


def test_zero_rhs_is_safe(tiny):
    S, m, lam = tiny
    x, hist = cg.cg(cg.normal_op(S, m, [lam]), np.zeros((1, 8, 6), np.complex128), 5)
    assert np.all(x == 0) and np.all(hist == 0)


def test_residual_history_matches_definition(rng, tiny):
    S, m, lam = tiny
    b = rand_c(rng, 1, 8, 6)
    op = cg.normal_op(S, m, [lam])
    x, hist = cg.cg(op, b, 4)
    r = b - op(x)
    assert abs(hist[0, -1] - np.vdot(r, r).real) < 1e-9 * hist[0, 0]
    assert abs(hist[0, 0] - np.vdot(b, b).real) < 1e-12 * hist[0, 0]


def test_cg_dc_solves_regularised_problem(rng, tiny):
    S, m, lam = tiny
    a = rand_c(rng, 1, 8, 6)
    z = rand_c(rng, 1, 8, 6)
    M = dense_normal(S, m, lam)
    ref = np.linalg.solve(M, (a + lam * z).ravel()).reshape(a.shape)
    x, _ = cg.cg_dc(a, z, S, m, [lam], 48)
    assert np.linalg.norm(x - ref) < 1e-10 * np.linalg.norm(ref)
    x0, _ = cg.cg_dc(a, None, S, m, [lam], 48)
    ref0 = np.linalg.solve(M, a.ravel()).reshape(a.shape)
    assert np.linalg.norm(x0 - ref0) < 1e-10 * np.linalg.norm(ref0)


def test_cg_dc_backward_matches_finite_differences(rng, tiny):
    """L = Re<c, x(a, z, lambda)>; its DF^H(1) gradient w.r.t. x is c."""
    S, m, lam = tiny
    n = 48
    a, z, c = rand_c(rng, 1, 8, 6), rand_c(rng, 1, 8, 6), rand_c(rng, 1, 8, 6)

    def L(a_, z_, lam_):
        x, _ = cg.cg_dc(a_, z_, S, m, [lam_], n)
        return np.real(np.vdot(c, x))

    x, _ = cg.cg_dc(a, z, S, m, [lam], n)
    ga, gz, gl = cg.cg_dc_backward(c, x, z, S, m, [lam], n)
    eps = 1e-6
    for g, which in ((ga, "a"), (gz, "z")):
        d = rand_c(rng, 1, 8, 6)
        if which == "a":
            fd = (L(a + eps * d, z, lam) - L(a - eps * d, z, lam)) / (2 * eps)
        else:
            fd = (L(a, z + eps * d, lam) - L(a, z - eps * d, lam)) / (2 * eps)
        an = np.real(np.vdot(g, d))
        assert abs(fd - an) < 1e-7 * max(1.0, abs(an))
    fd = (L(a, z, lam + eps) - L(a, z, lam - eps)) / (2 * eps)
    assert abs(fd - gl[0]) < 1e-7 * max(1.0, abs(gl[0]))


def test_cg_dc_backward_closed_form(rng, tiny):
    S, m, lam = tiny
    n = 48
    a, z, g = rand_c(rng, 1, 8, 6), rand_c(rng, 1, 8, 6), rand_c(rng, 1, 8, 6)
    M = dense_normal(S, m, lam)
    Minv = np.linalg.inv(M)
    x = (Minv @ (a + lam * z).ravel()).reshape(a.shape)
    ga, gz, gl = cg.cg_dc_backward(g, x, z, S, m, [lam], n)
    v = Minv @ g.ravel()
    assert np.linalg.norm(ga.ravel() - v) < 1e-10 * np.linalg.norm(v)
    assert np.linalg.norm(gz.ravel() - lam * v) < 1e-10 * np.linalg.norm(v)
    ref_l = np.real(np.vdot(v, (z - x).ravel()))
    assert abs(gl[0] - ref_l) < 1e-10 * abs(ref_l)
