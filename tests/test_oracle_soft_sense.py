"""Pins for the FP64 soft-SENSE oracle (several coil-map sets, Extensions to
the SENSE-Model subsection): one set reduces to SENSE, the adjoint identity,
the folding that the two-set layout of the synthetic inputs stands for (the
k-space of the folded coil images is every second line of the extended
k-space, the paper's reduced-FOV simulation), CG against a dense solve, and
finite differences of the soft MoDL reverse pass and the coil-image loss."""
import numpy as np
import pytest

from oracle import cg, sense
from oracle import soft_sense as ss
from synthetic import soft_slice_inputs


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_one_set_is_sense(rng):
    B, C, H, W = 2, 3, 8, 6
    x, S, y = rand_c(rng, B, H, W), rand_c(rng, B, C, H, W), rand_c(rng, B, C, H, W)
    m = (rng.random((B, H)) < 0.5).astype(np.float64)
    assert np.max(np.abs(ss.soft_fwd(x[:, None], S[:, None], m) - sense.sense_fwd(x, S, m))) < 1e-13
    assert np.max(np.abs(ss.soft_adj(y, S[:, None], m)[:, 0] - sense.sense_adj(y, S, m))) < 1e-13
    lam = [0.3, 0.7]
    assert np.max(np.abs(ss.soft_normal(x[:, None], S[:, None], m, lam)[:, 0]
                         - sense.sense_normal(x, S, m, lam))) < 1e-13
    a = sense.sense_adj(y, S, m)
    xs, hs = ss.soft_cg_dc(a[:, None], None, S[:, None], m, lam, 5)
    xc, hc = cg.cg_dc(a, None, S, m, lam, 5)
    assert np.max(np.abs(xs[:, 0] - xc)) < 1e-12 and np.max(np.abs(hs - hc)) < 1e-12 * hc.max()


def test_adjoint_identity_two_sets(rng):
    B, M, C, H, W = 2, 2, 3, 10, 12
    x, S, y = rand_c(rng, B, M, H, W), rand_c(rng, B, M, C, H, W), rand_c(rng, B, C, H, W)
    m = (rng.random((B, H)) < 0.5).astype(np.float64)
    lhs = np.vdot(ss.soft_fwd(x, S, m), y)
    rhs = np.vdot(x, ss.soft_adj(y, S, m))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_two_set_layout_is_the_fold_of_twice_the_field_of_view():
    """Coil images of the two-set layout = the extended coil images folded
    once along H (central H rows plus the rows H away), and their centered
    k-space = sqrt(2) x every second line of the extended centered k-space:
    the reduced-FOV data the paper's soft-SENSE experiment simulates."""
    H, W, C = 16, 12, 4
    d = soft_slice_inputs(3, H, W, C, 4, 4)
    u = d["S_ext"].astype(np.complex128) * d["x_ext"].astype(np.complex128)[None]  # [C, 2H, W]
    fold = np.array([u[:, (i + H // 2) % (2 * H)] + u[:, (i + 3 * H // 2) % (2 * H)] for i in range(H)])
    fold = np.moveaxis(fold, 0, 1)
    coil = ss.coil_images(d["x"][None], d["S"][None])[0]
    assert np.max(np.abs(coil - fold)) < 1e-6  # complex64 inputs
    k_fold = sense.fft1c(coil, 1)
    k_ext = sense.fft1c(u, 1)
    assert np.max(np.abs(k_fold - np.sqrt(2) * k_ext[:, ::2])) < 1e-6
    assert np.abs(d["x"][1]).max() > 0.05  # the object does exceed the field of view


def test_soft_cg_matches_dense_solve(rng):
    B, M, C, H, W = 1, 2, 3, 8, 6
    S = rand_c(rng, B, M, C, H, W) * 0.5
    m = np.zeros((B, H)); m[0, [0, 2, 3, 5]] = 1
    lam = [0.4]
    n = M * H * W
    A = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128); e[j] = 1
        A[:, j] = ss.soft_normal(e.reshape(1, M, H, W), S, m, lam).ravel()
    assert np.max(np.abs(A - A.conj().T)) < 1e-12
    b = rand_c(rng, B, M, H, W)
    x, _ = ss.soft_cg_dc(b, None, S, m, lam, n)
    ref = np.linalg.solve(A, b.ravel())
    assert np.max(np.abs(x.ravel() - ref)) < 1e-9 * np.max(np.abs(ref))


@pytest.fixture
def tiny_soft(rng):
    B, M, C, H, W = 1, 2, 2, 8, 8
    S = rand_c(rng, B, M, C, H, W) * 0.5
    m = np.zeros((B, H)); m[0, [0, 3, 4, 6]] = 1
    x_true = rand_c(rng, B, M, H, W)
    ref = ss.coil_images(x_true, S)
    aHy = ss.soft_adj(ss.soft_fwd(x_true, S, m), S, m)
    return S, m, aHy, ref


def test_coil_mse_gradient_finite_differences(rng, tiny_soft):
    S, m, aHy, ref = tiny_soft
    x = rand_c(rng, *aHy.shape)
    g = ss.coil_mse_grad(x, S, ref)
    d = rand_c(rng, *x.shape)
    eps = 1e-6
    fd = (ss.coil_mse(x + eps * d, S, ref) - ss.coil_mse(x - eps * d, S, ref)) / (2 * eps)
    an = np.real(np.vdot(g, d))
    assert abs(fd - an) < 1e-6 * max(1e-3, abs(an))


def test_soft_modl_backward_finite_differences(rng, tiny_soft):
    S, m, aHy, ref = tiny_soft
    w = [(rng.standard_normal((6, 2, 3, 3)) * 0.4, rng.standard_normal(6) * 0.1),
         (rng.standard_normal((2, 6, 3, 3)) * 0.4, rng.standard_normal(2) * 0.1)]
    lam, T, n = [0.7], 2, 128

    def loss(w_, lam_, a_=aHy):
        return ss.coil_mse(ss.modl_forward(a_, S, m, w_, lam_, T, n)[0], S, ref)

    xT, states, zs = ss.modl_forward(aHy, S, m, w, lam, T, n)
    gW, gl, ga = ss.modl_backward(ss.coil_mse_grad(xT, S, ref), states, zs, aHy, S, m, w, lam, T, n)
    eps = 1e-6
    for l in range(len(w)):
        dW, db = rng.standard_normal(w[l][0].shape), rng.standard_normal(w[l][1].shape)
        wp = [(Wt + (eps * dW if i == l else 0), b + (eps * db if i == l else 0)) for i, (Wt, b) in enumerate(w)]
        wm = [(Wt - (eps * dW if i == l else 0), b - (eps * db if i == l else 0)) for i, (Wt, b) in enumerate(w)]
        fd = (loss(wp, lam) - loss(wm, lam)) / (2 * eps)
        an = np.sum(gW[l][0] * dW) + np.sum(gW[l][1] * db)
        assert abs(fd - an) < 1e-6 * max(1e-3, abs(an)), (l, fd, an)
    fd = (loss(w, [lam[0] + eps]) - loss(w, [lam[0] - eps])) / (2 * eps)
    assert abs(fd - gl[0]) < 1e-6 * max(1e-3, abs(gl[0]))
    d = rand_c(rng, *aHy.shape)
    fd = (loss(w, lam, aHy + eps * d) - loss(w, lam, aHy - eps * d)) / (2 * eps)
    an = np.real(np.vdot(ga, d))
    assert abs(fd - an) < 1e-6 * max(1e-3, abs(an))


def test_network_updates_the_first_set_only(rng, tiny_soft):
    """One unroll: z = (D(x_1), x_2), so the second set's component of the
    data-consistency right-hand side is x_2 whatever the weights."""
    S, m, aHy, _ = tiny_soft
    w = [(rng.standard_normal((6, 2, 3, 3)), rng.standard_normal(6)),
         (rng.standard_normal((2, 6, 3, 3)), rng.standard_normal(2))]
    _, _, zs = ss.modl_forward(aHy, S, m, w, [0.5], 1, 4)
    assert np.array_equal(zs[0][:, 1], aHy[:, 1])
    assert np.max(np.abs(zs[0][:, 0] - aHy[:, 0])) > 1e-3
