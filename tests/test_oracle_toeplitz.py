"""Pins for the FP64 non-Cartesian oracle (Extensions to the SENSE-Model
subsection: the nuFFT SENSE operator and its normal operator as a PSF
convolution, the Toeplitz trick).

* the non-uniform DFT against brute-force sums written element by element;
* a trajectory on the Cartesian grid (the sampled rows of a row mask) gives
  the Cartesian SENSE operator of ``oracle.sense``, whose own pins (naive
  DFT, A^H A = I at full sampling) then carry over;
* the Toeplitz form equals the definition A^H A = F^H P^H P F on random
  off-grid trajectories (odd and even sizes, H != W);
* adjoint identity, Hermitian positive semi-definite normal operator, real
  PSF spectrum, the PSF at offset 0 is M / (HW);
* CG against a dense solve of the normal equations; MoDL's first unroll with
  an identity denoiser.
"""
import numpy as np
import pytest

from oracle import cg, sense
from oracle import toeplitz as tp
from synthetic import noncart_slice_inputs, radial_trajectory


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def rand_traj(rng, B, M, H, W):
    t = np.empty((B, M, 2))
    t[..., 0] = rng.uniform(-H / 2, H / 2, (B, M))
    t[..., 1] = rng.uniform(-W / 2, W / 2, (B, M))
    return t


def test_nudft_brute_force(rng):
    B, C, H, W, M = 1, 2, 5, 4, 7
    x, S = rand_c(rng, B, H, W), rand_c(rng, B, C, H, W)
    traj = rand_traj(rng, B, M, H, W)
    y = tp.nudft_fwd(x, S, traj)
    yb = np.zeros((B, C, M), dtype=complex)
    for c in range(C):
        for j in range(M):
            ky, kx = traj[0, j]
            acc = 0j
            for r in range(H):
                for s in range(W):
                    ph = -2 * np.pi * (ky * (r - H // 2) / H + kx * (s - W // 2) / W)
                    acc += S[0, c, r, s] * x[0, r, s] * complex(np.cos(ph), np.sin(ph))
            yb[0, c, j] = acc / np.sqrt(H * W)
    assert np.max(np.abs(y - yb)) < 1e-12 * np.max(np.abs(yb))
    g = rand_c(rng, B, C, M)
    xa = tp.nudft_adj(g, S, traj)
    xb = np.zeros((B, H, W), dtype=complex)
    for r in range(H):
        for s in range(W):
            acc = 0j
            for c in range(C):
                for j in range(M):
                    ky, kx = traj[0, j]
                    ph = 2 * np.pi * (ky * (r - H // 2) / H + kx * (s - W // 2) / W)
                    acc += np.conj(S[0, c, r, s]) * g[0, c, j] * complex(np.cos(ph), np.sin(ph))
            xb[0, r, s] = acc / np.sqrt(H * W)
    assert np.max(np.abs(xa - xb)) < 1e-12 * np.max(np.abs(xb))


@pytest.mark.parametrize("H,W", [(8, 6), (10, 10), (6, 9)])
def test_grid_trajectory_is_cartesian_sense(rng, H, W):
    """Sampled rows of a row mask as a trajectory: A, A^H and A^H A equal the
    Cartesian SENSE operator's (k-space sample (l, s) of the centred DFT is
    the point (l - H/2, s - W/2))."""
    B, C = 2, 3
    x, S = rand_c(rng, B, H, W), rand_c(rng, B, C, H, W)
    m = np.zeros((B, H))
    for b in range(B):
        m[b, rng.choice(H, size=H // 2, replace=False)] = 1.0
    rows = [np.flatnonzero(m[b]) for b in range(B)]
    traj = np.stack([np.array([(l - H // 2, s - W // 2) for l in rows[b] for s in range(W)], dtype=float)
                     for b in range(B)])
    y = tp.nudft_fwd(x, S, traj)
    yc = sense.sense_fwd(x, S, m)
    for b in range(B):
        assert np.max(np.abs(y[b] - yc[b][:, rows[b]].reshape(C, -1))) < 1e-12
    lam = [0.0, 0.4]
    ref = sense.sense_normal(x, S, m, lam)
    assert np.max(np.abs(tp.normal_direct(x, S, traj, lam) - ref)) < 1e-12
    assert np.max(np.abs(tp.normal(x, S, tp.psf(traj, H, W), lam) - ref)) < 1e-12


def test_full_grid_is_identity(rng):
    """Every grid point once, sum_c |S_c|^2 = 1: A^H A = I (the pin of the
    Cartesian oracle at full sampling, through the PSF form)."""
    H, W, C = 8, 10, 3
    S = rand_c(rng, 1, C, H, W)
    S /= np.sqrt(np.sum(np.abs(S) ** 2, axis=1, keepdims=True))
    traj = np.array([[(l - H // 2, s - W // 2) for l in range(H) for s in range(W)]], dtype=float)
    x = rand_c(rng, 1, H, W)
    assert np.max(np.abs(tp.normal(x, S, tp.psf(traj, H, W)) - x)) < 1e-12


@pytest.mark.parametrize("H,W,M", [(8, 8, 40), (7, 10, 33), (12, 6, 50)])
def test_toeplitz_equals_definition(rng, H, W, M):
    B, C = 2, 3
    x, S = rand_c(rng, B, H, W), rand_c(rng, B, C, H, W)
    traj = rand_traj(rng, B, M, H, W)
    lam = [0.1, 0.0]
    ref = tp.normal_direct(x, S, traj, lam)
    got = tp.normal(x, S, tp.psf(traj, H, W), lam)
    assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref))


def test_adjoint_identity_and_psd(rng):
    B, C, H, W, M = 2, 4, 9, 8, 60
    x, S = rand_c(rng, B, H, W), rand_c(rng, B, C, H, W)
    traj = rand_traj(rng, B, M, H, W)
    y = rand_c(rng, B, C, M)
    lhs = np.vdot(tp.nudft_fwd(x, S, traj), y)
    rhs = np.vdot(x, tp.nudft_adj(y, S, traj))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    P = tp.psf(traj, H, W)
    u = rand_c(rng, B, H, W)
    a = np.vdot(u, tp.normal(x, S, P))
    b = np.vdot(tp.normal(u, S, P), x)
    assert abs(a - b) < 1e-11 * abs(a)  # self-adjoint
    q = np.sum(np.conj(x) * tp.normal(x, S, P), axis=(1, 2))
    assert np.all(q.real > 0) and np.max(np.abs(q.imag) / q.real) < 1e-12


def test_psf_spectrum_real_and_centre(rng):
    H, W, M = 10, 8, 37
    traj = rand_traj(rng, 1, M, H, W)
    spec = tp.psf_spectrum(traj, H, W)
    assert np.max(np.abs(spec.imag)) < 1e-12 * np.max(np.abs(spec.real))
    h = tp.psf_kernel(traj[0], H, W)
    assert abs(h[0, 0] - M / (H * W)) < 1e-14
    assert np.all(h[H, :] == 0) and np.all(h[:, W] == 0)
    # Hermitian symmetry of the cyclic kernel
    idx_y, idx_x = (-np.arange(2 * H)) % (2 * H), (-np.arange(2 * W)) % (2 * W)
    assert np.max(np.abs(h - np.conj(h[np.ix_(idx_y, idx_x)]))) < 1e-15


def test_cg_dense_solve(rng):
    B, C, H, W, M = 1, 2, 5, 4, 30
    S = rand_c(rng, B, C, H, W)
    traj = rand_traj(rng, B, M, H, W)
    P = tp.psf(traj, H, W)
    lam = 0.05
    n = H * W
    Amat = np.zeros((n, n), dtype=complex)
    for i in range(n):
        e = np.zeros((1, H, W), dtype=complex)
        e.flat[i] = 1.0
        Amat[:, i] = tp.normal_direct(e, S, traj, lam).ravel()
    b = rand_c(rng, B, H, W)
    xd = np.linalg.solve(Amat, b.ravel()).reshape(1, H, W)
    xc, _ = tp.cg_dc(b, None, S, P, lam, 3 * n)
    assert np.max(np.abs(xc - xd)) < 1e-8 * np.max(np.abs(xd))


def test_modl_first_unroll_with_identity_denoiser(rng):
    """Zero weights make D the identity (residual network), so the first
    unroll is the data-consistency solve with z = x^0; T = 0 returns x^0."""
    B, C, H, W, M = 1, 2, 6, 6, 40
    S = rand_c(rng, B, C, H, W)
    traj = rand_traj(rng, B, M, H, W)
    P = tp.psf(traj, H, W)
    aHy = tp.nudft_adj(rand_c(rng, B, C, M), S, traj)
    x0 = tp.sense_init(aHy, S, P, 0.1, 3 * H * W)
    ch = [2, 64, 64, 64, 64, 2]
    zero = [(np.zeros((ch[l + 1], ch[l], 3, 3)), np.zeros(ch[l + 1])) for l in range(5)]
    out0, st0, _ = tp.modl_forward(x0, aHy, S, P, zero, 0.1, 0, 8)
    assert np.array_equal(out0, x0) and len(st0) == 1
    out, states, zs = tp.modl_forward(x0, aHy, S, P, zero, 0.1, 1, 8)
    assert np.max(np.abs(zs[0] - x0)) < 1e-15
    ref, _ = tp.cg_dc(aHy, x0, S, P, 0.1, 8)
    assert np.max(np.abs(out - ref)) < 1e-15
    # the SENSE start (CG run to convergence) solves the Tikhonov normal equations
    r = tp.normal(x0, S, P, 0.1) - aHy
    assert np.linalg.norm(r) < 1e-8 * np.linalg.norm(aHy)


def test_radial_generator_covers_the_extent():
    t = radial_trajectory(3, 32, 24, 11, 64)
    assert t.shape == (11 * 64, 2) and t.dtype == np.float32
    assert t[:, 0].min() >= -16 and t[:, 0].max() < 16 and t[:, 1].min() >= -12 and t[:, 1].max() < 12
    d = noncart_slice_inputs(5, 16, 16, 4, 5, 32)
    assert d["noise"].shape == (4, 160)


def test_adjoint_at_pixels_matches_full(rng):
    B, C, H, W, M = 2, 3, 7, 6, 25
    S = rand_c(rng, B, C, H, W)
    traj = rand_traj(rng, B, M, H, W)
    y = rand_c(rng, B, C, M)
    full = tp.nudft_adj(y, S, traj)
    pix = [(0, 0, 0), (1, 6, 5), (1, 3, 2), (0, 4, 1)]
    got = tp.nudft_adj_pixels(y, S, traj, pix)
    assert np.max(np.abs(got - np.array([full[b, r, s] for b, r, s in pix]))) < 1e-13


def test_modl_backward_finite_differences(rng):
    """g_lambda and one weight entry of the non-Cartesian MoDL reverse pass
    against central differences of L = Re<g, x^T>."""
    from oracle import cnn as ocnn
    B, C, H, W, M = 1, 2, 6, 6, 30
    S = rand_c(rng, B, C, H, W) * 0.5
    traj = rand_traj(rng, B, M, H, W)
    P = tp.psf(traj, H, W)
    aHy = tp.nudft_adj(rand_c(rng, B, C, M), S, traj)
    ch = [2, 4, 4, 4, 4, 2]
    wts = [(rng.standard_normal((ch[l + 1], ch[l], 3, 3)) * 0.3, rng.standard_normal(ch[l + 1]) * 0.1)
           for l in range(5)]
    lam, T, n = 0.3, 2, 60
    x0 = tp.sense_init(aHy, S, P, lam, n)
    g = rand_c(rng, B, H, W)
    xT, states, zs = tp.modl_forward(x0, aHy, S, P, wts, lam, T, n)
    gW, gl, _, _ = tp.modl_backward(g, states, zs, aHy, S, P, wts, lam, T, n)
    L = lambda x: np.sum(np.conj(g) * x).real
    eps = 1e-6
    lp = L(tp.modl_forward(x0, aHy, S, P, wts, lam + eps, T, n)[0])
    lm = L(tp.modl_forward(x0, aHy, S, P, wts, lam - eps, T, n)[0])
    assert abs((lp - lm) / (2 * eps) - gl[0]) < 1e-5 * max(1.0, abs(gl[0]))
    w2 = [(W_.copy(), b_.copy()) for W_, b_ in wts]
    w2[2][0][1, 3, 0, 2] += eps
    lp = L(tp.modl_forward(x0, aHy, S, P, w2, lam, T, n)[0])
    w2[2][0][1, 3, 0, 2] -= 2 * eps
    lm = L(tp.modl_forward(x0, aHy, S, P, w2, lam, T, n)[0])
    assert abs((lp - lm) / (2 * eps) - gW[2][0][1, 3, 0, 2]) < 1e-5 * max(1.0, abs(gW[2][0][1, 3, 0, 2]))


def test_forward_at_samples_matches_full(rng):
    B, C, H, W, M = 2, 3, 6, 8, 21
    x, S = rand_c(rng, B, H, W), rand_c(rng, B, C, H, W)
    traj = rand_traj(rng, B, M, H, W)
    full = tp.nudft_fwd(x, S, traj)
    sm = [(0, 0), (1, 20), (0, 7)]
    got = tp.nudft_fwd_samples(x, S, traj, sm)
    assert np.max(np.abs(got - np.array([full[b, :, j] for b, j in sm]))) < 1e-13
