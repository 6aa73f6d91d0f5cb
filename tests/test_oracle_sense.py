"""Pins for the FP64 SENSE oracle (oracle/sense.py) against facts fixed by
the mathematics: a brute-force centered DFT, the adjoint identity, unitarity
(A^H A = I at full sampling with sum |S|^2 = 1), the mask's null space and the
1-D decoupling identity the GPU kernels use."""
import cmath

import numpy as np
import pytest

from oracle import sense


def naive_centered_dft_1d(N):
    """Brute-force matrix of the centered unitary DFT, entry by entry:
    F[k, n] = exp(-2 pi i (k - N//2)(n - N//2) / N) / sqrt(N)."""
    c = N // 2
    F = np.empty((N, N), dtype=np.complex128)
    for k in range(N):
        for n in range(N):
            F[k, n] = cmath.exp(-2j * cmath.pi * (k - c) * (n - c) / N) / N ** 0.5
    return F


def naive_dft2(x):
    """2-D transform by explicit quadruple sum (tiny sizes only)."""
    H, W = x.shape
    FH, FW = naive_centered_dft_1d(H), naive_centered_dft_1d(W)
    out = np.zeros((H, W), dtype=np.complex128)
    for k in range(H):
        for l in range(W):
            s = 0j
            for n in range(H):
                for m in range(W):
                    s += FH[k, n] * FW[l, m] * x[n, m]
            out[k, l] = s
    return out


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def unit_coils(rng, B, C, H, W):
    S = rand_c(rng, B, C, H, W)
    return S / np.sqrt(np.sum(np.abs(S) ** 2, axis=1, keepdims=True))


@pytest.mark.parametrize("H,W", [(6, 10), (12, 15), (20, 18), (5, 8)])
def test_fft2c_matches_bruteforce_dft(rng, H, W):
    x = rand_c(rng, H, W)
    ref = naive_dft2(x)
    got = sense.fft2c(x)
    assert np.max(np.abs(got - ref)) < 1e-13 * max(1.0, np.max(np.abs(ref)))
    back = sense.ifft2c(got)
    assert np.max(np.abs(back - x)) < 1e-13


def test_constant_image_gives_centred_delta():
    H, W = 16, 12
    got = sense.fft2c(np.full((H, W), 2.0 + 0j))
    ref = np.zeros((H, W), dtype=np.complex128)
    ref[H // 2, W // 2] = 2.0 * np.sqrt(H * W)
    assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("N", [8, 12, 10, 6])
def test_centered_dft_checkerboard_form(rng, N):
    """For even N: F_c x = s * chk * FFT(chk * x) with chk = (-1)^n and
    s = +1 when N % 4 == 0, -1 when N % 4 == 2 (the form the GPU uses)."""
    x = rand_c(rng, N)
    chk = (-1.0) ** np.arange(N)
    s = 1.0 if N % 4 == 0 else -1.0
    ref = naive_centered_dft_1d(N) @ x
    got = s * chk * np.fft.fft(chk * x) / np.sqrt(N)
    assert np.max(np.abs(got - ref)) < 1e-13


def test_adjoint_identity(rng):
    B, C, H, W = 2, 3, 10, 12
    S = rand_c(rng, B, C, H, W)
    m = (rng.random((B, H)) < 0.5).astype(np.float64)
    x = rand_c(rng, B, H, W)
    y = rand_c(rng, B, C, H, W)
    lhs = np.vdot(y, sense.sense_fwd(x, S, m))          # <Ax, y>^*
    rhs = np.vdot(sense.sense_adj(y, S, m), x)          # <x, A^H y>^*
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_full_sampling_is_identity(rng):
    B, C, H, W = 2, 4, 12, 10
    S = unit_coils(rng, B, C, H, W)
    m = np.ones((B, H))
    x = rand_c(rng, B, H, W)
    got = sense.sense_normal(x, S, m, np.zeros(B))
    assert np.max(np.abs(got - x)) < 1e-14 * 10


def test_empty_mask_gives_lambda_identity(rng):
    B, C, H, W = 2, 3, 8, 6
    S = rand_c(rng, B, C, H, W)
    x = rand_c(rng, B, H, W)
    lam = np.array([0.3, 0.0])
    got = sense.sense_normal(x, S, np.zeros((B, H)), lam)
    assert np.max(np.abs(got - lam[:, None, None] * x)) < 1e-15


def test_forward_zero_on_unsampled_rows(rng):
    B, C, H, W = 1, 2, 10, 8
    S = rand_c(rng, B, C, H, W)
    m = np.zeros((B, H)); m[0, [1, 4, 5]] = 1
    y = sense.sense_fwd(rand_c(rng, B, H, W), S, m)
    assert np.all(y[:, :, m[0] == 0, :] == 0)
    assert np.all(np.abs(y[:, :, m[0] == 1, :]) > 0)


def test_normal_operator_hermitian_psd(rng):
    B, C, H, W = 1, 3, 8, 10
    S = rand_c(rng, B, C, H, W)
    m = (rng.random((B, H)) < 0.4).astype(np.float64)
    x, z = rand_c(rng, B, H, W), rand_c(rng, B, H, W)
    Nx = sense.sense_normal(x, S, m, [0.0])
    Nz = sense.sense_normal(z, S, m, [0.0])
    assert abs(np.vdot(z, Nx) - np.vdot(Nz, x)) < 1e-12 * abs(np.vdot(z, Nx))
    q = np.vdot(x, Nx)
    assert abs(q.imag) < 1e-12 * abs(q) and q.real >= 0


@pytest.mark.parametrize("H,W", [(8, 6), (12, 20), (10, 10)])
def test_decoupled_1d_normal_equals_2d(rng, H, W):
    B, C = 2, 3
    S = rand_c(rng, B, C, H, W)
    m = (rng.random((B, H)) < 0.5).astype(np.float64)
    x = rand_c(rng, B, H, W)
    lam = np.array([0.05, 1.0])
    a = sense.sense_normal(x, S, m, lam)
    b = sense.sense_normal_1d(x, S, m, lam)
    assert np.max(np.abs(a - b)) < 1e-13


def test_measure_adds_noise_only_on_sampled_rows(rng):
    B, C, H, W = 1, 2, 8, 8
    S = rand_c(rng, B, C, H, W)
    m = np.zeros((B, H)); m[0, ::2] = 1
    x = rand_c(rng, B, H, W)
    n = rand_c(rng, B, C, H, W)
    y = sense.measure(x, S, m, n)
    assert np.allclose(y - sense.sense_fwd(x, S, m), m[:, None, :, None] * n, atol=1e-13)
