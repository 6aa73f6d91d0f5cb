"""Pins for the FP64 CNN, MoDL and Adam oracles: library cross-correlation,
identity kernels, finite differences of every backward pass on tiny
converged problems, and Adam's closed-form first step."""
import numpy as np
import pytest
import scipy.signal

from oracle import adam, cg, cnn, modl, sense
from synthetic import cnn_weights


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_conv_matches_scipy_correlate(rng):
    B, H, W, Ci, Co = 2, 7, 9, 3, 4
    a = rng.standard_normal((B, H, W, Ci))
    Wt = rng.standard_normal((Co, Ci, 3, 3))
    bias = rng.standard_normal(Co)
    got = cnn.conv3x3(a, Wt, bias)
    for b in range(B):
        for o in range(Co):
            ref = bias[o] + sum(
                scipy.signal.correlate2d(a[b, :, :, i], Wt[o, i], mode="same", boundary="fill")
                for i in range(Ci))
            assert np.max(np.abs(got[b, :, :, o] - ref)) < 1e-12


def test_identity_kernel_returns_input(rng):
    a = rng.standard_normal((1, 5, 6, 3))
    Wt = np.zeros((3, 3, 3, 3))
    for i in range(3):
        Wt[i, i, 1, 1] = 1.0
    assert np.max(np.abs(cnn.conv3x3(a, Wt, np.zeros(3)) - a)) == 0


def test_conv_backward_finite_differences(rng):
    B, H, W, Ci, Co = 1, 5, 4, 2, 3
    a = rng.standard_normal((B, H, W, Ci))
    Wt = rng.standard_normal((Co, Ci, 3, 3))
    bias = rng.standard_normal(Co)
    g = rng.standard_normal((B, H, W, Co))
    ga, gW, gb = cnn.conv3x3_backward(a, Wt, g)
    L = lambda a_, W_, b_: np.sum(g * cnn.conv3x3(a_, W_, b_))
    eps = 1e-6
    da, dW, db = rng.standard_normal(a.shape), rng.standard_normal(Wt.shape), rng.standard_normal(Co)
    fd = (L(a + eps * da, Wt, bias) - L(a - eps * da, Wt, bias)) / (2 * eps)
    assert abs(fd - np.sum(ga * da)) < 1e-7 * max(1, abs(fd))
    fd = (L(a, Wt + eps * dW, bias) - L(a, Wt - eps * dW, bias)) / (2 * eps)
    assert abs(fd - np.sum(gW * dW)) < 1e-7 * max(1, abs(fd))
    fd = (L(a, Wt, bias + eps * db) - L(a, Wt, bias - eps * db)) / (2 * eps)
    assert abs(fd - np.sum(gb * db)) < 1e-7 * max(1, abs(fd))


def small_weights(rng, channels=(2, 8, 8, 2)):
    return [(rng.standard_normal((channels[l + 1], channels[l], 3, 3)) * 0.4,
             rng.standard_normal(channels[l + 1]) * 0.1) for l in range(len(channels) - 1)]


def test_denoiser_backward_finite_differences(rng):
    x = rand_c(rng, 1, 6, 5)
    w = small_weights(rng)
    g = rand_c(rng, 1, 6, 5)
    L = lambda x_, w_: np.real(np.vdot(g, cnn.denoise(x_, w_)))
    gx, gw = cnn.denoise_backward(x, w, g)
    eps = 1e-6
    d = rand_c(rng, 1, 6, 5)
    fd = (L(x + eps * d, w) - L(x - eps * d, w)) / (2 * eps)
    assert abs(fd - np.real(np.vdot(gx, d))) < 1e-7 * max(1, abs(fd))
    for l in range(len(w)):
        dW = rng.standard_normal(w[l][0].shape)
        wp = [(W + (eps * dW if i == l else 0), b) for i, (W, b) in enumerate(w)]
        wm = [(W - (eps * dW if i == l else 0), b) for i, (W, b) in enumerate(w)]
        fd = (L(x, wp) - L(x, wm)) / (2 * eps)
        assert abs(fd - np.sum(gw[l][0] * dW)) < 1e-7 * max(1, abs(fd))


def test_he_init_statistics():
    w = cnn_weights(7)
    assert [W.shape for W, _ in w] == [(64, 2, 3, 3), (64, 64, 3, 3), (64, 64, 3, 3),
                                       (64, 64, 3, 3), (2, 64, 3, 3)]
    W2 = w[1][0].astype(np.float64)
    assert abs(W2.std() - np.sqrt(2 / (9 * 64))) < 0.02 * np.sqrt(2 / (9 * 64))
    assert cnn.n_params((2, 64, 64, 64, 64, 2)) == 112896 + 258


@pytest.fixture
def tiny_problem(rng):
    B, C, H, W = 1, 2, 8, 8
    S = rand_c(rng, B, C, H, W) * 0.6
    m = np.zeros((B, H)); m[0, [0, 3, 4, 6]] = 1
    x_true = rand_c(rng, B, H, W)
    y = sense.sense_fwd(x_true, S, m)
    aHy = sense.sense_adj(y, S, m)
    return S, m, aHy, x_true


def test_modl_single_unroll_with_zero_net_is_dc_of_input(tiny_problem):
    """With all-zero weights N(x) = 0 so D(x) = x and one unroll is
    (A^H A + lam)^{-1} (A^H y + lam A^H y)."""
    S, m, aHy, _ = tiny_problem
    w = [(np.zeros((8, 2, 3, 3)), np.zeros(8)), (np.zeros((2, 8, 3, 3)), np.zeros(2))]
    lam = 0.5
    xT, _, _ = modl.forward(aHy, S, m, w, [lam], 1, 64)
    ref, _ = cg.cg_dc(aHy, aHy, S, m, [lam], 64)
    assert np.max(np.abs(xT - ref)) < 1e-13


def test_modl_backward_finite_differences(rng, tiny_problem):
    S, m, aHy, x_true = tiny_problem
    w = small_weights(rng)
    lam, T, n = [0.7], 2, 64

    def loss(w_, lam_):
        xT, _, _ = modl.forward(aHy, S, m, w_, lam_, T, n)
        return modl.mse(xT, x_true)

    xT, states, zs = modl.forward(aHy, S, m, w, lam, T, n)
    g = modl.mse_grad(xT, x_true)
    gW, gl, _ = modl.backward(g, states, zs, aHy, S, m, w, lam, T, n)
    eps = 1e-6
    for l in range(len(w)):
        dW = rng.standard_normal(w[l][0].shape)
        db = rng.standard_normal(w[l][1].shape)
        wp = [(W + (eps * dW if i == l else 0), b + (eps * db if i == l else 0)) for i, (W, b) in enumerate(w)]
        wm = [(W - (eps * dW if i == l else 0), b - (eps * db if i == l else 0)) for i, (W, b) in enumerate(w)]
        fd = (loss(wp, lam) - loss(wm, lam)) / (2 * eps)
        an = np.sum(gW[l][0] * dW) + np.sum(gW[l][1] * db)
        assert abs(fd - an) < 1e-6 * max(1e-3, abs(an)), (l, fd, an)
    fd = (loss(w, [lam[0] + eps]) - loss(w, [lam[0] - eps])) / (2 * eps)
    assert abs(fd - gl[0]) < 1e-6 * max(1e-3, abs(gl[0]))


def test_modl_input_gradient_finite_differences(rng, tiny_problem):
    S, m, aHy, x_true = tiny_problem
    w = small_weights(rng)
    lam, T, n = [0.7], 2, 64
    loss = lambda a_: modl.mse(modl.forward(a_, S, m, w, lam, T, n)[0], x_true)
    xT, states, zs = modl.forward(aHy, S, m, w, lam, T, n)
    _, _, ga = modl.backward(modl.mse_grad(xT, x_true), states, zs, aHy, S, m, w, lam, T, n)
    d = rand_c(rng, *aHy.shape)
    eps = 1e-6
    fd = (loss(aHy + eps * d) - loss(aHy - eps * d)) / (2 * eps)
    an = np.real(np.vdot(ga, d))
    assert abs(fd - an) < 1e-6 * max(1e-3, abs(an))


def test_mse_grad_finite_differences(rng):
    x, r = rand_c(rng, 2, 3, 4), rand_c(rng, 2, 3, 4)
    g = modl.mse_grad(x, r)
    d = rand_c(rng, 2, 3, 4)
    eps = 1e-6
    fd = (modl.mse(x + eps * d, r) - modl.mse(x - eps * d, r)) / (2 * eps)
    assert abs(fd - np.real(np.vdot(g, d))) < 1e-8


def test_adam_first_step_closed_form(rng):
    w0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 1e-3, 1e-8
    w1, m1, v1 = adam.step(w0, g, np.zeros(50), np.zeros(50), 1, lr=lr, eps=eps)
    assert np.max(np.abs(w1 - (w0 - lr * g / (np.abs(g) + eps)))) < 1e-15
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_adam_constant_gradient_moves_lr_per_step(rng):
    w = rng.standard_normal(10)
    g = np.sign(rng.standard_normal(10)) * 2.0
    m = v = np.zeros(10)
    w0 = w.copy()
    for t in range(1, 6):
        w, m, v = adam.step(w, g, m, v, t, lr=1e-2, eps=0.0)
    assert np.max(np.abs(w - (w0 - 5 * 1e-2 * np.sign(g)))) < 1e-12


def test_bf16_rounding_matches_torch_and_ties_to_even(rng):
    import torch
    a = rng.standard_normal(1000).astype(np.float32) * 10.0 ** rng.integers(-5, 5, 1000)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16_round(a), ref)
    one_plus_half_ulp = np.float32(1.0 + 2.0 ** -8)   # halfway between 1 and 1 + 2^-7
    three_halves = np.float32(1.0 + 3 * 2.0 ** -8)     # halfway between 1 + 2^-7 and 1 + 2^-6
    assert cnn.bf16_round(one_plus_half_ulp) == 1.0
    assert cnn.bf16_round(three_halves) == 1.0 + 2.0 ** -6


def hand_net():
    import json, os
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "denoise_hand_worked.json")))
    weights = []
    for cw, b in zip(d["centre_weights"], d["biases"]):
        cw = np.asarray(cw, dtype=np.float64)
        Wt = np.full(cw.shape + (3, 3), d["other_taps"])
        Wt[:, :, 1, 1] = cw
        weights.append((Wt, np.asarray(b, dtype=np.float64)))
    c = lambda a: np.array([complex(*v) for v in a]).reshape(-1, 1, 1)
    return d, weights, c


def test_denoise_hand_worked_example():
    """Values worked by hand (tests/golden/denoise_hand_worked.json): fails if
    the ReLU moves to the last layer, a ReLU, a bias or the residual is
    dropped, the channel order flips or the padding is not zero."""
    d, weights, c = hand_net()
    assert np.array_equal(cnn.denoise(c(d["x"]), weights), c(d["D"]))
    gx, grads = cnn.denoise_backward(c(d["x"]), weights, c(d["g"]))
    assert np.array_equal(gx, c(d["g_x"]))
    for l, (gW, gb) in enumerate(grads):
        want = np.zeros_like(gW)
        want[:, :, 1, 1] = d["grad_centre_weights_summed"][l]
        assert np.array_equal(gW, want), l
        assert np.array_equal(gb, d["grad_biases_summed"][l]), l


def test_bf16_mode_rounds_exactly_the_convolution_operands(rng):
    """Two-layer net computed independently with scipy's 2-D correlation and
    convolution: bf16 rounding of every convolution operand (layer inputs,
    weights, the gradients entering each reverse convolution), float64 for
    sums, biases, ReLU, bias gradients and the residual."""
    q = cnn.bf16_round
    B, H, W = 1, 5, 6
    x = rand_c(rng, B, H, W)
    g = rand_c(rng, B, H, W)
    w = small_weights(rng, (2, 3, 2))
    gx, grads = cnn.denoise_backward(x, w, g, bf16=True)
    out = cnn.denoise(x, w, bf16=True)
    corr = lambda a, k: scipy.signal.correlate2d(a, k, mode="same", boundary="fill")
    conv = lambda a, k: scipy.signal.convolve2d(a, k, mode="same", boundary="fill")
    wgrad = lambda d_, a: scipy.signal.correlate2d(np.pad(a, 1), d_, mode="valid")
    (W0, b0), (W1, b1) = w
    a0 = [q(x[0].real), q(x[0].imag)]
    pre0 = [b0[o] + sum(corr(a0[i], q(W0[o, i])) for i in range(2)) for o in range(3)]
    a1 = [q(np.maximum(p, 0)) for p in pre0]
    pre1 = [b1[o] + sum(corr(a1[i], q(W1[o, i])) for i in range(3)) for o in range(2)]
    assert np.max(np.abs(out[0] - (x[0] + pre1[0] + 1j * pre1[1]))) < 1e-12
    d1 = [g[0].real, g[0].imag]
    gb1 = [d1[o].sum() for o in range(2)]
    gW1 = np.array([[wgrad(q(d1[o]), a1[i]) for i in range(3)] for o in range(2)])
    ga1 = [sum(conv(q(d1[o]), q(W1[o, i])) for o in range(2)) for i in range(3)]
    d0 = [ga1[i] * (pre0[i] > 0) for i in range(3)]
    gb0 = [d0[o].sum() for o in range(3)]
    gW0 = np.array([[wgrad(q(d0[o]), a0[i]) for i in range(2)] for o in range(3)])
    ga0 = [sum(conv(q(d0[o]), q(W0[o, i])) for o in range(3)) for i in range(2)]
    assert np.max(np.abs(grads[1][0] - gW1)) < 1e-12
    assert np.max(np.abs(grads[1][1] - gb1)) < 1e-12
    assert np.max(np.abs(grads[0][0] - gW0)) < 1e-12
    assert np.max(np.abs(grads[0][1] - gb0)) < 1e-12
    assert np.max(np.abs(gx[0] - (g[0] + ga0[0] + 1j * ga0[1]))) < 1e-12


def test_bf16_mode_is_close_to_fp64(rng):
    x = rand_c(rng, 1, 12, 10)
    w = small_weights(rng)
    a = cnn.denoise(x, w)
    b = cnn.denoise(x, w, bf16=True)
    assert 0 < np.linalg.norm(a - b) / np.linalg.norm(a) < 2e-2
