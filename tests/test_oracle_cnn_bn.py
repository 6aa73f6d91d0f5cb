"""Pins for the FP64 denoiser with batch normalisation (oracle/cnn_bn.py):

* normalisation: the normalised values of every hidden layer have zero mean
  and variance var / (var + eps) per channel over the batch;
* reduction: with gamma = sqrt(var + eps) and beta = mu taken from the plain
  network's own pre-activations, batch normalisation is the identity and
  the output equals ``oracle.cnn`` without hidden biases (fails if the
  statistics run over a wrong axis, eps sits in the wrong place, or the
  normalisation moves relative to the ReLU);
* finite differences of g_gamma, g_beta, a weight and the input gradient
  (the batch-statistics terms of the reverse pass included);
* the slices of a batch are coupled: changing one changes the others."""
import numpy as np

from oracle import cnn, cnn_bn


def small_net(rng, ch=(2, 4, 4, 4, 4, 2), scale=0.5):
    return [(rng.standard_normal((ch[l + 1], ch[l], 3, 3)) * scale, rng.standard_normal(ch[l + 1]) * 0.1)
            for l in range(len(ch) - 1)]


def small_bn(rng, ch=(4, 4, 4, 4)):
    return [(1.0 + 0.3 * rng.standard_normal(c), 0.2 * rng.standard_normal(c)) for c in ch]


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_normalised_values(rng):
    x = rand_c(rng, 2, 6, 5)
    w, bn = small_net(rng), small_bn(rng)
    _, _, ys, yhats, istds = cnn_bn.net_forward(x, w, bn, keep=True)
    for y, yh in zip(ys, yhats):
        var = y.var(axis=(0, 1, 2))
        assert np.max(np.abs(yh.mean(axis=(0, 1, 2)))) < 1e-12
        assert np.max(np.abs(yh.var(axis=(0, 1, 2)) - var / (var + cnn_bn.EPS))) < 1e-12


def test_identity_normalisation_is_plain_network(rng):
    x = rand_c(rng, 3, 7, 6)
    w = small_net(rng)
    w0 = [(W, np.zeros_like(b)) if l < 4 else (W, b) for l, (W, b) in enumerate(w)]
    out, _, pres = cnn.net_forward(x, w0, keep=True)
    bn = []
    for l in range(4):
        y = pres[l]
        bn.append((np.sqrt(y.var(axis=(0, 1, 2)) + cnn_bn.EPS), y.mean(axis=(0, 1, 2))))
    got = cnn_bn.net_forward(x, w, bn)
    assert np.max(np.abs(got - out)) < 1e-12 * np.max(np.abs(out))


def test_backward_finite_differences(rng):
    x = rand_c(rng, 2, 5, 6)
    w, bn = small_net(rng), small_bn(rng)
    g = rand_c(rng, 2, 5, 6)
    L = lambda xx, ww, bb: np.sum(np.conj(g) * cnn_bn.denoise(xx, ww, bb)).real
    gx, grads, bng = cnn_bn.denoise_backward(x, w, bn, g)
    eps = 1e-6

    def fd(f):
        return (f(eps) - f(-eps)) / (2 * eps)

    for l, c in ((0, 1), (2, 3)):
        def fg(e, l=l, c=c):
            b2 = [(gg.copy(), bb.copy()) for gg, bb in bn]
            b2[l][0][c] += e
            return L(x, w, b2)

        def fb(e, l=l, c=c):
            b2 = [(gg.copy(), bb.copy()) for gg, bb in bn]
            b2[l][1][c] += e
            return L(x, w, b2)
        assert abs(fd(fg) - bng[l][0][c]) < 1e-6 * max(1.0, abs(bng[l][0][c]))
        assert abs(fd(fb) - bng[l][1][c]) < 1e-6 * max(1.0, abs(bng[l][1][c]))

    def fw(e):
        w2 = [(W.copy(), b.copy()) for W, b in w]
        w2[1][0][2, 3, 1, 0] += e
        return L(x, w2, bn)
    assert abs(fd(fw) - grads[1][0][2, 3, 1, 0]) < 1e-6 * max(1.0, abs(grads[1][0][2, 3, 1, 0]))

    def fwl(e):
        w2 = [(W.copy(), b.copy()) for W, b in w]
        w2[4][1][1] += e
        return L(x, w2, bn)
    assert abs(fd(fwl) - grads[4][1][1]) < 1e-6 * max(1.0, abs(grads[4][1][1]))
    for idx in ((0, 2, 3), (1, 4, 0)):
        for part in (1.0, 1j):
            def fx(e, idx=idx, part=part):
                x2 = x.copy()
                x2[idx] += e * part
                return L(x2, w, bn)
            got = gx[idx].real if part == 1.0 else gx[idx].imag
            assert abs(fd(fx) - got) < 1e-6 * max(1.0, abs(got))
    assert all(np.all(gb == 0) for _, gb in grads[:4])


def test_slices_are_coupled(rng):
    x = rand_c(rng, 2, 6, 6)
    w, bn = small_net(rng), small_bn(rng)
    a = cnn_bn.denoise(x, w, bn)
    x2 = x.copy()
    x2[1] *= 3.0
    b = cnn_bn.denoise(x2, w, bn)
    assert np.max(np.abs(a[0] - b[0])) > 1e-3
