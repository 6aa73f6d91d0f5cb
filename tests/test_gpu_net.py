"""Parity of the HIP denoiser (bf16 MFMA convolutions), the MoDL unrolled
network and its reverse pass, the MSE gradient and Adam against the FP64
oracle, through the C-ABI.

Forward: network outputs NRMSE <= 1e-2 against the plain FP64 oracle (bf16
operands, fp32 accumulation), per-pixel error <= 2e-2 of the largest value.

Reverse pass, reference of record: the oracle with bf16 convolution operands
(oracle.cnn, bf16=True: every operand of a convolution rounded to bf16, all
sums, biases, ReLU decisions and bias gradients in fp64).  Two correct
implementations of that definition that differ only in the order or width
of their sums do not agree to fp32 rounding: a stored activation whose fp32
and fp64 values straddle a bf16 rounding boundary differs by one bf16 step
(2^-7 relative), shifts the pre-activations it feeds, and so on -- in the
oracle itself, fp32 against fp64 accumulation gives 6, 45, 271 and 1656
differing activations in the four ReLU layers of one 320 x 320 phantom, and
the few of those that cross zero flip a ReLU decision, passing or blocking a
whole gradient value; in smooth image regions a channel's pre-activation
crosses zero along a contour, so flips come in clusters.  Measured between
the two oracle variants on the 4 x 320 x 320 phantom batch: J^T 2.6e-3
(per-pixel 3.5e-2), dW <= 2.0e-3, db <= 3.2e-3; on 320 x 320 noise images
3.4e-3.  Hence two bounds:
  * DECISION_FREE_TOL = 3e-3 where no ReLU decision is within reach of
    rounding (biases that keep every pre-activation half a standard
    deviation above zero): what remains is accumulation order and one-step
    rounding differences -- measured between the two oracle variants on the
    4 x 320 x 320 batch: <= 2.5e-4 except the last layer's dW, 9.0e-4 (its
    activations are large, so each one-step difference weighs more), with
    single entries at 3.3e-3; per-element bound 1e-2;
  * GRAD_TOL = 2e-2 with ReLU decisions (He-init weights, phantom inputs):
    about six times the largest spread measured between correct orders (a
    kernel is one more order, with its own flip clusters).
Bias gradients are fp32 sums of the unrounded gradients on both sides and
take the same bounds.
Plain FP64 is reported for every reverse pass; the kernels must be no further
from it than the bf16-operand definition itself plus the bound.  Per-pixel
bounds apply to forward outputs and decision-free reverse passes; with ReLU
decisions a flipped decision moves a neighbourhood by up to the local
gradient value, which the global bound covers and a per-pixel one cannot.

MoDL reverse pass: the oracle is driven with the HIP forward's own stored
states x^t, so each unroll's denoiser sees the same input on both sides; the
upstream gradients entering the denoiser then differ only by the fp32 CG error
(<= 1e-4): weight gradients <= GRAD_TOL; g_lambda and g_aHy <= 1e-3 (the
gradient tolerance; they are CG-adjoint terms).
Elementwise fp32 kernels (MSE, Adam): 1e-5.
"""
import numpy as np
import pytest
import torch

from oracle import adam as oadam
from oracle import cnn as ocnn
from oracle import modl as omodl
from oracle import sense as osense
from paper_2202_14005_amd import ops
from synthetic import cnn_weights
from tests.gpu_util import dev, host, inputs, maxrel, oracle_threads, rel, uneven

pytestmark = pytest.mark.gpu

NET_TOL = 1e-2
NET_PIXEL_TOL = 2e-2
GRAD_TOL = 2e-2           # reverse pass with ReLU decisions, against the bf16-operand oracle
DECISION_FREE_TOL = 3e-3  # reverse pass with no ReLU decision near zero
DECISION_FREE_ELEM_TOL = 1e-2
CG_GRAD_TOL = 1e-3        # g_lambda, g_aHy of the MoDL reverse pass


def weights(seed=7, last_scale=1.0):
    return cnn_weights(seed, last_scale=last_scale)


def all_active(xs, w, margin=0.5):
    """Biases for layers 1-4 that put every pre-activation at the inputs xs
    (complex slices of any shapes) at least `margin` of its channel's
    standard deviation above zero (batch statistics), computed layer by layer with the plain
    FP64 oracle; the last layer's bias is kept."""
    acts = [ocnn.to_channels(np.asarray(x, dtype=np.complex128)[None]) for x in xs]
    out = []
    for l, (Wt, b) in enumerate(w):
        if l < len(w) - 1:
            pres = [ocnn.conv3x3(a, Wt, np.zeros(len(b))) for a in acts]
            flat = np.concatenate([p.reshape(-1, len(b)) for p in pres])
            b = margin * flat.std(0) - flat.min(0)
            acts = [np.maximum(p + b, 0) for p in pres]
        out.append((Wt, np.asarray(b, dtype=np.float32)))
    return out


@pytest.mark.parametrize("B,H,W", [(2, 48, 40), (1, 320, 320), (2, 24, 16), (1, 96, 128)])
def test_cnn_forward_parity(B, H, W):
    d = inputs([300 + i for i in range(B)], H, W, 2)
    w = weights()
    plan = ops.Plan(H, W, 2, B=B, network=True)
    cnn = ops.CNN.from_numpy(w)
    z = host(plan.cnn_forward(dev(d["x"]), cnn))
    zref = ocnn.denoise(d["x"], w)
    nref = zref - d["x"]
    e_z, e_n, p_n = rel(z, zref), rel(z - d["x"], nref), maxrel(z - d["x"], nref)
    print(f"cnn fwd {B}x{H}x{W}: NRMSE z {e_z:.2e}, N(x) {e_n:.2e}, per-pixel N(x) {p_n:.2e}")
    assert e_z < NET_TOL
    assert e_n < NET_TOL
    assert p_n < NET_PIXEL_TOL


def cnn_backward_case(shapes, seed, w_fn):
    """HIP reverse pass of the denoiser on a batch of slices [(H, W), ...]
    (packed) and the oracle's, per slice, with bf16 operands and in plain
    FP64.  w_fn(xs) gives the weights.  Returns HIP (g_x, grads), the two
    oracle results (g_x packed, grads), the upstream gradient (packed) and
    the objects needed to call again."""
    rng = np.random.default_rng(seed)
    xs, gs = [], []
    for i, (H, W) in enumerate(shapes):
        xs.append(inputs([seed + i], H, W, 2)["x"][0])
        gs.append((rng.standard_normal((H, W)) + 1j * rng.standard_normal((H, W))).astype(np.complex64))
    w = w_fn(xs)
    plan = ops.Plan([s[0] for s in shapes], [s[1] for s in shapes], [2] * len(shapes), network=True)
    cnn = ops.CNN.from_numpy(w)
    grads = ops.CNNGrads(cnn)
    flat = lambda arrs: np.concatenate([a.ravel() for a in arrs])
    gx = host(plan.cnn_backward(dev(flat(xs)), dev(flat(gs)), cnn, grads)).ravel()
    got = (gx, [(host(grads.w[l]), host(grads.b[l])) for l in range(5)])
    refs = []
    with oracle_threads():
        for bf16 in (True, False):
            gxr, gw = [], None
            for x, g in zip(xs, gs):
                a, lg = ocnn.denoise_backward(x[None], w, g[None], bf16=bf16)
                gxr.append(a[0])
                gw = lg if gw is None else [(p[0] + q[0], p[1] + q[1]) for p, q in zip(gw, lg)]
            refs.append((flat(gxr), gw))
    return got, refs, flat(gs), (plan, cnn, grads, xs, gs)


BACKWARD_SHAPES = [
    ("2x48x40", [(48, 40)] * 2),
    # the training batch: 3200 weight-gradient tiles, ~12.5 per workgroup of
    # the 256-workgroup kernel and ~3 per workgroup of the 1024-workgroup ones
    ("4x320x320", [(320, 320)] * 4),
    # uneven: workgroup tile ranges cross slice boundaries, ragged 40-column slice
    ("uneven", [(320, 320), (192, 256), (48, 40), (96, 128)]),
]


def check_backward(name, got, refs, g, tol, pixel_tol):
    (gx, gw), (ref, ref64) = got, refs
    e, p = rel(gx - g, ref[0] - g), maxrel(gx - g, ref[0] - g)
    e_def, e64 = rel(ref[0] - g, ref64[0] - g), rel(gx - g, ref64[0] - g)
    print(f"cnn bwd {name} J^T gz: vs bf16-operand oracle {e:.2e} (per-pixel {p:.2e}); "
          f"vs fp64 {e64:.2e} (bf16-operand oracle vs fp64 {e_def:.2e})")
    assert e < tol
    assert pixel_tol is None or p < pixel_tol
    assert e64 < e_def + tol
    for l in range(5):
        (w_, b_), (wr, br) = gw[l], ref[1][l]
        ew, pw, eb = rel(w_, wr), maxrel(w_, wr), rel(b_, br)
        ew64, ed = rel(w_, ref64[1][l][0]), rel(wr, ref64[1][l][0])
        print(f"  layer {l}: dW {ew:.2e} (max {pw:.2e}) db {eb:.2e}; dW vs fp64 {ew64:.2e} "
              f"(bf16-operand oracle vs fp64 {ed:.2e})")
        assert ew < tol and eb < tol
        assert pixel_tol is None or pw < pixel_tol
        assert ew64 < ed + tol


@pytest.mark.parametrize("name,shapes", BACKWARD_SHAPES)
def test_cnn_backward_parity(name, shapes):
    got, refs, g, _ = cnn_backward_case(shapes, 310, lambda xs: weights())
    check_backward(name, got, refs, g, GRAD_TOL, None)


@pytest.mark.parametrize("name,shapes", BACKWARD_SHAPES)
def test_cnn_backward_decision_free(name, shapes):
    """No ReLU decision within reach of rounding: biases keep every
    pre-activation of layers 1-4 above zero by half of its channel's standard
    deviation in FP64 (at least a tenth with bf16 operands, against ~1e-6
    of accumulation-order noise), so the comparison sees the convolution
    arithmetic alone (weight-gradient tile walks included)."""
    got, refs, g, (plan, cnn, grads, xs, gs) = cnn_backward_case(
        shapes, 330, lambda xs: all_active(xs, weights()))
    w = cnn.numpy()
    with oracle_threads():
        pres = [ocnn.net_forward(x[None], w, keep=True, bf16=True)[2][:4] for x in xs]
    margin = min(float(np.min(np.concatenate([q[l].reshape(-1, 64) for q in pres]).min(0)
                              / np.concatenate([q[l].reshape(-1, 64) for q in pres]).std(0))) for l in range(4))
    print(f"decision-free {name}: smallest pre-activation {margin:.3f} of its channel's standard deviation")
    assert margin > 0.1
    check_backward(name, got, refs, g, DECISION_FREE_TOL, DECISION_FREE_ELEM_TOL)


def test_cnn_backward_accumulates():
    got, refs, g, (plan, cnn, grads, xs, gs) = cnn_backward_case([(48, 40)] * 2, 310, lambda xs: weights())
    plan.cnn_backward(dev(np.stack(xs)), dev(np.stack(gs)), cnn, grads, accumulate=True)
    for l in range(5):
        assert rel(host(grads.w[l]), 2 * got[1][l][0]) < 1e-6
        assert rel(host(grads.b[l]), 2 * got[1][l][1]) < 1e-6


def test_cnn_uneven_batch():
    shapes = [(48, 40, 2), (32, 64, 2), (96, 48, 2)]
    sl, pk = uneven(shapes, seed0=700)
    w = weights()
    plan = ops.Plan([s[0] for s in shapes], [s[1] for s in shapes], [s[2] for s in shapes], network=True)
    cnn = ops.CNN.from_numpy(w)
    z = host(plan.cnn_forward(dev(pk["x"]), cnn))
    o = 0
    for (H, W, _), s in zip(shapes, sl):
        zref = ocnn.denoise(s["x"][None], w)
        assert rel(z[o:o + H * W], zref) < NET_TOL
        o += H * W


def modl_case(B, H, W, C, seed=400):
    d = inputs([seed + i for i in range(B)], H, W, C)
    y = osense.measure(d["x"], d["S"], d["mask"], d["noise"])
    aHy = osense.sense_adj(y, d["S"], d["mask"]).astype(np.complex64)
    return d, aHy


@pytest.mark.parametrize("B,H,W,C,T", [(2, 48, 40, 4, 2), (1, 320, 320, 15, 5), (2, 48, 40, 4, 10)])
def test_modl_forward_parity(B, H, W, C, T):
    d, aHy = modl_case(B, H, W, C)
    w = weights(last_scale=0.1)
    lam = np.full(B, 0.05, dtype=np.float32)
    plan = ops.Plan(H, W, C, B=B, network=True)
    cnn = ops.CNN.from_numpy(w)
    x, st = plan.modl_forward(dev(aHy), dev(d["S"]), dev(d["mask"]), cnn, torch.tensor(lam), T, 10, states=True)
    xref, sref, _ = omodl.forward(aHy, d["S"], d["mask"], w, lam, T, 10)
    e = rel(host(x), xref)
    print(f"modl fwd {B}x{H}x{W} T={T}: NRMSE {e:.2e}")
    assert e < NET_TOL
    assert np.array_equal(host(st)[T], host(x))
    assert np.array_equal(host(st)[0], aHy)


@pytest.mark.parametrize("B,H,W,C,T", [(2, 48, 40, 4, 5), (1, 320, 320, 15, 2)])
def test_modl_backward_parity(B, H, W, C, T):
    """The oracle's reverse pass driven from the HIP forward's stored states
    x^0..x^T (and z^t = D(x^t) recomputed by the oracle), so each unroll's
    denoiser sees the same input on both sides."""
    d, aHy = modl_case(B, H, W, C, seed=420)
    w = weights(last_scale=0.1)
    lam = np.full(B, 0.05, dtype=np.float32)
    plan = ops.Plan(H, W, C, B=B, network=True)
    cnn = ops.CNN.from_numpy(w)
    S, m = dev(d["S"]), dev(d["mask"])
    xT, st = plan.modl_forward(dev(aHy), S, m, cnn, torch.tensor(lam), T, 10, states=True)
    loss, g = plan.mse_grad(xT, dev(d["x"]))
    grads = ops.CNNGrads(cnn)
    gl, ga = plan.modl_backward(g, st, dev(aHy), S, m, cnn, torch.tensor(lam), T, 10, grads, need_aHy=True)
    states = [s.astype(np.complex128) for s in host(st)]
    gref = omodl.mse_grad(states[T], d["x"])
    assert abs(float(host(loss)[0]) - omodl.mse(states[T], d["x"])) < 1e-5 * omodl.mse(states[T], d["x"])
    res = {}
    with oracle_threads():
        for bf16 in (True, False):
            zs = [ocnn.denoise(states[t], w, bf16=bf16) for t in range(T)]
            res[bf16] = omodl.backward(gref, states, zs, aHy, d["S"], d["mask"], w, lam, T, 10, bf16=bf16)
    (gw_ref, gl_ref, ga_ref), (gw64, gl64, ga64) = res[True], res[False]
    for l in range(5):
        ew, eb = rel(host(grads.w[l]), gw_ref[l][0]), rel(host(grads.b[l]), gw_ref[l][1])
        pw = maxrel(host(grads.w[l]), gw_ref[l][0])
        ew64, ed = rel(host(grads.w[l]), gw64[l][0]), rel(gw_ref[l][0], gw64[l][0])
        print(f"modl layer {l}: dW {ew:.2e} (max {pw:.2e}) db {eb:.2e}; dW vs fp64 {ew64:.2e} "
              f"(bf16-operand oracle vs fp64 {ed:.2e})")
        assert ew < GRAD_TOL and eb < GRAD_TOL and pw < GRAD_TOL
        assert ew64 < ed + GRAD_TOL
    el = np.max(np.abs(host(gl) - gl_ref) / np.abs(gl_ref))
    ea, pa = rel(host(ga), ga_ref), maxrel(host(ga), ga_ref)
    el64 = np.max(np.abs(host(gl) - gl64) / np.abs(gl64))
    ea64, ead = rel(host(ga), ga64), rel(ga_ref, ga64)
    print(f"modl g_lambda {el:.2e} (vs fp64 {el64:.2e}) g_aHy {ea:.2e} (per-pixel {pa:.2e}; vs fp64 {ea64:.2e}, "
          f"bf16-operand oracle vs fp64 {ead:.2e})")
    assert el < CG_GRAD_TOL and ea < CG_GRAD_TOL and pa < 2 * CG_GRAD_TOL
    assert ea64 < ead + CG_GRAD_TOL


def test_mse_grad_parity():
    B, H, W = 2, 64, 48
    d = inputs([500, 501], H, W, 2)
    rng = np.random.default_rng(9)
    x = (d["x"] + 0.1 * rng.standard_normal(d["x"].shape)).astype(np.complex64)
    plan = ops.Plan(H, W, 2, B=B, network=True)
    loss, g = plan.mse_grad(dev(x), dev(d["x"]))
    assert abs(float(host(loss)[0]) - omodl.mse(x, d["x"])) < 1e-5 * omodl.mse(x, d["x"])
    assert rel(host(g), omodl.mse_grad(x, d["x"])) < 1e-6


def test_adam_parity():
    w = cnn_weights(3)
    cnn = ops.CNN.from_numpy(w)
    opt = ops.Adam(cnn, lr=1e-3)
    rng = np.random.default_rng(2)
    grads = ops.CNNGrads(cnn)
    ref = [p.copy().astype(np.float64) for pair in w for p in pair]
    m = [np.zeros_like(r) for r in ref]
    v = [np.zeros_like(r) for r in ref]
    for t in range(1, 4):
        gs = [rng.standard_normal(r.shape).astype(np.float32) for r in ref]
        for gt, g in zip(grads.params(), gs):
            gt.copy_(torch.from_numpy(g))
        opt.step(grads)
        for i in range(len(ref)):
            ref[i], m[i], v[i] = oadam.step(ref[i], gs[i], m[i], v[i], t, lr=1e-3)
    for p, r in zip(cnn.params(), ref):
        assert np.max(np.abs(host(p) - r)) < 1e-6
    assert cnn.version == 3


def test_sub_batch_plans_on_two_streams_equal_one_plan():
    """Slices are independent: the batch run as two sub-batch plans on two
    concurrent streams (same column schedule) gives the single plan's MoDL
    output bit for bit -- no state is shared between plans or launches."""
    B, H, W, C, T = 4, 48, 40, 4, 2
    d, aHy = modl_case(B, H, W, C)
    cnn = ops.CNN.from_numpy(weights(last_scale=0.1))
    lam = 0.05
    S, m, a = dev(d["S"]), dev(d["mask"]), dev(aHy)
    sched = ops.schedules(H)[0]
    plan = ops.Plan(H, W, C, B=B, network=True)
    plan.set_schedule(H, sched)
    ref = plan.modl_forward(a, S, m, cnn, plan.lam(lam), T, 10)
    main = torch.cuda.current_stream()
    parts = []
    for j in range(2):
        sl = slice(2 * j, 2 * j + 2)
        p = ops.Plan(H, W, C, B=2, network=True)
        p.set_schedule(H, sched)
        parts.append((p, a[sl], S[sl], m[sl], torch.cuda.Stream()))
    for rep in range(3):
        outs = []
        for p, a_j, S_j, m_j, s_j in parts:
            s_j.wait_stream(main)
            with torch.cuda.stream(s_j):
                outs.append(p.modl_forward(a_j, S_j, m_j, cnn, p.lam(lam), T, 10))
        for *_, s_j in parts:
            main.wait_stream(s_j)
        assert torch.equal(torch.cat(outs, 0), ref), rep


@pytest.mark.parametrize("B,H,W,C", [(2, 48, 40, 4), (1, 320, 320, 15), (3, 24, 16, 3)])
def test_modl_fused_first_layers_equal_separate_kernels(B, H, W, C):
    """MoDL inference runs the first two denoiser layers as one kernel (the
    first layer's activation stays in LDS); the reverse pass and
    cnn_forward use the separate kernels.  Both round the first layer's
    output to bf16 the same way, so one unroll of modl_forward equals
    cnn_forward followed by cg_dc bit for bit (ragged tiles included)."""
    d, aHy = modl_case(B, H, W, C)
    cnn = ops.CNN.from_numpy(weights(last_scale=0.1))
    plan = ops.Plan(H, W, C, B=B, network=True)
    S, m, a = dev(d["S"]), dev(d["mask"]), dev(aHy)
    lam = plan.lam(0.05)
    fused = plan.modl_forward(a, S, m, cnn, lam, 1, 10)
    z = plan.cnn_forward(a, cnn)
    separate = plan.cg_dc(a, S, m, lam, 10, z=z)
    assert torch.equal(fused, separate)
