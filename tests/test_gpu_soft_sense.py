"""Soft-SENSE (two coil-map sets) on the GPU against the FP64 oracle
(oracle/soft_sense.py), through the C-ABI: the forward, adjoint and normal
operators (<= 1e-5), the CG solve (<= 1e-4), MoDL with the network on the
first set (output NRMSE <= 1e-2 against plain FP64; reverse pass from the
HIP states against the bf16-operand definition, the bounds of
tests/test_gpu_net.py), the coil-image loss and its gradient (<= 1e-5), and
the reduced-FOV property the paper's soft-SENSE experiment shows: with the
object larger than the field of view, two map sets recover the coil images
better than the first set alone."""
import numpy as np
import pytest
import torch

from oracle import cg as ocg
from oracle import cnn as ocnn
from oracle import sense as osense
from oracle import soft_sense as oss
from paper_2202_14005_amd import ops
from synthetic import cnn_weights, soft_batch_inputs
from tests.gpu_util import dev, host, maxrel, oracle_threads, rel

pytestmark = pytest.mark.gpu

OP_TOL = 1e-5
CG_TOL = 1e-4
NET_TOL = 1e-2
GRAD_TOL = 2e-2
CG_GRAD_TOL = 1e-3


def case(B, H, W, C, seed):
    d = soft_batch_inputs([seed + i for i in range(B)], H, W, C, 4, max(2, min(24, H // 8)))
    return d


@pytest.mark.parametrize("B,H,W,C", [(2, 48, 40, 4), (1, 96, 80, 6), (8, 320, 320, 15), (1, 240, 288, 5),
                                     (2, 48, 40, 1), (1, 48, 40, 2)])
def test_soft_operators_and_cg(B, H, W, C):
    """The CG steps split each column tile's coils over three workgroups:
    with one or two coils some of them get none."""
    d = case(B, H, W, C, 11000)
    x, S, m = d["x"], d["S"], d["mask"]
    plan = ops.Plan(H, W, C, B=B, soft=True)
    xt, St, mt = dev(x), dev(S), dev(m)
    with oracle_threads():
        y = host(plan.soft_sense_fwd(xt, St, mt))
        yref = oss.soft_fwd(x, S, m)
        yc = yref.astype(np.complex64)
        a = host(plan.soft_sense_adj(dev(yc), St, mt))
        aref = oss.soft_adj(yc, S, m)
        q = host(plan.soft_sense_normal(xt, St, mt, 0.05))
        qref = oss.soft_normal(x, S, m, 0.05)
        ac = aref.astype(np.complex64)
        xs = host(plan.soft_cg_dc(dev(ac), St, mt, 0.05, 10))
        xref, _ = oss.soft_cg_dc(ac, None, S, m, np.full(B, 0.05, dtype=np.float32), 10)
    errs = {"fwd": rel(y, yref), "adj": rel(a, aref), "normal": rel(q, qref), "cg": rel(xs, xref)}
    pix = {"fwd": maxrel(y, yref), "adj": maxrel(a, aref), "normal": maxrel(q, qref), "cg": maxrel(xs, xref)}
    print(f"soft {B}x{H}x{W}x{C}:", {k: f"{v:.1e}" for k, v in errs.items()}, "per-pixel",
          {k: f"{v:.1e}" for k, v in pix.items()})
    for k in ("fwd", "adj", "normal"):
        assert errs[k] < OP_TOL and pix[k] < 2 * OP_TOL, k
    assert errs["cg"] < CG_TOL and pix["cg"] < 2 * CG_TOL


def test_soft_uneven_batch_matches_oracle_per_slice():
    """Slices of several sizes and coil counts in one soft plan: per size
    group one launch whose workgroups map to (slice, column tile, coil
    split); narrower slices of a group leave tiles idle, and the 192^2
    two-coil slice leaves coil-split workgroups without coils.  Every
    operator and the CG solve, slice by slice, against the oracle."""
    from synthetic import soft_slice_inputs
    shapes = [(320, 320, 15), (192, 192, 10), (320, 256, 6), (48, 40, 3), (192, 192, 2)]
    sl = [soft_slice_inputs(12000 + i, H, W, C, 4, max(2, min(24, H // 8)))
          for i, (H, W, C) in enumerate(shapes)]
    pk = {k: np.concatenate([d[k].ravel() for d in sl]) for k in ("x", "S", "mask")}
    plan = ops.Plan([q[0] for q in shapes], [q[1] for q in shapes], [q[2] for q in shapes], soft=True)
    xt, St, mt = dev(pk["x"]), dev(pk["S"]), dev(pk["mask"])
    lam = np.full(len(shapes), 0.05, dtype=np.float32)
    y = host(plan.soft_sense_fwd(xt, St, mt))
    a = host(plan.soft_sense_adj(dev(y), St, mt))
    q = host(plan.soft_sense_normal(xt, St, mt, torch.tensor(lam)))
    xs = host(plan.soft_cg_dc(dev(a), St, mt, torch.tensor(lam), 10))
    xo = so = 0
    with oracle_threads():
        for (H, W, C), d in zip(shapes, sl):
            ni, nc = 2 * H * W, C * H * W
            x1, S1, m1 = d["x"][None], d["S"][None], d["mask"][None]
            yref = oss.soft_fwd(x1, S1, m1)
            aref = oss.soft_adj(y[so:so + nc].reshape(1, C, H, W), S1, m1)
            qref = oss.soft_normal(x1, S1, m1, 0.05)
            a1 = a[xo:xo + ni].reshape(1, 2, H, W)
            xref, _ = oss.soft_cg_dc(a1, None, S1, m1, lam[:1], 10)
            errs = {"fwd": rel(y[so:so + nc], yref), "adj": rel(a[xo:xo + ni], aref),
                    "normal": rel(q[xo:xo + ni], qref), "cg": rel(xs[xo:xo + ni], xref)}
            print(f"soft uneven {H}x{W}x{C}:", {k: f"{v:.1e}" for k, v in errs.items()})
            for k in ("fwd", "adj", "normal"):
                assert errs[k] < OP_TOL, k
            assert errs["cg"] < CG_TOL
            xo += ni
            so += nc


def test_soft_with_empty_second_set_is_sense():
    """With the second set's maps zero the soft operators give the SENSE
    operators of the first set (different kernels, so to fp32 rounding)."""
    B, H, W, C = 2, 64, 48, 4
    d = case(B, H, W, C, 11100)
    S = d["S"].copy()
    S[:, 1] = 0
    x, m = d["x"], d["mask"]
    sp = ops.Plan(H, W, C, B=B, soft=True)
    pl = ops.Plan(H, W, C, B=B)
    y_soft = host(sp.soft_sense_fwd(dev(x), dev(S), dev(m)))
    y_sense = host(pl.sense_fwd(dev(np.ascontiguousarray(x[:, 0])), dev(np.ascontiguousarray(S[:, 0])), dev(m)))
    assert rel(y_soft, y_sense) < OP_TOL
    q = host(sp.soft_sense_normal(dev(x), dev(S), dev(m), 0.1))
    q1 = host(pl.sense_normal(dev(np.ascontiguousarray(x[:, 0])), dev(np.ascontiguousarray(S[:, 0])), dev(m), 0.1))
    assert rel(q[:, 0], q1) < OP_TOL
    assert rel(q[:, 1], 0.1 * x[:, 1]) < OP_TOL


def test_soft_coil_mse_parity():
    B, H, W, C = 2, 48, 40, 4
    d = case(B, H, W, C, 11200)
    rng = np.random.default_rng(3)
    x = (d["x"] + 0.1 * (rng.standard_normal(d["x"].shape) + 1j * rng.standard_normal(d["x"].shape))).astype(
        np.complex64)
    ref = oss.coil_images(d["x"], d["S"]).astype(np.complex64)
    plan = ops.Plan(H, W, C, B=B, soft=True, network=True)
    loss, g = plan.soft_coil_mse_grad(dev(x), dev(d["S"]), dev(ref))
    lref = oss.coil_mse(x, d["S"], ref)
    assert abs(float(host(loss)[0]) - lref) < 1e-5 * lref
    assert rel(host(g), oss.coil_mse_grad(x, d["S"], ref)) < 1e-5


@pytest.mark.parametrize("B,H,W,C,T", [(2, 48, 40, 4, 2), (1, 320, 320, 15, 2)])
def test_soft_modl_forward_parity(B, H, W, C, T):
    d = case(B, H, W, C, 11300)
    with oracle_threads():
        y = oss.soft_measure(d["x"], d["S"], d["mask"], d["noise"])
        aHy = oss.soft_adj(y, d["S"], d["mask"]).astype(np.complex64)
    w = cnn_weights(7, last_scale=0.1)
    lam = np.full(B, 0.05, dtype=np.float32)
    plan = ops.Plan(H, W, C, B=B, soft=True, network=True)
    cnn = ops.CNN.from_numpy(w)
    x, st = plan.soft_modl_forward(dev(aHy), dev(d["S"]), dev(d["mask"]), cnn, torch.tensor(lam), T, 10,
                                   states=True)
    with oracle_threads():
        xref, _, _ = oss.modl_forward(aHy, d["S"], d["mask"], w, lam, T, 10)
    e, p = rel(host(x), xref), maxrel(host(x), xref)
    print(f"soft modl fwd {B}x{H}x{W} T={T}: NRMSE {e:.2e} per-pixel {p:.2e}")
    assert e < NET_TOL and p < 2 * NET_TOL
    assert np.array_equal(host(st)[T], host(x)) and np.array_equal(host(st)[0], aHy)


def test_soft_modl_backward_parity():
    """Reverse pass of soft MoDL with the coil-image loss; the oracle is
    driven from the HIP forward's stored states."""
    B, H, W, C, T = 2, 48, 40, 4, 2
    d = case(B, H, W, C, 11400)
    y = oss.soft_measure(d["x"], d["S"], d["mask"], d["noise"])
    aHy = oss.soft_adj(y, d["S"], d["mask"]).astype(np.complex64)
    ref = oss.coil_images(d["x"], d["S"]).astype(np.complex64)
    w = cnn_weights(7, last_scale=0.1)
    lam = np.full(B, 0.05, dtype=np.float32)
    plan = ops.Plan(H, W, C, B=B, soft=True, network=True)
    cnn = ops.CNN.from_numpy(w)
    S, m = dev(d["S"]), dev(d["mask"])
    xT, st = plan.soft_modl_forward(dev(aHy), S, m, cnn, torch.tensor(lam), T, 10, states=True)
    loss, g = plan.soft_coil_mse_grad(xT, S, dev(ref))
    grads = ops.CNNGrads(cnn)
    gl, ga = plan.soft_modl_backward(g, st, dev(aHy), S, m, cnn, torch.tensor(lam), T, 10, grads, need_aHy=True)
    states = [s.astype(np.complex128) for s in host(st)]
    gref = oss.coil_mse_grad(states[T], d["S"], ref)
    zs = []
    for t in range(T):
        z = states[t].copy()
        z[:, 0] = ocnn.denoise(states[t][:, 0], w, bf16=True)
        zs.append(z)
    gw_ref, gl_ref, ga_ref = oss.modl_backward(gref, states, zs, aHy, d["S"], d["mask"], w, lam, T, 10, bf16=True)
    for l in range(5):
        ew, eb = rel(host(grads.w[l]), gw_ref[l][0]), rel(host(grads.b[l]), gw_ref[l][1])
        print(f"soft modl layer {l}: dW {ew:.2e} db {eb:.2e}")
        assert ew < GRAD_TOL and eb < GRAD_TOL
    el = np.max(np.abs(host(gl) - gl_ref) / np.abs(gl_ref))
    ea = rel(host(ga), ga_ref)
    print(f"soft modl g_lambda {el:.2e} g_aHy {ea:.2e}")
    assert el < CG_GRAD_TOL and ea < CG_GRAD_TOL


def test_two_map_sets_recover_the_folded_object_better():
    """Reduced field of view (object twice the FOV, folded once): CG-SENSE
    with both map sets reconstructs the coil images closer to the truth than
    with the first set alone."""
    B, H, W, C = 4, 128, 128, 8
    d = case(B, H, W, C, 11500)
    x, S, m, noise = d["x"], d["S"], d["mask"], d["noise"]
    coil_true = oss.coil_images(x, S)
    soft = ops.Plan(H, W, C, B=B, soft=True)
    one = ops.Plan(H, W, C, B=B)
    St, mt = dev(S), dev(m)
    y = soft.soft_sense_fwd(dev(x), St, mt, noise=dev(noise))
    xs = host(soft.soft_cg_dc(soft.soft_sense_adj(y, St, mt), St, mt, 0.01, 30))
    S1 = dev(np.ascontiguousarray(S[:, 0]))
    x1 = host(one.cg_dc(one.sense_adj(y, S1, mt), S1, mt, 0.01, 30))
    e_soft = rel(oss.coil_images(xs, S), coil_true)
    e_one = rel(S[:, 0] * x1[:, None], coil_true)
    print(f"coil-image NRMSE: two sets {e_soft:.3f}, first set only {e_one:.3f}")
    assert e_soft < 0.8 * e_one
