"""The torch.autograd bindings (CGDC, MoDLFunction, MoDLNet) against the FP64
oracle's reverse passes and against finite differences of the HIP forward.

Tolerances: gradients 1e-3 (CG adjoint, fp32); the MoDL module's gradients
equal one direct library reverse pass, and for T = 1 (no CG error in the
denoiser's input) meet the denoiser bound 2e-2 against the bf16-operand
oracle (ReLU decisions within accumulation-order noise of zero flip; see
tests/test_gpu_net.py).
Finite differences are taken on a well-conditioned problem (lambda = 1, so
cond(A^H A + lambda I) <= 2 and 10 CG steps reach fp32 accuracy), where the
truncated CG map and its adjoint-CG derivative coincide.
"""
import numpy as np
import pytest
import torch

from oracle import cg as ocg
from oracle import modl as omodl
from oracle import sense as osense
from paper_2202_14005_amd import autograd, ops
from tests.gpu_util import dev, host, inputs, rel

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-3
NET_GRAD_TOL = 2e-2   # denoiser reverse pass with ReLU decisions, against the bf16-operand oracle


def problem(B, H, W, C, seed):
    d = inputs([seed + i for i in range(B)], H, W, C)
    y = osense.measure(d["x"], d["S"], d["mask"], d["noise"])
    aHy = osense.sense_adj(y, d["S"], d["mask"]).astype(np.complex64)
    return d, y, aHy


def cplx(rng, shape, scale=1.0):
    return (scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))).astype(np.complex64)


def inner(g, x):
    """Re<g, x> summed, as a torch scalar (test-side loss)."""
    return (torch.view_as_real(g) * torch.view_as_real(x)).sum(dtype=torch.float64)


def test_cgdc_autograd_vs_oracle():
    B, H, W, C, n = 2, 48, 40, 4, 10
    d, _, aHy = problem(B, H, W, C, 700)
    rng = np.random.default_rng(21)
    z = cplx(rng, aHy.shape, 0.3)
    g = cplx(rng, aHy.shape)
    lam = np.array([0.05, 0.1], dtype=np.float32)
    plan = ops.Plan(H, W, C, B=B)
    a_t = dev(aHy).requires_grad_()
    z_t = dev(z).requires_grad_()
    l_t = dev(lam).requires_grad_()
    x = autograd.cg_dc(plan, a_t, dev(d["S"]), dev(d["mask"]), l_t, n, z=z_t)
    inner(dev(g), x).backward()
    xr, _ = ocg.cg_dc(aHy, z, d["S"], d["mask"], lam, n)
    assert rel(host(x), xr) < 1e-4
    ga, gz, gl = ocg.cg_dc_backward(g, xr, z, d["S"], d["mask"], lam, n)
    errs = {"aHy": rel(host(a_t.grad), ga), "z": rel(host(z_t.grad), gz),
            "lam": float(np.max(np.abs(host(l_t.grad) - gl) / np.abs(gl)))}
    print("cgdc autograd", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v < GRAD_TOL, k


def test_cgdc_autograd_scalar_lambda_and_no_z():
    B, H, W, C, n = 2, 32, 48, 3, 8
    d, _, aHy = problem(B, H, W, C, 720)
    g = cplx(np.random.default_rng(2), aHy.shape)
    plan = ops.Plan(H, W, C, B=B)
    l_t = torch.tensor(0.07, device="cuda", requires_grad=True)
    a_t = dev(aHy).requires_grad_()
    x = autograd.cg_dc(plan, a_t, dev(d["S"]), dev(d["mask"]), l_t, n)
    inner(dev(g), x).backward()
    lam = np.full(B, 0.07, dtype=np.float32)
    xr, _ = ocg.cg_dc(aHy, None, d["S"], d["mask"], lam, n)
    ga, _, gl = ocg.cg_dc_backward(g, xr, None, d["S"], d["mask"], lam, n)
    assert l_t.grad.shape == l_t.shape
    assert abs(float(l_t.grad) - gl.sum()) < GRAD_TOL * abs(gl.sum())
    assert rel(host(a_t.grad), ga) < GRAD_TOL


def test_cgdc_autograd_finite_differences():
    B, H, W, C, n = 1, 32, 32, 4, 10
    d, _, aHy = problem(B, H, W, C, 740)
    rng = np.random.default_rng(5)
    z = cplx(rng, aHy.shape, 0.3)
    g = dev(cplx(rng, aHy.shape))
    plan = ops.Plan(H, W, C, B=B)
    S, m = dev(d["S"]), dev(d["mask"])
    lam0 = 1.0
    a_t, z_t = dev(aHy).requires_grad_(), dev(z).requires_grad_()
    l_t = torch.tensor([lam0], device="cuda", requires_grad=True)
    inner(g, autograd.cg_dc(plan, a_t, S, m, l_t, n, z=z_t)).backward()

    def L(a, zz, lam):
        with torch.no_grad():
            return float(inner(g, plan.cg_dc(a, S, m, torch.tensor([lam], device="cuda"), n, z=zz)))

    a0, z0 = dev(aHy), dev(z)
    da, dz = dev(cplx(rng, aHy.shape)), dev(cplx(rng, aHy.shape))
    # linear in aHy and z: a unit step is exact up to rounding
    fd_a = (L(a0 + da, z0, lam0) - L(a0 - da, z0, lam0)) / 2
    fd_z = (L(a0, z0 + dz, lam0) - L(a0, z0 - dz, lam0)) / 2
    h = 1e-2
    fd_l = (L(a0, z0, lam0 + h) - L(a0, z0, lam0 - h)) / (2 * h)
    an_a = float(inner(da, a_t.grad))
    an_z = float(inner(dz, z_t.grad))
    an_l = float(l_t.grad)
    print(f"fd aHy {fd_a:.6e} vs {an_a:.6e}; z {fd_z:.6e} vs {an_z:.6e}; lam {fd_l:.6e} vs {an_l:.6e}")
    assert abs(fd_a - an_a) < GRAD_TOL * abs(an_a)
    assert abs(fd_z - an_z) < GRAD_TOL * abs(an_z)
    assert abs(fd_l - an_l) < GRAD_TOL * abs(an_l)


def _modlnet(B, H, W, C, T, n, seed):
    d, y, aHy = problem(B, H, W, C, seed)
    plan = ops.Plan(H, W, C, B=B, network=True)
    net = autograd.MoDLNet(plan, T=T, n_cg=n, lam=0.05, learn_lam=True)
    with torch.no_grad():
        net.weights[4].mul_(0.1)
        net.biases[4].mul_(0.1)
    return d, y.astype(np.complex64), aHy, plan, net


def _mse(x, ref):
    diff = x - ref
    return (torch.view_as_real(diff) ** 2).sum() / diff.numel()


def test_modlnet_autograd_equals_library_reverse_pass():
    """Through autograd, T = 2: the gradients are exactly those of one direct
    mrx_modl_backward call (same kernels, fixed-order reductions)."""
    B, H, W, C, T, n = 2, 48, 40, 4, 2, 10
    d, y, aHy, plan, net = _modlnet(B, H, W, C, T, n, 760)
    S, m, ref, a = dev(d["S"]), dev(d["mask"]), dev(d["x"]), dev(aHy)
    a.requires_grad_()
    x = net.forward_from_adjoint(a, S, m)
    _mse(x, ref).backward()
    xT, st = plan.modl_forward(dev(aHy), S, m, net.cnn, 0.05, T, n, states=True)
    assert torch.equal(xT, x.detach())
    _, g = plan.mse_grad(xT, ref)
    grads = ops.CNNGrads(net.cnn)
    gl, ga = plan.modl_backward(g, st, dev(aHy), S, m, net.cnn, 0.05, T, n, grads, need_aHy=True)
    for l in range(5):
        assert torch.allclose(net.weights[l].grad, grads.w[l], rtol=1e-6, atol=0), l
        assert torch.allclose(net.biases[l].grad, grads.b[l], rtol=1e-6, atol=0), l
    assert torch.allclose(net.lam.grad, gl.sum().reshape(1), rtol=1e-6)
    assert torch.allclose(a.grad, ga, rtol=1e-6, atol=1e-12)


def test_modlnet_autograd_vs_oracle_and_optimizer_step():
    """T = 1 (the denoiser sees x^0 = A^H y, identical on both sides, so no
    bf16 ReLU decision differs): gradients against the bf16-operand oracle to
    the denoiser bound 2e-2 (tests/test_gpu_net.py derives it); an optimizer step then changes the weights in
    place and the next forward must use them."""
    B, H, W, C, T, n = 2, 48, 40, 4, 1, 10
    d, y, aHy, plan, net = _modlnet(B, H, W, C, T, n, 780)
    S, m = dev(d["S"]), dev(d["mask"])
    x = net.forward_from_adjoint(dev(aHy), S, m)
    _mse(x, dev(d["x"])).backward()
    w = [(wt.detach().cpu().numpy(), bt.detach().cpu().numpy()) for wt, bt in zip(net.weights, net.biases)]
    lam = np.full(B, 0.05, dtype=np.float32)
    xr, sr, zr = omodl.forward(aHy, d["S"], d["mask"], w, lam, T, n, bf16=True)
    assert rel(host(x), omodl.forward(aHy, d["S"], d["mask"], w, lam, T, n)[0]) < 1e-2
    gref = omodl.mse_grad(xr, d["x"])
    gw_ref, gl_ref, _ = omodl.backward(gref, sr, zr, aHy, d["S"], d["mask"], w, lam, T, n, bf16=True)
    for l in range(5):
        ew, eb = rel(host(net.weights[l].grad), gw_ref[l][0]), rel(host(net.biases[l].grad), gw_ref[l][1])
        print(f"modlnet layer {l}: dW {ew:.2e} db {eb:.2e}")
        assert ew < NET_GRAD_TOL and eb < NET_GRAD_TOL
    assert abs(float(net.lam.grad) - gl_ref.sum()) < NET_GRAD_TOL * abs(gl_ref.sum())
    opt = torch.optim.SGD(net.parameters(), lr=1e-2)
    opt.step()
    x2 = net.forward_from_adjoint(dev(aHy), S, m)
    w2 = [(wt.detach().cpu().numpy(), bt.detach().cpu().numpy()) for wt, bt in zip(net.weights, net.biases)]
    lam2 = np.full(B, float(net.lam.detach()), dtype=np.float32)
    xr2, _, _ = omodl.forward(aHy, d["S"], d["mask"], w2, lam2, T, n)
    assert rel(host(x2), xr2) < 1e-2
    assert rel(host(x2), host(x)) > 1e-6
    # the k-space entry point computes A^H y itself
    assert rel(host(net(dev(y), S, m)), host(x2)) < 1e-3
