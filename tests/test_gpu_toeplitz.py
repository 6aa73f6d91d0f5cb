"""Non-Cartesian SENSE through the Toeplitz normal operator on the GPU
against the FP64 oracle (oracle/toeplitz.py), through the C-ABI.

* the one-off steps: the non-uniform DFT forward model and adjoint, and the
  PSF spectrum on the twice-padded grid (<= 1e-5; spot checks of single
  pixels and samples at the full 320 x 320, 15-coil, 44-spoke size);
* the three-pass normal operator on a PSF both sides share (<= 1e-5
  overall and per pixel), and end to end with each side's own PSF;
* CG (10 steps, also at the full size, and the paper's 30): within 1e-4,
  or within three times the distance of the same CG in plain fp32
  arithmetic from the FP64 CG where that is larger (these radial problems
  can converge past what fp32 follows), with a normal-equation residual as
  small as the oracle's;
* MoDL from the SENSE start (output NRMSE <= 1e-2 against plain FP64) and
  its reverse pass from the HIP states against the bf16-operand oracle
  (the bounds of the Cartesian reverse-pass tests).
Sizes span several row and column tiles with ragged tails (H, W not
multiples of the tiles), H != W, and an uneven batch."""
import numpy as np
import pytest
import torch

from oracle import cg as ocg
from oracle import cnn as ocnn
from oracle import modl as omodl
from oracle import toeplitz as otp
from paper_2202_14005_amd import ops
from synthetic import cnn_weights, noncart_batch_inputs, noncart_slice_inputs
from tests.gpu_util import dev, host, maxrel, oracle_threads, rel

pytestmark = pytest.mark.gpu

OP_TOL = 1e-5
CG_TOL = 1e-4
NET_TOL = 1e-2
GRAD_TOL = 2e-2
CG_GRAD_TOL = 1e-3


def case(B, H, W, C, spokes, nread, seed):
    return noncart_batch_inputs([seed + i for i in range(B)], H, W, C, spokes, nread)


def cg_fp32(apply_S, b, n):
    """The oracle's CG recipe (textbook Hestenes-Stiefel from x0 = 0) with
    every vector rounded to complex64 and every inner product and scalar to
    float32 after each step: plain single-precision arithmetic, to measure
    how far fp32 rounding alone moves the solve (test instrument, not the
    reference)."""
    c64 = lambda a: a.astype(np.complex64).astype(np.complex128)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    dot = lambda u, v: f32(np.sum(np.conj(u) * v, axis=(-2, -1)).real)
    b = c64(b)
    x, r = np.zeros_like(b), b.copy()
    p, rho = r.copy(), dot(r, r)
    for _ in range(n):
        q = c64(apply_S(p))
        alpha = f32(rho / dot(p, q))
        x = c64(x + alpha[:, None, None] * p)
        r = c64(r - alpha[:, None, None] * q)
        rho_new = dot(r, r)
        p = c64(r + f32(rho_new / rho)[:, None, None] * p)
        rho = rho_new
    return x


def cg_reference(b, S, P, lam, x_gpu, n):
    """CG on these underdetermined radial problems can run the residual
    down by 1e9 and more (the paper's 30 steps; on the smallest grids
    already 10), past what single precision can follow, so the fp32 solve is
    compared with the FP64 one within fp32's own reach: ``spread`` is the
    distance of the same CG in plain fp32 arithmetic (``cg_fp32``) from the
    FP64 CG.  Also returns the relative normal-equation residuals
    ||(A^H A + lambda I) x - b|| / ||b|| of the GPU solution and of the FP64
    one."""
    lamv = np.full(b.shape[0], lam)
    ref, _ = otp.cg_dc(b, None, S, P, lamv, n)
    op = lambda v: otp.normal(v, S, P, lamv)
    res = lambda x: float(np.linalg.norm(op(x) - b) / np.linalg.norm(b))
    return ref, rel(cg_fp32(op, b, n), ref), res(x_gpu.astype(np.complex128)), res(ref)


@pytest.mark.parametrize("B,H,W,C,spokes,nread", [
    (2, 32, 48, 4, 13, 64), (1, 64, 40, 3, 9, 96), (3, 16, 16, 2, 7, 32), (1, 96, 80, 5, 11, 160)])
def test_toeplitz_operators_and_cg(B, H, W, C, spokes, nread):
    d = case(B, H, W, C, spokes, nread, 31000 + H)
    x, S, traj = d["x"], d["S"], d["traj"]
    plan = ops.Plan(H, W, C, B=B, toeplitz=True)
    xt, St, tt = dev(x), dev(S), dev(traj)
    with oracle_threads():
        y = host(plan.nufft_fwd(xt, St, tt))
        yref = otp.nudft_fwd(x, S, traj)
        yc = yref.astype(np.complex64)
        a = host(plan.nufft_adj(dev(yc), St, tt))
        aref = otp.nudft_adj(yc, S, traj)
        P = host(plan.toeplitz_psf(tt))
        Pref = otp.psf(traj, H, W)
        Pc = Pref.astype(np.float32)
        q = host(plan.sense_normal(xt, St, dev(Pc), 0.05))
        qref = otp.normal(x, S, Pc, 0.05)
        q_own = host(plan.sense_normal(xt, St, dev(P), 0.05))
        qdef = otp.normal_direct(x, S, traj, 0.05)
        ac = aref.astype(np.complex64)
        xs = host(plan.cg_dc(dev(ac), St, dev(Pc), 0.05, 10))
        xref, spread10, _, _ = cg_reference(ac, S, Pc, 0.05, xs, 10)
        xs30 = host(plan.cg_dc(dev(ac), St, dev(Pc), 0.05, 30))
        xref30, spread, res_gpu, res_ref = cg_reference(ac, S, Pc, 0.05, xs30, 30)
    errs = {"fwd": rel(y, yref), "adj": rel(a, aref), "psf": rel(P, Pref), "normal": rel(q, qref),
            "normal_own_psf": rel(q_own, qdef), "cg": rel(xs, xref), "cg30": rel(xs30, xref30)}
    pix = {"fwd": maxrel(y, yref), "adj": maxrel(a, aref), "psf": maxrel(P, Pref), "normal": maxrel(q, qref),
           "cg": maxrel(xs, xref)}
    print(f"toeplitz {B}x{H}x{W}x{C} M={spokes * nread}:", {k: f"{v:.1e}" for k, v in errs.items()},
          "per-pixel", {k: f"{v:.1e}" for k, v in pix.items()},
          f"fp32-CG spread cg {spread10:.1e} cg30 {spread:.1e}, cg30 residual gpu {res_gpu:.1e} "
          f"oracle {res_ref:.1e}")
    for k in ("fwd", "adj", "psf", "normal"):
        assert errs[k] < OP_TOL and pix[k] < 2 * OP_TOL, k
    assert errs["normal_own_psf"] < 2 * OP_TOL
    tol10 = max(CG_TOL, 3 * spread10)
    assert errs["cg"] < tol10 and pix["cg"] < 2 * tol10
    assert errs["cg30"] < max(CG_TOL, 3 * spread)
    assert res_gpu < max(1e-4, 10 * res_ref)


def test_toeplitz_uneven_batch():
    shapes = [(32, 48, 3), (64, 64, 5), (32, 48, 2), (16, 32, 4)]
    sl = [noncart_slice_inputs(32100 + i, H, W, C, 9, 64) for i, (H, W, C) in enumerate(shapes)]
    plan = ops.Plan([s[0] for s in shapes], [s[1] for s in shapes], [s[2] for s in shapes], toeplitz=True)
    M = sl[0]["traj"].shape[0]
    traj = np.stack([s["traj"] for s in sl])
    xp = np.concatenate([s["x"].ravel() for s in sl])
    Sp = np.concatenate([s["S"].ravel() for s in sl])
    St, tt = dev(Sp), dev(traj)
    P = host(plan.toeplitz_psf(tt))
    q = host(plan.sense_normal(dev(xp), St, dev(P), 0.1))
    o, oq = 0, 0
    for s, (H, W, C) in zip(sl, shapes):
        Pr = otp.psf(s["traj"][None], H, W)
        n = H * W
        ep = rel(P[4 * o:4 * (o + n)].reshape(2 * H, 2 * W), Pr[0])
        qr = otp.normal(s["x"][None], s["S"][None], Pr, 0.1)[0]
        eq = rel(q[o:o + n].reshape(H, W), qr)
        print(f"uneven {H}x{W}x{C}: psf {ep:.1e} normal {eq:.1e}")
        assert ep < OP_TOL and eq < 2 * OP_TOL
        o += n
    assert M == 9 * 64


def test_toeplitz_full_size_spot_checks():
    """320 x 320, 15 coils, 44 spokes of 640 samples (the paper's radial
    setting): PSF and normal operator in full, CG (10 steps) in full, the
    forward model and adjoint at sampled entries."""
    H = W = 320
    C, spokes, nread = 15, 44, 640
    d = case(1, H, W, C, spokes, nread, 33000)
    x, S, traj = d["x"], d["S"], d["traj"]
    plan = ops.Plan(H, W, C, B=1, toeplitz=True)
    xt, St, tt = dev(x), dev(S), dev(traj)
    rng = np.random.default_rng(1)
    with oracle_threads():
        P = host(plan.toeplitz_psf(tt))
        Pref = otp.psf(traj, H, W)
        ep, pp = rel(P, Pref), maxrel(P, Pref)
        y = host(plan.nufft_fwd(xt, St, tt, noise=dev(d["noise"])))
        js = [(0, int(j)) for j in rng.choice(spokes * nread, 24, replace=False)]
        yref = otp.nudft_fwd_samples(x, S, traj, js) + np.array([d["noise"][0, :, j] for _, j in js])
        ey = rel(np.array([y[0, :, j] for _, j in js]), yref)
        a = host(plan.nufft_adj(dev(y), St, tt))
        px = [(0, int(r), int(s)) for r, s in zip(rng.integers(0, H, 24), rng.integers(0, W, 24))]
        aref = otp.nudft_adj_pixels(y, S, traj, px)
        ea = rel(np.array([a[0, r, s] for _, r, s in px]), aref)
        Pc = Pref.astype(np.float32)
        q = host(plan.sense_normal(xt, St, dev(Pc), 0.05))
        qref = otp.normal(x, S, Pc, 0.05)
        eq, pq = rel(q, qref), maxrel(q, qref)
        aHy = a.astype(np.complex64)
        xs = host(plan.cg_dc(dev(aHy), St, dev(Pc), 0.05, 10))
        xref, _ = otp.cg_dc(aHy, None, S, Pc, 0.05, 10)
        ec, pc = rel(xs, xref), maxrel(xs, xref)
    print(f"toeplitz 320x320x15, 44 spokes: psf {ep:.1e} ({pp:.1e}) fwd {ey:.1e} adj {ea:.1e} "
          f"normal {eq:.1e} ({pq:.1e}) cg {ec:.1e} ({pc:.1e})")
    assert ep < OP_TOL and pp < 2 * OP_TOL
    assert ey < OP_TOL and ea < OP_TOL
    assert eq < OP_TOL and pq < 2 * OP_TOL
    assert ec < CG_TOL and pc < 2 * CG_TOL


def test_toeplitz_modl_forward_and_backward():
    B, H, W, C, T, n = 2, 48, 32, 4, 2, 8
    d = case(B, H, W, C, 11, 96, 34000)
    x, S, traj = d["x"], d["S"], d["traj"]
    w = cnn_weights(7, last_scale=0.1)
    lam = np.full(B, 0.05, dtype=np.float32)
    plan = ops.Plan(H, W, C, B=B, network=True, toeplitz=True)
    cnn = ops.CNN.from_numpy(w)
    St, tt = dev(S), dev(traj)
    Pref = otp.psf(traj, H, W)
    Pc = Pref.astype(np.float32)
    Pt = dev(Pc)
    y = plan.nufft_fwd(dev(x), St, tt, noise=dev(d["noise"]))
    aHy = plan.nufft_adj(y, St, tt)
    x0 = plan.cg_dc(aHy, St, Pt, torch.tensor(lam), n)
    xT, st = plan.modl_forward(aHy, St, Pt, cnn, torch.tensor(lam), T, n, states=True, x0=x0)
    a_h, x0_h = host(aHy).astype(np.complex128), host(x0).astype(np.complex128)
    with oracle_threads():
        x0_ref, spread0, _, _ = cg_reference(a_h, S, Pc, 0.05, x0_h, n)
        xT_ref, _, _ = otp.modl_forward(x0_h, a_h, S, Pc, w, lam, T, n)
    e0, eT = rel(x0_h, x0_ref), rel(host(xT), xT_ref)
    print(f"toeplitz MoDL: SENSE start {e0:.1e} (fp32-CG spread {spread0:.1e}), x^T NRMSE {eT:.1e}")
    assert e0 < max(CG_TOL, 3 * spread0) and eT < NET_TOL
    assert np.array_equal(host(st)[0], host(x0))
    # reverse pass from the HIP states
    loss, g = plan.mse_grad(xT, dev(x))
    grads = ops.CNNGrads(cnn)
    gl, _ = plan.modl_backward(g, st, aHy, St, Pt, cnn, torch.tensor(lam), T, n, grads)
    states = [s.astype(np.complex128) for s in host(st)]
    gref = omodl.mse_grad(states[T], x)
    with oracle_threads():
        zs = [ocnn.denoise(states[t], w, bf16=True) for t in range(T)]
        gw_ref, gl_ref, _, _ = otp.modl_backward(gref, states, zs, a_h, S, Pc, w, lam, T, n, bf16=True)
    for l in range(5):
        ew, eb = rel(host(grads.w[l]), gw_ref[l][0]), rel(host(grads.b[l]), gw_ref[l][1])
        print(f"toeplitz MoDL layer {l}: dW {ew:.2e} db {eb:.2e}")
        assert ew < GRAD_TOL and eb < GRAD_TOL
    el = np.max(np.abs(host(gl) - gl_ref) / np.abs(gl_ref))
    print(f"toeplitz MoDL g_lambda {el:.2e}")
    assert el < CG_GRAD_TOL
