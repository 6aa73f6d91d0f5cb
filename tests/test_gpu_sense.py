"""Parity of the HIP SENSE operators and CG data-consistency solve (through
the C-ABI) against the FP64 oracle on seeded inputs.

Tolerances (relative L2 error over the whole output): each operator 1e-5,
after CG 1e-4, CG reverse pass 1e-4.
"""
import numpy as np
import pytest
import torch

from oracle import cg as ocg
from oracle import sense as osense
from paper_2202_14005_amd.ops import Plan
from tests.gpu_util import dev, host, inputs, rel, uneven

pytestmark = pytest.mark.gpu

OP_TOL = 1e-5
CG_TOL = 1e-4

# (H, W, C, mask kind): 128/320/384 are the configurations' sizes; 40x24 and
# 16x16 have ragged column tiles (W not a multiple of the tile width) and
# tiny transforms; 192x256 has H != W.
CASES = [
    (128, 128, 8, "uniform"),
    (320, 320, 15, "vd"),
    (384, 320, 15, "regular"),
    (192, 256, 10, "vd"),
    (40, 24, 3, "uniform"),
    (16, 16, 2, "uniform"),
    (256, 96, 4, "vd"),
    (512, 160, 3, "vd"),
]


def case_inputs(H, W, C, kind, B=2, seed=100):
    d = inputs([seed + i for i in range(B)], H, W, C, 4, None, kind)
    return d


@pytest.mark.parametrize("H,W,C,kind", CASES)
def test_sense_normal_parity(H, W, C, kind):
    d = case_inputs(H, W, C, kind)
    B = d["x"].shape[0]
    lam = np.array([0.01, 0.5], dtype=np.float32)[:B]
    plan = Plan(H, W, C, B=B)
    q = plan.sense_normal(dev(d["x"]), dev(d["S"]), dev(d["mask"]), torch.tensor(lam))
    ref = osense.sense_normal(d["x"], d["S"], d["mask"], lam)
    assert rel(host(q), ref) < OP_TOL


@pytest.mark.parametrize("H,W,C,kind", CASES)
def test_sense_fwd_adj_parity(H, W, C, kind):
    d = case_inputs(H, W, C, kind)
    plan = Plan(H, W, C, B=2)
    x, S, m, n = dev(d["x"]), dev(d["S"]), dev(d["mask"]), dev(d["noise"])
    y = plan.sense_fwd(x, S, m)
    assert rel(host(y), osense.sense_fwd(d["x"], d["S"], d["mask"])) < OP_TOL
    yn = plan.sense_fwd(x, S, m, noise=n)
    yref = osense.measure(d["x"], d["S"], d["mask"], d["noise"])
    assert rel(host(yn), yref) < OP_TOL
    yh = host(yn)
    for b in range(2):
        assert np.all(yh[b][:, d["mask"][b] == 0, :] == 0)
    y64 = yref.astype(np.complex64)
    a = plan.sense_adj(dev(y64), S, m)
    assert rel(host(a), osense.sense_adj(y64, d["S"], d["mask"])) < OP_TOL


@pytest.mark.parametrize("H,W,C,kind", CASES[:5])
def test_cg_dc_parity(H, W, C, kind):
    d = case_inputs(H, W, C, kind)
    y = osense.measure(d["x"], d["S"], d["mask"], d["noise"])
    aHy = osense.sense_adj(y, d["S"], d["mask"]).astype(np.complex64)
    z = (0.9 * d["x"]).astype(np.complex64)
    lam = np.array([0.05, 0.01], dtype=np.float32)
    plan = Plan(H, W, C, B=2)
    x, h = plan.cg_dc(dev(aHy), dev(d["S"]), dev(d["mask"]), torch.tensor(lam), 10, z=dev(z), hist=True)
    xref, href = ocg.cg_dc(aHy, z, d["S"], d["mask"], lam, 10)
    assert rel(host(x), xref) < CG_TOL
    assert np.max(np.abs(host(h) - href) / href[:, :1]) < CG_TOL
    # plain CG-SENSE (z = 0)
    x0 = plan.cg_dc(dev(aHy), dev(d["S"]), dev(d["mask"]), torch.tensor(lam), 10)
    x0ref, _ = ocg.cg_dc(aHy, None, d["S"], d["mask"], lam, 10)
    assert rel(host(x0), x0ref) < CG_TOL
    assert int(plan.status().abs().sum()) == 0


@pytest.mark.parametrize("H,W,C,kind", [(128, 128, 8, "uniform"), (320, 320, 15, "vd"), (40, 24, 3, "uniform")])
def test_cg_dc_backward_parity(H, W, C, kind):
    d = case_inputs(H, W, C, kind)
    y = osense.measure(d["x"], d["S"], d["mask"], d["noise"])
    aHy = osense.sense_adj(y, d["S"], d["mask"]).astype(np.complex64)
    z = (0.8 * d["x"]).astype(np.complex64)
    lam = np.array([0.05, 0.2], dtype=np.float32)
    xref, _ = ocg.cg_dc(aHy, z, d["S"], d["mask"], lam, 10)
    x64 = xref.astype(np.complex64)
    rng = np.random.default_rng(3)
    g = (rng.standard_normal(aHy.shape) + 1j * rng.standard_normal(aHy.shape)).astype(np.complex64) * 1e-3
    plan = Plan(H, W, C, B=2)
    ga, gz, gl = plan.cg_dc_backward(dev(g), dev(x64), dev(d["S"]), dev(d["mask"]), torch.tensor(lam), 10,
                                     z=dev(z))
    ra, rz, rl = ocg.cg_dc_backward(g, x64, z, d["S"], d["mask"], lam, 10)
    assert rel(host(ga), ra) < CG_TOL
    assert rel(host(gz), rz) < CG_TOL
    assert np.max(np.abs(host(gl) - rl) / np.abs(rl)) < 1e-3


def test_full_sampling_is_identity():
    H, W, C = 128, 96, 6
    d = case_inputs(H, W, C, "uniform")
    m = np.ones_like(d["mask"])
    plan = Plan(H, W, C, B=2)
    q = plan.sense_normal(dev(d["x"]), dev(d["S"]), dev(m))
    # sum |S|^2 = 1 up to complex64 rounding of S
    assert rel(host(q), d["x"]) < 2e-6


def test_empty_mask_and_zero_rhs():
    H, W, C = 64, 64, 4
    d = case_inputs(H, W, C, "uniform")
    m = np.zeros_like(d["mask"])
    plan = Plan(H, W, C, B=2)
    lam = torch.tensor([0.5, 2.0])
    q = plan.sense_normal(dev(d["x"]), dev(d["S"]), dev(m), lam)
    assert rel(host(q), d["x"] * np.array([0.5, 2.0])[:, None, None]) < 1e-6
    x = plan.cg_dc(dev(d["x"]), dev(d["S"]), dev(m), lam, 5)
    assert rel(host(x), d["x"] / np.array([0.5, 2.0])[:, None, None]) < 1e-6
    xz = plan.cg_dc(torch.zeros_like(dev(d["x"])), dev(d["S"]), dev(d["mask"]), lam, 5)
    assert np.all(host(xz) == 0)
    assert int(plan.status().abs().sum()) == 0


def test_nonfinite_input_sets_status_and_terminates():
    H, W, C = 64, 64, 4
    d = case_inputs(H, W, C, "uniform")
    aHy = d["x"].copy()
    aHy[1, 3, 5] = np.nan
    plan = Plan(H, W, C, B=2)
    x = plan.cg_dc(dev(aHy), dev(d["S"]), dev(d["mask"]), 0.05, 10)
    st = host(plan.status(clear=True))
    assert st[0] == 0 and (st[1] & 1) == 1
    assert np.all(np.isfinite(host(x)[0]))
    assert int(plan.status().abs().sum()) == 0


def test_uneven_batch_matches_oracle_per_slice():
    shapes = [(128, 128, 8), (192, 192, 10), (320, 320, 15), (384, 320, 12), (128, 128, 3)]
    sl, pk = uneven(shapes)
    plan = Plan([s[0] for s in shapes], [s[1] for s in shapes], [s[2] for s in shapes])
    lam = np.array([0.05] * len(shapes), dtype=np.float32)
    x, S, m, n = dev(pk["x"]), dev(pk["S"]), dev(pk["mask"]), dev(pk["noise"])
    q = host(plan.sense_normal(x, S, m, torch.tensor(lam)))
    y = host(plan.sense_fwd(x, S, m, noise=n))
    a = host(plan.sense_adj(dev(y), S, m))
    xs = host(plan.cg_dc(dev(a), S, m, torch.tensor(lam), 10))
    xo = so = 0
    for (H, W, C), s in zip(shapes, sl):
        ni, nc = H * W, C * H * W
        args = (s["x"][None], s["S"][None], s["mask"][None])
        assert rel(q[xo:xo + ni], osense.sense_normal(*args, [0.05])) < OP_TOL
        yref = osense.measure(*args, s["noise"][None])
        assert rel(y[so:so + nc], yref) < OP_TOL
        aref = osense.sense_adj(y[so:so + nc].reshape(1, C, H, W), s["S"][None], s["mask"][None])
        assert rel(a[xo:xo + ni], aref) < OP_TOL
        xref, _ = ocg.cg_dc(a[xo:xo + ni].reshape(1, H, W), None, s["S"][None], s["mask"][None], [0.05], 10)
        assert rel(xs[xo:xo + ni], xref) < CG_TOL
        xo += ni
        so += nc


def test_uneven_batch_split_operator_matches_oracle():
    """The operator applications of an uneven batch under coil-split
    schedules: every size group with a split schedule writes its partial
    planes (one group has fewer coils than splits), the 128^2 group has no
    split schedule and runs unsplit, and a fixed-order sum adds the planes;
    the normal operator and the CG solve per slice against the oracle."""
    from paper_2202_14005_amd import ops
    shapes = [(192, 192, 10), (320, 320, 15), (384, 320, 12), (128, 128, 3), (256, 256, 2)]
    sl, pk = uneven(shapes, seed0=5100)
    plan = Plan([s[0] for s in shapes], [s[1] for s in shapes], [s[2] for s in shapes])
    for H in (192, 256, 320, 384):
        name = [n for n in ops.schedules(H) if n.endswith("_w16_k3")][0]
        plan.set_schedule(H, name)
    lam = np.array([0.05] * len(shapes), dtype=np.float32)
    x, S, m = dev(pk["x"]), dev(pk["S"]), dev(pk["mask"])
    q = host(plan.sense_normal(x, S, m, torch.tensor(lam)))
    a = host(plan.sense_adj(plan.sense_fwd(x, S, m, noise=dev(pk["noise"])), S, m))
    xs = host(plan.cg_dc(dev(a), S, m, torch.tensor(lam), 10))
    xo = 0
    for (H, W, C), s in zip(shapes, sl):
        ni = H * W
        args = (s["x"][None], s["S"][None], s["mask"][None])
        e_q = rel(q[xo:xo + ni], osense.sense_normal(*args, [0.05]))
        xref, _ = ocg.cg_dc(a[xo:xo + ni].reshape(1, H, W), None, s["S"][None], s["mask"][None], [0.05], 10)
        e_x = rel(xs[xo:xo + ni], xref)
        print(f"{H}x{W}x{C} ({plan.schedule(shapes.index((H, W, C)))}): normal {e_q:.1e} cg {e_x:.1e}")
        assert e_q < OP_TOL and e_x < CG_TOL
        xo += ni


def test_bitwise_reproducible():
    H, W, C = 320, 320, 15
    d = case_inputs(H, W, C, "vd")
    plan = Plan(H, W, C, B=2)
    args = (dev(d["x"]), dev(d["S"]), dev(d["mask"]), 0.05, 10)
    x1 = host(plan.cg_dc(*args))
    x2 = host(plan.cg_dc(*args))
    assert np.array_equal(x1.view(np.uint32), x2.view(np.uint32))


def test_full_size_batch_parity():
    """The benchmark's batch: 8 slices of 320 x 320 with 15 coils, R = 4
    variable density with 24 centre lines, lambda = 0.05, 10 CG iterations."""
    H = W = 320
    C, B = 15, 8
    d = inputs([2000 + i for i in range(B)], H, W, C, 4, 24, "vd")
    plan = Plan(H, W, C, B=B)
    x, S, m, n = dev(d["x"]), dev(d["S"]), dev(d["mask"]), dev(d["noise"])
    y = plan.sense_fwd(x, S, m, noise=n)
    a = plan.sense_adj(y, S, m)
    xs = plan.cg_dc(a, S, m, 0.05, 10)
    yref = osense.measure(d["x"], d["S"], d["mask"], d["noise"])
    assert rel(host(y), yref) < OP_TOL
    aref = osense.sense_adj(host(y), d["S"], d["mask"])
    assert rel(host(a), aref) < OP_TOL
    xref, _ = ocg.cg_dc(host(a), None, d["S"], d["mask"], np.full(B, 0.05), 10)
    assert rel(host(xs), xref) < CG_TOL


@pytest.mark.parametrize("H,W,C", [(320, 24, 5), (384, 40, 4), (256, 16, 7), (192, 24, 3), (128, 40, 6)])
def test_every_schedule_normal_and_cg(H, W, C):
    """Each registered column schedule of a length (workgroup-tiled and
    wave-local variants) against the oracle; W = 24 and 40 leave a ragged last
    tile for the 16-column schedules."""
    from paper_2202_14005_amd import ops
    B = 2
    d = inputs([1700 + i for i in range(B)], H, W, C)
    y = osense.measure(d["x"], d["S"], d["mask"], d["noise"])
    aHy = osense.sense_adj(y, d["S"], d["mask"]).astype(np.complex64)
    q_ref = osense.sense_normal(d["x"], d["S"], d["mask"], 0.1)
    x_ref, _ = ocg.cg_dc(aHy, None, d["S"], d["mask"], np.full(B, 0.05), 10)
    S, m = dev(d["S"]), dev(d["mask"])
    names = ops.schedules(H)
    assert names
    for name in names:
        plan = Plan(H, W, C, B=B)
        plan.set_schedule(H, name)
        assert plan.schedule(0) == name
        e_q = rel(host(plan.sense_normal(dev(d["x"]), S, m, 0.1)), q_ref)
        e_x = rel(host(plan.cg_dc(dev(aHy), S, m, 0.05, 10)), x_ref)
        print(f"{name}: normal {e_q:.2e} cg {e_x:.2e}")
        assert e_q < OP_TOL, name
        assert e_x < CG_TOL, name


@pytest.mark.parametrize("H,W,C", [(320, 24, 1), (320, 40, 2), (320, 24, 64), (128, 24, 64), (384, 40, 1)])
def test_every_schedule_coil_count_edges(H, W, C):
    """The smallest and largest coil counts a plan accepts (1, 2 and 64)
    under every column schedule of a length: coil splits and coil groups
    that get no coil at all (C < split count) and splits of 21-22 coils; the
    forward and adjoint operators at the same counts."""
    from paper_2202_14005_amd import ops
    B = 2
    d = inputs([1800 + i for i in range(B)], H, W, C)
    y_ref = osense.sense_fwd(d["x"], d["S"], d["mask"])
    y = osense.measure(d["x"], d["S"], d["mask"], d["noise"])
    aHy = osense.sense_adj(y, d["S"], d["mask"]).astype(np.complex64)
    q_ref = osense.sense_normal(d["x"], d["S"], d["mask"], 0.1)
    x_ref, _ = ocg.cg_dc(aHy, None, d["S"], d["mask"], np.full(B, 0.05), 10)
    S, m = dev(d["S"]), dev(d["mask"])
    plan = Plan(H, W, C, B=B)
    assert rel(host(plan.sense_fwd(dev(d["x"]), S, m)), y_ref) < OP_TOL
    a_ref = osense.sense_adj(y.astype(np.complex64), d["S"], d["mask"])
    assert rel(host(plan.sense_adj(dev(y.astype(np.complex64)), S, m)), a_ref) < OP_TOL
    names = ops.schedules(H)
    assert names
    for name in names:
        plan = Plan(H, W, C, B=B)
        plan.set_schedule(H, name)
        e_q = rel(host(plan.sense_normal(dev(d["x"]), S, m, 0.1)), q_ref)
        e_x = rel(host(plan.cg_dc(dev(aHy), S, m, 0.05, 10)), x_ref)
        print(f"C={C} {name}: normal {e_q:.2e} cg {e_x:.2e}")
        assert e_q < OP_TOL, name
        assert e_x < CG_TOL, name


def test_kernel_timing_records_each_launch():
    """Per-launch event timing: one record per normal-operator launch and CG
    update of a solve, none once switched off; the solve's result is the
    same with timing on."""
    H, W, C, B, n = 64, 48, 4, 2, 7
    d = case_inputs(H, W, C, "uniform", B=B, seed=1900)
    S, m, x = dev(d["S"]), dev(d["mask"]), dev(d["x"])
    plan = Plan(H, W, C, B=B)
    ref = plan.cg_dc(x, S, m, 0.05, n)
    plan.kernel_timing(True)
    out = plan.cg_dc(x, S, m, 0.05, n)
    t_n, c_n = plan.kernel_time(plan.KERNEL_NORMAL)
    t_u, c_u = plan.kernel_time(plan.KERNEL_CG_UPDATE)
    assert (c_n, c_u) == (n, n) and t_n > 0 and t_u > 0
    assert torch.equal(out, ref)
    plan.sense_normal(x, S, m, 0.1)
    assert plan.kernel_time(plan.KERNEL_NORMAL)[1] == n + 1
    assert plan.kernel_time(plan.KERNEL_CONV_MID) == (0.0, 0)
    plan.kernel_timing(False)
    plan.cg_dc(x, S, m, 0.05, n)
    assert plan.kernel_time(plan.KERNEL_NORMAL) == (0.0, 0)
