"""The allocation-free CG solve (mrx_cg_dc_noalloc), called through the
C-ABI, against mrx_cg_dc on the same plan: two calls in a row, the second
on a smaller batch, must give mrx_cg_dc's solution and residual history bit
for bit (the same kernels, in the same order, on other buffers) and the FP64
oracle's solution to the CG bound 1e-4; status bits are per call; a plan
whose CG buffers exceed the fixed scratch is refused before any work."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import cg as ocg
from oracle import sense as osense
from paper_2202_14005_amd import ops
from paper_2202_14005_amd._lib import lib
from tests.gpu_util import dev, host, inputs, oracle_threads, rel

pytestmark = pytest.mark.gpu

CG_TOL = 1e-4
NONFINITE = 1


def ptr(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def noalloc_call(plan, aHy, S, m, lam, n, z, x, hist, flags):
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return lib().mrx_cg_dc_noalloc(plan._h, ptr(aHy), ptr(z), ptr(S), ptr(m), ptr(lam), n, ptr(x), ptr(hist),
                                   ptr(flags), stream)


def solve_pair(B, H, W, C, seed, poison=None):
    d = inputs([seed + i for i in range(B)], H, W, C)
    y = osense.measure(d["x"], d["S"], d["mask"], d["noise"])
    aHy = osense.sense_adj(y, d["S"], d["mask"]).astype(np.complex64)
    rng = np.random.default_rng(seed)
    z = (aHy + 0.05 * (rng.standard_normal(aHy.shape) + 1j * rng.standard_normal(aHy.shape))).astype(np.complex64)
    if poison is not None:
        aHy[poison, 3, 5] = np.nan
    plan = ops.Plan(H, W, C, B=B)
    S, m, a, zt = dev(d["S"]), dev(d["mask"]), dev(aHy), dev(z)
    lam = plan.lam(0.05)
    n = 10
    x_ref, h_ref = plan.cg_dc(a, S, m, lam, n, z=zt, hist=True)
    x = torch.full_like(x_ref, float("nan"))
    hist = torch.empty_like(h_ref)
    flags = torch.full((B,), 0xFFFF, dtype=torch.int32, device=a.device)
    code = noalloc_call(plan, a, S, m, lam, n, zt, x, hist, flags)
    assert code == 0, lib().mrx_last_error().decode()
    torch.cuda.synchronize()
    return d, aHy, z, x_ref, h_ref, x, hist, host(flags)


def test_noalloc_equals_cg_dc_two_calls_second_smaller():
    for B, H, W, C, seed in [(4, 320, 320, 15, 7000), (2, 192, 192, 8, 7100)]:
        print(f"case B={B} {H}x{W} C={C}", flush=True)
        d, aHy, z, x_ref, h_ref, x, hist, flags = solve_pair(B, H, W, C, seed)
        assert torch.equal(x, x_ref)
        assert torch.equal(hist, h_ref)
        assert np.all(flags == 0), flags
        with oracle_threads():
            xo, _ = ocg.cg_dc(aHy, z, d["S"], d["mask"], np.full(B, 0.05, dtype=np.float32), 10)
        e = rel(host(x), xo)
        print(f"  noalloc vs oracle {e:.2e}")
        assert e < CG_TOL


def test_noalloc_status_bits_are_per_call():
    *_, flags = solve_pair(2, 48, 40, 4, 7200, poison=1)
    assert flags[0] == 0 and flags[1] & NONFINITE, flags
    *_, flags = solve_pair(2, 48, 40, 4, 7300)
    assert np.all(flags == 0), flags


def test_noalloc_refuses_a_plan_beyond_the_scratch():
    B, H, W, C = 40, 320, 320, 2
    plan = ops.Plan(H, W, C, B=B)
    a = torch.zeros((B, H, W), dtype=torch.complex64, device="cuda")
    S = torch.zeros((B, C, H, W), dtype=torch.complex64, device="cuda")
    m = torch.ones((B, H), dtype=torch.float32, device="cuda")
    x = torch.full_like(a, 7.0)
    code = noalloc_call(plan, a, S, m, plan.lam(0.05), 10, None, x, None, None)
    msg = lib().mrx_last_error().decode()
    torch.cuda.synchronize()
    assert code == -1 and "scratch" in msg, (code, msg)
    assert bool((x == 7.0).all())
