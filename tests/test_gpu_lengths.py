"""Every supported transform length against the FP64 oracle, through the
C-ABI: the forward, adjoint and normal operators (relative error <= 1e-5)
and the CG solve (<= 1e-4, 10 iterations), with the length along H (column
transforms and the normal operator) and along W (row transforms), on one
slice of three coils; and an uneven batch of generic lengths.  Lengths
without a tuned schedule run the build's generic one."""
import numpy as np
import pytest

from oracle import cg as ocg
from oracle import sense as osense
from paper_2202_14005_amd import _lib, ops
from tests.gpu_util import dev, host, inputs, rel, uneven

pytestmark = pytest.mark.gpu

OP_TOL = 1e-5
CG_TOL = 1e-4
LENGTHS = [n for n in range(8, 1025, 2) if _lib.lib().mrx_supported_length(n)]


def check_slice(H, W, C, seed):
    d = inputs([seed], H, W, C, 4, max(2, min(24, H // 8)))
    x, S, m = d["x"], d["S"], d["mask"]
    plan = ops.Plan(H, W, C, B=1)
    xt, St, mt = dev(x), dev(S), dev(m)
    y = plan.sense_fwd(xt, St, mt)
    yref = osense.sense_fwd(x, S, m)
    e_f = rel(host(y), yref)
    yc = yref.astype(np.complex64)
    a = plan.sense_adj(dev(yc), St, mt)
    aref = osense.sense_adj(yc, S, m)
    e_a = rel(host(a), aref)
    q = plan.sense_normal(xt, St, mt, 0.05)
    e_n = rel(host(q), osense.sense_normal(x, S, m, 0.05))
    ac = aref.astype(np.complex64)
    xs = plan.cg_dc(dev(ac), St, mt, 0.05, 10)
    xref, _ = ocg.cg_dc(ac, None, S, m, np.full(1, 0.05, dtype=np.float32), 10)
    e_c = rel(host(xs), xref)
    return e_f, e_a, e_n, e_c, plan.schedule(0)


@pytest.mark.parametrize("n", LENGTHS)
def test_length_parity(n):
    for H, W in ((n, 24), (24, n)):
        e_f, e_a, e_n, e_c, sched = check_slice(H, W, 3, 9000 + n)
        print(f"{H}x{W} [{sched}]: fwd {e_f:.1e} adj {e_a:.1e} normal {e_n:.1e} cg {e_c:.1e}")
        assert e_f < OP_TOL and e_a < OP_TOL and e_n < OP_TOL, (H, W)
        assert e_c < CG_TOL, (H, W)


def test_uneven_generic_lengths_cg():
    shapes = [(240, 288, 4), (640, 96, 3), (1024, 8, 2), (54, 250, 3)]
    sl, pk = uneven(shapes, seed0=9500)
    plan = ops.Plan([s[0] for s in shapes], [s[1] for s in shapes], [s[2] for s in shapes])
    S, m = dev(pk["S"]), dev(pk["mask"])
    aHy = np.concatenate([osense.sense_adj(osense.sense_fwd(s["x"][None], s["S"][None], s["mask"][None]),
                                           s["S"][None], s["mask"][None]).ravel() for s in sl]).astype(np.complex64)
    x = host(plan.cg_dc(dev(aHy), S, m, 0.05, 10))
    q = host(plan.sense_normal(dev(pk["x"]), S, m, 0.05))
    o = 0
    for (H, W, C), s in zip(shapes, sl):
        a = aHy[o:o + H * W].reshape(1, H, W)
        xref, _ = ocg.cg_dc(a, None, s["S"][None], s["mask"][None], np.full(1, 0.05, dtype=np.float32), 10)
        qref = osense.sense_normal(s["x"][None], s["S"][None], s["mask"][None], 0.05)
        e_c, e_n = rel(x[o:o + H * W], xref), rel(q[o:o + H * W], qref)
        print(f"{H}x{W}x{C}: cg {e_c:.1e} normal {e_n:.1e}")
        assert e_c < CG_TOL and e_n < OP_TOL
        o += H * W
