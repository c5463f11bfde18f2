"""q1_pcg_noalloc (workspace in the library's static device array, for callers
that cannot allocate) against q1_pcg on the same operators: two calls in a row,
the second on a smaller problem, must give the same iterations, statuses and
iterates.  The default operators are bitwise reproducible, so the iterates are
compared for equality; the bar of the FP64 parity tests (1e-12) is checked too."""
import numpy as np
import pytest

import seeded_inputs as si
from helpers import dev, make_op, problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q1():
    import torch
    assert torch.cuda.is_available()
    import paper_2308_09839_amd as q1
    return q1


def _rhs(n, mask, dpn, seed):
    b = si.vec_uniform(n * dpn, seed, si.STREAM_RHS)
    b[np.repeat(mask.astype(bool), dpn)] = 0.0
    return b


def test_pcg_noalloc_matches_pcg(q1, orc):
    import torch
    cases = [(1, (24, 20, 18), 0.1, 0, 1e-10),   # larger first
             (1, (32, 16, 8), 0.0, 0, 1e-10),    # owner-computes tiles (one partial per tile)
             (3, (8, 7, 6), 0.1, 0, 1e-10),      # then a smaller one (elasticity)
             (1, (9, 8, 7), 0.0, 1, 1e-5),       # an FP32 operator
             (1, (16, 8, 4), 0.0, 1, 1e-5)]      # and an FP32 owner-computes one
    for physics, n, jitter, dtype, rtol in cases:
        print(f"\n[noalloc] physics={physics} n={n} dtype={dtype}", flush=True)
        pr = problem(physics, n, jitter, 91, True)
        dpn = 1 if physics == 1 else 3
        nn = pr["xyz"].shape[1]
        b = _rhs(nn, pr["mask"], dpn, 91)
        op = make_op(pr, dtype, 0)
        t = torch.float64 if dtype == 0 else torch.float32
        bd = dev(b, t)
        x_ref = torch.full_like(bd, 3.0)
        x_na = torch.full_like(bd, -5.0)  # overwritten: x0 = 0 in both
        st_ref = q1.q1_pcg(op, 1, bd, x_ref, rtol, 5000)
        st_na = q1.q1_pcg_noalloc(op, 1, bd, x_na, rtol, 5000)
        torch.cuda.synchronize()
        for key in ("status", "iters"):
            assert st_na[key] == st_ref[key], (key, st_na[key], st_ref[key])
        assert st_na["status"] == 0
        xr, xn = x_ref.double().cpu().numpy(), x_na.double().cpu().numpy()
        assert np.linalg.norm(xn - xr) <= 1e-12 * np.linalg.norm(xr)
        assert np.array_equal(xn, xr)
        assert st_na["true_rel_res"] == st_ref["true_rel_res"]
        A = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
        assert orc.true_rel_res(A, xr, b) <= rtol * 1.01


def test_pcg_noalloc_limits(q1):
    """Beyond the static workspace the call returns Q1_EINVAL before any launch;
    b = 0 gives x = 0 at once; maxit = 0 reports no convergence."""
    import torch
    m = 146  # 147^3 nodes > Q1_NOALLOC_MAX_DOF
    assert (m + 1) ** 3 > q1.Q1_NOALLOC_MAX_DOF
    xyz, conn = si.box_mesh(m, m, m)
    k = np.ones((1, m ** 3))
    op = q1.q1_op_create(1, 0, 1, dev(xyz), dev(conn.astype(np.int32)), dev(k))
    bd = torch.zeros(xyz.shape[1], dtype=torch.float64, device="cuda")
    xd = torch.empty_like(bd)
    with pytest.raises(q1.Q1Error):
        q1.q1_pcg_noalloc(op, 1, bd, xd, 1e-8, 10)
    op.destroy()
    pr = problem(1, (5, 4, 3), 0.1, 92, True)
    op = make_op(pr, 0, 0)
    bd = torch.zeros(pr["xyz"].shape[1], dtype=torch.float64, device="cuda")
    xd = torch.full_like(bd, 1.0)
    st = q1.q1_pcg_noalloc(op, 1, bd, xd, 1e-8, 10)
    assert st["status"] == 0 and st["iters"] == 0 and float(xd.abs().max()) == 0.0
    b = _rhs(pr["xyz"].shape[1], pr["mask"], 1, 92)
    st = q1.q1_pcg_noalloc(op, 1, dev(b), xd, 1e-8, 0)
    assert st["status"] == q1.Q1_ENOCONV
