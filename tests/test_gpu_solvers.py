"""GPU parity of the CSR comparison path and the Krylov solvers against the
CPU oracle: pattern bit-equal, values and SpMV to 1e-13/1e-12, the first PCG
iterates to 1e-10, converged solves judged by the oracle's operator,
flexible PCG reducing to PCG for a fixed SPD preconditioner and following the
oracle's flexible PCG and FCG(m) for one that changes between calls, iterative
refinement to 1e-10, and the failure paths (zero right-hand side, breakdown,
iteration limit, failing preconditioner)."""
import numpy as np
import pytest

import seeded_inputs as si
from helpers import (TOL, HostPrecond, dev, dpn_of, gpu_apply, make_op, problem, rel_err,
                     torch_dtype)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q1():
    import torch
    assert torch.cuda.is_available()
    import paper_2308_09839_amd as q1
    return q1


def rhs(A, pr, seed):
    b = si.vec_uniform(A.n, seed, si.STREAM_RHS)
    if pr.get("mask") is not None:
        b[si.dof_mask(pr["mask"], dpn_of(pr["physics"])) == 1] = 0.0
    return b


# -- CSR ------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("physics,n,jitter,mask", [(1, (16, 16, 16), 0.1, True),
                                                   (1, (7, 5, 3), 0.0, False),
                                                   (3, (6, 5, 4), 0.1, True),
                                                   (2, (6, 5, 4), 0.1, True)])
def test_csr_parity(q1, orc, physics, n, jitter, mask, dtype):
    print(f"\n[csr] physics={physics} n={n} dtype={dtype}", flush=True)
    pr = problem(physics, n, jitter, 51, mask)
    A = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    op = make_op(pr, dtype, 0)
    csr = q1.q1_csr_create(op)
    rowptr, col, val = q1.q1_csr_export(csr)
    assert np.array_equal(rowptr.astype(np.int64), A.rowptr)
    assert np.array_equal(col, A.col)
    tol = 1e-13 if dtype == 0 else 2e-6
    assert np.max(np.abs(val - A.val)) <= tol * np.max(np.abs(A.val))
    x = si.vec_uniform(A.n, 52, si.STREAM_X)
    ref = A.matvec(x)
    y_csr = gpu_apply(csr, x, dtype)
    y_mf = gpu_apply(op, x, dtype)
    assert rel_err(y_csr, ref) <= TOL[dtype]
    assert rel_err(y_mf, y_csr) <= 2 * TOL[dtype]
    nb, fl = csr.bytes()
    assert fl == 2.0 * A.nnz


# -- PCG ------------------------------------------------------------------------

def solve_gpu(q1, op, b, dtype, pc=1, rtol=1e-8, maxit=20000):
    import torch
    t = torch_dtype(dtype)
    bd = dev(b, t)
    xd = torch.empty_like(bd)
    st = q1.q1_pcg(op, pc, bd, xd, rtol, maxit)
    return xd.double().cpu().numpy(), st


@pytest.mark.parametrize("csr,jitter", [(False, 0.1), (True, 0.1), (False, 0.0)])
def test_pcg_first_iterates(q1, orc, csr, jitter):
    """The first ten iterates against the oracle's; undistorted, the default
    operator takes the owner-computes tiles, whose apply also forms the p.q
    partials the iteration reduces."""
    print(f"\n[pcg iterates] csr={csr} jitter={jitter}", flush=True)
    pr = problem(1, (16, 16, 16), jitter, 2308, True)
    A = orc.assemble(1, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    b = rhs(A, pr, 2308)
    op = make_op(pr, 0, 0)
    if csr:
        op = q1.q1_csr_create(op)
    for k in range(1, 11):
        ref = orc.pcg(A, b, rtol=0.0, maxit=k)
        x, st = solve_gpu(q1, op, b, 0, rtol=0.0, maxit=k)
        assert st["status"] == -4 and st["iters"] == k
        assert np.linalg.norm(x - ref.x) <= 1e-10 * np.linalg.norm(ref.x), k


@pytest.mark.parametrize("physics,n,jitter", [(1, (16, 16, 16), 0.1), (1, (13, 11, 7), 0.0),
                                              (3, (8, 8, 8), 0.1), (2, (10, 9, 8), 0.1)])
def test_pcg_converged(q1, orc, physics, n, jitter):
    print(f"\n[pcg converged] physics={physics} n={n}", flush=True)
    pr = problem(physics, n, jitter, 2308, True)
    A = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    b = rhs(A, pr, 61)
    ref = orc.pcg(A, b, rtol=1e-8)
    x, st = solve_gpu(q1, make_op(pr, 0, 0), b, 0, rtol=1e-8)
    assert st["status"] == 0
    assert orc.true_rel_res(A, x, b) <= 1e-8 * (1 + 1e-3)
    assert abs(st["iters"] - ref.iters) <= 0.02 * ref.iters + 2
    assert abs(st["true_rel_res"] - orc.true_rel_res(A, x, b)) <= 1e-12


def test_pcg_fp32_operator(q1, orc):
    print("\n[pcg fp32]", flush=True)
    pr = problem(1, (12, 12, 12), 0.1, 63, True)
    A = orc.assemble(1, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    b = rhs(A, pr, 63)
    x, st = solve_gpu(q1, make_op(pr, 1, 0), b, 1, rtol=1e-5)
    assert st["status"] == 0
    assert orc.true_rel_res(A, x, b) <= 1e-4


def test_pcg_edge_cases(q1, orc):
    print("\n[pcg edge cases]", flush=True)
    pr = problem(1, (5, 4, 3), 0.1, 64, True)
    A = orc.assemble(1, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    op = make_op(pr, 0, 0)
    # zero right-hand side
    x, st = solve_gpu(q1, op, np.zeros(A.n), 0)
    assert st["status"] == 0 and st["iters"] == 0 and np.all(x == 0)
    # iteration limit: status ENOCONV, x = the oracle's iterate
    b = rhs(A, pr, 64)
    x, st = solve_gpu(q1, op, b, 0, rtol=1e-14, maxit=3)
    ref = orc.pcg(A, b, rtol=0.0, maxit=3)
    assert st["status"] == -4 and st["iters"] == 3
    assert np.linalg.norm(x - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    # negative definite operator: breakdown at the first p^T A p
    prn = dict(pr)
    prn["coef"] = -pr["coef"]
    x, st = solve_gpu(q1, make_op(prn, 0, 0), b, 0, pc=0)
    assert st["status"] == -5


# -- flexible PCG -----------------------------------------------------------------

def test_fpcg_with_jacobi_equals_pcg(q1, orc):
    import torch
    print("\n[fpcg = pcg]", flush=True)
    pr = problem(1, (12, 10, 8), 0.1, 71, True)
    A = orc.assemble(1, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    b = rhs(A, pr, 71)
    op = make_op(pr, 0, 0)
    J = q1.q1_jacobi_create(op)
    for k in (1, 5, 20):
        bd = dev(b, torch.float64)
        xd = torch.empty_like(bd)
        st = q1.q1_fpcg(op, J, bd, xd, 0.0, k)
        ref = orc.pcg(A, b, rtol=0.0, maxit=k)
        x = xd.cpu().numpy()
        assert st["iters"] == k and st["fallback_at"] == -1
        assert np.linalg.norm(x - ref.x) <= 1e-10 * np.linalg.norm(ref.x), k
    bd = dev(b, torch.float64)
    xd = torch.empty_like(bd)
    st = q1.q1_fpcg(op, J, bd, xd, 1e-8, 5000)
    assert st["status"] == 0
    assert orc.true_rel_res(A, xd.cpu().numpy(), b) <= 1e-8 * (1 + 1e-3)


@pytest.mark.parametrize("m", [2, 8])
def test_fcg_with_jacobi_equals_pcg(q1, orc, m):
    """For a fixed SPD preconditioner the extra orthogonalisations of FCG(m)
    vanish: the iterates are the PCG iterates."""
    import torch
    print(f"\n[fcg({m}) = pcg]", flush=True)
    pr = problem(1, (12, 10, 8), 0.1, 73, True)
    A = orc.assemble(1, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    b = rhs(A, pr, 73)
    op = make_op(pr, 0, 0)
    J = q1.q1_jacobi_create(op)
    for k in (1, 3, 12):
        bd = dev(b, torch.float64)
        xd = torch.empty_like(bd)
        st = q1.q1_fcg(op, J, bd, xd, 0.0, k, trunc_m=m)
        ref = orc.pcg(A, b, rtol=0.0, maxit=k)
        assert st["iters"] == k and st["fallback_at"] == -1
        assert np.linalg.norm(xd.cpu().numpy() - ref.x) <= 1e-10 * np.linalg.norm(ref.x), k
    bd = dev(b, torch.float64)
    xd = torch.empty_like(bd)
    st = q1.q1_fcg(op, J, bd, xd, 1e-8, 5000, trunc_m=m)
    assert st["status"] == 0
    assert orc.true_rel_res(A, xd.cpu().numpy(), b) <= 1e-8 * (1 + 1e-3)
    with pytest.raises(q1.Q1Error):
        q1.q1_fcg(op, J, bd, xd, 1e-8, 10, trunc_m=9)


def _varying(d, seed):
    """Jacobi scaled per entry by seeded factors that change at every call."""
    calls = [0]

    def f(r):
        k = calls[0]
        calls[0] += 1
        return si.varying_factors(r.shape[0], k, seed) * r / d

    return f


@pytest.mark.parametrize("m", [1, 2, 8])
def test_fcg_varying_preconditioner_matches_oracle(q1, orc, m):
    """With a preconditioner that changes between calls, q1_fpcg (m = 1) and
    q1_fcg(m) follow the oracle's Golub-Ye FPCG and FCG(m) iterates."""
    import torch
    print(f"\n[fcg({m}) varying preconditioner]", flush=True)
    pr = problem(1, (12, 10, 8), 0.1, 74, True)
    A = orc.assemble(1, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    b = rhs(A, pr, 74)
    d = A.diag()
    op = make_op(pr, 0, 0)
    for k in (1, 4, 10):
        bd = dev(b, torch.float64)
        xd = torch.empty_like(bd)
        M = HostPrecond(_varying(d, 81), A.n)
        st = q1.q1_fcg(op, M, bd, xd, 0.0, k, trunc_m=m)
        if m == 1:
            ref = orc.fpcg(A, b, _varying(d, 81), rtol=0.0, maxit=k)
        else:
            ref = orc.fcg(A, b, _varying(d, 81), m, rtol=0.0, maxit=k)
        assert st["iters"] == k and st["fallback_at"] == -1 and M.calls == k
        x = xd.cpu().numpy()
        assert np.linalg.norm(x - ref.x) <= 1e-10 * np.linalg.norm(ref.x), (m, k)
    bd = dev(b, torch.float64)
    xd = torch.empty_like(bd)
    st = q1.q1_fcg(op, HostPrecond(_varying(d, 82), A.n), bd, xd, 1e-8, 5000, trunc_m=m)
    ref = orc.fcg(A, b, _varying(d, 82), m, rtol=1e-8, maxit=5000)
    assert st["status"] == 0 and st["fallback_at"] == -1
    assert abs(st["iters"] - ref.iters) <= 0.02 * ref.iters + 2
    assert orc.true_rel_res(A, xd.cpu().numpy(), b) <= 1e-8 * (1 + 1e-3)


def test_fpcg_safeguard_fallback(q1, orc):
    import torch
    print("\n[fpcg safeguard]", flush=True)
    pr = problem(1, (10, 10, 10), 0.1, 72, True)
    A = orc.assemble(1, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    b = rhs(A, pr, 72)
    op = make_op(pr, 0, 0)
    bd = dev(b, torch.float64)
    xd = torch.empty_like(bd)
    calls = []

    def failing(r, z, s):  # reports failure without touching z
        calls.append(1)
        return 1

    st = q1.q1_fpcg(op, failing, bd, xd, 1e-8, 5000)
    assert st["status"] == 0 and st["fallback_at"] == 0 and len(calls) == 1
    assert orc.true_rel_res(A, xd.cpu().numpy(), b) <= 1e-8 * (1 + 1e-3)
    ref = orc.pcg(A, b, rtol=1e-8)
    assert abs(st["iters"] - ref.iters) <= 0.02 * ref.iters + 2


# -- mixed-precision iterative refinement ---------------------------------------------

@pytest.mark.parametrize("physics,n", [(1, (16, 16, 16)), (3, (10, 10, 10))])
def test_ir_reaches_fp64_tolerance(q1, orc, physics, n):
    import torch
    print(f"\n[ir] physics={physics} n={n}", flush=True)
    pr = problem(physics, n, 0.1 if physics == 1 else 0.0, 81, True)
    A = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    b = rhs(A, pr, 81)
    op64 = make_op(pr, 0, 0)
    op32 = make_op(pr, 1, 0)
    bd = dev(b, torch.float64)
    xd = torch.empty_like(bd)
    st = q1.q1_ir_solve(op64, op32, bd, xd, 1e-10, 1e-4)
    assert st["status"] == 0 and st["outer_iters"] >= 2
    assert orc.true_rel_res(A, xd.cpu().numpy(), b) <= 1e-10 * (1 + 1e-3)


# -- mixed-precision PCG with reliable updates ---------------------------------------

@pytest.mark.parametrize("physics,n,jitter", [(1, (16, 16, 16), 0.1), (3, (10, 10, 10), 0.0),
                                              (1, (32, 16, 8), 0.0)])
def test_mpcg_reaches_fp64_tolerance(q1, orc, physics, n, jitter):
    """FP32 recurrences with FP64 refreshes reach an FP64 tolerance that FP32
    PCG alone cannot, in about the iterations of FP64 PCG (undistorted 32 x 16 x 8:
    both operators on owner-computes tiles)."""
    import torch
    print(f"\n[mpcg] physics={physics} n={n} jitter={jitter}", flush=True)
    pr = problem(physics, n, jitter, 82, True)
    A = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    b = rhs(A, pr, 82)
    op64, op32 = make_op(pr, 0, 0), make_op(pr, 1, 0)
    bd = dev(b, torch.float64)
    xd = torch.full_like(bd, 7.0)  # x is overwritten, not used as a guess
    st = q1.q1_mpcg(op64, op32, bd, xd, 1e-10, 0.1, 20000)
    x = xd.cpu().numpy()
    assert st["status"] == 0 and st["outer_iters"] >= 2
    t = orc.true_rel_res(A, x, b)
    assert t <= 1e-10 * (1 + 1e-3)
    assert abs(st["true_rel_res"] - t) <= 1e-13
    ref = orc.pcg(A, b, rtol=1e-10)
    assert st["iters"] <= 1.25 * ref.iters + 5, (st["iters"], ref.iters)


def test_mpcg_edge_cases(q1, orc):
    import torch
    print("\n[mpcg edge cases]", flush=True)
    pr = problem(1, (6, 5, 4), 0.1, 83, True)
    A = orc.assemble(1, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    op64, op32 = make_op(pr, 0, 0), make_op(pr, 1, 0)
    bd = dev(np.zeros(A.n), torch.float64)
    xd = torch.full_like(bd, 3.0)
    st = q1.q1_mpcg(op64, op32, bd, xd, 1e-10, 0.1, 100)
    assert st["status"] == 0 and st["iters"] == 0 and bool((xd == 0).all())
    # iteration limit: ENOCONV with x the FP64 sum of the corrections so far
    b = rhs(A, pr, 83)
    bd = dev(b, torch.float64)
    st = q1.q1_mpcg(op64, op32, bd, xd, 1e-14, 0.1, 4)
    assert st["status"] == -4 and st["iters"] == 4
    ref = orc.pcg(A, b, rtol=0.0, maxit=4)
    x = xd.cpu().numpy()
    assert np.linalg.norm(x - ref.x) <= 1e-5 * np.linalg.norm(ref.x)
    assert abs(st["true_rel_res"] - orc.true_rel_res(A, x, b)) <= 1e-12
    with pytest.raises(q1.Q1Error):
        q1.q1_mpcg(op64, op32, bd, xd, 1e-10, 1.5, 100)
    with pytest.raises(q1.Q1Error):
        q1.q1_mpcg(op32, op64, bd, xd, 1e-10, 0.1, 100)


def test_pcg_trace_snapshots(q1, orc):
    """Recorded iterates equal the oracle's PCG iterates after the same number
    of iterations; snapshots past convergence hold the final x."""
    import torch
    print("\n[pcg trace]", flush=True)
    pr = problem(1, (10, 9, 8), 0.1, 91, True)
    A = orc.assemble(1, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    b = rhs(A, pr, 91)
    op = make_op(pr, 0, 0)
    bd = dev(b, torch.float64)
    xd = torch.empty_like(bd)
    its = [0, 1, 2, 5, 9, 9, 30, 100000]
    snaps = [torch.full_like(bd, 5.0) for _ in its]
    st = q1.q1_pcg_trace(op, 1, bd, xd, 1e-8, 5000, its, snaps)
    assert st["status"] == 0
    for k, s in zip(its, snaps):
        if k == 0:
            assert bool((s == 0).all())
            continue
        ref = orc.pcg(A, b, rtol=0.0, maxit=min(k, st["iters"]))
        x = s.cpu().numpy()
        assert np.linalg.norm(x - ref.x) <= 1e-10 * np.linalg.norm(ref.x), k
    assert torch.equal(snaps[-1], xd)


# -- fused single-workgroup PCG (small problems) ----------------------------------

def solve_fused(q1, op, b, pc=1, rtol=1e-8, maxit=20000):
    import torch
    bd = dev(b, torch.float64)
    xd = torch.empty_like(bd)
    st = q1.q1_pcg_fused(op, pc, bd, xd, rtol, maxit)
    return xd.cpu().numpy(), st


def test_fused_pcg_iterates(q1, orc):
    """Truncated fused solves equal the oracle's PCG iterates."""
    print("\n[fused pcg iterates] 16^3 jittered", flush=True)
    pr = problem(1, (16, 16, 16), 0.1, 2308, True)
    A = orc.assemble(1, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    b = rhs(A, pr, 2308)
    op = make_op(pr, 0, 0)
    for k in (1, 2, 5, 10):
        ref = orc.pcg(A, b, rtol=0.0, maxit=k)
        x, st = solve_fused(q1, op, b, rtol=0.0, maxit=k)
        assert st["status"] == -4 and st["iters"] == k
        assert np.linalg.norm(x - ref.x) <= 1e-10 * np.linalg.norm(ref.x), k


@pytest.mark.parametrize("physics,n,jitter", [(1, (16, 16, 16), 0.1), (2, (9, 8, 7), 0.1),
                                              (3, (7, 6, 5), 0.1), (1, (5, 4, 3), 0.0)])
def test_fused_pcg_converged(q1, orc, physics, n, jitter):
    print(f"\n[fused pcg] physics={physics} n={n}", flush=True)
    pr = problem(physics, n, jitter, 91, True)
    A = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    b = rhs(A, pr, 92)
    ref = orc.pcg(A, b, rtol=1e-8)
    x, st = solve_fused(q1, make_op(pr, 0, 0), b)
    tr = orc.true_rel_res(A, x, b)
    assert st["status"] == 0
    assert tr <= 1e-8 * (1 + 1e-3)
    assert abs(st["iters"] - ref.iters) <= 0.02 * ref.iters + 2, (st["iters"], ref.iters)
    assert abs(st["true_rel_res"] - tr) <= 1e-12


def test_fused_pcg_limits(q1):
    import torch
    print("\n[fused pcg limits]", flush=True)
    pr = problem(1, (24, 24, 24), 0.0, 93, True)  # 15,625 DOF: beyond the LDS capacity
    op = make_op(pr, 0, 0)
    bd = torch.ones(pr["xyz"].shape[1], dtype=torch.float64, device="cuda")
    with pytest.raises(q1.Q1Error) as ei:
        q1.q1_pcg_fused(op, 1, bd, torch.empty_like(bd), 1e-8, 100)
    assert ei.value.code == -6
    pr = problem(1, (4, 4, 4), 0.0, 94, True)
    op = make_op(pr, 0, 0)
    bd = torch.zeros(pr["xyz"].shape[1], dtype=torch.float64, device="cuda")
    xd = torch.full_like(bd, 3.0)
    st = q1.q1_pcg_fused(op, 1, bd, xd, 1e-8, 100)
    assert st["status"] == 0 and st["iters"] == 0 and torch.all(xd == 0)
    op32 = make_op(pr, 1, 0)
    with pytest.raises(q1.Q1Error):
        q1.q1_pcg_fused(op32, 1, bd, xd, 1e-8, 100)


# -- the dot-product study ------------------------------------------------------

@pytest.mark.parametrize("n", [1, 255, 4913, 2_146_689])
@pytest.mark.parametrize("dtype", [0, 1])
def test_dot_variants(q1, n, dtype):
    """Both dot implementations against an exact-enough host sum (math.fsum of
    the FP64 products); the two-stage one is bitwise reproducible."""
    import math

    import torch
    print(f"\n[dot] n={n} dtype={dtype}", flush=True)
    a = si.vec_uniform(n, 11, si.STREAM_X)
    b = si.vec_uniform(n, 12, si.STREAM_X)
    t = torch_dtype(dtype)
    ad, bd = dev(a, t), dev(b, t)
    ah, bh = ad.double().cpu().numpy(), bd.double().cpu().numpy()  # the rounded operands
    ref = math.fsum(ah * bh)
    scale = float(np.abs(ah) @ np.abs(bh))
    work = torch.empty(1024, dtype=torch.float64, device="cuda")
    outs = []
    for variant in (q1.Q1_DOT_TWO_STAGE, q1.Q1_DOT_ATOMIC):
        for nb in (0, 1, 7, 1024):
            out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
            q1.q1_dot(ad, bd, out, variant, nb, work)
            torch.cuda.synchronize()
            v = float(out.item())
            assert abs(v - ref) <= 1e-13 * scale + 1e-300, (variant, nb, v, ref)
            if variant == q1.Q1_DOT_TWO_STAGE and nb == 0:
                outs.append(v)
    out = torch.empty((1,), dtype=torch.float64, device="cuda")
    q1.q1_dot(ad, bd, out, q1.Q1_DOT_TWO_STAGE, 0, work)
    torch.cuda.synchronize()
    assert float(out.item()) == outs[0]
    with pytest.raises(q1.Q1Error):
        q1.q1_dot(ad, bd, out, q1.Q1_DOT_TWO_STAGE, 1025, work)


def test_solves_bitwise_reproducible(q1, orc):
    """On the default (block) operators two identical solves take the same
    iterations and return bitwise-identical iterates: the apply, the diagonal and
    every reduction add in a fixed order."""
    import torch
    for physics, n, jitter in ((1, (16, 16, 16), 0.1), (3, (10, 10, 10), 0.1),
                               (1, (32, 16, 8), 0.0)):
        print(f"\n[reproducible solve] physics={physics} n={n} jitter={jitter}", flush=True)
        pr = problem(physics, n, jitter, 83, True)
        A = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
        b = rhs(A, pr, 83)
        op64, op32 = make_op(pr, 0, 0), make_op(pr, 1, 0)
        assert op64.reproducible() and op32.reproducible()
        bd = dev(b, torch.float64)
        for solve in (lambda x: q1.q1_pcg(op64, 1, bd, x, 1e-10, 20000),
                      lambda x: q1.q1_mpcg(op64, op32, bd, x, 1e-10, 0.1, 20000)):
            xs, its = [], []
            for _ in range(2):
                xd = torch.empty_like(bd)
                st = solve(xd)
                assert st["status"] == 0
                its.append(st["iters"])
                xs.append(xd.cpu().numpy())
            assert its[0] == its[1]
            assert np.array_equal(xs[0], xs[1])
