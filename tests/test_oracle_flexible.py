"""Pins of the oracle's flexible Krylov solvers (CPU only).

The flexible solvers run with a preconditioner that changes from one call to
the next: z = f_k * r / diag(A), where f_k holds seeded factors in [0.5, 1.5)
that differ per call k.  With such a preconditioner the flexible choices of
beta (Golub-Ye) and of the A-orthogonalisation (Notay's FCG(m)) are no longer
equivalent to the standard PCG beta, so each pin below fails for a plausible
mistake in them:

* consecutive steps are A-conjugate (the flexible beta enforces it exactly;
  the standard beta rho_{k+1}/rho_k gives a conjugacy defect of order 1);
* FCG with every direction kept is the Galerkin (energy-minimising) solution
  on the span of its directions, and so reaches the dense solve in at most n
  steps;
* FCG(m) keeps every direction A-conjugate to its m predecessors, and its
  energy error decreases monotonically;
* FCG(1) and Golub-Ye flexible PCG, two different formulas, give the same
  iterates; for a fixed SPD preconditioner FCG(m) gives the PCG iterates.
"""
from __future__ import annotations

import numpy as np
import pytest

import seeded_inputs as si

from test_oracle_pins import dirichlet_problem


def varying_jacobi(d: np.ndarray, seed: int):
    calls = [0]

    def M(r):
        k = calls[0]
        calls[0] += 1
        return si.varying_factors(r.shape[0], k, seed) * r / d

    return M


def energy(Ad, v):
    return float(v @ Ad @ v)


def conjugacy_defect(Ad, u, v):
    return abs(float(u @ Ad @ v)) / np.sqrt(energy(Ad, u) * energy(Ad, v))


def test_fpcg_consecutive_steps_conjugate(orc):
    A, b = dirichlet_problem(orc, 1, (4, 3, 3), 41)
    Ad = A.to_dense()
    res = orc.fpcg(A, b, varying_jacobi(A.diag(), 77), rtol=0.0, maxit=15, record=True)
    assert res.status == -4 and res.iters == 15
    steps = np.diff(res.iterates, axis=0)  # x_{k+1} - x_k = alpha_k p_k
    worst = max(conjugacy_defect(Ad, steps[k + 1], steps[k]) for k in range(len(steps) - 1))
    assert worst <= 1e-10, worst


def test_fcg1_equals_golub_ye_fpcg(orc):
    A, b = dirichlet_problem(orc, 1, (4, 4, 3), 42)
    d = A.diag()
    g = orc.fpcg(A, b, varying_jacobi(d, 78), rtol=0.0, maxit=25, record=True)
    f = orc.fcg(A, b, varying_jacobi(d, 78), 1, rtol=0.0, maxit=25, record=True)
    assert g.iters == f.iters == 25
    scale = np.max(np.abs(g.iterates))
    assert np.max(np.abs(g.iterates - f.iterates)) <= 1e-10 * scale


@pytest.mark.parametrize("physics,n", [(1, (2, 2, 2)), (3, (1, 1, 2))])
def test_full_fcg_is_galerkin_and_finite(orc, physics, n):
    A, b = dirichlet_problem(orc, physics, n, 43)
    Ad = A.to_dense()
    xs = np.linalg.solve(Ad, b)
    N = A.n
    res = orc.fcg(A, b, varying_jacobi(A.diag(), 79), N, rtol=1e-13, maxit=N, record=True)
    assert res.status == 0 and res.iters <= N
    assert np.linalg.norm(res.x - xs) <= 1e-9 * np.linalg.norm(xs)
    steps = np.diff(res.iterates, axis=0)
    for k in range(1, res.iters + 1):
        D = steps[:k].T  # directions p_0 .. p_{k-1}, up to scale
        gal = D @ np.linalg.solve(D.T @ Ad @ D, D.T @ b)
        assert np.linalg.norm(res.iterates[k] - gal) <= 1e-9 * np.linalg.norm(gal), k
    # steps at roundoff level (the last ones, as a difference of iterates) carry
    # no conjugacy information
    big = [k for k in range(res.iters) if np.linalg.norm(steps[k]) > 1e-6 * np.linalg.norm(xs)]
    assert len(big) >= 8
    for i in big:
        for j in big:
            if j < i:
                assert conjugacy_defect(Ad, steps[i], steps[j]) <= 1e-8, (i, j)


@pytest.mark.parametrize("m", [1, 2, 4])
def test_truncated_fcg_window_conjugacy_and_energy(orc, m):
    A, b = dirichlet_problem(orc, 1, (4, 3, 3), 44)
    Ad = A.to_dense()
    xs = np.linalg.solve(Ad, b)
    res = orc.fcg(A, b, varying_jacobi(A.diag(), 80), m, rtol=0.0, maxit=20, record=True)
    assert res.iters == 20
    steps = np.diff(res.iterates, axis=0)
    for i in range(len(steps)):
        for j in range(max(0, i - m), i):
            assert conjugacy_defect(Ad, steps[i], steps[j]) <= 1e-9, (m, i, j)
    err = [energy(Ad, xs - x) for x in res.iterates]
    assert all(err[k + 1] < err[k] for k in range(len(err) - 1))
    if m == 1:
        # beyond the window the directions are not conjugate: the truncation is real
        assert max(conjugacy_defect(Ad, steps[i], steps[i - 2]) for i in range(2, 20)) > 1e-3


@pytest.mark.parametrize("m", [2, 8])
def test_fcg_fixed_preconditioner_equals_pcg(orc, m):
    A, b = dirichlet_problem(orc, 1, (4, 3, 3), 45)
    d = A.diag()
    ref = orc.pcg(A, b, rtol=0.0, maxit=20)
    got = orc.fcg(A, b, lambda r: r / d, m, rtol=0.0, maxit=20)
    assert ref.iters == got.iters == 20
    assert np.linalg.norm(got.x - ref.x) <= 1e-10 * np.linalg.norm(ref.x)


def test_fcg_edge_cases(orc):
    A, b = dirichlet_problem(orc, 1, (2, 2, 2), 46)
    res = orc.fcg(A, np.zeros_like(b), lambda r: r, 3, rtol=1e-8, maxit=10)
    assert res.status == 0 and res.iters == 0 and np.all(res.x == 0)
    res = orc.fcg(A, b, lambda r: r * np.nan, 3, rtol=1e-8, maxit=10)
    assert res.status == -5
    # negative definite operator: breakdown at the first p^T A p
    A.val = -A.val
    res = orc.fcg(A, b, lambda r: r, 2, rtol=1e-8, maxit=10)
    assert res.status == -5
