"""Pins of the oracle's linear-tetrahedron and triquadratic-hexahedron operators
(the simplicial and quadratic elements of the paper's conclusions, Section 7)
against facts fixed by the mathematics:

* the reference tetrahedron's Laplace matrix and the 7-point stencil that the
  Kuhn split of a uniform grid assembles to;
* the triquadratic box element matrices as Kronecker products of exact 1-D
  integrals of the quadratic Lagrange polynomials (numpy polynomial algebra,
  independent of the oracle's quadrature and Jacobian code), axis-aligned and
  rotated;
* constant and rigid-body null spaces, linear patch tests and the energy
  identity on jittered meshes, a quadratic patch test for the triquadratic
  element, symmetry, definiteness and a dense solve.
"""
import numpy as np
import pytest
from numpy.polynomial import polynomial as P

import seeded_inputs as si

from test_oracle_pins import abs_bound, hex_volume_divergence, rigid_modes, rotation


def lattice_interior(n, step=1):
    """Node ids of the interior lattice points of an (n*step)^3-node-interval box."""
    N = [m * step for m in n]
    ids = []
    for k in range(1, N[2]):
        for j in range(1, N[1]):
            for i in range(1, N[0]):
                ids.append(i + (N[0] + 1) * (j + (N[1] + 1) * k))
    return np.array(ids)


# -- linear tetrahedra ------------------------------------------------------------

def test_tet_reference_laplace(orc):
    X = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    ref = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]]) / 6.0
    assert np.max(np.abs(orc.ke_tet(1, X, 1.0) - ref)) < 1e-15
    # scaled by s, rotated and moved: the Laplace matrix scales by s, k enters linearly
    R, s, k = rotation(5), 1.7, 0.3
    Y = s * X @ R.T + np.array([2.0, -1.0, 0.5])
    assert np.max(np.abs(orc.ke_tet(1, Y, k) - k * s * ref)) < 1e-14


def test_tet_kuhn_split_seven_point_stencil(orc):
    n, h, kc = 4, 2.0, 3.0
    xyz, conn = si.tet_mesh(n, n, n, h, 0.0, 1)
    A = orc.assemble(1, xyz, conn, np.full((1, conn.shape[1]), kc)).to_dense()
    for (i, j, k) in [(1, 1, 1), (2, 1, 3), (2, 2, 2)]:
        nid = i + (n + 1) * (j + (n + 1) * k)
        expect = np.zeros(A.shape[0])
        expect[nid] = 6.0 * kc * h
        for d in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
            for sgn in (-1, 1):
                m = (i + sgn * d[0]) + (n + 1) * ((j + sgn * d[1]) + (n + 1) * (k + sgn * d[2]))
                expect[m] = -kc * h
        assert np.max(np.abs(A[nid] - expect)) < 1e-13 * kc * h


def _tet_problem(physics, n, seed, jitter=0.1, const=None):
    xyz, conn = si.tet_mesh(*n, 1.0, jitter, seed)
    ne = conn.shape[1]
    if physics == 1:
        coef = (np.full((1, ne), const) if const is not None
                else si.field_lognormal(ne, 0.0, 1.0, seed)[None])
    else:
        coef = (np.stack([np.full(ne, const[0]), np.full(ne, const[1])]) if const is not None
                else np.stack(si.lame_from_E_nu(*si.field_elastic(ne, seed))))
    return xyz, conn, coef


def test_tet_null_spaces(orc):
    xyz, conn, coef = _tet_problem(1, (3, 4, 2), 21)
    A = orc.assemble(1, xyz, conn, coef)
    one = np.ones(A.n)
    assert np.max(np.abs(A.matvec(one))) <= abs_bound(A, one)
    xyz, conn, coef = _tet_problem(3, (3, 2, 3), 22)
    A = orc.assemble(3, xyz, conn, coef)
    for u in rigid_modes(xyz):
        assert np.max(np.abs(A.matvec(u))) <= abs_bound(A, u)
    u = np.random.default_rng(0).standard_normal(A.n)
    assert np.linalg.norm(A.matvec(u)) > 1e-3


def test_tet_patch_and_energy(orc):
    n = (4, 3, 3)
    V = float(np.prod(n))  # the jitter keeps the box
    xyz, conn, coef = _tet_problem(1, n, 23, const=2.5)
    A = orc.assemble(1, xyz, conn, coef)
    a = np.array([0.3, -1.1, 0.7])
    u = a @ xyz + 0.4
    r = A.matvec(u)[lattice_interior(n)]
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(A.val)) * np.max(np.abs(u))
    ul = a @ xyz
    assert abs(ul @ A.matvec(ul) - 2.5 * (a @ a) * V) < 1e-12 * 2.5 * (a @ a) * V
    lam, mu = 1.7, 0.6
    xyz, conn, coef = _tet_problem(3, n, 24, const=(lam, mu))
    A = orc.assemble(3, xyz, conn, coef)
    B = np.array([[0.2, -0.5, 0.1], [0.4, 0.3, -0.2], [-0.6, 0.05, 0.9]])
    u = (B @ xyz).T + np.array([0.1, 0.2, -0.3])
    r = A.matvec(u.ravel()).reshape(-1, 3)[lattice_interior(n)]
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(A.val)) * np.max(np.abs(u))
    ul = (B @ xyz).T.ravel()
    eps = 0.5 * (B + B.T)
    energy = V * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))
    assert abs(ul @ A.matvec(ul) - energy) < 1e-12 * energy


@pytest.mark.parametrize("physics", [1, 3])
def test_tet_symmetry_definiteness_dense_solve(orc, physics):
    xyz, conn, coef = _tet_problem(physics, (2, 2, 2), 25)
    mask = si.face_mask(2, 2, 2, "z0")
    A = orc.assemble(physics, xyz, conn, coef, mask)
    Ad = A.to_dense()
    assert np.max(np.abs(Ad - Ad.T)) < 1e-14 * np.max(np.abs(Ad))
    assert np.linalg.eigvalsh(Ad).min() > 0
    b = si.vec_uniform(A.n, 25, si.STREAM_RHS)
    b[si.dof_mask(mask, 1 if physics == 1 else 3) == 1] = 0.0
    res = orc.pcg(A, b, rtol=1e-13, maxit=10 * A.n)
    xs = np.linalg.solve(Ad, b)
    assert res.status == 0 and np.linalg.norm(res.x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_tet_inverted_rejected(orc):
    X = np.array([[0.0, 0, 0], [0, 1, 0], [1, 0, 0], [0, 0, 1]])  # negative orientation
    with pytest.raises(ValueError):
        orc.ke_tet(1, X, 1.0)


# -- triquadratic hexahedra ---------------------------------------------------------

# quadratic Lagrange polynomials on [0, 1] with nodes 0, 1/2, 1 (coefficients in t)
LQ = [np.array([1.0, -3.0, 2.0]), np.array([0.0, 4.0, -4.0]), np.array([0.0, -1.0, 2.0])]


def _int01(c):
    ci = P.polyint(c)
    return P.polyval(1.0, ci) - P.polyval(0.0, ci)


def q2_1d(h):
    """Exact 1-D matrices on an interval of length h: mass M, stiffness S and the
    mixed E_ij = int phi_i' phi_j (independent of h)."""
    D = [P.polyder(c) for c in LQ]
    M = np.array([[h * _int01(P.polymul(a, b)) for b in LQ] for a in LQ])
    S = np.array([[_int01(P.polymul(a, b)) / h for b in D] for a in D])
    E = np.array([[_int01(P.polymul(a, b)) for b in LQ] for a in D])
    return M, S, E


def kron3(fx, fy, fz):  # local node a = i + 3j + 9k: x index fastest
    return np.kron(fz, np.kron(fy, fx))


def q2_box_nodes(hx, hy, hz, R=None, shift=(0.0, 0.0, 0.0)):
    X = np.array([[(a % 3) * hx / 2, ((a // 3) % 3) * hy / 2, (a // 9) * hz / 2]
                  for a in range(27)])
    if R is not None:
        X = X @ R.T
    return X + np.asarray(shift)


def test_q2_1d_matrices_textbook():
    M, S, _ = q2_1d(1.0)
    assert np.allclose(M, np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) / 30, atol=1e-15)
    assert np.allclose(S, np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 3, atol=1e-14)


@pytest.mark.parametrize("rot", [False, True])
def test_q2_laplace_box_closed_form(orc, rot):
    h, k = (0.7, 1.3, 2.1), 0.37
    R = rotation() if rot else None
    Ke = orc.ke_q2(1, q2_box_nodes(*h, R, (5.0, -2.0, 1.0)), k)
    (Mx, Sx, _), (My, Sy, _), (Mz, Sz, _) = (q2_1d(v) for v in h)
    ref = k * (kron3(Sx, My, Mz) + kron3(Mx, Sy, Mz) + kron3(Mx, My, Sz))
    assert np.max(np.abs(Ke - ref)) < 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("rot", [False, True])
def test_q2_elasticity_box_closed_form(orc, rot):
    h, lam, mu = (0.9, 1.4, 0.6), 2.7, 0.8
    R = rotation(7) if rot else np.eye(3)
    Ke = orc.ke_q2(3, q2_box_nodes(*h, R if rot else None), lam, mu)
    one = [q2_1d(v) for v in h]

    def D(a, b):  # int d_a phi_i d_b phi_j, a product of 1-D factors
        fs = []
        for d in range(3):
            M, S, E = one[d]
            fs.append(S if a == d and b == d else E if a == d else E.T if b == d else M)
        return kron3(*fs)

    Dm = [[D(a, b) for b in range(3)] for a in range(3)]
    lap = Dm[0][0] + Dm[1][1] + Dm[2][2]
    ref = np.zeros((81, 81))
    for i in range(3):
        for j in range(3):
            ref[i::3, j::3] = lam * Dm[i][j] + mu * ((lap if i == j else 0.0) + Dm[j][i])
    if rot:
        T = np.kron(np.eye(27), R)
        ref = T @ ref @ T.T
    assert np.max(np.abs(Ke - ref)) < 1e-13 * np.max(np.abs(ref))


def _q2_problem(physics, n, seed, jitter=0.1, h=1.0, const=None):
    xyz, conn = si.q2_box_mesh(*n, h, jitter, seed)
    ne = conn.shape[1]
    if physics == 1:
        coef = (np.full((1, ne), const) if const is not None
                else si.field_lognormal(ne, 0.0, 1.0, seed)[None])
    else:
        coef = (np.stack([np.full(ne, const[0]), np.full(ne, const[1])]) if const is not None
                else np.stack(si.lame_from_E_nu(*si.field_elastic(ne, seed))))
    return xyz, conn, coef


def test_q2_null_spaces(orc):
    xyz, conn, coef = _q2_problem(1, (3, 2, 2), 31)
    A = orc.assemble(1, xyz, conn, coef)
    one = np.ones(A.n)
    assert np.max(np.abs(A.matvec(one))) <= abs_bound(A, one)
    xyz, conn, coef = _q2_problem(3, (2, 2, 2), 32)
    A = orc.assemble(3, xyz, conn, coef)
    for u in rigid_modes(xyz):
        assert np.max(np.abs(A.matvec(u))) <= abs_bound(A, u)


def test_q2_linear_patch_and_energy(orc):
    """On the jittered (trilinear-geometry) mesh the 3x3x3 rule integrates the
    linear-field residual and the energy exactly."""
    n = (3, 2, 3)
    xyz, conn, coef = _q2_problem(1, n, 33, const=2.5)
    A = orc.assemble(1, xyz, conn, coef)
    a = np.array([0.3, -1.1, 0.7])
    u = a @ xyz + 0.4
    r = A.matvec(u)[lattice_interior(n, 2)]
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(A.val)) * np.max(np.abs(u))
    # heterogeneous k: u = a.x has energy |a|^2 sum_e k_e |Omega_e|, volumes from the
    # element vertices by the divergence theorem
    _, conn, coef = _q2_problem(1, n, 33)
    A = orc.assemble(1, xyz, conn, coef)
    corners = [0, 2, 6, 8, 18, 20, 24, 26]  # the vertices in the trilinear order
    vols = np.array([hex_volume_divergence(xyz[:, conn[corners, e]].T)
                     for e in range(conn.shape[1])])
    ul = a @ xyz
    ref = (a @ a) * np.sum(coef[0] * vols)
    assert abs(ul @ A.matvec(ul) - ref) < 1e-12 * ref
    lam, mu = 1.7, 0.6
    xyz, conn, coef = _q2_problem(3, n, 34, const=(lam, mu))
    A = orc.assemble(3, xyz, conn, coef)
    B = np.array([[0.2, -0.5, 0.1], [0.4, 0.3, -0.2], [-0.6, 0.05, 0.9]])
    u = (B @ xyz).T + np.array([0.1, 0.2, -0.3])
    r = A.matvec(u.ravel()).reshape(-1, 3)[lattice_interior(n, 2)]
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(A.val)) * np.max(np.abs(u))


def test_q2_quadratic_patch(orc):
    """u = x^2 + 2 y^2 - z^2 + xy (so -Laplace u = -4) on an undistorted box: at an
    interior node, (A u)_i = -4 k int phi_i, the integral a product of the 1-D
    Simpson weights h/6, 2h/3 (and h/3 at a vertex shared by two intervals)."""
    n, h, k = (3, 3, 2), 0.7, 1.9
    xyz, conn, coef = _q2_problem(1, n, 35, jitter=0.0, h=h, const=k)
    A = orc.assemble(1, xyz, conn, coef)
    x, y, z = xyz
    u = x ** 2 + 2 * y ** 2 - z ** 2 + x * y
    r = A.matvec(u)
    N = [2 * m + 1 for m in n]
    for nid in lattice_interior(n, 2):
        I, J, K = nid % N[0], (nid // N[0]) % N[1], nid // (N[0] * N[1])
        w = np.prod([h / 3 if c % 2 == 0 else 2 * h / 3 for c in (I, J, K)])
        assert abs(r[nid] - (-4.0 * k * w)) < 1e-12 * np.max(np.abs(A.val)) * np.max(np.abs(u))


@pytest.mark.parametrize("physics", [1, 3])
def test_q2_symmetry_definiteness_dense_solve(orc, physics):
    xyz, conn, coef = _q2_problem(physics, (2, 1, 2), 36)
    mask = si.q2_face_mask(2, 1, 2, "z0")
    A = orc.assemble(physics, xyz, conn, coef, mask)
    Ad = A.to_dense()
    assert np.max(np.abs(Ad - Ad.T)) < 1e-13 * np.max(np.abs(Ad))
    assert np.linalg.eigvalsh(Ad).min() > 0
    b = si.vec_uniform(A.n, 36, si.STREAM_RHS)
    b[si.dof_mask(mask, 1 if physics == 1 else 3) == 1] = 0.0
    res = orc.pcg(A, b, rtol=1e-13, maxit=20 * A.n)
    xs = np.linalg.solve(Ad, b)
    assert res.status == 0 and np.linalg.norm(res.x - xs) <= 1e-8 * np.linalg.norm(xs)


@pytest.mark.parametrize("physics,nloc", [(1, 4), (3, 4), (1, 27), (3, 27)])
def test_apply_rows_equals_assembled_rows(orc, physics, nloc):
    if nloc == 4:
        xyz, conn, coef = _tet_problem(physics, (2, 3, 2), 37)
        mask = si.face_mask(2, 3, 2, "z0")
    else:
        xyz, conn, coef = _q2_problem(physics, (2, 2, 1), 37)
        mask = si.q2_face_mask(2, 2, 1, "z0")
    A = orc.assemble(physics, xyz, conn, coef, mask)
    x = si.vec_uniform(A.n, 37, si.STREAM_X)
    y = orc.apply_rows(physics, xyz, conn, coef, mask, x, np.arange(A.n))
    assert np.max(np.abs(y - A.matvec(x))) <= 1e-13 * np.max(np.abs(y))
