"""Pins of the oracle's tricubic (Q3) hexahedron operators (the higher-order
elements of the paper's conclusions, Section 7) against facts fixed by the
mathematics:

* the textbook 1-D mass and stiffness matrices of the cubic Lagrange element
  (equispaced nodes), from exact polynomial integrals;
* the tricubic box element matrices as Kronecker products of those exact 1-D
  integrals (numpy polynomial algebra, independent of the oracle's quadrature
  and Jacobian code), axis-aligned and rotated, Laplace and elasticity;
* constant and rigid-body null spaces, linear patch tests and the energy
  identity on jittered (trilinear-geometry) meshes, a cubic patch test with
  Simpson's 3/8 weights on an undistorted box, symmetry, definiteness and a
  dense solve, and the element-by-element rows equal to the assembled ones.
"""
import numpy as np
import pytest
from numpy.polynomial import polynomial as P

import seeded_inputs as si

from test_oracle_elements import lattice_interior
from test_oracle_pins import abs_bound, hex_volume_divergence, rigid_modes, rotation

# cubic Lagrange polynomials on [0, 1] with nodes 0, 1/3, 2/3, 1 (coefficients,
# lowest degree first), built as products of the node factors
_NODES = [0.0, 1.0 / 3.0, 2.0 / 3.0, 1.0]


def _lagrange(i):
    c = np.array([1.0])
    for m, t in enumerate(_NODES):
        if m != i:
            c = P.polymul(c, np.array([-t, 1.0]) / (_NODES[i] - t))
    return c


LC = [_lagrange(i) for i in range(4)]


def _int01(c):
    ci = P.polyint(c)
    return P.polyval(1.0, ci) - P.polyval(0.0, ci)


def q3_1d(h):
    """Exact 1-D matrices on an interval of length h: mass M, stiffness S and the
    mixed E_ij = int phi_i' phi_j."""
    D = [P.polyder(c) for c in LC]
    M = np.array([[h * _int01(P.polymul(a, b)) for b in LC] for a in LC])
    S = np.array([[_int01(P.polymul(a, b)) / h for b in D] for a in D])
    E = np.array([[_int01(P.polymul(a, b)) for b in LC] for a in D])
    return M, S, E


def kron3(fx, fy, fz):  # local node a = i + 4j + 16k: x index fastest
    return np.kron(fz, np.kron(fy, fx))


def q3_box_nodes(hx, hy, hz, R=None, shift=(0.0, 0.0, 0.0)):
    X = np.array([[(a % 4) * hx / 3, ((a // 4) % 4) * hy / 3, (a // 16) * hz / 3]
                  for a in range(64)])
    if R is not None:
        X = X @ R.T
    return X + np.asarray(shift)


def test_q3_1d_matrices_textbook():
    M, S, _ = q3_1d(1.0)
    Mt = np.array([[128, 99, -36, 19], [99, 648, -81, -36], [-36, -81, 648, 99],
                   [19, -36, 99, 128]]) / 1680
    St = np.array([[148, -189, 54, -13], [-189, 432, -297, 54], [54, -297, 432, -189],
                   [-13, 54, -189, 148]]) / 40
    assert np.allclose(M, Mt, atol=1e-15)
    assert np.allclose(S, St, atol=1e-13)


@pytest.mark.parametrize("rot", [False, True])
def test_q3_laplace_box_closed_form(orc, rot):
    h, k = (0.7, 1.3, 2.1), 0.37
    R = rotation() if rot else None
    Ke = orc.ke_q3(1, q3_box_nodes(*h, R, (5.0, -2.0, 1.0)), k)
    (Mx, Sx, _), (My, Sy, _), (Mz, Sz, _) = (q3_1d(v) for v in h)
    ref = k * (kron3(Sx, My, Mz) + kron3(Mx, Sy, Mz) + kron3(Mx, My, Sz))
    assert np.max(np.abs(Ke - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("rot", [False, True])
def test_q3_elasticity_box_closed_form(orc, rot):
    h, lam, mu = (0.9, 1.4, 0.6), 2.7, 0.8
    R = rotation(7) if rot else np.eye(3)
    Ke = orc.ke_q3(3, q3_box_nodes(*h, R if rot else None), lam, mu)
    one = [q3_1d(v) for v in h]

    def D(a, b):  # int d_a phi_i d_b phi_j, a product of 1-D factors
        fs = []
        for d in range(3):
            M, S, E = one[d]
            fs.append(S if a == d and b == d else E if a == d else E.T if b == d else M)
        return kron3(*fs)

    Dm = [[D(a, b) for b in range(3)] for a in range(3)]
    lap = Dm[0][0] + Dm[1][1] + Dm[2][2]
    ref = np.zeros((192, 192))
    for i in range(3):
        for j in range(3):
            ref[i::3, j::3] = lam * Dm[i][j] + mu * ((lap if i == j else 0.0) + Dm[j][i])
    if rot:
        T = np.kron(np.eye(64), R)
        ref = T @ ref @ T.T
    assert np.max(np.abs(Ke - ref)) < 1e-12 * np.max(np.abs(ref))


def _q3_problem(physics, n, seed, jitter=0.1, h=1.0, const=None):
    xyz, conn = si.q3_box_mesh(*n, h, jitter, seed)
    ne = conn.shape[1]
    if physics == 1:
        coef = (np.full((1, ne), const) if const is not None
                else si.field_lognormal(ne, 0.0, 1.0, seed)[None])
    else:
        coef = (np.stack([np.full(ne, const[0]), np.full(ne, const[1])]) if const is not None
                else np.stack(si.lame_from_E_nu(*si.field_elastic(ne, seed))))
    return xyz, conn, coef


def test_q3_mesh_layout():
    """Element vertices are box_mesh's nodes; the other nodes interpolate them."""
    n = (2, 3, 1)
    xyz, conn = si.q3_box_mesh(*n, 1.0, 0.1, 5)
    vxyz, vconn = si.box_mesh(*n, 1.0, 0.1, 5)
    corners = [0, 3, 12, 15, 48, 51, 60, 63]  # the vertices in the trilinear order
    for e in range(conn.shape[1]):
        assert np.array_equal(xyz[:, conn[corners, e]], vxyz[:, vconn[:, e]])
    assert xyz.shape[1] == si.q3_box_sizes(*n)[0] == 7 * 10 * 4


def test_q3_null_spaces(orc):
    xyz, conn, coef = _q3_problem(1, (2, 2, 2), 41)
    A = orc.assemble(1, xyz, conn, coef)
    one = np.ones(A.n)
    assert np.max(np.abs(A.matvec(one))) <= abs_bound(A, one)
    xyz, conn, coef = _q3_problem(3, (2, 1, 2), 42)
    A = orc.assemble(3, xyz, conn, coef)
    for u in rigid_modes(xyz):
        assert np.max(np.abs(A.matvec(u))) <= abs_bound(A, u)


def test_q3_linear_patch_and_energy(orc):
    """On the jittered (trilinear-geometry) mesh the 4x4x4 rule integrates the
    linear-field residual and the energy exactly."""
    n = (2, 2, 3)
    xyz, conn, coef = _q3_problem(1, n, 43, const=2.5)
    A = orc.assemble(1, xyz, conn, coef)
    a = np.array([0.3, -1.1, 0.7])
    u = a @ xyz + 0.4
    r = A.matvec(u)[lattice_interior(n, 3)]
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(A.val)) * np.max(np.abs(u))
    _, conn, coef = _q3_problem(1, n, 43)
    A = orc.assemble(1, xyz, conn, coef)
    corners = [0, 3, 12, 15, 48, 51, 60, 63]
    vols = np.array([hex_volume_divergence(xyz[:, conn[corners, e]].T)
                     for e in range(conn.shape[1])])
    ul = a @ xyz
    ref = (a @ a) * np.sum(coef[0] * vols)
    assert abs(ul @ A.matvec(ul) - ref) < 1e-12 * ref
    lam, mu = 1.7, 0.6
    xyz, conn, coef = _q3_problem(3, n, 44, const=(lam, mu))
    A = orc.assemble(3, xyz, conn, coef)
    B = np.array([[0.2, -0.5, 0.1], [0.4, 0.3, -0.2], [-0.6, 0.05, 0.9]])
    u = (B @ xyz).T + np.array([0.1, 0.2, -0.3])
    r = A.matvec(u.ravel()).reshape(-1, 3)[lattice_interior(n, 3)]
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(A.val)) * np.max(np.abs(u))


def test_q3_cubic_patch(orc):
    """u = x^3 - 3 x y^2 + x^2 + 2 y^2 - z^2 + yz (Laplacian 4) on an undistorted
    box: at an interior node, (A u)_i = -4 k int phi_i, the integral a product of
    the 1-D weights of Simpson's 3/8 rule, 3h/8 at an interval's inner nodes and
    2 h/8 at a vertex shared by two intervals."""
    n, h, k = (2, 3, 2), 0.7, 1.9
    xyz, conn, coef = _q3_problem(1, n, 45, jitter=0.0, h=h, const=k)
    A = orc.assemble(1, xyz, conn, coef)
    x, y, z = xyz
    u = x ** 3 - 3 * x * y ** 2 + x ** 2 + 2 * y ** 2 - z ** 2 + y * z
    r = A.matvec(u)
    N = [3 * m + 1 for m in n]
    for nid in lattice_interior(n, 3):
        I, J, K = nid % N[0], (nid // N[0]) % N[1], nid // (N[0] * N[1])
        w = np.prod([h / 4 if c % 3 == 0 else 3 * h / 8 for c in (I, J, K)])
        assert abs(r[nid] - (-4.0 * k * w)) < 1e-12 * np.max(np.abs(A.val)) * np.max(np.abs(u))


@pytest.mark.parametrize("physics", [1, 3])
def test_q3_symmetry_definiteness_dense_solve(orc, physics):
    xyz, conn, coef = _q3_problem(physics, (2, 1, 1), 46)
    mask = si.q3_face_mask(2, 1, 1, "z0")
    A = orc.assemble(physics, xyz, conn, coef, mask)
    Ad = A.to_dense()
    assert np.max(np.abs(Ad - Ad.T)) < 1e-13 * np.max(np.abs(Ad))
    assert np.linalg.eigvalsh(Ad).min() > 0
    b = si.vec_uniform(A.n, 46, si.STREAM_RHS)
    b[si.dof_mask(mask, 1 if physics == 1 else 3) == 1] = 0.0
    res = orc.pcg(A, b, rtol=1e-13, maxit=20 * A.n)
    xs = np.linalg.solve(Ad, b)
    assert res.status == 0 and np.linalg.norm(res.x - xs) <= 1e-8 * np.linalg.norm(xs)


@pytest.mark.parametrize("physics", [1, 3])
def test_q3_apply_rows_equals_assembled_rows(orc, physics):
    xyz, conn, coef = _q3_problem(physics, (2, 1, 2), 47)
    mask = si.q3_face_mask(2, 1, 2, "z0")
    A = orc.assemble(physics, xyz, conn, coef, mask)
    x = si.vec_uniform(A.n, 47, si.STREAM_X)
    y = orc.apply_rows(physics, xyz, conn, coef, mask, x, np.arange(A.n))
    assert np.max(np.abs(y - A.matvec(x))) <= 1e-13 * np.max(np.abs(y))
