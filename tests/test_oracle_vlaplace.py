"""Pins of the oracle's vector Laplace operator (Section 2, the vector Laplace
element matrix: the double contraction of e_k (x) grad phi_i with
e_l (x) grad phi_j, times the cell coefficient).  Each check is a fact of the
continuous operator or an independent closed form: the element matrix of a
rotated box from exact 1-D integrals, the three constant null vectors, exact
reproduction of linear fields, the energy of a linear field with volumes from
the divergence theorem, symmetry and definiteness, and a dense solve."""
import numpy as np
import pytest

import seeded_inputs as si
from test_oracle_pins import (abs_bound, box_nodes, hex_volume_divergence, interior_nodes,
                              laplace_box_closed_form, rotation)


@pytest.mark.parametrize("rot", [False, True])
def test_vlaplace_box_closed_form(orc, rot):
    # components do not couple: K[3a+i, 3b+j] = delta_ij * (scalar box matrix)[a, b],
    # and the scalar Laplacian does not see a rotation of the box
    hx, hy, hz, k = 0.8, 1.6, 0.45, 2.3
    Ke = orc.ke_vlaplace(box_nodes(hx, hy, hz, rotation(5) if rot else None, (1.0, 2.0, -3.0)), k)
    ref = np.kron(laplace_box_closed_form(hx, hy, hz, k), np.eye(3))
    assert np.max(np.abs(Ke - ref)) < 1e-13 * np.max(np.abs(ref))


def test_vlaplace_constant_nullspace(orc):
    xyz, conn = si.box_mesh(3, 2, 4, 1.0, 0.1, 41)
    k = si.field_lognormal(24, 0.0, 1.0, 41)
    A = orc.assemble(2, xyz, conn, k[None])
    for c in range(3):
        u = np.zeros((xyz.shape[1], 3))
        u[:, c] = 1.0
        u = u.ravel()
        assert np.max(np.abs(A.matvec(u))) <= abs_bound(A, u)
    # a rotation field is not in the null space (unlike elasticity)
    w = np.cross(np.broadcast_to([0.0, 0.0, 1.0], (xyz.shape[1], 3)), xyz.T).ravel()
    assert np.linalg.norm(A.matvec(w)) > 1e-3


def test_vlaplace_patch(orc):
    n = (3, 4, 3)
    xyz, conn = si.box_mesh(*n, 1.0, 0.1, 42)
    A = orc.assemble(2, xyz, conn, np.full((1, int(np.prod(n))), 1.9))
    B = np.array([[0.3, -0.2, 0.5], [-0.7, 0.1, 0.4], [0.2, 0.9, -0.3]])
    u = (B @ xyz).T + np.array([0.5, -0.1, 0.2])
    r = A.matvec(u.ravel()).reshape(-1, 3)[interior_nodes(n)]
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(A.val)) * np.max(np.abs(u))


def test_vlaplace_energy(orc):
    # u = B x: u^T A u = |B|_F^2 sum_e k_e |Omega_e|
    n = (2, 3, 3)
    xyz, conn = si.box_mesh(*n, 1.0, 0.1, 43)
    ne = int(np.prod(n))
    k = si.field_lognormal(ne, 0.0, 1.0, 43)
    A = orc.assemble(2, xyz, conn, k[None])
    vols = np.array([hex_volume_divergence(xyz[:, conn[:, e]].T) for e in range(ne)])
    B = np.array([[0.3, -0.2, 0.5], [-0.7, 0.1, 0.4], [0.2, 0.9, -0.3]])
    u = (B @ xyz).T.ravel()
    ref = np.sum(B * B) * np.dot(k, vols)
    assert abs(u @ A.matvec(u) - ref) < 1e-12 * ref


def test_vlaplace_symmetry_definiteness_and_solve(orc):
    n = (2, 3, 2)
    xyz, conn = si.box_mesh(*n, 1.0, 0.1, 44)
    k = si.field_lognormal(12, 0.0, 1.0, 44)[None]
    A = orc.assemble(2, xyz, conn, k).to_dense()
    assert np.max(np.abs(A - A.T)) < 1e-14 * np.max(np.abs(A))
    ev = np.linalg.eigvalsh(A)
    assert np.all(np.abs(ev[:3]) < 1e-12 * ev[-1]) and np.all(ev[3:] > 1e-8 * ev[-1])
    mask = si.face_mask(*n, "z0")
    Ad = orc.assemble(2, xyz, conn, k, mask)
    D = Ad.to_dense()
    assert np.linalg.eigvalsh(D)[0] > 0.0
    fixed = np.nonzero(si.dof_mask(mask, 3))[0]
    assert np.all(D[fixed][:, fixed] == np.eye(len(fixed)))
    b = si.vec_uniform(Ad.n, 44, si.STREAM_RHS)
    b[fixed] = 0.0
    xs = np.linalg.solve(D, b)
    res = orc.pcg(Ad, b, rtol=1e-13, maxit=10 * Ad.n)
    assert res.status == 0
    assert np.linalg.norm(res.x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_vlaplace_apply_rows_equals_assembled_rows(orc):
    n = (2, 3, 2)
    xyz, conn = si.box_mesh(*n, 1.0, 0.1, 45)
    k = si.field_lognormal(12, 0.0, 1.0, 45)[None]
    mask = si.face_mask(*n, "z0")
    A = orc.assemble(2, xyz, conn, k, mask)
    x = si.vec_uniform(A.n, 45, si.STREAM_X)
    rows = np.arange(A.n)
    y = orc.apply_rows(2, xyz, conn, k, mask, x, rows)
    assert np.max(np.abs(y - A.matvec(x))) < 1e-13 * np.max(np.abs(y))
