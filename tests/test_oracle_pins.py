"""Pins of the CPU oracle against facts fixed by the paper and the mathematics.

Each test checks the oracle against something other than its own code: a
closed form derived from exact 1-D integrals, an invariant of the continuous
operator (null spaces, linear-field reproduction, energy), a divergence-theorem
volume, or a dense library solve.  A dropped term, a sign error, a transposed
Jacobian or a wrong index in the oracle fails at least one of them.
"""
import numpy as np
import pytest

import seeded_inputs as si

S = np.array([[1.0, -1.0], [-1.0, 1.0]])
M = np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0
# int phi_i' phi_j dx on one 1-D linear element (independent of length)
E = np.array([[-0.5, -0.5], [0.5, 0.5]])


def kron3(fx, fy, fz):
    # local node a = i + 2j + 4k: x index fastest
    return np.kron(fz, np.kron(fy, fx))


def box_nodes(hx, hy, hz, R=None, shift=(0.0, 0.0, 0.0)):
    X = np.array([[(a & 1) * hx, ((a >> 1) & 1) * hy, ((a >> 2) & 1) * hz] for a in range(8)])
    if R is not None:
        X = X @ R.T
    return X + np.asarray(shift)


def rotation(seed=3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


# -- P1: closed-form Laplace element matrix of a (rotated) rectangular box --

def laplace_box_closed_form(hx, hy, hz, k):
    return k * (hy * hz / hx * kron3(S, M, M) + hx * hz / hy * kron3(M, S, M)
                + hx * hy / hz * kron3(M, M, S))


def test_p1_unit_cube_entries(orc):
    # side h cube: entries k h {1/3, 0, -1/12, -1/12} by Hamming distance 0..3
    h, k = 2.0, 3.0
    Ke = orc.ke_laplace(box_nodes(h, h, h), k)
    for a in range(8):
        for b in range(8):
            d = bin(a ^ b).count("1")
            expect = k * h * [1.0 / 3.0, 0.0, -1.0 / 12.0, -1.0 / 12.0][d]
            assert abs(Ke[a, b] - expect) < 1e-14 * k * h


@pytest.mark.parametrize("rot", [False, True])
def test_p1_box_closed_form(orc, rot):
    hx, hy, hz, k = 0.7, 1.3, 2.1, 0.37
    R = rotation() if rot else None
    Ke = orc.ke_laplace(box_nodes(hx, hy, hz, R, (5.0, -2.0, 1.0)), k)
    ref = laplace_box_closed_form(hx, hy, hz, k)
    assert np.max(np.abs(Ke - ref)) < 1e-13 * np.max(np.abs(ref))


# -- P2: closed-form elasticity element matrix of a (rotated) box ------------

def elasticity_box_closed_form(h, lam, mu):
    def D(a, b):
        # int d_a phi_i d_b phi_j over the box, product of 1-D factors
        fs = []
        for d in range(3):
            if a == d and b == d:
                fs.append(S / h[d])
            elif a == d:
                fs.append(E)
            elif b == d:
                fs.append(E.T)
            else:
                fs.append(h[d] * M)
        return kron3(*fs)
    Dm = [[D(a, b) for b in range(3)] for a in range(3)]
    K = np.zeros((24, 24))
    lap = Dm[0][0] + Dm[1][1] + Dm[2][2]
    for i in range(3):
        for j in range(3):
            blk = lam * Dm[i][j] + mu * ((lap if i == j else 0.0) + Dm[j][i])
            K[i::3, j::3] = blk
    return K


def rotate_elasticity(K, R):
    # K in rotated frame: T K T^T with T = blockdiag(R) over the 8 nodes
    T = np.kron(np.eye(8), R)
    return T @ K @ T.T


@pytest.mark.parametrize("rot", [False, True])
def test_p2_elasticity_closed_form(orc, rot):
    h = (0.9, 1.4, 0.6)
    lam, mu = 2.7, 0.8
    R = rotation(7) if rot else np.eye(3)
    Ke = orc.ke_elasticity(box_nodes(*h, R=R if rot else None), lam, mu)
    ref = elasticity_box_closed_form(h, lam, mu)
    if rot:
        ref = rotate_elasticity(ref, R)
    assert np.max(np.abs(Ke - ref)) < 1e-13 * np.max(np.abs(ref))


# -- P3: assembled 27-point stencil on a uniform grid -----------------------

def test_p3_assembled_stencil(orc):
    n, h, kc = 4, 2.0, 3.0
    xyz, conn = si.box_mesh(n, n, n, h, 0.0, 1)
    A = orc.assemble(1, xyz, conn, np.full((1, n ** 3), kc))
    Ad = A.to_dense()
    for (i, j, k) in [(1, 1, 1), (2, 1, 3), (2, 2, 2)]:
        nid = i + (n + 1) * (j + (n + 1) * k)
        row = Ad[nid]
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                for dk in (-1, 0, 1):
                    m = (i + di) + (n + 1) * ((j + dj) + (n + 1) * (k + dk))
                    d = abs(di) + abs(dj) + abs(dk)
                    expect = kc * h * [8.0 / 3.0, 0.0, -1.0 / 6.0, -1.0 / 12.0][d]
                    assert abs(row[m] - expect) < 1e-13 * kc * h
        assert np.count_nonzero(np.abs(row) > 1e-14) == 1 + 12 + 8
        assert abs(row.sum()) < 1e-13 * kc * h
    # 27-point pattern: nnz of the full grid is (3n+1)^3 for an n^3 box
    assert A.nnz == (3 * n + 1) ** 3


# -- P4: null spaces on jittered meshes with heterogeneous coefficients ------

def abs_bound(A, x):
    Aabs = A.to_scipy().copy()
    Aabs.data = np.abs(Aabs.data)
    return 64 * np.finfo(float).eps * np.max(Aabs @ np.abs(x))


def test_p4_laplace_constant_nullspace(orc):
    xyz, conn = si.box_mesh(3, 4, 2, 1.0, 0.1, 11)
    k = si.field_lognormal(24, 0.0, 1.0, 11)
    A = orc.assemble(1, xyz, conn, k[None])
    one = np.ones(A.n)
    assert np.max(np.abs(A.matvec(one))) <= abs_bound(A, one)


def rigid_modes(xyz):
    nn = xyz.shape[1]
    modes = []
    for c in range(3):
        u = np.zeros((nn, 3)); u[:, c] = 1.0
        modes.append(u.ravel())
    for w in np.eye(3):
        u = np.cross(np.broadcast_to(w, (nn, 3)), xyz.T)
        modes.append(u.ravel())
    return modes


def test_p4_elasticity_rigid_modes(orc):
    xyz, conn = si.box_mesh(3, 2, 3, 1.0, 0.1, 12)
    E, nu = si.field_elastic(18, 12)
    lam, mu = si.lame_from_E_nu(E, nu)
    A = orc.assemble(3, xyz, conn, np.stack([lam, mu]))
    for u in rigid_modes(xyz):
        assert np.max(np.abs(A.matvec(u))) <= abs_bound(A, u)
    # a non-rigid field is not in the null space
    u = np.random.default_rng(0).standard_normal(A.n)
    assert np.linalg.norm(A.matvec(u)) > 1e-3


# -- P5: linear patch tests on a jittered mesh ---------------------------------

def interior_nodes(n):
    idx = []
    for k in range(1, n[2]):
        for j in range(1, n[1]):
            for i in range(1, n[0]):
                idx.append(i + (n[0] + 1) * (j + (n[1] + 1) * k))
    return np.array(idx)


def test_p5_laplace_patch(orc):
    n = (4, 3, 3)
    xyz, conn = si.box_mesh(*n, 1.0, 0.1, 13)
    A = orc.assemble(1, xyz, conn, np.full((1, np.prod(n)), 2.5))
    a = np.array([0.3, -1.1, 0.7])
    u = a @ xyz + 0.4
    r = A.matvec(u)[interior_nodes(n)]
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(A.val)) * np.max(np.abs(u))


def test_p5_elasticity_patch(orc):
    n = (3, 3, 4)
    xyz, conn = si.box_mesh(*n, 1.0, 0.1, 14)
    ne = int(np.prod(n))
    A = orc.assemble(3, xyz, conn, np.stack([np.full(ne, 1.7), np.full(ne, 0.6)]))
    B = np.array([[0.2, -0.5, 0.1], [0.4, 0.3, -0.2], [-0.6, 0.05, 0.9]])
    u = (B @ xyz).T + np.array([0.1, 0.2, -0.3])
    r = A.matvec(u.ravel()).reshape(-1, 3)[interior_nodes(n)]
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(A.val)) * np.max(np.abs(u))


# -- P6: energy identity with volumes from the divergence theorem -------------

def hex_volume_divergence(X):
    """Volume of the trilinear hexahedron X[8,3] as (1/3) of the flux of x
    through its six bilinear faces; Simpson's 3x3 rule is exact for the
    biquadratic flux integrand."""
    sp = np.array([0.0, 0.5, 1.0]); sw = np.array([1.0, 4.0, 1.0]) / 6.0
    vol = 0.0
    # (fixed axis, value, param axes in right-handed order)
    for ax, (p1, p2) in ((0, (1, 2)), (1, (2, 0)), (2, (0, 1))):
        for val, sign in ((0, -1.0), (1, 1.0)):
            def node(c1, c2):
                idx = [0, 0, 0]
                idx[ax] = val; idx[p1] = c1; idx[p2] = c2
                return X[idx[0] + 2 * idx[1] + 4 * idx[2]]
            P00, P10, P01, P11 = node(0, 0), node(1, 0), node(0, 1), node(1, 1)
            for s, ws in zip(sp, sw):
                for t, wt in zip(sp, sw):
                    x = (1 - s) * (1 - t) * P00 + s * (1 - t) * P10 + (1 - s) * t * P01 + s * t * P11
                    xs = (1 - t) * (P10 - P00) + t * (P11 - P01)
                    xt = (1 - s) * (P01 - P00) + s * (P11 - P10)
                    vol += sign * ws * wt * np.dot(x, np.cross(xs, xt))
    return vol / 3.0


def test_divergence_volume_of_box():
    assert abs(hex_volume_divergence(box_nodes(0.7, 1.3, 2.1, rotation())) - 0.7 * 1.3 * 2.1) < 1e-14


def test_p6_laplace_energy(orc):
    n = (3, 3, 3)
    xyz, conn = si.box_mesh(*n, 1.0, 0.1, 15)
    k = si.field_lognormal(27, 0.0, 1.0, 15)
    A = orc.assemble(1, xyz, conn, k[None])
    vols = np.array([hex_volume_divergence(xyz[:, conn[:, e]].T) for e in range(27)])
    assert abs(vols.sum() - 27.0) < 1e-12  # jitter keeps the box
    a = np.array([0.8, -0.3, 1.9])
    u = a @ xyz
    assert abs(u @ A.matvec(u) - a @ a * np.dot(k, vols)) < 1e-12 * a @ a * np.dot(k, vols)


def test_p6_elasticity_energy(orc):
    n = (2, 3, 2)
    xyz, conn = si.box_mesh(*n, 1.0, 0.1, 16)
    E, nu = si.field_elastic(12, 16)
    lam, mu = si.lame_from_E_nu(E, nu)
    A = orc.assemble(3, xyz, conn, np.stack([lam, mu]))
    vols = np.array([hex_volume_divergence(xyz[:, conn[:, e]].T) for e in range(12)])
    B = np.array([[0.2, -0.5, 0.1], [0.4, 0.3, -0.2], [-0.6, 0.05, 0.9]])
    eps = 0.5 * (B + B.T)
    dens = lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps)
    u = (B @ xyz).T.ravel()
    ref = np.dot(dens, vols)
    assert abs(u @ A.matvec(u) - ref) < 1e-12 * ref


# -- P7: symmetry and definiteness ------------------------------------------

@pytest.mark.parametrize("physics", [1, 3])
def test_p7_symmetry_definiteness(orc, physics):
    n = (2, 2, 2)
    xyz, conn = si.box_mesh(*n, 1.0, 0.1, 17)
    if physics == 1:
        coef = si.field_lognormal(8, 0.0, 1.0, 17)[None]
    else:
        coef = np.stack(si.lame_from_E_nu(*si.field_elastic(8, 17)))
    A = orc.assemble(physics, xyz, conn, coef).to_dense()
    assert np.max(np.abs(A - A.T)) < 1e-14 * np.max(np.abs(A))
    ev = np.linalg.eigvalsh(A)
    nnull = 1 if physics == 1 else 6
    assert np.all(ev[nnull:] > 1e-8 * ev[-1])
    assert np.all(np.abs(ev[:nnull]) < 1e-12 * ev[-1])
    mask = si.face_mask(*n, "z0")
    Ad = orc.assemble(physics, xyz, conn, coef, mask).to_dense()
    assert np.max(np.abs(Ad - Ad.T)) < 1e-14 * np.max(np.abs(Ad))
    assert np.linalg.eigvalsh(Ad)[0] > 0.0
    fixed = np.nonzero(si.dof_mask(mask, physics))[0]
    assert np.all(Ad[fixed][:, fixed] == np.eye(len(fixed)))
    free = np.setdiff1d(np.arange(A.shape[0]), fixed)
    assert np.all(Ad[np.ix_(fixed, free)] == 0.0)
    assert np.allclose(Ad[np.ix_(free, free)], A[np.ix_(free, free)], rtol=0, atol=0)


# -- P8/P11/P12: solvers against dense solves -------------------------------

def dirichlet_problem(orc, physics, n, seed):
    xyz, conn = si.box_mesh(*n, 1.0, 0.1, seed)
    ne = int(np.prod(n))
    if physics == 1:
        coef = si.field_lognormal(ne, 0.0, 1.0, seed)[None]
    else:
        coef = np.stack(si.lame_from_E_nu(*si.field_elastic(ne, seed)))
    mask = si.face_mask(*n, "z0")
    A = orc.assemble(physics, xyz, conn, coef, mask)
    b = si.vec_uniform(A.n, seed, si.STREAM_RHS)
    b[si.dof_mask(mask, physics) == 1] = 0.0
    return A, b


@pytest.mark.parametrize("physics,n", [(1, (3, 2, 2)), (1, (4, 4, 4)), (3, (2, 2, 3))])
def test_pcg_matches_dense_solve(orc, physics, n):
    A, b = dirichlet_problem(orc, physics, n, 21)
    xs = np.linalg.solve(A.to_dense(), b)
    res = orc.pcg(A, b, rtol=1e-13, maxit=10 * A.n)
    assert res.status == 0
    assert np.linalg.norm(res.x - xs) <= 1e-9 * np.linalg.norm(xs)
    assert orc.true_rel_res(A, res.x, b) < 1e-12
    # recurrence residual history is the true one at convergence
    assert res.history[-1] / res.history[0] <= 1e-13


def test_pcg_first_iterate_closed_form(orc):
    A, b = dirichlet_problem(orc, 1, (3, 3, 2), 22)
    d = A.diag()
    z = b / d
    Ad = A.to_dense()
    alpha = (b @ z) / (z @ Ad @ z)
    res = orc.pcg(A, b, rtol=0.0, maxit=1)
    assert res.status == -4 and res.iters == 1
    assert np.max(np.abs(res.x - alpha * z)) <= 1e-14 * np.max(np.abs(alpha * z))
    # plain CG (no preconditioner) terminates in at most n steps in exact
    # arithmetic; after n + a few it is at roundoff
    res = orc.pcg(A, b, rtol=1e-12, maxit=A.n + 20, jacobi=False)
    assert res.status == 0


def test_fpcg_with_fixed_preconditioner_equals_pcg(orc):
    A, b = dirichlet_problem(orc, 1, (4, 3, 3), 23)
    d = A.diag()
    ref = orc.pcg(A, b, rtol=0.0, maxit=20)
    got = orc.fpcg(A, b, lambda r: r / d, rtol=0.0, maxit=20)
    assert ref.iters == got.iters == 20
    assert np.linalg.norm(got.x - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    assert np.max(np.abs(got.history - ref.history)) <= 1e-10 * ref.history[0]


def test_fpcg_failing_preconditioner_is_breakdown(orc):
    A, b = dirichlet_problem(orc, 1, (2, 2, 2), 24)
    res = orc.fpcg(A, b, lambda r: r * np.nan, rtol=1e-8, maxit=10)
    assert res.status == -5


def test_pcg_zero_rhs(orc):
    A, b = dirichlet_problem(orc, 1, (2, 2, 2), 25)
    res = orc.pcg(A, np.zeros_like(b), rtol=1e-8, maxit=10)
    assert res.status == 0 and res.iters == 0 and np.all(res.x == 0)


def test_bad_element_rejected(orc):
    X = box_nodes(1, 1, 1)
    X[[0, 1]] = X[[1, 0]]  # inverted element
    with pytest.raises(ValueError):
        orc.ke_laplace(X, 1.0)


# -- generator invariants ------------------------------------------------------

def test_generator_reproducible_and_planar():
    xyz1, conn1 = si.box_mesh(5, 4, 3, 1.0, 0.1, 2308)
    xyz2, conn2 = si.box_mesh(5, 4, 3, 1.0, 0.1, 2308)
    assert np.array_equal(xyz1, xyz2) and np.array_equal(conn1, conn2)
    xyz3, _ = si.box_mesh(5, 4, 3, 1.0, 0.1, 2309)
    assert not np.array_equal(xyz1, xyz3)
    # surface nodes are exactly on the box faces
    for c, n in zip(range(3), (5, 4, 3)):
        assert xyz1[c].min() == 0.0 and xyz1[c].max() == float(n)
    base, _ = si.box_mesh(5, 4, 3, 1.0, 0.0, 0)
    assert np.max(np.abs(xyz1 - base)) <= 0.1


def test_splitmix64_published_sequence():
    # SplitMix64 with state 0: the first outputs of the reference generator
    # (state advanced by the golden gamma before mixing).
    z = si.splitmix64(np.arange(3, dtype=np.uint64) * np.uint64(si.GOLDEN))
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_normals_have_unit_moments():
    z = si.normal(5, 1, np.arange(200000, dtype=np.uint64))
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01


@pytest.mark.parametrize("physics", [1, 3])
def test_apply_rows_equals_assembled_rows(orc, physics):
    # the element-by-element row product and the assembled CSR product are two
    # independent routes through the oracle's element matrices
    n = (3, 2, 3)
    xyz, conn = si.box_mesh(*n, 1.0, 0.1, 31)
    ne = int(np.prod(n))
    coef = (si.field_lognormal(ne, 0.0, 1.0, 31)[None] if physics == 1
            else np.stack(si.lame_from_E_nu(*si.field_elastic(ne, 31))))
    mask = si.face_mask(*n, "z0")
    A = orc.assemble(physics, xyz, conn, coef, mask)
    x = si.vec_uniform(A.n, 31, si.STREAM_X)
    rows = np.arange(A.n)
    y = orc.apply_rows(physics, xyz, conn, coef, mask, x, rows)
    assert np.max(np.abs(y - A.matvec(x))) <= 1e-13 * np.max(np.abs(y))
