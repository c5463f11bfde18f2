"""GPU parity of the matrix-free apply and diagonal against the CPU oracle.

Bars: relative error <= 1e-12 for FP64 applies and <= 2e-5 for FP32
applies (FP32 coordinates, coefficients, vectors and arithmetic compared with
the FP64 oracle on the FP64 inputs)."""
import numpy as np
import pytest

import seeded_inputs as si
from helpers import (TOL, dev, gpu_apply, gpu_diag, make_op, problem, rel_err, rigid_modes,
                     torch_dtype)

pytestmark = pytest.mark.gpu

VARIANTS = [1, 2, 3, 5]  # atomic scatter, colour classes, LDS tiles, block-staged tiles


@pytest.fixture(scope="module")
def q1():
    import torch
    assert torch.cuda.is_available()
    import paper_2308_09839_amd as q1
    return q1


CASES = [
    # physics, elements, jitter, mask
    (1, (16, 16, 16), 0.1, True),   # the 16^3 jittered validation problem
    (1, (13, 11, 7), 0.1, True),    # ragged tail of a 256-element block
    (1, (5, 3, 4), 0.0, False),     # undistorted (affine path), pure Neumann
    (1, (1, 1, 1), 0.0, False),
    (3, (8, 8, 8), 0.1, True),
    (3, (13, 11, 7), 0.0, True),    # affine elasticity, ragged
    (3, (3, 2, 2), 0.1, False),
    (2, (9, 7, 6), 0.1, True),      # vector Laplace
    (2, (13, 11, 7), 0.0, False),   # affine vector Laplace, ragged
    (2, (1, 1, 1), 0.1, True),
]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("physics,n,jitter,mask", CASES)
def test_apply_parity(q1, orc, physics, n, jitter, mask, dtype, variant):
    print(f"\n[apply parity] physics={physics} n={n} jitter={jitter} dtype={dtype} "
          f"variant={variant}", flush=True)
    pr = problem(physics, n, jitter, 2308, mask)
    A = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    x = si.vec_uniform(A.n, 2308, si.STREAM_X)
    ref = A.matvec(x)
    op = make_op(pr, dtype, variant)
    y = gpu_apply(op, x, dtype)
    err = rel_err(y, ref)
    assert err <= TOL[dtype], err
    assert np.max(np.abs(y - ref)) <= 10 * TOL[dtype] * np.max(np.abs(ref))


# Boxes made of whole default tiles: the block variant's instances with the tile
# shape built in, for parallelepipeds and general hexahedra, with and without
# Dirichlet nodes (whose tiles load their node words instead of computing them).
# Scalar kind: 16 x 8 x 4 tiles; 3-DOF kinds: 16 x 4 x 4 tiles.
FIXED_TILE_CASES = [
    # physics, elements, jitter, mask
    (1, (16, 8, 4), 0.0, False),
    (1, (16, 8, 16), 0.0, True),
    (1, (32, 16, 16), 0.1, False),
    (1, (32, 16, 8), 0.0, False),
    (1, (32, 16, 8), 0.0, True),
    (1, (48, 24, 12), 0.0, True),
    (1, (32, 16, 8), 0.1, True),
    (3, (32, 8, 8), 0.0, True),
    (3, (32, 8, 8), 0.1, False),
    (2, (16, 4, 8), 0.0, True),
    (2, (16, 4, 8), 0.1, True),
]


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("physics,n,jitter,mask", FIXED_TILE_CASES)
def test_apply_parity_whole_tiles(q1, orc, physics, n, jitter, mask, dtype):
    print(f"\n[apply parity, whole tiles] physics={physics} n={n} jitter={jitter} mask={mask} "
          f"dtype={dtype}", flush=True)
    pr = problem(physics, n, jitter, 2311, mask)
    A = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    x = si.vec_uniform(A.n, 2311, si.STREAM_X)
    ref = A.matvec(x)
    op = make_op(pr, dtype, 0)
    assert op.reproducible()
    ys = [gpu_apply(op, x, dtype) for _ in range(3)]
    assert all(np.array_equal(ys[0], y) for y in ys[1:])
    assert rel_err(ys[0], ref) <= TOL[dtype]
    assert np.max(np.abs(ys[0] - ref)) <= 10 * TOL[dtype] * np.max(np.abs(ref))
    ds = [gpu_diag(op, A.n, dtype) for _ in range(2)]
    assert np.array_equal(ds[0], ds[1])
    assert rel_err(ds[0], A.diag()) <= TOL[dtype]


# Owner-computes tiles (the default for the scalar kind on box lattices of
# parallelepipeds whose element counts are multiples of 16, 8, 4): each tile owns
# a 16 x 8 x 4 node box, the last tile in a direction also the mesh's last node
# plane.  Dirichlet nodes are drawn at random so that they fall on tile borders,
# box corners and the last planes.
OWNER_CASES = [(16, 8, 4), (32, 8, 4), (16, 16, 8), (32, 16, 12), (48, 24, 8)]


@pytest.mark.parametrize("jitter", [0.0, 0.1])
@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("mask", ["none", "random", "all_faces"])
@pytest.mark.parametrize("n", OWNER_CASES)
def test_owner_tiles_parity(q1, orc, monkeypatch, n, mask, dtype, jitter):
    """Parallelepipeds (jitter 0) take the closed-form element; these small jittered
    meshes take the owner tiles with the general element."""
    print(f"\n[owner tiles] n={n} mask={mask} dtype={dtype} jitter={jitter}", flush=True)
    pr = problem(1, n, jitter, 2317, False)
    nn = pr["xyz"].shape[1]
    if mask == "random":
        pr["mask"] = (np.random.default_rng(2317).random(nn) < 0.15).astype(np.uint8)
    elif mask == "all_faces":
        m = np.zeros(nn, np.uint8)
        for f in ("x0", "x1", "y0", "y1", "z0", "z1"):
            m |= si.face_mask(*n, f).astype(np.uint8)
        pr["mask"] = m
    A = orc.assemble(1, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    x = si.vec_uniform(A.n, 2317, si.STREAM_X)
    ref = A.matvec(x)
    op = make_op(pr, dtype, 0)
    assert op.reproducible()
    ys = [gpu_apply(op, x, dtype) for _ in range(3)]
    assert all(np.array_equal(ys[0], y) for y in ys[1:])
    assert rel_err(ys[0], ref) <= TOL[dtype]
    assert np.max(np.abs(ys[0] - ref)) <= 10 * TOL[dtype] * np.max(np.abs(ref))
    if pr["mask"] is not None:
        fixed = pr["mask"] == 1
        assert np.array_equal(ys[0][fixed], x[fixed].astype(ys[0].dtype)) or dtype == 1
    # the halo-slot tiles of the same operator agree to the same bar (they add in
    # another order, so the two results are not bitwise equal: the owner path ran)
    monkeypatch.setenv("Q1_OWNER_TILE", "0")
    y_halo = gpu_apply(make_op(pr, dtype, 0), x, dtype)
    monkeypatch.delenv("Q1_OWNER_TILE")
    assert rel_err(y_halo, ref) <= TOL[dtype]
    assert not np.array_equal(y_halo, ys[0])


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("physics,n", [(1, (1, 1, 1)), (1, (2, 2, 2)), (1, (3, 2, 2)),
                                       (3, (1, 1, 1)), (3, (2, 2, 1)), (2, (2, 1, 1))])
def test_brute_force_dense(q1, orc, physics, n, variant):
    """Apply to every unit vector: the columns form the assembled matrix."""
    print(f"\n[dense] physics={physics} n={n}", flush=True)
    import torch
    pr = problem(physics, n, 0.1, 41, mask=True)
    A = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"]).to_dense()
    op = make_op(pr, 0, variant)
    N = A.shape[0]
    cols = np.empty((N, N))
    xd = torch.zeros(N, device="cuda", dtype=torch.float64)
    yd = torch.empty_like(xd)
    for j in range(N):
        xd.zero_(); xd[j] = 1.0
        op.apply(xd, yd)
        cols[:, j] = yd.cpu().numpy()
    assert np.max(np.abs(cols - A)) <= 1e-13 * np.max(np.abs(A))


@pytest.mark.parametrize("variant", VARIANTS + [6])
@pytest.mark.parametrize("dtype", [0, 1])
def test_null_spaces(q1, orc, dtype, variant):
    print(f"\n[null spaces] dtype={dtype}", flush=True)
    bound = 1e-13 if dtype == 0 else 2e-6
    pr = problem(1, (9, 7, 6), 0.1, 43, mask=False)
    op = make_op(pr, dtype, variant)
    nn = pr["xyz"].shape[1]
    y = gpu_apply(op, np.ones(nn), dtype)
    kmax = pr["coef"].max()
    assert np.max(np.abs(y)) <= bound * kmax * 8
    pr = problem(3, (5, 6, 4), 0.1, 44, mask=False)
    op = make_op(pr, dtype, variant)
    A = orc.assemble(3, pr["xyz"], pr["conn"], pr["coef"])
    scale = np.max(np.abs(A.val))
    for u in rigid_modes(pr["xyz"]):
        y = gpu_apply(op, u, dtype)
        assert np.max(np.abs(y)) <= bound * scale * np.max(np.abs(u)) * 30


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("physics,n,jitter", [(1, (16, 16, 16), 0.1), (1, (7, 5, 3), 0.0),
                                              (3, (7, 6, 5), 0.1), (3, (4, 4, 4), 0.0),
                                              (2, (7, 6, 5), 0.1), (2, (4, 4, 4), 0.0)])
def test_diag_parity(q1, orc, physics, n, jitter, dtype):
    print(f"\n[diag] physics={physics} n={n} dtype={dtype}", flush=True)
    pr = problem(physics, n, jitter, 45, mask=True)
    A = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    d = gpu_diag(make_op(pr, dtype), A.n, dtype)
    ref = A.diag()
    assert np.max(np.abs(d - ref) / np.abs(ref)) <= (1e-13 if dtype == 0 else 2e-5)


@pytest.mark.parametrize("variant", VARIANTS)
def test_full_size_laplace_sampled(q1, orc, variant):
    """128^3 undistorted layered-coefficient Laplace, FP64 and FP32, in the
    benchmark's launch configuration: sampled rows against the oracle's
    element-by-element rows, and A 1 = 0 over the whole grid."""
    print("\n[full-size laplace 128^3]", flush=True)
    pr = si.problem_laplace_layered(128, si.seed_for(1))
    nn = pr["xyz"].shape[1]
    x = si.vec_uniform(nn, si.seed_for(1), si.STREAM_X)
    rng = np.random.default_rng(0)
    rows = np.unique(np.concatenate([rng.integers(0, nn, 3000), [0, nn - 1, 129 * 129 * 64 + 64]]))
    ref = orc.apply_rows(1, pr["xyz"], pr["conn"], pr["coef"], None, x, rows)
    for dtype in (0, 1):
        op = make_op(pr, dtype, variant)
        y = gpu_apply(op, x, dtype)
        err = np.linalg.norm(y[rows] - ref) / np.linalg.norm(ref)
        assert err <= TOL[dtype], (dtype, err)
        y1 = gpu_apply(op, np.ones(nn), dtype)
        assert np.max(np.abs(y1)) <= (1e-12 if dtype == 0 else 1e-4) * pr["coef"].max()
        del op


@pytest.mark.parametrize("variant", VARIANTS)
def test_full_size_elasticity_sampled(q1, orc, variant):
    print("\n[full-size elasticity 96^3]", flush=True)
    pr = si.problem_elasticity(96, si.seed_for(2))
    nn = pr["xyz"].shape[1]
    x = si.vec_uniform(3 * nn, si.seed_for(2), si.STREAM_X)
    rng = np.random.default_rng(1)
    rows = np.unique(np.concatenate([rng.integers(0, 3 * nn, 3000), [0, 3 * nn - 1]]))
    ref = orc.apply_rows(3, pr["xyz"], pr["conn"], pr["coef"], pr["mask"], x, rows)
    for dtype in (0, 1):
        op = make_op(pr, dtype, variant)
        y = gpu_apply(op, x, dtype)
        err = np.linalg.norm(y[rows] - ref) / np.linalg.norm(ref)
        assert err <= TOL[dtype], (dtype, err)
        del op


@pytest.mark.parametrize("variant", VARIANTS)
def test_full_size_vlaplace_sampled(q1, orc, variant):
    """96^3 undistorted vector Laplace (the 3-DOF Laplace workload), FP64 and
    FP32: sampled rows against the oracle's element-by-element rows, and the
    three constant fields in the null space over the whole grid."""
    print("\n[full-size vector laplace 96^3]", flush=True)
    pr = si.problem_vlaplace(96, si.seed_for(5))
    nn = pr["xyz"].shape[1]
    x = si.vec_uniform(3 * nn, si.seed_for(5), si.STREAM_X)
    rng = np.random.default_rng(2)
    rows = np.unique(np.concatenate([rng.integers(0, 3 * nn, 3000), [0, 3 * nn - 1]]))
    ref = orc.apply_rows(2, pr["xyz"], pr["conn"], pr["coef"], pr["mask"], x, rows)
    for dtype in (0, 1):
        op = make_op(pr, dtype, variant)
        y = gpu_apply(op, x, dtype)
        err = np.linalg.norm(y[rows] - ref) / np.linalg.norm(ref)
        assert err <= TOL[dtype], (dtype, err)
        del op
    pr_n = dict(pr, mask=None)
    op = make_op(pr_n, 0, variant)
    for c in range(3):
        u = np.zeros((nn, 3))
        u[:, c] = 1.0
        y = gpu_apply(op, u.ravel(), 0)
        assert np.max(np.abs(y)) <= 1e-12 * pr["coef"].max()


@pytest.mark.parametrize("jitter", [0.0, 0.1])
def test_full_size_laplace_full_vector(q1, orc, jitter):
    """128^3 layered-coefficient Laplace in the benchmark's launch configuration
    (default operator), FP64 and FP32, undistorted (parallelepiped element path)
    and jittered (general hexahedra): every entry of y against the oracle's
    assembled CSR matrix (57,066,625 non-zeros)."""
    print(f"\n[full-vector laplace 128^3] jitter={jitter}", flush=True)
    seed = si.seed_for(1)
    pr = si.problem_laplace_layered(128, seed)
    if jitter:
        pr["xyz"], _ = si.box_mesh(128, 128, 128, 1.0, jitter, seed)
    nn = pr["xyz"].shape[1]
    A = orc.assemble(1, pr["xyz"], pr["conn"], pr["coef"])
    assert A.nnz == 385 ** 3
    x = si.vec_uniform(nn, seed, si.STREAM_X)
    ref = A.matvec(x)
    del A
    for dtype in (0, 1):
        op = make_op(pr, dtype, 0)
        y = gpu_apply(op, x, dtype)
        op.destroy()
        assert rel_err(y, ref) <= TOL[dtype], (dtype, rel_err(y, ref))
        assert np.max(np.abs(y - ref)) <= 10 * TOL[dtype] * np.max(np.abs(ref))


def test_full_size_elasticity_jittered(q1, orc):
    """96^3 jittered elasticity (the general-hexahedron instance), FP64 and FP32:
    sampled rows against the oracle's element-by-element rows, and, without the
    Dirichlet condition, the six rigid-body modes in the null space over the
    whole grid."""
    print("\n[full-size jittered elasticity 96^3]", flush=True)
    seed = si.seed_for(2)
    pr = si.problem_elasticity(96, seed)
    pr["xyz"], _ = si.box_mesh(96, 96, 96, 1.0, 0.1, seed)
    nn = pr["xyz"].shape[1]
    x = si.vec_uniform(3 * nn, seed, si.STREAM_X)
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([rng.integers(0, 3 * nn, 3000), [0, 3 * nn - 1]]))
    ref = orc.apply_rows(3, pr["xyz"], pr["conn"], pr["coef"], pr["mask"], x, rows)
    for dtype in (0, 1):
        op = make_op(pr, dtype, 0)
        y = gpu_apply(op, x, dtype)
        op.destroy()
        err = np.linalg.norm(y[rows] - ref) / np.linalg.norm(ref)
        assert err <= TOL[dtype], (dtype, err)
    op = make_op(dict(pr, mask=None), 0, 0)
    scale = np.max(pr["coef"]) * 1.0
    for m in rigid_modes(pr["xyz"]):
        y = gpu_apply(op, m, 0)
        assert np.max(np.abs(y)) <= 1e-10 * scale * max(1.0, np.max(np.abs(m)))
    op.destroy()


# -- partial assembly (quadrature data stored at set-up) ----------------------------

PA_CASES = CASES


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("physics,n,jitter,mask", PA_CASES)
def test_partial_assembly_parity(q1, orc, physics, n, jitter, mask, dtype):
    print(f"\n[partial assembly] physics={physics} n={n} jitter={jitter} dtype={dtype}",
          flush=True)
    pr = problem(physics, n, jitter, 2308, mask)
    A = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    x = si.vec_uniform(A.n, 2308, si.STREAM_X)
    ref = A.matvec(x)
    y = gpu_apply(make_op(pr, dtype, 6), x, dtype)
    assert rel_err(y, ref) <= TOL[dtype], rel_err(y, ref)


def test_partial_assembly_full_size(q1, orc):
    """128^3 layered-coefficient Laplace through partial assembly, FP64 and FP32:
    sampled rows against the oracle, and the constant null vector."""
    print("\n[partial assembly 128^3]", flush=True)
    pr = si.problem_laplace_layered(128, si.seed_for(1))
    nn = pr["xyz"].shape[1]
    x = si.vec_uniform(nn, si.seed_for(1), si.STREAM_X)
    rows = np.unique(np.random.default_rng(3).integers(0, nn, 3000))
    ref = orc.apply_rows(1, pr["xyz"], pr["conn"], pr["coef"], None, x, rows)
    for dtype in (0, 1):
        op = make_op(pr, dtype, 6)
        y = gpu_apply(op, x, dtype)
        assert np.linalg.norm(y[rows] - ref) / np.linalg.norm(ref) <= TOL[dtype]
        y1 = gpu_apply(op, np.ones(nn), dtype)
        assert np.max(np.abs(y1)) <= (1e-12 if dtype == 0 else 1e-4) * pr["coef"].max()
        del op


def test_partial_assembly_elasticity_full_size(q1, orc):
    """96^3 elasticity through partial assembly (the scaled adjugate per point),
    FP64 and FP32, undistorted and jittered: sampled rows against the oracle's
    element-by-element rows, and the six rigid-body modes in the kernel of the
    pure-Neumann operator."""
    print("\n[partial assembly elasticity 96^3]", flush=True)
    rng = np.random.default_rng(4)
    for jitter in (0.0, 0.1):
        pr = si.problem_elasticity(96, si.seed_for(2), jitter=jitter)
        nn = pr["xyz"].shape[1]
        x = si.vec_uniform(3 * nn, si.seed_for(2), si.STREAM_X)
        rows = np.unique(rng.integers(0, 3 * nn, 3000))
        ref = orc.apply_rows(3, pr["xyz"], pr["conn"], pr["coef"], pr["mask"], x, rows)
        prn = dict(pr, mask=None)
        for dtype in (0, 1):
            y = gpu_apply(make_op(pr, dtype, 6), x, dtype)
            assert np.linalg.norm(y[rows] - ref) / np.linalg.norm(ref) <= TOL[dtype], (jitter,
                                                                                      dtype)
        opn = make_op(prn, 0, 6)
        scale = pr["coef"].max() * 8
        for m in rigid_modes(pr["xyz"]):
            ym = gpu_apply(opn, m, 0)
            assert np.max(np.abs(ym)) <= 1e-10 * scale * max(1.0, np.max(np.abs(m)))


def test_empty_mesh_and_errors(q1):
    import torch
    print("\n[edge cases]", flush=True)
    # no elements: y = x on masked nodes, 0 elsewhere
    xyz = dev(np.zeros((3, 4)), torch.float64)
    conn = torch.zeros((8, 0), dtype=torch.int32, device="cuda")
    coef = torch.zeros((1, 0), dtype=torch.float64, device="cuda")
    mask = dev(np.array([1, 0, 1, 0], dtype=np.uint8))
    op = q1.q1_op_create(1, 0, 1, xyz, conn, coef, mask)
    x = dev(np.array([1.0, 2.0, 3.0, 4.0]))
    y = torch.full_like(x, 7.0)
    op.apply(x, y)
    assert y.cpu().tolist() == [1.0, 0.0, 3.0, 0.0]
    with pytest.raises(q1.Q1Error) as ei:
        op.apply(x, x)
    assert ei.value.code == -1
    # host memory is rejected
    pr = problem(1, (2, 2, 2), 0.0, 1, mask=False)
    t = torch_dtype(0)
    with pytest.raises(q1.Q1Error):
        import ctypes
        h = ctypes.c_void_p()
        xyz_h = np.ascontiguousarray(pr["xyz"])
        rc = q1.lib().q1_op_create(ctypes.byref(h), 1, 0, 1, xyz_h.shape[1], 8,
                                   xyz_h.ctypes.data_as(ctypes.c_void_p),
                                   ctypes.c_void_p(dev(pr["conn"]).data_ptr()),
                                   ctypes.c_void_p(dev(pr["coef"], t).data_ptr()), None, None)
        q1._lib.check(rc)
    with pytest.raises(q1.Q1Error):  # no physics kind 4
        q1.q1_op_create(4, 0, 1, dev(pr["xyz"], t), dev(pr["conn"]), dev(pr["coef"], t))


@pytest.mark.parametrize("variant", VARIANTS + [6])
@pytest.mark.parametrize("physics", [1, 2, 3])
def test_apply_permuted_numbering(q1, orc, physics, variant):
    """Nodes renumbered by a random permutation: tiles are no longer lattices in
    id order, so the block kernels read their corner indices from the planner's
    tables instead of computing them."""
    print(f"\n[permuted numbering] physics={physics} variant={variant}", flush=True)
    pr = problem(physics, (9, 7, 6), 0.1, 47, True)
    nn = pr["xyz"].shape[1]
    perm = np.random.default_rng(5).permutation(nn)  # new id of old node i = perm[i]
    inv = np.argsort(perm)
    pp = dict(pr, xyz=pr["xyz"][:, inv], conn=perm[pr["conn"]].astype(np.int32),
              mask=pr["mask"][inv])
    A = orc.assemble(physics, pp["xyz"], pp["conn"], pp["coef"], pp["mask"])
    x = si.vec_uniform(A.n, 47, si.STREAM_X)
    ref = A.matvec(x)
    for dtype in (0, 1):
        y = gpu_apply(make_op(pp, dtype, variant), x, dtype)
        assert rel_err(y, ref) <= TOL[dtype], (dtype, rel_err(y, ref))


def _with_orphan(pr, masked: bool):
    """The problem with one extra node, numbered in the middle, that no element
    references."""
    nn = pr["xyz"].shape[1]
    k = nn // 2
    out = dict(pr)
    out["xyz"] = np.insert(pr["xyz"], k, np.array([0.5, 0.5, 0.5]), axis=1)
    out["conn"] = (pr["conn"] + (pr["conn"] >= k)).astype(np.int32)
    out["mask"] = np.insert(pr["mask"], k, np.uint8(1 if masked else 0))
    return out, k


@pytest.mark.parametrize("masked", [False, True])
@pytest.mark.parametrize("variant", VARIANTS + [6])
@pytest.mark.parametrize("physics", [1, 3])
def test_unreferenced_node(q1, orc, physics, variant, masked):
    """A node no element references has a zero row: every variant writes y = 0
    there (y = x when masked), whatever y held before; diag 0 (1 if masked)."""
    import torch
    print(f"\n[orphan] physics={physics} variant={variant} masked={masked}", flush=True)
    pr = problem(physics, (6, 5, 4), 0.1, 2308, True)
    dpn = 1 if physics == 1 else 3
    A = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    pr2, k = _with_orphan(pr, masked)
    n2 = pr2["xyz"].shape[1] * dpn
    x2 = si.vec_uniform(n2, 2308, si.STREAM_X)
    x = np.delete(x2, np.arange(k * dpn, (k + 1) * dpn))
    ref = np.insert(A.matvec(x), k * dpn,
                    x2[k * dpn:(k + 1) * dpn] if masked else np.zeros(dpn))
    dref = np.insert(A.diag(), k * dpn, np.full(dpn, 1.0 if masked else 0.0))
    op = make_op(pr2, 0, variant)
    xd = dev(x2, torch.float64)
    yd = torch.full_like(xd, float("nan"))
    op.apply(xd, yd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    assert np.all(np.isfinite(y))
    assert np.array_equal(y[k * dpn:(k + 1) * dpn], ref[k * dpn:(k + 1) * dpn])
    assert rel_err(y, ref) <= TOL[0]
    d = gpu_diag(op, n2, 0)
    assert np.max(np.abs(d - dref)) <= 1e-13 * np.max(np.abs(dref))


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 5, 6])
def test_connectivity_out_of_range_rejected(q1, variant):
    """q1_op_create checks every connectivity entry on the device."""
    pr = problem(1, (4, 3, 2), 0.0, 7, True)
    nn = pr["xyz"].shape[1]
    for bad in (-1, nn, 2 ** 31 - 1):
        conn = pr["conn"].copy()
        conn[3, 5] = bad
        with pytest.raises(q1.Q1Error) as ei:
            make_op(dict(pr, conn=conn), 0, variant)
        assert ei.value.code == -1, (variant, bad, str(ei.value))


REPRO_CASES = [
    # physics, elements, jitter, variant
    (1, (16, 16, 16), 0.1, 5),  # general hexahedra
    (1, (37, 19, 11), 0.0, 5),  # parallelepipeds, ragged tiles on every side
    (2, (9, 7, 6), 0.1, 5),
    (3, (8, 8, 8), 0.1, 5),
    (3, (21, 9, 7), 0.0, 5),
    (1, (13, 11, 7), 0.1, 6),   # partial assembly
    (3, (8, 8, 8), 0.1, 6),
]


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("physics,n,jitter,variant", REPRO_CASES)
def test_block_apply_bitwise_reproducible(q1, orc, physics, n, jitter, variant, dtype):
    """The block and partial-assembly variants add every node's contributions in a
    fixed order (split accumulation, halo slots summed in tile order): repeated
    applies and diagonals are bitwise identical, and still match the oracle."""
    print(f"\n[reproducible] physics={physics} n={n} variant={variant} dtype={dtype}", flush=True)
    pr = problem(physics, n, jitter, 2308, True)
    A = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    op = make_op(pr, dtype, variant)
    assert op.reproducible()
    x = si.vec_uniform(A.n, 2309, si.STREAM_X)
    ys = [gpu_apply(op, x, dtype) for _ in range(4)]
    assert all(np.array_equal(ys[0], y) for y in ys[1:])
    assert rel_err(ys[0], A.matvec(x)) <= TOL[dtype]
    ds = [gpu_diag(op, A.n, dtype) for _ in range(3)]
    assert all(np.array_equal(ds[0], d) for d in ds[1:])
    assert rel_err(ds[0], A.diag()) <= TOL[dtype]


def test_atomic_variant_not_reproducible_flag(q1):
    pr = problem(1, (4, 4, 4), 0.1, 2308, True)
    assert not make_op(pr, 0, 1).reproducible()
    assert not make_op(pr, 0, 3).reproducible()
    assert make_op(pr, 0, 0).reproducible()  # the default is the block variant
