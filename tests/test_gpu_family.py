"""GPU parity of the linear-tetrahedron, triquadratic- and tricubic-hexahedron operators
(q1_op_create_elem) against the CPU oracle's assembled matrices: applies and
diagonals at 1e-12 (FP64) and 2e-5 (FP32), null spaces, full-size sampled
rows, Jacobi-PCG through the generic solvers, and the unsupported requests."""
import numpy as np
import pytest

import seeded_inputs as si
from helpers import TOL, dev, rel_err, rigid_modes, torch_dtype

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q1():
    import torch
    assert torch.cuda.is_available()
    import paper_2308_09839_amd as q1
    return q1


def family_problem(elem, physics, n, jitter, seed, mask=True, h=1.0):
    if elem == 4:
        xyz, conn = si.tet_mesh(*n, h, jitter, seed)
        m = si.face_mask(*n, "z0") if mask else None
    elif elem == 27:
        xyz, conn = si.q2_box_mesh(*n, h, jitter, seed)
        m = si.q2_face_mask(*n, "z0") if mask else None
    else:
        xyz, conn = si.q3_box_mesh(*n, h, jitter, seed)
        m = si.q3_face_mask(*n, "z0") if mask else None
    ne = conn.shape[1]
    if physics == 1:
        coef = si.field_lognormal(ne, 0.0, 1.0, seed)[None]
    else:
        coef = np.stack(si.lame_from_E_nu(*si.field_elastic(ne, seed)))
    return dict(elem=elem, physics=physics, xyz=xyz, conn=conn, coef=coef, mask=m)


def make_family_op(q1, pr, dtype=0, variant=0):
    t = torch_dtype(dtype)
    mask = dev(pr["mask"].astype(np.uint8)) if pr.get("mask") is not None else None
    return q1.q1_op_create_elem(pr["elem"], pr["physics"], dtype, variant, dev(pr["xyz"], t),
                                dev(pr["conn"].astype(np.int32)), dev(pr["coef"], t), mask)


def apply(op, x, dtype):
    import torch
    xd = dev(x, torch_dtype(dtype))
    yd = torch.full_like(xd, float("nan"))
    op.apply(xd, yd)
    torch.cuda.synchronize()
    return yd.double().cpu().numpy()


CASES = [
    # elem, physics, elements, jitter, mask
    (4, 1, (6, 5, 4), 0.1, True),
    (4, 1, (7, 3, 5), 0.0, False),   # 630 tetrahedra: a ragged last block
    (4, 3, (5, 4, 3), 0.1, True),
    (4, 3, (1, 1, 1), 0.1, False),
    (27, 1, (4, 3, 3), 0.1, True),
    (27, 1, (5, 2, 1), 0.0, False),  # 10 elements: one full block of 9 and one of 1
    (27, 3, (3, 3, 2), 0.1, True),
    (27, 3, (1, 1, 1), 0.1, False),
    (64, 1, (3, 3, 2), 0.1, True),
    (64, 1, (3, 2, 1), 0.0, False),  # 6 elements: one full block of 4 and one of 2
    (64, 3, (2, 2, 2), 0.1, True),
    (64, 3, (1, 1, 1), 0.1, False),
]


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("elem,physics,n,jitter,mask", CASES)
def test_family_apply_parity(q1, orc, elem, physics, n, jitter, mask, dtype, variant):
    print(f"\n[family apply] elem={elem} physics={physics} n={n} dtype={dtype} "
          f"variant={variant}", flush=True)
    pr = family_problem(elem, physics, n, jitter, 2308, mask)
    A = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    x = si.vec_uniform(A.n, 2308, si.STREAM_X)
    ref = A.matvec(x)
    op = make_family_op(q1, pr, dtype, variant)
    y = apply(op, x, dtype)
    assert rel_err(y, ref) <= TOL[dtype], rel_err(y, ref)
    assert np.max(np.abs(y - ref)) <= 10 * TOL[dtype] * np.max(np.abs(ref))
    d = torch_empty(A.n, dtype)
    op.diag(d)
    import torch
    torch.cuda.synchronize()
    dref = A.diag()
    assert np.max(np.abs(d.double().cpu().numpy() - dref)) <= 10 * TOL[dtype] * np.max(np.abs(dref))
    # the default: block tiles for tetrahedra, the atomic scatter for the hexahedra
    assert op.info()["variant"] == (5 if elem == 4 and variant == 0 else 1)


def torch_empty(n, dtype):
    import torch
    return torch.empty(n, dtype=torch_dtype(dtype), device="cuda")


@pytest.mark.parametrize("elem", [4, 27, 64])
def test_family_dense(q1, orc, elem):
    """Apply to every unit vector: the columns are the assembled matrix."""
    import torch
    for physics in (1, 3):
        n = {4: (2, 1, 2), 27: (1, 2, 1), 64: (1, 1, 1)}[elem]
        pr = family_problem(elem, physics, n, 0.1, 41)
        Ad = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"]).to_dense()
        op = make_family_op(q1, pr)
        N = Ad.shape[0]
        xd = torch.zeros(N, dtype=torch.float64, device="cuda")
        yd = torch.empty_like(xd)
        cols = np.empty((N, N))
        for j in range(N):
            xd.zero_()
            xd[j] = 1.0
            op.apply(xd, yd)
            cols[:, j] = yd.cpu().numpy()
        assert np.max(np.abs(cols - Ad)) <= 1e-13 * np.max(np.abs(Ad))


@pytest.mark.parametrize("elem", [4, 27, 64])
@pytest.mark.parametrize("dtype", [0, 1])
def test_family_null_spaces(q1, orc, elem, dtype):
    bound = 1e-13 if dtype == 0 else 2e-6
    pr = family_problem(elem, 1, (4, 3, 3) if elem != 64 else (3, 2, 2), 0.1, 43, mask=False)
    A = orc.assemble(1, pr["xyz"], pr["conn"], pr["coef"])
    y = apply(make_family_op(q1, pr, dtype), np.ones(pr["xyz"].shape[1]), dtype)
    assert np.max(np.abs(y)) <= bound * np.max(np.abs(A.val)) * 30
    pr = family_problem(elem, 3, (3, 3, 2) if elem != 64 else (2, 2, 1), 0.1, 44, mask=False)
    A = orc.assemble(3, pr["xyz"], pr["conn"], pr["coef"])
    op = make_family_op(q1, pr, dtype)
    for u in rigid_modes(pr["xyz"]):
        y = apply(op, u, dtype)
        assert np.max(np.abs(y)) <= bound * np.max(np.abs(A.val)) * np.max(np.abs(u)) * 30


@pytest.mark.parametrize("elem", [4, 27, 64])
def test_family_full_size_rows(q1, orc, elem):
    """The benchmark sizes (Kuhn-split 128^3 box, 12,582,912 tetrahedra;
    64^3 triquadratic box, 2,146,689 nodes; 42^3 tricubic box, 2,048,383
    nodes) with the layered coefficient, FP64 and FP32: sampled rows against
    the oracle's element-by-element rows."""
    print(f"\n[family full size] elem={elem}", flush=True)
    if elem == 4:
        n = 128
        xyz, conn = si.tet_mesh(n, n, n)
        k = np.repeat(si.field_layered(n, n, n, 4, 1.5, 0.5, si.seed_for(1)), 6)
    elif elem == 27:
        n = 64
        xyz, conn = si.q2_box_mesh(n, n, n)
        k = si.field_layered(n, n, n, 2, 1.5, 0.5, si.seed_for(1))
    else:
        n = 42
        xyz, conn = si.q3_box_mesh(n, n, n)
        k = si.field_layered(n, n, n, 1, 1.5, 0.5, si.seed_for(1))
    pr = dict(elem=elem, physics=1, xyz=xyz, conn=conn, coef=k[None], mask=None)
    nn = xyz.shape[1]
    x = si.vec_uniform(nn, si.seed_for(1), si.STREAM_X)
    rows = np.unique(np.random.default_rng(6).integers(0, nn, 2000))
    ref = orc.apply_rows(1, xyz, conn, pr["coef"], None, x, rows)
    for dtype in (0, 1):
        for variant in ((0, 1) if elem == 4 else (0,)):
            y = apply(make_family_op(q1, pr, dtype, variant), x, dtype)
            assert np.linalg.norm(y[rows] - ref) / np.linalg.norm(ref) <= TOL[dtype], dtype


@pytest.mark.parametrize("elem,physics", [(4, 1), (4, 3), (27, 1), (27, 3), (64, 1), (64, 3)])
def test_family_pcg(q1, orc, elem, physics):
    """Jacobi-PCG through the generic solver: the first iterates are the oracle's,
    the converged solution has the requested residual under the oracle's matrix."""
    import torch
    n = {4: (6, 5, 4), 27: (3, 3, 3), 64: (2, 2, 2)}[elem]
    pr = family_problem(elem, physics, n, 0.1, 61)
    A = orc.assemble(physics, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    b = si.vec_uniform(A.n, 61, si.STREAM_RHS)
    b[si.dof_mask(pr["mask"], 1 if physics == 1 else 3) == 1] = 0.0
    op = make_family_op(q1, pr)
    bd = dev(b, torch.float64)
    for k in (1, 5, 10):
        xd = torch.empty_like(bd)
        st = q1.q1_pcg(op, 1, bd, xd, 0.0, k)
        ref = orc.pcg(A, b, rtol=0.0, maxit=k)
        assert st["iters"] == k
        assert np.linalg.norm(xd.cpu().numpy() - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    xd = torch.empty_like(bd)
    st = q1.q1_pcg(op, 1, bd, xd, 1e-8, 20000)
    assert st["status"] == 0
    assert orc.true_rel_res(A, xd.cpu().numpy(), b) <= 1e-8 * (1 + 1e-3)


def test_family_unsupported_and_invalid(q1):
    pr = family_problem(4, 1, (2, 2, 2), 0.0, 1)
    for variant in (2, 3, 6):
        with pytest.raises(q1.Q1Error) as ei:
            make_family_op(q1, pr, 0, variant)
        assert ei.value.code == -6
    pr27 = family_problem(27, 1, (2, 2, 2), 0.0, 1)
    for variant in (2, 3, 5, 6):
        with pytest.raises(q1.Q1Error) as ei:
            make_family_op(q1, pr27, 0, variant)
        assert ei.value.code == -6
    with pytest.raises(q1.Q1Error) as ei:
        make_family_op(q1, dict(pr, physics=2, coef=pr["coef"]))
    assert ei.value.code == -6
    op = make_family_op(q1, pr)
    with pytest.raises(q1.Q1Error) as ei:
        q1.q1_csr_create(op)
    assert ei.value.code == -6
    bad = dict(pr, conn=pr["conn"].copy())
    bad["conn"][2, 7] = pr["xyz"].shape[1]
    with pytest.raises(q1.Q1Error) as ei:
        make_family_op(q1, bad)
    assert ei.value.code == -1
    with pytest.raises(q1.Q1Error) as ei:
        make_family_op(q1, dict(pr, elem=5))
    assert ei.value.code == -1


# Tetrahedra of a Kuhn-split box lattice whose cell counts are multiples of 16, 8, 4:
# the scalar operator takes the owner-computes tiles, each cell's six tetrahedra
# evaluated as one element (bitwise reproducible apply and diagonal).
@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("mask", ["none", "random", "all_faces"])
@pytest.mark.parametrize("n,jitter", [((16, 8, 4), 0.0), ((32, 16, 8), 0.1), ((48, 8, 12), 0.1)])
def test_owner_tets(q1, orc, monkeypatch, n, jitter, mask, dtype):
    import torch
    print(f"\n[owner tets] n={n} jitter={jitter} mask={mask} dtype={dtype}", flush=True)
    pr = family_problem(4, 1, n, jitter, 2319, False)
    nn = pr["xyz"].shape[1]
    if mask == "random":
        pr["mask"] = (np.random.default_rng(2319).random(nn) < 0.15).astype(np.uint8)
    elif mask == "all_faces":
        m = np.zeros(nn, np.uint8)
        for f in ("x0", "x1", "y0", "y1", "z0", "z1"):
            m |= si.face_mask(*n, f).astype(np.uint8)
        pr["mask"] = m
    A = orc.assemble(1, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    x = si.vec_uniform(A.n, 2319, si.STREAM_X)
    ref = A.matvec(x)
    op = make_family_op(q1, pr, dtype)
    assert op.reproducible()
    ys = [apply(op, x, dtype) for _ in range(3)]
    assert all(np.array_equal(ys[0], y) for y in ys[1:])
    assert rel_err(ys[0], ref) <= TOL[dtype], rel_err(ys[0], ref)
    assert np.max(np.abs(ys[0] - ref)) <= 10 * TOL[dtype] * np.max(np.abs(ref))
    ds = []
    for _ in range(2):
        d = torch_empty(A.n, dtype)
        op.diag(d)
        torch.cuda.synchronize()
        ds.append(d.double().cpu().numpy())
    assert np.array_equal(ds[0], ds[1])
    dref = A.diag()
    assert np.max(np.abs(ds[0] - dref)) <= 10 * TOL[dtype] * np.max(np.abs(dref))
    # the block tiles of the same operator agree to the same bar, in another order
    monkeypatch.setenv("Q1_OWNER_TILE", "0")
    opb = make_family_op(q1, pr, dtype)
    monkeypatch.delenv("Q1_OWNER_TILE")
    assert not opb.reproducible()
    yb = apply(opb, x, dtype)
    assert rel_err(yb, ref) <= TOL[dtype]
    assert not np.array_equal(yb, ys[0])


def test_owner_tets_pcg(q1, orc):
    """Jacobi-PCG on owner-computes tetrahedra (the apply forms the p.q partials):
    the first iterates are the oracle's, and two solves are bitwise identical."""
    import torch
    pr = family_problem(4, 1, (32, 16, 8), 0.1, 62)
    A = orc.assemble(1, pr["xyz"], pr["conn"], pr["coef"], pr["mask"])
    b = si.vec_uniform(A.n, 62, si.STREAM_RHS)
    b[pr["mask"] == 1] = 0.0
    op = make_family_op(q1, pr)
    assert op.reproducible()
    bd = dev(b, torch.float64)
    for k in (1, 5, 10):
        xd = torch.empty_like(bd)
        st = q1.q1_pcg(op, 1, bd, xd, 0.0, k)
        ref = orc.pcg(A, b, rtol=0.0, maxit=k)
        assert st["iters"] == k
        assert np.linalg.norm(xd.cpu().numpy() - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    xs, its = [], []
    for _ in range(2):
        xd = torch.empty_like(bd)
        st = q1.q1_pcg(op, 1, bd, xd, 1e-8, 20000)
        assert st["status"] == 0
        its.append(st["iters"])
        xs.append(xd.cpu().numpy())
    assert its[0] == its[1] and np.array_equal(xs[0], xs[1])
    assert orc.true_rel_res(A, xs[0], b) <= 1e-8 * (1 + 1e-3)
