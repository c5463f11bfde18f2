"""GPU parity of the learned preconditioner's kernels against the FP64 network
oracle on identical BF16-rounded operands: convolution forward,
backward-data and backward-weight to 1e-4 of the largest entry (FP32
accumulation of up to 27 x 96 products), the whole network forward and
gradient with the oracle rounding every stored tensor as the library does,
the loss, Adam, and the preconditioner's encoding."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import unet_oracle as U

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q1():
    import torch
    assert torch.cuda.is_available()
    import paper_2308_09839_amd as q1
    return q1


def rnd(shape, seed, lo=-1.0, hi=1.0):
    n = int(np.prod(shape))
    return (lo + (hi - lo) * si.uniform(seed, si.STREAM_X, np.arange(n, dtype=np.uint64))).reshape(shape)


def bf(a):
    """BF16 device tensor of a (torch's round-to-nearest-even conversion)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).cuda()


def f32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    return t.double().cpu().numpy()


def maxrel(x, ref):
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-30))


def normrel(x, ref):
    return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-30))


# -- single layers ---------------------------------------------------------------

FWD_CASES = [  # B, fine grid, ca, up_a, cb, cout, relu
    (2, (5, 6, 7), 16, 0, 0, 16, 0),
    (1, (8, 8, 8), 8, 0, 0, 16, 1),
    (1, (6, 8, 10), 64, 1, 32, 32, 1),
    (2, (4, 6, 4), 32, 1, 16, 16, 0),
    (1, (5, 5, 5), 64, 0, 0, 64, 0),
    (1, (3, 5, 9), 16, 0, 0, 48, 0),
    (1, (4, 4, 5), 16, 0, 0, 96, 1),
]


@pytest.mark.parametrize("B,grid,ca,up,cb,cout,relu", FWD_CASES)
def test_conv_forward(q1, B, grid, ca, up, cb, cout, relu):
    print(f"\n[conv fwd] B={B} grid={grid} ca={ca} up={up} cb={cb} cout={cout}", flush=True)
    D, H, W = grid
    ga = (B, D // 2, H // 2, W // 2, ca) if up else (B, D, H, W, ca)
    a = U.bf16_round(rnd(ga, 1))
    b = U.bf16_round(rnd((B, D, H, W, cb), 2)) if cb else None
    w = rnd((27, ca + cb, cout), 3) * 0.2
    bias = rnd((cout,), 4)
    y = q1.q1_conv3d_forward(bf(a), ca, f32(w), cout, bias=f32(bias), b=bf(b) if cb else None,
                             cb=cb, up_a=up, relu=relu)
    x = U.up2(a) if up else a
    if cb:
        x = np.concatenate([x, b], axis=4)
    ref = U.conv3d(x, U.bf16_round(w), bias.astype(np.float32))
    if relu:
        ref = U.relu(ref)
    assert maxrel(host(y), ref) <= 1e-4


BWD_CASES = [  # B, grid, cout (gradient channels in), cin (out)
    (2, (5, 6, 7), 16, 16), (1, (6, 4, 6), 32, 96), (1, (5, 7, 4), 16, 48),
    (1, (5, 5, 5), 64, 64), (2, (4, 4, 6), 32, 16), (1, (3, 3, 3), 64, 32)]


@pytest.mark.parametrize("B,grid,cout,cin", BWD_CASES)
def test_conv_backward_data(q1, B, grid, cout, cin):
    print(f"\n[conv bwd data] B={B} grid={grid} cout={cout} cin={cin}", flush=True)
    gy = U.bf16_round(rnd((B,) + grid + (cout,), 5))
    w = rnd((27, cin, cout), 6) * 0.2
    gx = q1.q1_conv3d_backward_data(bf(gy), cout, f32(w), cin)
    ref = U.conv3d_backward_data(gy, U.bf16_round(w))
    assert maxrel(host(gx), ref) <= 1e-4


WG_CASES = [  # B, fine grid, ca, up_a, cb, cout
    (2, (5, 6, 7), 16, 0, 0, 16), (1, (8, 8, 8), 8, 0, 0, 16), (1, (6, 8, 10), 64, 1, 32, 32),
    (2, (4, 6, 4), 32, 1, 16, 16), (1, (5, 5, 5), 64, 0, 0, 64), (3, (3, 4, 5), 32, 0, 0, 32)]


@pytest.mark.parametrize("B,grid,ca,up,cb,cout", WG_CASES)
def test_conv_backward_weight(q1, B, grid, ca, up, cb, cout):
    print(f"\n[conv bwd weight] B={B} grid={grid} ca={ca} up={up} cb={cb} cout={cout}", flush=True)
    D, H, W = grid
    ga = (B, D // 2, H // 2, W // 2, ca) if up else (B, D, H, W, ca)
    a = U.bf16_round(rnd(ga, 7))
    b = U.bf16_round(rnd((B, D, H, W, cb), 8)) if cb else None
    gy = U.bf16_round(rnd((B, D, H, W, cout), 9))
    gw, gb = q1.q1_conv3d_backward_weight(bf(a), ca, bf(gy), cout, b=bf(b) if cb else None, cb=cb,
                                          up_a=up)
    x = U.up2(a) if up else a
    if cb:
        x = np.concatenate([x, b], axis=4)
    rw, rb = U.conv3d_backward_weight(x, gy)
    assert maxrel(host(gw), rw) <= 1e-4
    assert maxrel(host(gb), rb) <= 1e-5


def test_conv_argument_errors(q1):
    import torch
    a = torch.zeros((1, 4, 4, 4, 16), dtype=torch.bfloat16, device="cuda")
    w = torch.zeros((27, 16, 24), dtype=torch.float32, device="cuda")
    with pytest.raises(q1.Q1Error):
        q1.q1_conv3d_forward(a, 16, w, 24)  # unsupported output width
    with pytest.raises(q1.Q1Error):
        q1.q1_conv3d_forward(a, 12, w, 16)  # channels not a multiple of 8


# -- the whole network ------------------------------------------------------------

def net_inputs(B, D, H, W, seed):
    x = np.zeros((B, D, H, W, 8))
    x[..., :2] = rnd((B, D, H, W, 2), seed) * np.array([1.0, 0.5])
    return U.bf16_round(x)


def oracle_theta(seed):
    th = U.init_params(seed) * 0.8
    lay, _ = U.param_layout()
    for name, wo, ws, bo, co in lay:
        th[bo:bo + co] = rnd((co,), seed + wo % 101, -0.05, 0.1)
    return th.astype(np.float32).astype(np.float64)


def test_unet_forward_backward(q1):
    import torch
    B, D, H, W = 2, 8, 8, 12
    print(f"\n[unet] B={B} grid={D}x{H}x{W}", flush=True)
    th = oracle_theta(31)
    net = q1.UNet(D, H, W, B, seed=1)
    assert net.nparams == th.size
    net.set_params(f32(th))
    assert np.array_equal(host(net.get(0)), th)
    x = net_inputs(B, D, H, W, 32)
    xd = bf(x)
    out = torch.empty((B, D, H, W), dtype=torch.float32, device="cuda")
    net.forward(xd, out, B)
    ref, cache = U.unet_forward(th, x[..., :2], bf16=True)
    print(f"  forward: {normrel(host(out), ref):.2e}")
    # observed 1.5e-5: the two sides round the same BF16 activations at every layer
    assert normrel(host(out), ref) <= 1e-4, normrel(host(out), ref)
    # loss kernel on seeded values (not on the network output)
    o_s = rnd((B, D, H, W), 35).astype(np.float32).astype(np.float64)
    tgt = rnd((B, D, H, W), 33).astype(np.float32).astype(np.float64)
    wgt = (rnd((B, D, H, W), 34, 0, 1) > 0.25).astype(np.float64)
    dout = torch.empty_like(out)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.mse(f32(o_s), f32(tgt), f32(wgt), dout, loss)
    L_ref, g_ref = U.mse_loss(o_s, tgt, wgt)
    assert abs(float(loss.item()) - L_ref) <= 1e-5 * L_ref
    assert maxrel(host(dout), g_ref) <= 1e-5
    # parameter gradient for a seeded dL/dout, oracle on the same stored roundings
    g_out = (rnd((B, D, H, W), 36) * 1e-2).astype(np.float32).astype(np.float64)
    net.backward(f32(g_out))
    g = host(net.get(1))
    gr = U.unet_backward(th, cache, g_out, bf16=True)
    lay, _ = U.param_layout()
    for name, wo, ws, bo, co in lay:
        sz = int(np.prod(ws))
        e_w = normrel(g[wo:wo + sz], gr[wo:wo + sz])
        e_b = normrel(g[bo:bo + co], gr[bo:bo + co])
        print(f"  {name}: w {e_w:.2e} b {e_b:.2e}")
        # observed at most 1.1e-3 (the encoder's first levels, deepest in the
        # backward pass through BF16-rounded activations)
        assert e_w <= 4e-3 and e_b <= 4e-3, name


def test_unet_adam_step(q1):
    B, D, H, W = 1, 4, 4, 4
    th = oracle_theta(41)
    net = q1.UNet(D, H, W, B, seed=2)
    net.set_params(f32(th))
    g = rnd(th.shape, 44, -1e-2, 1e-2).astype(np.float32).astype(np.float64)
    m = np.zeros_like(g)
    v = np.zeros_like(g)
    ref = th
    for step in (1, 2, 3):
        net.set_grad(f32(g))
        net.adam_step(1e-3, step)
        ref, m, v = U.adam_step(ref, g, m, v, step, 1e-3, 0.9, 0.999, 1e-8)
        t = host(net.get(0))
        assert np.max(np.abs(t - ref)) <= 1e-6 * 1e-3 + 1e-6 * np.max(np.abs(th)), step
        g = g[::-1].copy()


def test_unet_training_lowers_the_loss(q1):
    import torch
    B, D, H, W = 2, 8, 8, 8
    print("\n[unet training]", flush=True)
    net = q1.UNet(D, H, W, B, seed=3)
    x = bf(net_inputs(B, D, H, W, 51))
    tgt = f32(rnd((B, D, H, W), 52) * 0.5)
    wgt = torch.ones_like(tgt)
    out = torch.empty_like(tgt)
    dout = torch.empty_like(tgt)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for step in range(1, 61):
        net.forward(x, out, B)
        net.mse(out, tgt, wgt, dout, loss)
        hist.append(float(loss.item()))
        net.backward(dout)
        net.adam_step(3e-3, step)
    print("  loss", hist[0], "->", hist[-1])
    assert all(np.isfinite(hist)) and hist[-1] < 0.5 * hist[0]


# -- the preconditioner ------------------------------------------------------------

def test_unet_encoding_and_precond(q1, orc):
    import torch
    nx, ny, nz = 6, 5, 4
    D, H, W = 8, 8, 8
    print("\n[unet precond encoding]", flush=True)
    k = si.field_lognormal(nx * ny * nz, 0.0, 2.0, 61)
    mask = si.face_mask(nx, ny, nz, "z0")
    nn = (nx + 1) * (ny + 1) * (nz + 1)
    r = si.vec_uniform(nn, 62, si.STREAM_RHS)
    free = mask == 0
    net = q1.UNet(D, H, W, 1, seed=4)
    th = oracle_theta(63)
    net.set_params(f32(th))
    kd = torch.from_numpy(k).cuda()
    md = torch.from_numpy(mask.astype(np.uint8)).cuda()
    pc = q1.UNetPrecond(net, nx, ny, nz, kd, md)
    rd = torch.from_numpy(r).cuda()
    inp = torch.zeros((D, H, W, 8), dtype=torch.bfloat16, device="cuda")
    pc.encode(rd, inp)
    kap = U.nodal_mean_log(nx, ny, nz, k)
    ref_in = U.encode_input(r, free, kap, nx, ny, nz, D, H, W)[0]
    got = host(inp)
    assert np.all(got[..., 2:] == 0)
    assert np.array_equal(got[..., :2], U.bf16_round(ref_in.astype(np.float32)))
    tg = torch.empty((D, H, W), dtype=torch.float32, device="cuda")
    wg = torch.empty_like(tg)
    pc.encode_target(rd, tg, wg)
    ref_t = U.encode_input(r, free, kap, nx, ny, nz, D, H, W)[0, ..., 0]
    assert maxrel(host(tg), ref_t) <= 1e-6
    ref_w = np.zeros((D, H, W))
    ref_w[:nz + 1, :ny + 1, :nx + 1] = free.reshape(nz + 1, ny + 1, nx + 1)
    assert np.array_equal(host(wg), ref_w)
    # z = decode(N(encode(r)))
    z = torch.empty_like(rd)
    assert q1.lib().q1_unet_precond(pc.handle, q1._dptr(rd), q1._dptr(z),
                                     q1._stream(None)) == 0
    out, _ = U.unet_forward(th, U.bf16_round(ref_in[None].astype(np.float32)), bf16=True)
    zr = U.decode_output(out, free, nx, ny, nz)
    print(f"  z: {normrel(host(z), zr):.2e}")
    assert normrel(host(z), zr) <= 1e-6  # observed 5.3e-8 (FP32 decode of the same network output)
    assert np.all(host(z)[~free] == 0)


def test_fpcg_with_untrained_network_still_converges(q1, orc):
    """An untrained network is a poor preconditioner; flexible PCG with its
    safeguards must still reach the tolerance under the oracle's operator."""
    import torch
    from helpers import make_op
    nx = ny = nz = 6
    print("\n[fpcg untrained net]", flush=True)
    xyz, conn = si.box_mesh(nx, ny, nz)
    k = si.field_lognormal(nx * ny * nz, 0.0, 2.0, 71)
    mask = si.face_mask(nx, ny, nz, "z0")
    pr = dict(physics=1, xyz=xyz, conn=conn, coef=k[None], mask=mask)
    A = orc.assemble(1, xyz, conn, k[None], mask)
    b = si.vec_uniform(A.n, 72, si.STREAM_RHS)
    b[mask == 1] = 0.0
    op = make_op(pr, 0, 0)
    net = q1.UNet(8, 8, 8, 1, seed=5)
    kd = torch.from_numpy(k).cuda()
    md = torch.from_numpy(mask.astype(np.uint8)).cuda()
    pc = q1.UNetPrecond(net, nx, ny, nz, kd, md)
    bd = torch.from_numpy(b).cuda()
    xd = torch.empty_like(bd)
    st = q1.q1_fpcg(op, pc, bd, xd, 1e-8, 2000, safeguard_m=20)
    assert st["status"] == 0
    assert orc.true_rel_res(A, xd.cpu().numpy(), b) <= 1e-8 * (1 + 1e-3)


def test_two_level_precond(q1, orc):
    """Two-level form against its composition from the oracle: damped Jacobi
    with the assembled diagonal, the network oracle as the correction, the
    energy-optimal scale, and the assembled operator."""
    import torch
    from helpers import make_op
    nx, ny, nz = 6, 5, 4
    D = H = W = 8
    omega = 0.6
    print("\n[unet two-level]", flush=True)
    xyz, conn = si.box_mesh(nx, ny, nz)
    k = si.field_lognormal(nx * ny * nz, 0.0, 2.0, 81)
    mask = si.face_mask(nx, ny, nz, "z0")
    free = mask == 0
    A = orc.assemble(1, xyz, conn, k[None], mask)
    r = si.vec_uniform(A.n, 82, si.STREAM_RHS)
    r[~free] = 0.0
    th = oracle_theta(83)
    net = q1.UNet(D, H, W, 1, seed=6)
    net.set_params(f32(th))
    op = make_op(dict(physics=1, xyz=xyz, conn=conn, coef=k[None], mask=mask), 0, 0)
    pc = q1.UNetPrecond(net, nx, ny, nz, torch.from_numpy(k).cuda(),
                        torch.from_numpy(mask.astype(np.uint8)).cuda())
    pc.two_level(op, omega)
    rd = torch.from_numpy(r).cuda()
    z = torch.empty_like(rd)
    assert q1.lib().q1_unet_precond(pc.handle, q1._dptr(rd), q1._dptr(z), q1._stream(None)) == 0
    # oracle composition
    w = 1.0 / A.diag()
    z1 = omega * w * r
    r1 = r - A.matvec(z1)
    kap = U.nodal_mean_log(nx, ny, nz, k)
    x_in = U.encode_input(r1, free, kap, nx, ny, nz, D, H, W)
    out, _ = U.unet_forward(th, U.bf16_round(x_in.astype(np.float32)), bf16=True)
    d = U.decode_output(out, free, nx, ny, nz)
    Ad = A.matvec(d)
    c = (d @ r1) / (d @ Ad)
    zr = z1 + c * d + omega * w * (r1 - c * Ad)
    print(f"  z: {normrel(host(z), zr):.2e}")
    assert normrel(host(z), zr) <= 1e-8  # observed 2.5e-10
    assert np.all(host(z)[~free] == 0)


def test_two_level_schedule(q1, orc):
    """With schedule period 3 the context evaluates the network on calls 0, 3, ...
    and the plain Jacobi step D^-1 r (the oracle's diagonal) on the others."""
    import torch
    from helpers import make_op
    nx, ny, nz = 6, 5, 4
    xyz, conn = si.box_mesh(nx, ny, nz)
    k = si.field_lognormal(nx * ny * nz, 0.0, 2.0, 85)
    mask = si.face_mask(nx, ny, nz, "z0")
    A = orc.assemble(1, xyz, conn, k[None], mask)
    r = si.vec_uniform(A.n, 86, si.STREAM_RHS)
    r[mask == 1] = 0.0
    net = q1.UNet(8, 8, 8, 1, seed=7)
    op = make_op(dict(physics=1, xyz=xyz, conn=conn, coef=k[None], mask=mask), 0, 0)
    pc = q1.UNetPrecond(net, nx, ny, nz, torch.from_numpy(k).cuda(),
                        torch.from_numpy(mask.astype(np.uint8)).cuda())
    with pytest.raises(q1.Q1Error):  # a period above 1 needs the two-level form
        pc.schedule(3)
    pc.two_level(op, 0.6)
    rd = torch.from_numpy(r).cuda()
    outs = []
    for per in (1, 3):
        pc.schedule(per)
        for _ in range(4):
            z = torch.empty_like(rd)
            assert q1.lib().q1_unet_precond(pc.handle, q1._dptr(rd), q1._dptr(z),
                                            q1._stream(None)) == 0
            outs.append(host(z))
    net_z = outs[0]
    assert all(np.array_equal(o, net_z) for o in outs[1:4])  # period 1: the network each call
    jac = r / A.diag()
    assert np.array_equal(outs[4], net_z) and np.array_equal(outs[7], net_z)
    for o in (outs[5], outs[6]):
        assert np.max(np.abs(o - jac)) <= 1e-15 * np.max(np.abs(jac))


def test_unet_pairs(q1, orc):
    """The training pairs against the oracle: e = x* - x_k, r = A e, then one
    damped-Jacobi step e1 = e - omega D^-1 r, r1 = A e1 (FP32 outputs)."""
    import torch
    from helpers import make_op
    n = 9
    xyz, conn = si.box_mesh(n, n, n)
    k = si.field_lognormal(n ** 3, 0.0, 2.0, 87)
    mask = si.face_mask(n, n, n, "z0")
    A = orc.assemble(1, xyz, conn, k[None], mask)
    b = si.vec_uniform(A.n, 88, si.STREAM_RHS)
    b[mask == 1] = 0.0
    op = make_op(dict(physics=1, xyz=xyz, conn=conn, coef=k[None], mask=mask), 0, 0)
    bd = torch.from_numpy(b).cuda()
    xs = torch.empty_like(bd)
    its = [1, 5, 20]
    snaps = [torch.empty_like(bd) for _ in its]
    q1.q1_pcg_trace(op, 1, bd, xs, 1e-12, 10000, its, snaps)
    for omega in (0.0, 0.6):
        e_out = [torch.empty(A.n, dtype=torch.float32, device="cuda") for _ in its]
        r_out = [torch.empty_like(e_out[0]) for _ in its]
        q1.q1_unet_pairs(op, xs, snaps, omega, e_out, r_out)
        torch.cuda.synchronize()
        for i in range(len(its)):
            e = xs.cpu().numpy() - snaps[i].cpu().numpy()
            r = A.matvec(e)
            if omega > 0:
                e = e - omega * r / A.diag()
                r = A.matvec(e)
            assert maxrel(host(e_out[i]), e) <= 1e-6
            assert normrel(host(r_out[i]), r) <= 1e-6
