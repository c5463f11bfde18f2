"""Pins of the network oracle to facts outside its own code: a library
correlation for the convolution, central finite differences for every
gradient (the network is piecewise quadratic in each parameter, so central
differences are exact up to rounding away from ReLU kinks), explicit loops
for pooling and upsampling, the closed form of Adam's first steps, and torch's
own float -> bfloat16 conversion for the rounding."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import unet_oracle as U


def rnd(shape, seed, lo=-1.0, hi=1.0):
    n = int(np.prod(shape))
    return (lo + (hi - lo) * si.uniform(seed, si.STREAM_X, np.arange(n, dtype=np.uint64))).reshape(shape)


def test_bf16_round_matches_torch():
    import torch
    x = np.concatenate([rnd((4000,), 1, -3, 3), np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8,
                                                          -1.0 - 2.0 ** -8, 0.0, 65504.0])])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(U.bf16_round(x), ref)


def test_conv3d_matches_library_correlation():
    from scipy import ndimage
    x = rnd((2, 5, 6, 7, 3), 2)
    w = rnd((27, 3, 4), 3)
    b = rnd((4,), 4)
    y = U.conv3d(x, w, b)
    for bi in range(2):
        for co in range(4):
            ref = b[co] + sum(ndimage.correlate(x[bi, ..., ci], w[:, ci, co].reshape(3, 3, 3),
                                                mode="constant", cval=0.0) for ci in range(3))
            assert np.max(np.abs(y[bi, ..., co] - ref)) <= 1e-13


def test_conv3d_delta_kernel_is_a_shift():
    x = rnd((1, 4, 5, 6, 2), 5)
    for t in (0, 4, 13, 22, 26):
        w = np.zeros((27, 2, 2))
        w[t] = np.eye(2)
        dz, dy, dx = U.TAPS[t]
        y = U.conv3d(x, w, np.zeros(2))
        for z in range(4):
            for yy in range(5):
                for xx in range(6):
                    zz, y2, x2 = z + dz, yy + dy, xx + dx
                    inside = 0 <= zz < 4 and 0 <= y2 < 5 and 0 <= x2 < 6
                    ref = x[0, zz, y2, x2] if inside else np.zeros(2)
                    assert np.array_equal(y[0, z, yy, xx], ref)


def central(f, v, i, h=1e-5):
    old = v.flat[i]
    v.flat[i] = old + h
    fp = f()
    v.flat[i] = old - h
    fm = f()
    v.flat[i] = old
    return (fp - fm) / (2 * h)


def test_conv_gradients_by_finite_differences():
    x = rnd((2, 4, 5, 3, 3), 6)
    w = rnd((27, 3, 5), 7)
    b = rnd((5,), 8)
    gy = rnd((2, 4, 5, 3, 5), 9)
    f = lambda: float((U.conv3d(x, w, b) * gy).sum())
    gx = U.conv3d_backward_data(gy, w)
    gw, gb = U.conv3d_backward_weight(x, gy)
    for arr, g in ((x, gx), (w, gw), (b, gb)):
        for i in np.linspace(0, arr.size - 1, 23).astype(int):
            assert abs(central(f, arr, i) - g.flat[i]) <= 1e-7 * (1 + abs(g.flat[i]))


def test_pool_and_upsample_by_loops():
    x = rnd((2, 4, 6, 2, 3), 10)
    p = U.pool2(x)
    u = U.up2(p)
    for b in range(2):
        for z in range(2):
            for y in range(3):
                for xx in range(1):
                    blk = x[b, 2 * z:2 * z + 2, 2 * y:2 * y + 2, 2 * xx:2 * xx + 2]
                    assert np.allclose(p[b, z, y, xx], blk.reshape(-1, 3).mean(axis=0), atol=1e-15)
                    for c in range(8):
                        assert np.array_equal(u[b, 2 * z + (c >> 2), 2 * y + ((c >> 1) & 1),
                                                2 * xx + (c & 1)], p[b, z, y, xx])
    # adjoints: <pool x, g> = <x, pool^T g>, <up p, g> = <p, up^T g>
    g = rnd(p.shape, 11)
    assert abs((p * g).sum() - (x * U.pool2_adjoint(g)).sum()) <= 1e-12
    g2 = rnd(u.shape, 12)
    assert abs((u * g2).sum() - (p * U.up2_adjoint(g2)).sum()) <= 1e-12


def test_param_layout_counts():
    lay, n = U.param_layout()
    expect = sum(27 * ci * co + co for _, ci, co, _ in U.LAYERS) + 17
    assert n == expect == 353713
    assert lay[0][2] == (27, 2, 16) and lay[6][2] == (27, 96, 32) and lay[-1][2] == (16,)


@pytest.mark.parametrize("bf16", [False])
def test_unet_gradient_by_finite_differences(bf16):
    th = U.init_params(3) * 0.7
    lay, n = U.param_layout()
    x = rnd((2, 4, 4, 8, 2), 13)
    tgt = rnd((2, 4, 4, 8), 14)
    wgt = (rnd((2, 4, 4, 8), 15, 0, 1) > 0.3).astype(np.float64)
    # biases away from zero so that ReLU kinks are not straddled
    for name, wo, ws, bo, co in lay:
        th[bo:bo + co] = rnd((co,), 16 + wo % 97, 0.05, 0.2)

    def loss():
        out, _ = U.unet_forward(th, x)
        return U.mse_loss(out, tgt, wgt)[0]

    out, cache = U.unet_forward(th, x)
    _, gout = U.mse_loss(out, tgt, wgt)
    g = U.unet_backward(th, cache, gout)
    scale = np.max(np.abs(g))
    idx = []
    for name, wo, ws, bo, co in lay:
        sz = int(np.prod(ws))
        idx += list(wo + np.linspace(0, sz - 1, 4).astype(int)) + [bo, bo + co - 1]
    for i in idx:
        fd = central(loss, th, i, h=1e-6)
        assert abs(fd - g[i]) <= 1e-6 * abs(g[i]) + 1e-8 * scale, (i, fd, g[i])


def test_mse_gradient():
    o, t = rnd((1, 2, 2, 4), 17), rnd((1, 2, 2, 4), 18)
    w = np.ones_like(o)
    L, g = U.mse_loss(o, t, w)
    assert abs(L - np.mean((o - t) ** 2)) <= 1e-15
    w = (rnd(o.shape, 19, 0, 1) > 0.5).astype(float)
    f = lambda: U.mse_loss(o, t, w)[0]
    L, g = U.mse_loss(o, t, w)
    for i in range(o.size):
        assert abs(central(f, o, i) - g.flat[i]) <= 1e-9


def test_adam_closed_form():
    th = rnd((50,), 20)
    g = rnd((50,), 21)
    m = np.zeros(50)
    v = np.zeros(50)
    lr, eps = 1e-3, 1e-8
    t1, m, v = U.adam_step(th, g, m, v, 1, lr, 0.9, 0.999, eps)
    assert np.allclose(t1, th - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    # with a constant gradient the bias-corrected moments are exact, so every
    # step moves by the same amount
    t = t1
    for s in range(2, 6):
        t_new, m, v = U.adam_step(t, g, m, v, s, lr, 0.9, 0.999, eps)
        assert np.allclose(t - t_new, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)
        t = t_new


def test_nodal_mean_log_and_encoding():
    nx, ny, nz = 3, 2, 2
    k = np.full(nx * ny * nz, np.e ** 1.5)
    assert np.allclose(U.nodal_mean_log(nx, ny, nz, k), 1.5, atol=1e-15)
    # one cell different: a corner node sees only cell 0
    k = np.ones(nx * ny * nz)
    k[0] = np.e ** 4
    kap = U.nodal_mean_log(nx, ny, nz, k)
    assert abs(kap[0] - 4.0) <= 1e-15 and abs(kap[1] - 2.0) <= 1e-15  # node 1 touches cells 0, 1
    assert abs(kap[(nx + 1) * (ny + 1) + (nx + 1) + 1] - 0.5) <= 1e-15  # centre node: 8 cells
    nn = (nx + 1) * (ny + 1) * (nz + 1)
    r = rnd((nn,), 22)
    free = np.ones(nn, dtype=bool)
    free[: (nx + 1) * (ny + 1)] = False
    x = U.encode_input(r, free, kap, nx, ny, nz, 4, 4, 8)
    ch0 = x[0, :nz + 1, :ny + 1, :nx + 1, 0].ravel()
    assert abs(np.sqrt(np.mean(ch0[free] ** 2)) - 1.0) <= 1e-14 and np.all(ch0[~free] == 0)
    assert np.all(x[0, nz + 1:] == 0) and np.all(x[0, :, :, nx + 1:] == 0)
    z = U.decode_output(x[..., 0], free, nx, ny, nz)
    assert np.array_equal(z, ch0)
