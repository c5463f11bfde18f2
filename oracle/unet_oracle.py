"""Plain FP64 CPU oracle of the learned preconditioner's network.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it; the product library never imports or calls it, and
nothing here calls the product library.

The paper's conclusions (Section 7) name matrix-free preconditioners as
future work and say nothing of learned ones: the learned preconditioner is
this project's own addition.  What is computed here is the network this
project defines for it:

* a 3-level 3-D convolutional U-Net on the node grid, channels 16/32/64,
  3x3x3 zero-padded convolutions with bias, ReLU after every 3x3x3
  convolution, 2x2x2 average pooling down, nearest-neighbour 2x upsampling
  and channel concatenation with the skip tensor up, and a 1x1 head;
* the mean-squared error against a target field on a weighted set of nodes;
* Adam (Kingma and Ba, 2015) with bias correction;
* the input encoding of a residual r on a box mesh: r scaled to unit RMS over
  the free nodes and the nodal mean of ln k scaled by 1/2.

Everything is written as the definitions: a convolution is a sum over its 27
taps of a shifted input times a Cin x Cout matrix (the matrix product is a
library primitive), and each backward function is the adjoint of its forward
function written out.  Tensors are [B, D, H, W, C] (z, y, x, channel) in
float64; a convolution weight is [27, Cin, Cout] with tap
t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1).

Pins (CPU tests): convolutions against scipy.ndimage.correlate, every
gradient against central finite differences of the forward function, pooling
and upsampling against numpy.repeat and block means, Adam's first step against
its closed form, BF16 rounding against torch's conversion.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]

# name, input channels, output channels, grid level (1 = finest)
LAYERS = [
    ("enc1a", 2, 16, 1), ("enc1b", 16, 16, 1),
    ("enc2a", 16, 32, 2), ("enc2b", 32, 32, 2),
    ("enc3a", 32, 64, 3), ("enc3b", 64, 64, 3),
    ("dec2a", 64 + 32, 32, 2), ("dec2b", 32, 32, 2),
    ("dec1a", 32 + 16, 16, 1), ("dec1b", 16, 16, 1),
]
HEAD = ("head", 16, 1)
IN_CHANNELS = 2


def param_layout():
    """[(name, w_offset, w_shape, b_offset, cout)] of the flat parameter vector:
    per layer the weight [27, Cin, Cout] then the bias [Cout]; the head's weight
    is [Cin] then its bias [1]."""
    out, off = [], 0
    for name, ci, co, _ in LAYERS:
        out.append((name, off, (27, ci, co), off + 27 * ci * co, co))
        off += 27 * ci * co + co
    out.append((HEAD[0], off, (HEAD[1],), off + HEAD[1], 1))
    off += HEAD[1] + 1
    return out, off


def unpack_params(theta):
    lay, n = param_layout()
    assert theta.size == n
    P = {}
    for name, wo, ws, bo, co in lay:
        P[name] = (theta[wo:wo + int(np.prod(ws))].reshape(ws), theta[bo:bo + co])
    return P


def pack_grads(G):
    lay, n = param_layout()
    g = np.zeros(n)
    for name, wo, ws, bo, co in lay:
        gw, gb = G[name]
        g[wo:wo + int(np.prod(ws))] = gw.ravel()
        g[bo:bo + co] = gb
    return g


# -- BF16 storage ---------------------------------------------------------------

def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    The value is first rounded to float32, which is how the stored operands
    are produced on the other side as well."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


# -- elementary operators ---------------------------------------------------------

def shift(x, d):
    """y[b, z, y, x] = x[b, z + dz, y + dy, x + dx], zero outside the grid."""
    dz, dy, dx = d
    _, D, H, W, _ = x.shape
    y = np.zeros_like(x)
    zs, ys, xs = (slice(max(0, -dz), D - max(0, dz)), slice(max(0, -dy), H - max(0, dy)),
                  slice(max(0, -dx), W - max(0, dx)))
    zt, yt, xt = (slice(max(0, dz), D - max(0, -dz)), slice(max(0, dy), H - max(0, -dy)),
                  slice(max(0, dx), W - max(0, -dx)))
    y[:, zs, ys, xs] = x[:, zt, yt, xt]
    return y


def conv3d(x, w, b):
    """y = sum_t shift(x, t) W_t + b (3x3x3 'same' correlation with zero padding)."""
    y = np.zeros(x.shape[:4] + (w.shape[2],))
    for t, d in enumerate(TAPS):
        y += shift(x, d) @ w[t]
    return y + b


def conv3d_backward_data(gy, w):
    """Adjoint of x -> conv3d(x, w, 0): gx = sum_t shift(gy W_t^T, -t)."""
    gx = np.zeros(gy.shape[:4] + (w.shape[1],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        gx += shift(gy @ w[t].T, (-dz, -dy, -dx))
    return gx


def conv3d_backward_weight(x, gy):
    """dW_t = sum over voxels of shift(x, t)^T gy; db = sum over voxels of gy."""
    ci, co = x.shape[4], gy.shape[4]
    G = gy.reshape(-1, co)
    gw = np.zeros((27, ci, co))
    for t, d in enumerate(TAPS):
        gw[t] = shift(x, d).reshape(-1, ci).T @ G
    return gw, G.sum(axis=0)


def relu(x):
    return np.maximum(x, 0.0)


def pool2(x):
    """2x2x2 average pooling (even D, H, W)."""
    B, D, H, W, C = x.shape
    return x.reshape(B, D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4, 6))


def pool2_adjoint(g):
    """Adjoint of pool2: every fine voxel receives 1/8 of its parent's value."""
    return up2(g) / 8.0


def up2(x):
    """Nearest-neighbour 2x upsampling: the child voxel takes its parent's value."""
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def up2_adjoint(g):
    """Adjoint of up2: the parent receives the sum of its 8 children."""
    B, D, H, W, C = g.shape
    return g.reshape(B, D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4, 6))


# -- the network --------------------------------------------------------------------

def unet_forward(theta, x, bf16=False):
    """Network output [B, D, H, W] and the cache for the backward pass.

    With bf16=True the operands are rounded the way they are stored for the
    matrix cores: weights, every activation the convolutions read, and every
    pooled tensor to BF16; biases, the head and the output stay in full
    precision."""
    P = unpack_params(theta)
    rnd = bf16_round if bf16 else (lambda a: a)
    W = {k: (rnd(v[0]), v[1]) for k, v in P.items()}
    c = {"x": rnd(x)}

    def layer(name, inp):
        y = relu(conv3d(inp, *W[name]))
        c[name] = rnd(y)
        return c[name]

    s1 = layer("enc1b", layer("enc1a", c["x"]))
    c["p1"] = rnd(pool2(s1))
    s2 = layer("enc2b", layer("enc2a", c["p1"]))
    c["p2"] = rnd(pool2(s2))
    b3 = layer("enc3b", layer("enc3a", c["p2"]))
    c["cat2"] = np.concatenate([up2(b3), s2], axis=4)
    t2 = layer("dec2b", layer("dec2a", c["cat2"]))
    c["cat1"] = np.concatenate([up2(t2), s1], axis=4)
    t1 = layer("dec1b", layer("dec1a", c["cat1"]))
    wh, bh = P["head"]
    out = t1 @ wh + bh[0]
    return out, c


def unet_backward(theta, c, gout, bf16=False):
    """Gradient of the flat parameter vector for dL/dout = gout [B, D, H, W].

    With bf16=True the gradients that the matrix cores read (dL/d pre-activation
    of every convolution) are rounded to BF16, and the weights are the BF16
    copies used by the forward pass."""
    P = unpack_params(theta)
    rnd = bf16_round if bf16 else (lambda a: a)
    W = {k: rnd(v[0]) for k, v in P.items()}
    G = {}
    wh, _ = P["head"]
    t1 = c["dec1b"]
    G["head"] = ((t1 * gout[..., None]).reshape(-1, t1.shape[4]).sum(axis=0),
                 np.array([gout.sum()]))
    g = gout[..., None] * wh  # dL/d t1

    def back(name, inp, g_out, need_data=True):
        gpre = rnd(g_out * (c[name] > 0))
        gw, gb = conv3d_backward_weight(inp, gpre)
        G[name] = (gw, gb)
        return conv3d_backward_data(gpre, W[name]) if need_data else None

    g = back("dec1b", c["dec1a"], g)
    g = back("dec1a", c["cat1"], g)
    ct2 = P["dec2b"][0].shape[2]
    g_t2, g_s1 = up2_adjoint(g[..., :ct2]), g[..., ct2:]
    g = back("dec2b", c["dec2a"], g_t2)
    g = back("dec2a", c["cat2"], g)
    cb3 = P["enc3b"][0].shape[2]
    g_b3, g_s2 = up2_adjoint(g[..., :cb3]), g[..., cb3:]
    g = back("enc3b", c["enc3a"], g_b3)
    g = back("enc3a", c["p2"], g)
    g = back("enc2b", c["enc2a"], g_s2 + pool2_adjoint(g))
    g = back("enc2a", c["p1"], g)
    g = back("enc1b", c["enc1a"], g_s1 + pool2_adjoint(g))
    back("enc1a", c["x"], g, need_data=False)
    return pack_grads(G)


def mse_loss(out, target, weight):
    """L = sum(weight (out - target)^2) / sum(weight) and dL/dout."""
    den = weight.sum()
    d = out - target
    return float((weight * d * d).sum() / den), 2.0 * weight * d / den


def adam_step(theta, grad, m, v, step, lr, b1, b2, eps):
    """One Adam step (step counts from 1) with bias-corrected moments."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; a reference set
    for tests (the library draws its own initial weights)."""
    rng = np.random.default_rng(seed)
    lay, n = param_layout()
    th = np.zeros(n)
    for name, wo, ws, bo, co in lay:
        fan_in = int(np.prod(ws[:-1])) if len(ws) == 3 else ws[0]
        th[wo:wo + int(np.prod(ws))] = rng.standard_normal(int(np.prod(ws))) * np.sqrt(2.0 / fan_in)
    return th


# -- input encoding of a residual on a box mesh ---------------------------------------

def nodal_mean_log(nx, ny, nz, k):
    """Mean of ln k over the cells adjacent to each node; k is per cell, cells
    x-fastest, nodes x-fastest."""
    lk = np.log(np.asarray(k, dtype=np.float64)).reshape(nz, ny, nx)
    s = np.zeros((nz + 1, ny + 1, nx + 1))
    n = np.zeros_like(s)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                s[dz:dz + nz, dy:dy + ny, dx:dx + nx] += lk
                n[dz:dz + nz, dy:dy + ny, dx:dx + nx] += 1.0
    return (s / n).ravel()


def encode_input(r, free, kappa, nx, ny, nz, D, H, W):
    """Input [1, D, H, W, 2]: channel 0 is r on the free nodes scaled to unit
    RMS over them, channel 1 is kappa / 2 on every mesh node; the node grid
    sits at the origin of the D x H x W grid and the rest is zero."""
    free = np.asarray(free, dtype=bool)
    nf = free.sum()
    rr = np.where(free, r, 0.0)
    nrm = np.sqrt((rr * rr).sum())
    x = np.zeros((1, D, H, W, 2))
    g = (nz + 1, ny + 1, nx + 1)
    x[0, :g[0], :g[1], :g[2], 0] = (rr * (np.sqrt(nf) / nrm if nrm > 0 else 0.0)).reshape(g)
    x[0, :g[0], :g[1], :g[2], 1] = (np.asarray(kappa) / 2.0).reshape(g)
    return x


def decode_output(out, free, nx, ny, nz):
    """z on the nodes: the network output on free nodes, zero on Dirichlet nodes."""
    g = (nz + 1, ny + 1, nx + 1)
    z = out[0, :g[0], :g[1], :g[2]].ravel().copy()
    z[~np.asarray(free, dtype=bool)] = 0.0
    return z
