"""MI355X-native matrix-free Q1 hexahedral finite-element operators.

Thin Python binding of ``libq1mf.so`` (C ABI in ``include/q1mf.h``).  The
functions keep the C names; they only marshal arguments: torch tensors are
passed as raw device pointers, numpy arrays as host pointers, and the current
torch (HIP) stream is used unless one is given.  Every computation runs in
the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import sys

import numpy as np

from . import _lib as _libmod
from ._lib import (PRECOND_FN, Q1_EBREAKDOWN, Q1_ELASTICITY, Q1_ENOCONV, Q1_F32, Q1_F64,
                   Q1_HEX8, Q1_HEX27, Q1_HEX64, Q1_TET4,
                   Q1_LAPLACE, Q1_OK, Q1_VLAPLACE, Q1_PC_JACOBI, Q1_PC_NONE, Q1_V_ATOMIC, Q1_V_AUTO, Q1_V_COLOR,
                   Q1_V_CSR, Q1_V_LDS_TILE, Q1Error, Q1Stats, check, last_error, lib)

__all__ = [
    "Q1_PC_NONE", "Q1_PC_JACOBI", "q1_dot", "Q1_DOT_TWO_STAGE", "Q1_DOT_ATOMIC", "Q1Stats", "q1_pcg", "q1_pcg_noalloc", "Q1_NOALLOC_MAX_DOF", "q1_pcg_fused", "q1_pcg_trace", "q1_batched_pcg", "q1_batched_mpcg", "q1_mpcg", "q1_fpcg", "q1_fcg", "q1_ir_solve", "Jacobi",
    "q1_jacobi_create", "Q1_OK", "Q1_ENOCONV", "Q1_EBREAKDOWN", "Q1Error", "Q1_LAPLACE", "Q1_VLAPLACE", "Q1_ELASTICITY", "Q1_F64", "Q1_F32", "Q1_V_AUTO", "Q1_V_ATOMIC",
    "Q1_V_COLOR", "Q1_V_LDS_TILE", "Q1_V_CSR", "q1_csr_create", "q1_csr_info", "q1_csr_export", "lib", "last_error", "q1_version", "q1_box_sizes", "q1_box_mesh",
    "q1_face_mask", "q1_field_lognormal", "q1_field_layered", "q1_field_elastic",
    "q1_lame_from_E_nu", "q1_vec_uniform", "q1_op_create", "q1_op_create_elem", "Q1_HEX8", "Q1_TET4", "Q1_HEX27", "Q1_HEX64", "q1_op_apply", "q1_op_diag",
    "q1_op_info", "q1_op_bytes", "q1_op_reproducible", "q1_op_destroy", "q1_model_bytes", "Op",
    "q1_conv3d_forward", "q1_conv3d_backward_data", "q1_conv3d_backward_weight", "UNet",
    "q1_unet_create", "UNetPrecond", "q1_unet_pc_create", "q1_unet_pairs",
]


# ---- helpers -------------------------------------------------------------

def _hptr(a: np.ndarray) -> ctypes.c_void_p:
    return a.ctypes.data_as(ctypes.c_void_p)


def _dptr(t) -> ctypes.c_void_p | None:
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device (cuda/HIP) tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def q1_version() -> int:
    return lib().q1_version()


# ---- generators (host) ---------------------------------------------------

def q1_box_sizes(nx: int, ny: int, nz: int) -> tuple[int, int]:
    nn, ne = ctypes.c_int64(), ctypes.c_int64()
    check(lib().q1_box_sizes(nx, ny, nz, ctypes.byref(nn), ctypes.byref(ne)))
    return nn.value, ne.value


def q1_box_mesh(nx, ny, nz, h=1.0, jitter_frac=0.0, seed=0):
    nn, ne = q1_box_sizes(nx, ny, nz)
    xyz = np.empty((3, nn)); conn = np.empty((8, ne), dtype=np.int32)
    check(lib().q1_box_mesh(nx, ny, nz, h, jitter_frac, seed, _hptr(xyz), _hptr(conn)))
    return xyz, conn


def q1_face_mask(nx, ny, nz, face: int):
    nn, _ = q1_box_sizes(nx, ny, nz)
    m = np.empty(nn, dtype=np.uint8)
    check(lib().q1_face_mask(nx, ny, nz, face, _hptr(m)))
    return m


def q1_field_lognormal(n, mu, sigma, seed, stream=1):
    out = np.empty(n)
    check(lib().q1_field_lognormal(n, mu, sigma, seed, stream, _hptr(out)))
    return out


def q1_field_layered(nx, ny, nz, layer_cells, s_layer, s_cell, seed):
    out = np.empty(nx * ny * nz)
    check(lib().q1_field_layered(nx, ny, nz, layer_cells, s_layer, s_cell, seed, _hptr(out)))
    return out


def q1_field_elastic(n, seed):
    E = np.empty(n); nu = np.empty(n)
    check(lib().q1_field_elastic(n, seed, _hptr(E), _hptr(nu)))
    return E, nu


def q1_lame_from_E_nu(E, nu):
    E = np.ascontiguousarray(E, dtype=np.float64); nu = np.ascontiguousarray(nu, dtype=np.float64)
    lam = np.empty_like(E); mu = np.empty_like(E)
    check(lib().q1_lame_from_E_nu(E.size, _hptr(E), _hptr(nu), _hptr(lam), _hptr(mu)))
    return lam, mu


def q1_vec_uniform(n, seed, stream, lo=-1.0, hi=1.0):
    out = np.empty(n)
    check(lib().q1_vec_uniform(n, seed, stream, lo, hi, _hptr(out)))
    return out


def q1_model_bytes(kind: int, physics: int, real_bytes: int, coef_bytes: int, n_nodes: int,
                   n_elems: int, cache: int) -> float:
    b = ctypes.c_double()
    check(lib().q1_model_bytes(kind, physics, real_bytes, coef_bytes, n_nodes, n_elems, cache,
                               ctypes.byref(b)))
    return b.value


# ---- operators -----------------------------------------------------------

class Op:
    """Owning wrapper of a ``q1_op*``; keeps the referenced tensors alive."""

    def __init__(self, handle: ctypes.c_void_p, keep: tuple):
        self.handle = handle
        self._keep = keep

    def apply(self, x, y, stream=None):
        return q1_op_apply(self, x, y, stream)

    def diag(self, d, stream=None):
        return q1_op_diag(self, d, stream)

    def info(self):
        return q1_op_info(self)

    def bytes(self):
        return q1_op_bytes(self)

    def reproducible(self) -> bool:
        return q1_op_reproducible(self)

    def destroy(self):
        if self.handle:
            q1_op_destroy(self)

    def __del__(self):
        # at interpreter shutdown the process releases device memory itself:
        # no library call is made from a finaliser then (and once the module's
        # globals are cleared, the check itself raises and is ignored)
        try:
            if _can_release():
                self.destroy()
        except Exception:
            pass


def q1_op_create(physics: int, dtype: int, variant: int, xyz, conn, coef, mask=None,
                 stream=None) -> Op:
    """xyz [3, n_nodes], conn int32 [8, n_elems], coef [ncoef, n_elems], mask uint8 [n_nodes]:
    device tensors of the operator's dtype (conn and mask excepted)."""
    h = ctypes.c_void_p()
    n_nodes = xyz.shape[-1]
    n_elems = conn.shape[-1]
    check(lib().q1_op_create(ctypes.byref(h), physics, dtype, variant, n_nodes, n_elems,
                             _dptr(xyz), _dptr(conn), _dptr(coef), _dptr(mask), _stream(stream)))
    return Op(h, (xyz, conn, coef, mask))


def q1_op_create_elem(elem: int, physics: int, dtype: int, variant: int, xyz, conn, coef,
                      mask=None, stream=None) -> Op:
    """Operator of an element family: Q1_HEX8 (conn [8, n_elems]), Q1_TET4
    (conn [4, n_elems]), Q1_HEX27 (conn [27, n_elems]) or Q1_HEX64 (conn [64, n_elems])."""
    h = ctypes.c_void_p()
    n_nodes = xyz.shape[-1]
    n_elems = conn.shape[-1]
    check(lib().q1_op_create_elem(ctypes.byref(h), elem, physics, dtype, variant, n_nodes, n_elems,
                                  _dptr(xyz), _dptr(conn), _dptr(coef), _dptr(mask),
                                  _stream(stream)))
    return Op(h, (xyz, conn, coef, mask))


def q1_op_apply(op: Op, x, y, stream=None) -> None:
    check(lib().q1_op_apply(op.handle, _dptr(x), _dptr(y), _stream(stream)))


def q1_op_diag(op: Op, d, stream=None) -> None:
    check(lib().q1_op_diag(op.handle, _dptr(d), _stream(stream)))


def q1_op_info(op: Op) -> dict:
    ph, dt, va = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    nn, ne = ctypes.c_int64(), ctypes.c_int64()
    check(lib().q1_op_info(op.handle, ctypes.byref(ph), ctypes.byref(dt), ctypes.byref(va),
                           ctypes.byref(nn), ctypes.byref(ne)))
    return dict(physics=ph.value, dtype=dt.value, variant=va.value, n_nodes=nn.value,
                n_elems=ne.value)


def q1_op_bytes(op: Op) -> tuple[float, float]:
    b, f = ctypes.c_double(), ctypes.c_double()
    check(lib().q1_op_bytes(op.handle, ctypes.byref(b), ctypes.byref(f)))
    return b.value, f.value


def q1_op_reproducible(op: Op) -> bool:
    r = ctypes.c_int()
    check(lib().q1_op_reproducible(op.handle, ctypes.byref(r)))
    return bool(r.value)


def q1_op_destroy(op: Op) -> None:
    if op.handle:
        check(lib().q1_op_destroy(op.handle))
        op.handle = ctypes.c_void_p()


# ---- CSR comparison --------------------------------------------------------

def q1_csr_create(like: Op, stream=None) -> Op:
    h = ctypes.c_void_p()
    check(lib().q1_csr_create(ctypes.byref(h), like.handle, _stream(stream)))
    return Op(h, like._keep)


def q1_csr_info(op: Op) -> tuple[int, int]:
    nr, nz = ctypes.c_int64(), ctypes.c_int64()
    check(lib().q1_csr_info(op.handle, ctypes.byref(nr), ctypes.byref(nz)))
    return nr.value, nz.value


def q1_csr_export(op: Op):
    """(rowptr int32, col int32, val) as host numpy arrays."""
    nr, nz = q1_csr_info(op)
    info = q1_op_info(op)
    rowptr = np.empty(nr + 1, dtype=np.int32)
    col = np.empty(nz, dtype=np.int32)
    val = np.empty(nz, dtype=np.float64 if info["dtype"] == Q1_F64 else np.float32)
    check(lib().q1_csr_export(op.handle, _hptr(rowptr), _hptr(col), _hptr(val)))
    return rowptr, col, val


# ---- solvers ---------------------------------------------------------------

def _solve_rc(rc: int) -> int:
    """Non-convergence and breakdown are outcomes reported in the stats."""
    if rc not in (Q1_OK, Q1_ENOCONV, Q1_EBREAKDOWN):
        check(rc)
    return rc


Q1_DOT_TWO_STAGE = 0
Q1_DOT_ATOMIC = 1
Q1_NOALLOC_MAX_DOF = 3145728  # the static workspace of q1_pcg_noalloc (include/q1mf.h)


def q1_dot(a, b, out, variant: int = Q1_DOT_TWO_STAGE, nblocks: int = 0, work=None,
           stream=None) -> None:
    """out (device FP64 scalar tensor) = a.b for device vectors a, b (FP64 or FP32);
    work: device FP64 buffer of >= 1024 entries for the two-stage variant."""
    import torch
    dtype = Q1_F64 if a.dtype == torch.float64 else Q1_F32
    check(lib().q1_dot(a.numel(), dtype, _dptr(a), _dptr(b), _dptr(out), variant, nblocks,
                       _dptr(work), _stream(stream)))


def q1_pcg(op: Op, pc: int, b, x, rtol: float, maxit: int, stream=None) -> dict:
    st = Q1Stats()
    _solve_rc(lib().q1_pcg(op.handle, pc, _dptr(b), _dptr(x), rtol, maxit, ctypes.byref(st),
                           _stream(stream)))
    return st.as_dict()


def q1_pcg_noalloc(op: Op, pc: int, b, x, rtol: float, maxit: int, stream=None) -> dict:
    """q1_pcg with its workspace in the library's static device array (no allocation)."""
    st = Q1Stats()
    _solve_rc(lib().q1_pcg_noalloc(op.handle, pc, _dptr(b), _dptr(x), rtol, maxit,
                                   ctypes.byref(st), _stream(stream)))
    return st.as_dict()


def q1_pcg_trace(op: Op, pc: int, b, x, rtol: float, maxit: int, snap_iters, snaps,
                 stream=None) -> dict:
    """q1_pcg recording x after the given iterations into the device vectors `snaps`."""
    n = len(snap_iters)
    it = (ctypes.c_int * max(n, 1))(*[int(k) for k in snap_iters])
    ptr = (ctypes.c_void_p * max(n, 1))(*[_dptr(v) for v in snaps])
    st = Q1Stats()
    _solve_rc(lib().q1_pcg_trace(op.handle, pc, _dptr(b), _dptr(x), rtol, maxit, n, it, ptr,
                                 ctypes.byref(st), _stream(stream)))
    return st.as_dict()


class Jacobi:
    """Device Jacobi preconditioner (z = D^{-1} r) usable with q1_fpcg."""

    def __init__(self, op: Op, stream=None):
        self.handle = ctypes.c_void_p()
        check(lib().q1_jacobi_create(ctypes.byref(self.handle), op.handle, _stream(stream)))
        self._op = op
        self.fn = ctypes.cast(lib().q1_precond_jacobi, ctypes.c_void_p)

    def destroy(self):
        if self.handle:
            lib().q1_jacobi_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            if _can_release():
                self.destroy()
        except Exception:
            pass


def q1_jacobi_create(op: Op, stream=None) -> Jacobi:
    return Jacobi(op, stream)


def q1_fpcg(op: Op, precond, b, x, rtol: float, maxit: int, safeguard_m: int = 0,
            stream=None, trunc_m: int = 1) -> dict:
    """precond: a Jacobi/learned preconditioner object with .fn and .handle, a
    (function pointer, ctx) pair, or a Python callable f(r_ptr, z_ptr, stream_ptr) -> int
    that enqueues z = M(r) on the stream.  trunc_m > 1 runs FCG(trunc_m) (q1_fcg)."""
    keep = None
    if hasattr(precond, "fn") and hasattr(precond, "handle"):
        fn, ctx = precond.fn, precond.handle
    elif isinstance(precond, tuple):
        fn, ctx = precond
    elif precond is None:
        fn, ctx = None, None
    else:
        def _cb(_ctx, r, z, s, _f=precond):
            try:
                return int(_f(r, z, s))
            except Exception:
                return -1
        keep = PRECOND_FN(_cb)
        fn, ctx = ctypes.cast(keep, ctypes.c_void_p), None
    st = Q1Stats()
    if trunc_m == 1:
        _solve_rc(lib().q1_fpcg(op.handle, fn, ctx, _dptr(b), _dptr(x), rtol, maxit, safeguard_m,
                                ctypes.byref(st), _stream(stream)))
    else:
        _solve_rc(lib().q1_fcg(op.handle, fn, ctx, _dptr(b), _dptr(x), rtol, maxit, safeguard_m,
                               trunc_m, ctypes.byref(st), _stream(stream)))
    del keep
    return st.as_dict()


def q1_fcg(op: Op, precond, b, x, rtol: float, maxit: int, safeguard_m: int = 0,
           trunc_m: int = 4, stream=None) -> dict:
    """Flexible CG with truncated orthogonalisation against the last trunc_m directions."""
    return q1_fpcg(op, precond, b, x, rtol, maxit, safeguard_m, stream, trunc_m)


def q1_mpcg(op64: Op, op32: Op, b, x, rtol: float, delta: float = 0.1, maxit: int = 50000,
            stream=None) -> dict:
    st = Q1Stats()
    _solve_rc(lib().q1_mpcg(op64.handle, op32.handle, _dptr(b), _dptr(x), rtol, delta, maxit,
                            ctypes.byref(st), _stream(stream)))
    return st.as_dict()


def q1_pcg_fused(op: Op, pc: int, b, x, rtol: float, maxit: int, stream=None) -> dict:
    """Jacobi-PCG in one launch of one workgroup (small problems: the DOF vector
    must fit in 64 KB of LDS)."""
    st = Q1Stats()
    _solve_rc(lib().q1_pcg_fused(op.handle, pc, _dptr(b), _dptr(x), rtol, maxit,
                                 ctypes.byref(st), _stream(stream)))
    return st.as_dict()


def q1_ir_solve(op64: Op, op32: Op, b, x, rtol: float, inner_rtol: float = 1e-4,
                max_outer: int = 50, max_inner: int = 20000, stream=None) -> dict:
    st = Q1Stats()
    _solve_rc(lib().q1_ir_solve(op64.handle, op32.handle, _dptr(b), _dptr(x), rtol, inner_rtol,
                                max_outer, max_inner, ctypes.byref(st), _stream(stream)))
    return st.as_dict()


def q1_batched_pcg(ops, b, x, rtol: float, maxit: int, stream=None) -> list[dict]:
    """ops: list of operators; b, x: lists (one per problem) of lists of
    nrhs device vectors.  One persistent kernel solves all of them."""
    nprob = len(ops)
    nrhs = len(b[0])
    VP = ctypes.c_void_p
    opa = (VP * nprob)(*[o.handle for o in ops])
    ba = (VP * (nprob * nrhs))(*[_dptr(v) for row in b for v in row])
    xa = (VP * (nprob * nrhs))(*[_dptr(v) for row in x for v in row])
    st = (Q1Stats * (nprob * nrhs))()
    _solve_rc(lib().q1_batched_pcg(nprob, ctypes.cast(opa, VP), nrhs, ctypes.cast(ba, VP),
                                   ctypes.cast(xa, VP), rtol, maxit, ctypes.cast(st, VP),
                                   _stream(stream)))
    return [s_.as_dict() for s_ in st]


def q1_batched_mpcg(ops, b, x, rtol: float, maxit: int, delta: float = 0.1,
                    stream=None) -> list[dict]:
    """Mixed-precision batched PCG (FP32 applies and directions, FP64 x, r,
    dots and true-residual refreshes), same layout as q1_batched_pcg."""
    nprob = len(ops)
    nrhs = len(b[0])
    VP = ctypes.c_void_p
    opa = (VP * nprob)(*[o.handle for o in ops])
    ba = (VP * (nprob * nrhs))(*[_dptr(v) for row in b for v in row])
    xa = (VP * (nprob * nrhs))(*[_dptr(v) for row in x for v in row])
    st = (Q1Stats * (nprob * nrhs))()
    _solve_rc(lib().q1_batched_mpcg(nprob, ctypes.cast(opa, VP), nrhs, ctypes.cast(ba, VP),
                                    ctypes.cast(xa, VP), rtol, delta, maxit, ctypes.cast(st, VP),
                                    _stream(stream)))
    return [s_.as_dict() for s_ in st]


# ---- learned preconditioner ------------------------------------------------------

def q1_conv3d_forward(a, ca: int, w, cout: int, bias=None, b=None, cb: int = 0, up_a: int = 0,
                      relu: int = 0, y=None, stream=None):
    """y (FP32 [B, D, H, W, cout]) = conv3d(concat(up?(a), b)); a, b BF16 channel-last;
    the output grid is b's, or a's (doubled when up_a)."""
    import torch
    ref = b if b is not None else a
    B, D, H, W = ref.shape[:4]
    if b is None and up_a:
        D, H, W = 2 * D, 2 * H, 2 * W
    if y is None:
        y = torch.empty((B, D, H, W, cout), dtype=torch.float32, device=a.device)
    check(lib().q1_conv3d_forward(B, D, H, W, _dptr(a), ca, up_a, _dptr(b), cb, _dptr(w),
                                  _dptr(bias), cout, relu, _dptr(y), _stream(stream)))
    return y


def q1_conv3d_backward_data(gy, cout: int, w, cin: int, stream=None):
    import torch
    B, D, H, W = gy.shape[:4]
    gx = torch.empty((B, D, H, W, cin), dtype=torch.float32, device=gy.device)
    check(lib().q1_conv3d_backward_data(B, D, H, W, _dptr(gy), cout, _dptr(w), cin, _dptr(gx),
                                        _stream(stream)))
    return gx


def q1_conv3d_backward_weight(a, ca: int, gy, cout: int, b=None, cb: int = 0, up_a: int = 0,
                              stream=None):
    import torch
    B, D, H, W = gy.shape[:4]
    gw = torch.empty((27, ca + cb, cout), dtype=torch.float32, device=gy.device)
    gb = torch.empty((cout,), dtype=torch.float32, device=gy.device)
    check(lib().q1_conv3d_backward_weight(B, D, H, W, _dptr(a), ca, up_a, _dptr(b), cb, _dptr(gy),
                                          cout, _dptr(gw), _dptr(gb), _stream(stream)))
    return gw, gb


class UNet:
    """Handle of the network (q1_unet_*).  theta/grad are views of the
    library's FP32 parameter and gradient vectors."""

    def __init__(self, D: int, H: int, W: int, batch: int, seed: int = 0, stream=None):
        import torch
        self.handle = ctypes.c_void_p()
        check(lib().q1_unet_create(ctypes.byref(self.handle), D, H, W, batch, seed,
                                   _stream(stream)))
        n = ctypes.c_int64()
        check(lib().q1_unet_info(self.handle, ctypes.byref(n), None, None, None, None))
        self.nparams, self.D, self.H, self.W, self.batch = n.value, D, H, W, batch

    def get(self, which: int = 0, stream=None):
        """Copy of the parameters (which=0) or gradients (which=1), FP32 on the device."""
        import torch
        buf = torch.empty(self.nparams, dtype=torch.float32, device="cuda")
        check(lib().q1_unet_copy(self.handle, which, 0, _dptr(buf), _stream(stream)))
        return buf

    def set_params(self, theta, stream=None):
        """Overwrite the parameters from a device FP32 vector and repack."""
        check(lib().q1_unet_copy(self.handle, 0, 1, _dptr(theta), _stream(stream)))
        self.commit(stream)

    def set_grad(self, grad, stream=None):
        """Overwrite the gradient vector (e.g. with gradients summed elsewhere)."""
        check(lib().q1_unet_copy(self.handle, 1, 1, _dptr(grad), _stream(stream)))

    def commit(self, stream=None):
        check(lib().q1_unet_commit(self.handle, _stream(stream)))

    def forward(self, inp, out, nbatch: int, stream=None):
        check(lib().q1_unet_forward(self.handle, _dptr(inp), _dptr(out), nbatch, _stream(stream)))

    def mse(self, out, target, weight, dout, loss=None, stream=None):
        check(lib().q1_unet_mse(self.handle, _dptr(out), _dptr(target), _dptr(weight), _dptr(dout),
                                _dptr(loss), _stream(stream)))

    def backward(self, dout, stream=None):
        check(lib().q1_unet_backward(self.handle, _dptr(dout), _stream(stream)))

    def adam_step(self, lr, step, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        check(lib().q1_unet_adam_step(self.handle, lr, b1, b2, eps, step, _stream(stream)))

    def destroy(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            lib().q1_unet_destroy(h)
        self.handle = None

    def __del__(self):
        try:
            if _can_release():
                self.destroy()
        except Exception:
            pass


def q1_unet_create(D, H, W, batch, seed=0, stream=None) -> UNet:
    return UNet(D, H, W, batch, seed, stream)


class UNetPrecond:
    """q1_unet_pc: the network as a q1_fpcg preconditioner on a box mesh."""

    def __init__(self, net: UNet, nx: int, ny: int, nz: int, k, mask=None, stream=None):
        self.net, self.k, self.mask = net, k, mask  # kept alive with the context
        self.handle = ctypes.c_void_p()
        check(lib().q1_unet_pc_create(ctypes.byref(self.handle), net.handle, nx, ny, nz, _dptr(k),
                                      _dptr(mask), _stream(stream)))
        self.fn = ctypes.cast(lib().q1_unet_precond, ctypes.c_void_p)

    def two_level(self, op: Op, omega: float = 0.6, stream=None):
        """Jacobi smoothing around the network's energy-scaled correction."""
        self.op = op
        check(lib().q1_unet_pc_two_level(self.handle, op.handle, omega, _stream(stream)))

    def schedule(self, period: int):
        """Network on every period-th call from now on, the Jacobi step otherwise
        (call before each solve to restart the count)."""
        check(lib().q1_unet_pc_schedule(self.handle, int(period)))

    def encode(self, r, inp, stream=None):
        check(lib().q1_unet_encode(self.handle, _dptr(r), _dptr(inp), _stream(stream)))

    def encode_target(self, e, target, weight=None, stream=None):
        check(lib().q1_unet_encode_target(self.handle, _dptr(e), _dptr(target), _dptr(weight),
                                          _stream(stream)))

    def destroy(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            lib().q1_unet_pc_destroy(h)
        self.handle = None

    def __del__(self):
        try:
            if _can_release():
                self.destroy()
        except Exception:
            pass


def q1_unet_pc_create(net, nx, ny, nz, k, mask=None, stream=None) -> UNetPrecond:
    return UNetPrecond(net, nx, ny, nz, k, mask, stream)


def q1_unet_pairs(op: Op, xstar, iterates, omega: float, e_out, r_out, stream=None) -> None:
    """Training pairs (FP32 e, r written to the device vectors e_out[i], r_out[i])
    from the FP64 iterates of one Jacobi-PCG trajectory and its converged xstar."""
    n = len(iterates)
    VP = ctypes.c_void_p
    xa = (VP * max(n, 1))(*[_dptr(v) for v in iterates])
    ea = (VP * max(n, 1))(*[_dptr(v) for v in e_out])
    ra = (VP * max(n, 1))(*[_dptr(v) for v in r_out])
    check(lib().q1_unet_pairs(op.handle, _dptr(xstar), n, ctypes.cast(xa, VP), omega,
                              ctypes.cast(ea, VP), ctypes.cast(ra, VP), _stream(stream)))


def _lib_loaded() -> bool:
    return _libmod._lib is not None


def _can_release() -> bool:
    """Whether a finaliser may call into the library: not during interpreter
    shutdown (the HIP runtime may already be tearing down), and only once the
    library is loaded."""
    try:
        return not sys.is_finalizing() and _lib_loaded()
    except Exception:  # module state already torn down
        return False

