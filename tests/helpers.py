"""Shared helpers of the GPU tests: device upload of seeded inputs, operator
creation through the binding, and the oracle references."""
from __future__ import annotations

import numpy as np

import seeded_inputs as si

TOL = {0: 1e-12, 1: 2e-5}  # relative error bound per dtype (F64, F32)


def torch_dtype(dtype: int):
    import torch
    return torch.float64 if dtype == 0 else torch.float32


def dev(a, dt=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to(device="cuda", dtype=dt) if dt is not None else t.to("cuda")


def make_op(prob: dict, dtype: int = 0, variant: int = 0):
    import paper_2308_09839_amd as q1
    t = torch_dtype(dtype)
    xyz = dev(prob["xyz"], t)
    conn = dev(prob["conn"].astype(np.int32))
    coef = dev(prob["coef"], t)
    mask = dev(prob["mask"].astype(np.uint8)) if prob.get("mask") is not None else None
    return q1.q1_op_create(prob["physics"], dtype, variant, xyz, conn, coef, mask)


def gpu_apply(op, x: np.ndarray, dtype: int) -> np.ndarray:
    import torch
    t = torch_dtype(dtype)
    xd = dev(x, t)
    yd = torch.empty_like(xd)
    op.apply(xd, yd)
    torch.cuda.synchronize()
    return yd.double().cpu().numpy()


def gpu_diag(op, n: int, dtype: int) -> np.ndarray:
    import torch
    d = torch.empty(n, device="cuda", dtype=torch_dtype(dtype))
    op.diag(d)
    torch.cuda.synchronize()
    return d.double().cpu().numpy()


def problem(physics: int, n, jitter: float, seed: int, mask: bool = True, coef_kind="iid"):
    xyz, conn = si.box_mesh(*n, 1.0, jitter, seed)
    ne = int(np.prod(n))
    if physics in (1, 2):  # scalar and vector Laplace: one coefficient k
        if coef_kind == "layered":
            coef = si.field_layered(*n, 4, 1.5, 0.5, seed)[None]
        else:
            coef = si.field_lognormal(ne, 0.0, 1.0, seed)[None]
    else:
        coef = np.stack(si.lame_from_E_nu(*si.field_elastic(ne, seed)))
    m = si.face_mask(*n, "z0") if mask else None
    return dict(physics=physics, n=tuple(n), xyz=xyz, conn=conn, coef=coef, mask=m)


def rel_err(y, ref):
    return float(np.linalg.norm(y - ref) / np.linalg.norm(ref))


def rigid_modes(xyz):
    nn = xyz.shape[1]
    out = []
    for c in range(3):
        u = np.zeros((nn, 3)); u[:, c] = 1.0
        out.append(u.ravel())
    for w in np.eye(3):
        out.append(np.cross(np.broadcast_to(w, (nn, 3)), xyz.T).ravel())
    return out


def dpn_of(physics: int) -> int:
    """DOF per node of a physics kind (1 scalar Laplace, 2 vector Laplace, 3 elasticity)."""
    return 1 if physics == 1 else 3


_HIP = None


def hip_runtime():
    """The HIP runtime already loaded in the process (by torch), through ctypes."""
    global _HIP
    if _HIP is None:
        import ctypes
        import torch  # noqa: F401  (loads libamdhip64 first)
        L = ctypes.CDLL("libamdhip64.so.7")
        L.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_int, ctypes.c_void_p]
        L.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
        _HIP = L
    return _HIP


class HostPrecond:
    """A preconditioner callback for the device flexible solvers whose z = f(r)
    is computed on the host by a numpy callable: r is copied to the host,
    f applied, z copied back (test code: the solvers see an ordinary callback
    that enqueues nothing asynchronous)."""

    def __init__(self, f, n: int):
        self.f, self.n, self.calls = f, n, 0

    def __call__(self, r_ptr, z_ptr, stream):
        import ctypes
        L = hip_runtime()
        h2d, d2h = 1, 2
        r = np.empty(self.n)
        if L.hipStreamSynchronize(stream):
            return 1
        if L.hipMemcpyAsync(r.ctypes.data, r_ptr, r.nbytes, d2h, stream):
            return 1
        if L.hipStreamSynchronize(stream):
            return 1
        z = np.ascontiguousarray(self.f(r), dtype=np.float64)
        self.calls += 1
        rc = L.hipMemcpyAsync(z_ptr, z.ctypes.data, z.nbytes, h2d, stream)
        rc = rc or L.hipStreamSynchronize(stream)
        return 1 if rc else 0
