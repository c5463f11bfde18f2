"""ctypes loader of libq1mf.so: argument marshalling only.

The shared library is built in-tree by ``paper_2308_09839_amd.build``; this
module refuses to run without it (there is no fallback implementation).
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libq1mf.so")

Q1_OK = 0
Q1_EINVAL = -1
Q1_ENOMEM = -2
Q1_EHIP = -3
Q1_ENOCONV = -4
Q1_EBREAKDOWN = -5
Q1_EUNSUPPORTED = -6

Q1_LAPLACE = 1
Q1_VLAPLACE = 2
Q1_ELASTICITY = 3
Q1_F64 = 0
Q1_F32 = 1
Q1_V_AUTO = 0
Q1_V_ATOMIC = 1
Q1_V_COLOR = 2
Q1_V_LDS_TILE = 3
Q1_V_CSR = 4
Q1_V_BLOCK = 5
Q1_V_PA = 6
Q1_HEX8 = 8
Q1_TET4 = 4
Q1_HEX27 = 27
Q1_HEX64 = 64

Q1_PC_NONE = 0
Q1_PC_JACOBI = 1


class Q1Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("true_rel_res", ctypes.c_double), ("seconds", ctypes.c_double),
                ("fallback_at", ctypes.c_int), ("outer_iters", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


PRECOND_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_void_p)

_STATUS = {0: "Q1_OK", -1: "Q1_EINVAL", -2: "Q1_ENOMEM", -3: "Q1_EHIP", -4: "Q1_ENOCONV",
           -5: "Q1_EBREAKDOWN", -6: "Q1_EUNSUPPORTED"}


class Q1Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None

c_int, c_i64, c_u64, c_dbl, c_vp = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
P = ctypes.POINTER
c_flt = ctypes.c_float

# name -> (restype, argtypes); the declarations of include/q1mf.h
PROTOTYPES = {
    "q1_last_error": (ctypes.c_char_p, []),
    "q1_version": (c_int, []),
    "q1_box_sizes": (c_int, [c_int, c_int, c_int, P(c_i64), P(c_i64)]),
    "q1_box_mesh": (c_int, [c_int, c_int, c_int, c_dbl, c_dbl, c_u64, c_vp, c_vp]),
    "q1_face_mask": (c_int, [c_int, c_int, c_int, c_int, c_vp]),
    "q1_field_lognormal": (c_int, [c_i64, c_dbl, c_dbl, c_u64, c_u64, c_vp]),
    "q1_field_layered": (c_int, [c_int, c_int, c_int, c_int, c_dbl, c_dbl, c_u64, c_vp]),
    "q1_field_elastic": (c_int, [c_i64, c_u64, c_vp, c_vp]),
    "q1_lame_from_E_nu": (c_int, [c_i64, c_vp, c_vp, c_vp, c_vp]),
    "q1_vec_uniform": (c_int, [c_i64, c_u64, c_u64, c_dbl, c_dbl, c_vp]),
    "q1_op_create": (c_int, [P(c_vp), c_int, c_int, c_int, c_i64, c_i64, c_vp, c_vp, c_vp, c_vp,
                             c_vp]),
    "q1_op_create_elem": (c_int, [P(c_vp), c_int, c_int, c_int, c_int, c_i64, c_i64, c_vp, c_vp,
                                  c_vp, c_vp, c_vp]),
    "q1_op_apply": (c_int, [c_vp, c_vp, c_vp, c_vp]),
    "q1_op_diag": (c_int, [c_vp, c_vp, c_vp]),
    "q1_op_info": (c_int, [c_vp, P(c_int), P(c_int), P(c_int), P(c_i64), P(c_i64)]),
    "q1_op_bytes": (c_int, [c_vp, P(c_dbl), P(c_dbl)]),
    "q1_op_reproducible": (c_int, [c_vp, P(c_int)]),
    "q1_op_destroy": (c_int, [c_vp]),
    "q1_model_bytes": (c_int, [c_int, c_int, c_int, c_int, c_i64, c_i64, c_int, P(c_dbl)]),
    "q1_csr_create": (c_int, [P(c_vp), c_vp, c_vp]),
    "q1_csr_info": (c_int, [c_vp, P(c_i64), P(c_i64)]),
    "q1_csr_export": (c_int, [c_vp, c_vp, c_vp, c_vp]),
    "q1_pcg": (c_int, [c_vp, c_int, c_vp, c_vp, c_dbl, c_int, P(Q1Stats), c_vp]),
    "q1_pcg_noalloc": (c_int, [c_vp, c_int, c_vp, c_vp, c_dbl, c_int, P(Q1Stats), c_vp]),
    "q1_pcg_trace": (c_int, [c_vp, c_int, c_vp, c_vp, c_dbl, c_int, c_int, c_vp, c_vp, P(Q1Stats),
                             c_vp]),
    "q1_fpcg": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_dbl, c_int, c_int, P(Q1Stats), c_vp]),
    "q1_fcg": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_dbl, c_int, c_int, c_int, P(Q1Stats),
                       c_vp]),
    "q1_jacobi_create": (c_int, [P(c_vp), c_vp, c_vp]),
    "q1_precond_jacobi": (c_int, [c_vp, c_vp, c_vp, c_vp]),
    "q1_jacobi_destroy": (c_int, [c_vp]),
    "q1_batched_pcg": (c_int, [c_int, c_vp, c_int, c_vp, c_vp, c_dbl, c_int, c_vp, c_vp]),
    "q1_batched_mpcg": (c_int, [c_int, c_vp, c_int, c_vp, c_vp, c_dbl, c_dbl, c_int, c_vp,
                                c_vp]),
    "q1_mpcg": (c_int, [c_vp, c_vp, c_vp, c_vp, c_dbl, c_dbl, c_int, P(Q1Stats), c_vp]),
    "q1_dot": (c_int, [c_i64, c_int, c_vp, c_vp, c_vp, c_int, c_int, c_vp, c_vp]),
    "q1_pcg_fused": (c_int, [c_vp, c_int, c_vp, c_vp, c_dbl, c_int, P(Q1Stats), c_vp]),
    "q1_ir_solve": (c_int, [c_vp, c_vp, c_vp, c_vp, c_dbl, c_dbl, c_int, c_int, P(Q1Stats), c_vp]),
    "q1_conv3d_forward": (c_int, [c_int, c_int, c_int, c_int, c_vp, c_int, c_int, c_vp, c_int,
                                  c_vp, c_vp, c_int, c_int, c_vp, c_vp]),
    "q1_conv3d_backward_data": (c_int, [c_int, c_int, c_int, c_int, c_vp, c_int, c_vp, c_int,
                                        c_vp, c_vp]),
    "q1_conv3d_backward_weight": (c_int, [c_int, c_int, c_int, c_int, c_vp, c_int, c_int, c_vp,
                                          c_int, c_vp, c_int, c_vp, c_vp, c_vp]),
    "q1_unet_create": (c_int, [P(c_vp), c_int, c_int, c_int, c_int, c_u64, c_vp]),
    "q1_unet_destroy": (c_int, [c_vp]),
    "q1_unet_info": (c_int, [c_vp, P(c_i64), P(c_int), P(c_int), P(c_int), P(c_int)]),
    "q1_unet_params": (c_int, [c_vp, P(c_vp), P(c_vp)]),
    "q1_unet_commit": (c_int, [c_vp, c_vp]),
    "q1_unet_copy": (c_int, [c_vp, c_int, c_int, c_vp, c_vp]),
    "q1_unet_forward": (c_int, [c_vp, c_vp, c_vp, c_int, c_vp]),
    "q1_unet_mse": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "q1_unet_backward": (c_int, [c_vp, c_vp, c_vp]),
    "q1_unet_adam_step": (c_int, [c_vp, c_flt, c_flt, c_flt, c_flt, c_int, c_vp]),
    "q1_unet_pc_create": (c_int, [P(c_vp), c_vp, c_int, c_int, c_int, c_vp, c_vp, c_vp]),
    "q1_unet_pc_destroy": (c_int, [c_vp]),
    "q1_unet_pc_two_level": (c_int, [c_vp, c_vp, c_dbl, c_vp]),
    "q1_unet_encode": (c_int, [c_vp, c_vp, c_vp, c_vp]),
    "q1_unet_encode_target": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "q1_unet_precond": (c_int, [c_vp, c_vp, c_vp, c_vp]),
    "q1_unet_pc_schedule": (c_int, [c_vp, c_int]),
    "q1_unet_pairs": (c_int, [c_vp, c_vp, c_int, c_vp, c_dbl, c_vp, c_vp, c_vp]),
}


def lib():
    """Load libq1mf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2308_09839_amd.build` (no fallback path exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().q1_last_error().decode(errors="replace")


def check(rc: int) -> int:
    if rc != Q1_OK:
        raise Q1Error(rc, last_error())
    return rc
