"""Python access to the plain FP64 CPU oracle (``q1_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  The product library never imports, links or calls
anything here, and nothing here calls the product library.

The oracle computes the operator by its plain definition: element matrices by
2x2x2 Gauss quadrature (paper Section 2), a CSR matrix summed element by
element (Section 3, assembly by column search and addition), and products
with that matrix.  ``pcg``/``fpcg`` are Hestenes-Stiefel PCG and flexible PCG
built from the CG operations of Table 4.  ``unet_oracle`` (numpy, FP64) is
the learned preconditioner's network written as its definitions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "q1_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")

PRECOND_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP over SpMV rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.orc_ke_laplace.argtypes = [_f64p, ctypes.c_double, _f64p]
        L.orc_ke_elasticity.argtypes = [_f64p, ctypes.c_double, ctypes.c_double, _f64p]
        L.orc_ke_vlaplace.argtypes = [_f64p, ctypes.c_double, _f64p]
        L.orc_csr_pattern.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, _i32p,
                                      _i64p, ctypes.c_void_p]
        L.orc_csr_pattern.restype = ctypes.c_int64
        L.orc_csr_assemble.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, _f64p,
                                       _i32p, _f64p, ctypes.c_void_p, _i64p, _i32p, _f64p]
        L.orc_csr_pattern_n.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                        ctypes.c_int64, _i32p, _i64p, ctypes.c_void_p]
        L.orc_csr_pattern_n.restype = ctypes.c_int64
        L.orc_csr_assemble_n.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                         ctypes.c_int64, _f64p, _i32p, _f64p, ctypes.c_void_p,
                                         _i64p, _i32p, _f64p]
        L.orc_apply_rows_n.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                       ctypes.c_int64, _f64p, _i32p, _f64p, ctypes.c_void_p,
                                       _f64p, ctypes.c_int64, _i64p, _f64p]
        L.orc_ke_tet_laplace.argtypes = [_f64p, ctypes.c_double, _f64p]
        L.orc_ke_tet_elasticity.argtypes = [_f64p, ctypes.c_double, ctypes.c_double, _f64p]
        L.orc_ke_q2_laplace.argtypes = [_f64p, ctypes.c_double, _f64p]
        L.orc_ke_q2_elasticity.argtypes = [_f64p, ctypes.c_double, ctypes.c_double, _f64p]
        L.orc_ke_q3_laplace.argtypes = [_f64p, ctypes.c_double, _f64p]
        L.orc_ke_q3_elasticity.argtypes = [_f64p, ctypes.c_double, ctypes.c_double, _f64p]
        L.orc_apply_rows.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, _f64p, _i32p,
                                     _f64p, ctypes.c_void_p, _f64p, ctypes.c_int64, _i64p, _f64p]
        L.orc_spmv.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, _f64p]
        L.orc_diag.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_pcg.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, _f64p,
                              ctypes.c_double, ctypes.c_int, ctypes.c_int,
                              ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                              ctypes.c_void_p]
        L.orc_fpcg.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, _f64p,
                               ctypes.c_double, ctypes.c_int, PRECOND_FN, ctypes.c_void_p,
                               ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                               ctypes.c_void_p, ctypes.c_void_p]
        L.orc_fcg.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, _f64p,
                              ctypes.c_double, ctypes.c_int, ctypes.c_int, PRECOND_FN,
                              ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                              ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_void_p]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def ke_laplace(X: np.ndarray, k: float = 1.0) -> np.ndarray:
    """8x8 scalar-Laplace element matrix of the hexahedron with nodes X[8,3]."""
    Ke = np.zeros(64)
    if lib().orc_ke_laplace(np.ascontiguousarray(X, dtype=np.float64).ravel(), float(k), Ke):
        raise ValueError("non-positive Jacobian determinant")
    return Ke.reshape(8, 8)


def ke_elasticity(X: np.ndarray, lam: float, mu: float) -> np.ndarray:
    """24x24 isotropic-elasticity element matrix, DOF 3*node + component."""
    Ke = np.zeros(576)
    if lib().orc_ke_elasticity(np.ascontiguousarray(X, dtype=np.float64).ravel(),
                               float(lam), float(mu), Ke):
        raise ValueError("non-positive Jacobian determinant")
    return Ke.reshape(24, 24)


def ke_vlaplace(X: np.ndarray, k: float = 1.0) -> np.ndarray:
    """24x24 vector-Laplace element matrix, DOF 3*node + component."""
    Ke = np.zeros(576)
    if lib().orc_ke_vlaplace(np.ascontiguousarray(X, dtype=np.float64).ravel(), float(k), Ke):
        raise ValueError("non-positive Jacobian determinant")
    return Ke.reshape(24, 24)


def ke_tet(physics: int, X: np.ndarray, c0: float, c1: float = 0.0) -> np.ndarray:
    """Linear-tetrahedron element matrix (X[4,3]): physics 1 (4x4, k = c0) or 3
    (12x12, lambda = c0, mu = c1)."""
    X = np.ascontiguousarray(X, dtype=np.float64).ravel()
    if physics == 1:
        Ke = np.zeros(16)
        rc = lib().orc_ke_tet_laplace(X, float(c0), Ke)
    else:
        Ke = np.zeros(144)
        rc = lib().orc_ke_tet_elasticity(X, float(c0), float(c1), Ke)
    if rc:
        raise ValueError("non-positive Jacobian determinant")
    m = 4 if physics == 1 else 12
    return Ke.reshape(m, m)


def ke_q2(physics: int, X: np.ndarray, c0: float, c1: float = 0.0) -> np.ndarray:
    """Triquadratic-hexahedron element matrix (X[27,3], local node i + 3j + 9k):
    physics 1 (27x27) or 3 (81x81)."""
    X = np.ascontiguousarray(X, dtype=np.float64).ravel()
    if physics == 1:
        Ke = np.zeros(729)
        rc = lib().orc_ke_q2_laplace(X, float(c0), Ke)
    else:
        Ke = np.zeros(6561)
        rc = lib().orc_ke_q2_elasticity(X, float(c0), float(c1), Ke)
    if rc:
        raise ValueError("non-positive Jacobian determinant")
    m = 27 if physics == 1 else 81
    return Ke.reshape(m, m)


def ke_q3(physics: int, X: np.ndarray, c0: float, c1: float = 0.0) -> np.ndarray:
    """Tricubic-hexahedron element matrix (X[64,3], local node i + 4j + 16k):
    physics 1 (64x64) or 3 (192x192)."""
    X = np.ascontiguousarray(X, dtype=np.float64).ravel()
    if physics == 1:
        Ke = np.zeros(4096)
        rc = lib().orc_ke_q3_laplace(X, float(c0), Ke)
    else:
        Ke = np.zeros(36864)
        rc = lib().orc_ke_q3_elasticity(X, float(c0), float(c1), Ke)
    if rc:
        raise ValueError("non-positive Jacobian determinant")
    m = 64 if physics == 1 else 192
    return Ke.reshape(m, m)


@dataclass
class CSR:
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def matvec(self, x: np.ndarray) -> np.ndarray:
        y = np.empty(self.n)
        lib().orc_spmv(self.n, self.rowptr, self.col, self.val,
                       np.ascontiguousarray(x, dtype=np.float64), y)
        return y

    def diag(self) -> np.ndarray:
        d = np.empty(self.n)
        lib().orc_diag(self.n, self.rowptr, self.col, self.val, d)
        return d

    def to_dense(self) -> np.ndarray:
        A = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        A[rows, self.col] = self.val
        return A

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))


def dpn_of(physics: int) -> int:
    """DOF per node: 1 for scalar Laplace, 3 for vector Laplace and elasticity."""
    return 1 if physics == 1 else 3


def csr_pattern(dpn: int, n_nodes: int, conn: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Pattern for the connectivity conn [nloc, n_elems] (nloc 8, 4, 27 or 64)."""
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    nloc, ne = conn.shape
    rowptr = np.zeros(n_nodes * dpn + 1, dtype=np.int64)
    nnz = lib().orc_csr_pattern_n(dpn, nloc, n_nodes, ne, conn.ravel(), rowptr, None)
    if nnz < 0:
        raise MemoryError("oracle pattern allocation failed")
    col = np.empty(nnz, dtype=np.int32)
    lib().orc_csr_pattern_n(dpn, nloc, n_nodes, ne, conn.ravel(), rowptr,
                            col.ctypes.data_as(ctypes.c_void_p))
    return rowptr, col


def assemble(physics: int, xyz: np.ndarray, conn: np.ndarray, coef: np.ndarray,
             mask: np.ndarray | None = None) -> CSR:
    """Assembled operator with Dirichlet elimination on the masked nodes.

    physics = 1 (scalar Laplace, coef [1, ne] = k), 2 (vector Laplace, 3 DOF
    per node, coef [1, ne] = k) or 3 (elasticity, coef [2, ne] = lambda, mu).
    xyz [3, nn], conn [nloc, ne] with nloc 8 (trilinear hexahedra), 4 (linear
    tetrahedra), 27 (triquadratic hexahedra) or 64 (tricubic hexahedra), mask
    uint8 [nn]."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    nn, ne = xyz.shape[1], conn.shape[1]
    rowptr, col = csr_pattern(dpn_of(physics), nn, conn)
    val = np.empty(col.shape[0])
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        mptr = mask.ctypes.data_as(ctypes.c_void_p)
    else:
        mptr = None
    rc = lib().orc_csr_assemble_n(conn.shape[0], physics, nn, ne, xyz.ravel(), conn.ravel(),
                                  coef.ravel(), mptr, rowptr, col, val)
    if rc == -1:
        raise ValueError("element with non-positive Jacobian determinant")
    if rc != 0:
        raise RuntimeError(f"oracle assembly failed ({rc})")
    return CSR(nn * dpn_of(physics), rowptr, col, val)


def apply_rows(physics: int, xyz: np.ndarray, conn: np.ndarray, coef: np.ndarray,
               mask: np.ndarray | None, x: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """Rows ``rows`` (DOF indices) of A x, summed element by element from the
    element matrices (no global matrix), with the Dirichlet elimination."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    y = np.empty(rows.shape[0])
    mptr = None
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        mptr = mask.ctypes.data_as(ctypes.c_void_p)
    rc = lib().orc_apply_rows_n(conn.shape[0], physics, xyz.shape[1], conn.shape[1],
                                xyz.ravel(), conn.ravel(), coef.ravel(), mptr, x, rows.shape[0],
                                rows, y)
    if rc:
        raise RuntimeError(f"oracle apply_rows failed ({rc})")
    return y


@dataclass
class SolveResult:
    x: np.ndarray
    status: int
    iters: int
    rel_res: float
    history: np.ndarray


def pcg(A: CSR, b: np.ndarray, rtol: float = 1e-8, maxit: int = 20000,
        jacobi: bool = True) -> SolveResult:
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    hist = np.zeros(maxit + 1)
    st = lib().orc_pcg(A.n, A.rowptr, A.col, A.val, b, x, float(rtol), int(maxit),
                       int(bool(jacobi)), ctypes.byref(it), ctypes.byref(rr),
                       hist.ctypes.data_as(ctypes.c_void_p))
    return SolveResult(x, int(st), it.value, rr.value, hist[: it.value + 1].copy())


@dataclass
class FlexResult(SolveResult):
    iterates: np.ndarray | None = None  # [iters+1, n] when recorded


def _precond_cb(precond):
    def _cb(_ctx, n, rp, zp):
        try:
            r = np.ctypeslib.as_array(rp, shape=(n,))
            z = np.ctypeslib.as_array(zp, shape=(n,))
            z[:] = precond(r.copy())
            return 0 if np.all(np.isfinite(z)) else 1
        except Exception:  # a failing preconditioner is a breakdown
            return 1
    return PRECOND_FN(_cb)


def _flex(which: str, A: CSR, b, precond, rtol: float, maxit: int, m: int,
          record: bool) -> FlexResult:
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n)
    cb = _precond_cb(precond)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    hist = np.zeros(maxit + 1)
    xh = np.zeros((maxit + 1, A.n)) if record else None
    xh_p = xh.ctypes.data_as(ctypes.c_void_p) if record else None
    hp = hist.ctypes.data_as(ctypes.c_void_p)
    if which == "fpcg":
        st = lib().orc_fpcg(A.n, A.rowptr, A.col, A.val, b, x, float(rtol), int(maxit), cb, None,
                            ctypes.byref(it), ctypes.byref(rr), hp, xh_p)
    else:
        st = lib().orc_fcg(A.n, A.rowptr, A.col, A.val, b, x, float(rtol), int(maxit), int(m),
                           cb, None, ctypes.byref(it), ctypes.byref(rr), hp, xh_p)
    k = it.value
    return FlexResult(x, int(st), k, rr.value, hist[: k + 1].copy(),
                      xh[: k + 1].copy() if record else None)


def fpcg(A: CSR, b: np.ndarray, precond, rtol: float = 1e-8, maxit: int = 20000,
         record: bool = False) -> FlexResult:
    """Flexible PCG (Golub-Ye beta); ``precond(r) -> z`` is any Python callable
    on numpy arrays, called once per iteration in order.  ``record`` keeps the
    iterates x_0 .. x_k."""
    return _flex("fpcg", A, b, precond, rtol, maxit, 1, record)


def fcg(A: CSR, b: np.ndarray, precond, m: int, rtol: float = 1e-8, maxit: int = 20000,
        record: bool = False) -> FlexResult:
    """FCG(m): flexible CG with A-orthogonalisation against the last m directions."""
    return _flex("fcg", A, b, precond, rtol, maxit, m, record)


def true_rel_res(A: CSR, x: np.ndarray, b: np.ndarray) -> float:
    r = b - A.matvec(x)
    return float(np.linalg.norm(r) / np.linalg.norm(b))
