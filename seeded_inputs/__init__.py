"""Seeded synthetic inputs for the Q1 hexahedral operators.

This module only draws random numbers and lays out a Cartesian box mesh; it
holds none of the finite-element arithmetic.  Both the CPU oracle tests and the
GPU tests take their inputs from here, so the two sides see identical arrays.

Counter-based generator (one definition, also implemented independently in the
C library's host generators):

* ``splitmix64`` is the published SplitMix64 finaliser (Steele, Lea & Flood,
  "Fast splittable pseudorandom number generators", OOPSLA 2014).
* draw(seed, stream, i) = splitmix64(key + i) with
  key = seed XOR (stream * 0x9E3779B97F4A7C15), all arithmetic modulo 2**64.
* U(0,1): (draw >> 11) * 2**-53.
* N(0,1): Box-Muller on the two uniforms u1 = U(2i), u2 = U(2i+1):
  sqrt(-2 log(1 - u1)) * cos(2 pi u2).

Streams: 0 node jitter, 1 cell coefficient (k or E), 2 second cell field
(Poisson ratio, or the per-cell factor of a layered field), 3 apply input x,
4 right-hand side / body force, 5 batch problem sizes, 6 the factors of a
preconditioner that changes from one call to the next (solver tests).

Mesh numbering (the paper's Cartesian example grids, Section 4): node
id = i + (nx+1)(j + (ny+1)k); element e = ex + nx(ey + ny ez); local node
a = di + 2 dj + 4 dk of an element is node (ex+di, ey+dj, ez+dk).  The
connectivity is stored structure-of-arrays, conn[a, e].
"""
from __future__ import annotations

import math

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

STREAM_JITTER = 0
STREAM_COEF = 1
STREAM_COEF2 = 2
STREAM_X = 3
STREAM_RHS = 4
STREAM_BATCH = 5
STREAM_PC = 6


def splitmix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied to counters ``z`` (uint64 array)."""
    z = np.asarray(z, dtype=np.uint64)
    z = z + np.uint64(GOLDEN)
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _key(seed: int, stream: int) -> np.uint64:
    return np.uint64((seed ^ ((stream * GOLDEN) & MASK64)) & MASK64)


def draw_u64(seed: int, stream: int, idx) -> np.ndarray:
    idx = np.asarray(idx, dtype=np.uint64)
    return splitmix64(_key(seed, stream) + idx)


def uniform(seed: int, stream: int, idx) -> np.ndarray:
    """U[0,1) with 53 random bits."""
    z = draw_u64(seed, stream, idx)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, stream: int, idx) -> np.ndarray:
    """N(0,1) by Box-Muller on the uniforms at counters 2i and 2i+1."""
    idx = np.asarray(idx, dtype=np.uint64)
    u1 = uniform(seed, stream, np.uint64(2) * idx)
    u2 = uniform(seed, stream, np.uint64(2) * idx + np.uint64(1))
    return np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * math.pi * u2)


def box_sizes(nx: int, ny: int, nz: int) -> tuple[int, int]:
    return (nx + 1) * (ny + 1) * (nz + 1), nx * ny * nz


def box_mesh(nx: int, ny: int, nz: int, h: float = 1.0, jitter_frac: float = 0.0,
             seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """Cartesian box of nx*ny*nz hexahedra with spacing h.

    Interior nodes move by U(-jitter_frac*h, jitter_frac*h) per coordinate
    (stream 0, counter 3*id + c); nodes on the domain surface stay put so the
    domain is exactly [0, nx h] x [0, ny h] x [0, nz h].

    Returns xyz as float64 [3, n_nodes] and conn as int32 [8, n_elems].
    """
    nn, ne = box_sizes(nx, ny, nz)
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                          indexing="ij")
    i = i.ravel(); j = j.ravel(); k = k.ravel()
    xyz = np.empty((3, nn), dtype=np.float64)
    xyz[0] = i.astype(np.float64) * h
    xyz[1] = j.astype(np.float64) * h
    xyz[2] = k.astype(np.float64) * h
    if jitter_frac != 0.0:
        interior = (i > 0) & (i < nx) & (j > 0) & (j < ny) & (k > 0) & (k < nz)
        ids = np.nonzero(interior)[0].astype(np.uint64)
        amp = jitter_frac * h
        for c in range(3):
            u = uniform(seed, STREAM_JITTER, np.uint64(3) * ids + np.uint64(c))
            xyz[c, ids] = xyz[c, ids] + (2.0 * u - 1.0) * amp
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex = ex.ravel(); ey = ey.ravel(); ez = ez.ravel()
    conn = np.empty((8, ne), dtype=np.int32)
    for a in range(8):
        di, dj, dk = a & 1, (a >> 1) & 1, (a >> 2) & 1
        conn[a] = (ex + di) + (nx + 1) * ((ey + dj) + (ny + 1) * (ez + dk))
    return xyz, conn


# The six tetrahedra of the Kuhn (Freudenthal) split of a hexahedron, as local
# corners a = di + 2 dj + 4 dk: each follows one path of unit steps from corner 0
# to corner 7 (x, y, z in some order), so neighbouring hexahedra split their
# shared faces the same way.  Listed with positive orientation on the unit cube.
KUHN_TETS = ((0, 1, 3, 7), (0, 5, 1, 7), (0, 3, 2, 7), (0, 2, 6, 7), (0, 6, 4, 7),
             (0, 4, 5, 7))


def tet_mesh(nx: int, ny: int, nz: int, h: float = 1.0, jitter_frac: float = 0.0,
             seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """Linear tetrahedra: every hexahedron of box_mesh (same nodes, same jitter)
    split into the six Kuhn tetrahedra; tetrahedron t of hexahedron e is element
    6 e + t.  Returns xyz [3, n_nodes] and conn int32 [4, 6 n_hex]."""
    xyz, hconn = box_mesh(nx, ny, nz, h, jitter_frac, seed)
    ne = hconn.shape[1]
    conn = np.empty((4, 6 * ne), dtype=np.int32)
    for t, corners in enumerate(KUHN_TETS):
        for v, a in enumerate(corners):
            conn[v, t::6] = hconn[a]
    return xyz, conn


def q2_box_sizes(nx: int, ny: int, nz: int) -> tuple[int, int]:
    return (2 * nx + 1) * (2 * ny + 1) * (2 * nz + 1), nx * ny * nz


def q2_box_mesh(nx: int, ny: int, nz: int, h: float = 1.0, jitter_frac: float = 0.0,
                seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """Triquadratic hexahedra on the box of nx*ny*nz elements.

    Nodes lie on the doubled lattice, id = I + (2nx+1)(J + (2ny+1)K).  The
    element vertices (even I, J, K) are box_mesh's nodes, jitter included; every
    other node sits at the trilinear interpolation of its element's vertices
    (at local coordinate 1/2 along each odd index), so each element is the
    trilinear image of the reference cube.  Local node a = di + 3 dj + 9 dk of
    element e = ex + nx(ey + ny ez) is lattice node (2ex+di, 2ey+dj, 2ez+dk).
    Returns xyz [3, n_nodes] and conn int32 [27, n_elems]."""
    vxyz, _ = box_mesh(nx, ny, nz, h, jitter_frac, seed)
    NX, NY, NZ = 2 * nx + 1, 2 * ny + 1, 2 * nz + 1
    K, J, I = np.meshgrid(np.arange(NZ), np.arange(NY), np.arange(NX), indexing="ij")
    I = I.ravel(); J = J.ravel(); K = K.ravel()
    xyz = np.zeros((3, NX * NY * NZ))

    def vid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    # the vertex of the lower corner and the parity (odd = halfway) per axis
    i0, j0, k0 = I // 2, J // 2, K // 2
    oi, oj, ok = I % 2, J % 2, K % 2
    for di in (0, 1):
        wi = np.where(oi == 1, 0.5, 1.0 - di)
        for dj in (0, 1):
            wj = np.where(oj == 1, 0.5, 1.0 - dj)
            for dk in (0, 1):
                wk = np.where(ok == 1, 0.5, 1.0 - dk)
                w = wi * wj * wk
                sel = w > 0
                v = vid(np.minimum(i0 + di, nx), np.minimum(j0 + dj, ny), np.minimum(k0 + dk, nz))
                xyz[:, sel] += w[sel] * vxyz[:, v[sel]]
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex = ex.ravel(); ey = ey.ravel(); ez = ez.ravel()
    conn = np.empty((27, nx * ny * nz), dtype=np.int32)
    for a in range(27):
        di, dj, dk = a % 3, (a // 3) % 3, a // 9
        conn[a] = (2 * ex + di) + NX * ((2 * ey + dj) + NY * (2 * ez + dk))
    return xyz, conn


def q2_face_mask(nx: int, ny: int, nz: int, face: int | str) -> np.ndarray:
    """uint8 per node of q2_box_mesh: 1 on the chosen face of the box."""
    if isinstance(face, str):
        face = FACES[face]
    NX, NY, NZ = 2 * nx + 1, 2 * ny + 1, 2 * nz + 1
    K, J, I = np.meshgrid(np.arange(NZ), np.arange(NY), np.arange(NX), indexing="ij")
    sel = [I.ravel() == 0, I.ravel() == NX - 1, J.ravel() == 0, J.ravel() == NY - 1,
           K.ravel() == 0, K.ravel() == NZ - 1][face]
    return sel.astype(np.uint8)


def q3_box_sizes(nx: int, ny: int, nz: int) -> tuple[int, int]:
    return (3 * nx + 1) * (3 * ny + 1) * (3 * nz + 1), nx * ny * nz


def q3_box_mesh(nx: int, ny: int, nz: int, h: float = 1.0, jitter_frac: float = 0.0,
                seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """Tricubic hexahedra on the box of nx*ny*nz elements.

    Nodes lie on the tripled lattice, id = I + (3nx+1)(J + (3ny+1)K).  The
    element vertices (I, J, K multiples of 3) are box_mesh's nodes, jitter
    included; every other node sits at the trilinear interpolation of its
    element's vertices at local coordinate (I mod 3)/3 (and likewise in y, z),
    so each element is the trilinear image of the reference cube.  Local node
    a = di + 4 dj + 16 dk of element e = ex + nx(ey + ny ez) is lattice node
    (3ex+di, 3ey+dj, 3ez+dk).  Returns xyz [3, n_nodes] and conn int32
    [64, n_elems]."""
    vxyz, _ = box_mesh(nx, ny, nz, h, jitter_frac, seed)
    NX, NY, NZ = 3 * nx + 1, 3 * ny + 1, 3 * nz + 1
    K, J, I = np.meshgrid(np.arange(NZ), np.arange(NY), np.arange(NX), indexing="ij")
    I = I.ravel(); J = J.ravel(); K = K.ravel()
    xyz = np.zeros((3, NX * NY * NZ))

    def vid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    # the vertex of the lower corner and the local coordinate per axis
    i0, j0, k0 = I // 3, J // 3, K // 3
    ti, tj, tk = (I % 3) / 3.0, (J % 3) / 3.0, (K % 3) / 3.0
    for di in (0, 1):
        wi = ti if di else 1.0 - ti
        for dj in (0, 1):
            wj = tj if dj else 1.0 - tj
            for dk in (0, 1):
                wk = tk if dk else 1.0 - tk
                w = wi * wj * wk
                sel = w > 0
                v = vid(np.minimum(i0 + di, nx), np.minimum(j0 + dj, ny), np.minimum(k0 + dk, nz))
                xyz[:, sel] += w[sel] * vxyz[:, v[sel]]
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex = ex.ravel(); ey = ey.ravel(); ez = ez.ravel()
    conn = np.empty((64, nx * ny * nz), dtype=np.int32)
    for a in range(64):
        di, dj, dk = a % 4, (a // 4) % 4, a // 16
        conn[a] = (3 * ex + di) + NX * ((3 * ey + dj) + NY * (3 * ez + dk))
    return xyz, conn


def q3_face_mask(nx: int, ny: int, nz: int, face: int | str) -> np.ndarray:
    """uint8 per node of q3_box_mesh: 1 on the chosen face of the box."""
    if isinstance(face, str):
        face = FACES[face]
    NX, NY, NZ = 3 * nx + 1, 3 * ny + 1, 3 * nz + 1
    K, J, I = np.meshgrid(np.arange(NZ), np.arange(NY), np.arange(NX), indexing="ij")
    sel = [I.ravel() == 0, I.ravel() == NX - 1, J.ravel() == 0, J.ravel() == NY - 1,
           K.ravel() == 0, K.ravel() == NZ - 1][face]
    return sel.astype(np.uint8)


FACES = {"x0": 0, "x1": 1, "y0": 2, "y1": 3, "z0": 4, "z1": 5}


def face_mask(nx: int, ny: int, nz: int, face: int | str) -> np.ndarray:
    """uint8 per node: 1 on the chosen face of the box (0:x0 1:x1 2:y0 3:y1 4:z0 5:z1)."""
    if isinstance(face, str):
        face = FACES[face]
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                          indexing="ij")
    sel = [i.ravel() == 0, i.ravel() == nx, j.ravel() == 0, j.ravel() == ny,
           k.ravel() == 0, k.ravel() == nz][face]
    return sel.astype(np.uint8)


def field_lognormal(n: int, mu: float, sigma: float, seed: int,
                    stream: int = STREAM_COEF) -> np.ndarray:
    """exp(mu + sigma * N(0,1)) per cell; sigma is the std-dev of the log."""
    return np.exp(mu + sigma * normal(seed, stream, np.arange(n, dtype=np.uint64)))


def field_layered(nx: int, ny: int, nz: int, layer_cells: int, s_layer: float,
                  s_cell: float, seed: int) -> np.ndarray:
    """k_e = exp(s_layer N_layer(ez // layer_cells)) * exp(s_cell N_cell(e)).

    Layer values come from stream 1 (counter = layer), cell factors from
    stream 2 (counter = e).
    """
    ne = nx * ny * nz
    e = np.arange(ne, dtype=np.int64)
    ez = e // (nx * ny)
    nlay = (nz + layer_cells - 1) // layer_cells
    lay = np.exp(s_layer * normal(seed, STREAM_COEF, np.arange(nlay, dtype=np.uint64)))
    cell = np.exp(s_cell * normal(seed, STREAM_COEF2, e.astype(np.uint64)))
    return lay[ez // layer_cells] * cell


def field_elastic(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """E = exp(N(ln 10, 1)) (stream 1) and nu ~ U(0.15, 0.35) (stream 2) per cell."""
    idx = np.arange(n, dtype=np.uint64)
    E = np.exp(math.log(10.0) + 1.0 * normal(seed, STREAM_COEF, idx))
    nu = 0.15 + 0.2 * uniform(seed, STREAM_COEF2, idx)
    return E, nu


def lame_from_E_nu(E: np.ndarray, nu: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Lame constants of an isotropic material from Young's modulus and Poisson ratio."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def vec_uniform(n: int, seed: int, stream: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """U(lo, hi) entries from the given stream."""
    u = uniform(seed, stream, np.arange(n, dtype=np.uint64))
    return lo + (hi - lo) * u


def batch_sizes(nprob: int, seed: int, lo: int = 16, hi: int = 64) -> np.ndarray:
    """Edge sizes n_p ~ U{lo..hi} inclusive (stream 5)."""
    u = uniform(seed, STREAM_BATCH, np.arange(nprob, dtype=np.uint64))
    return (lo + np.floor(u * (hi - lo + 1))).astype(np.int64)


def varying_factors(n: int, call: int, seed: int, lo: float = 0.5, hi: float = 1.5) -> np.ndarray:
    """Per-entry factors U(lo, hi) for the call-th use (from 0) of a
    preconditioner that changes between calls: stream 6, counters call*n + i."""
    idx = np.uint64(call) * np.uint64(n) + np.arange(n, dtype=np.uint64)
    return lo + (hi - lo) * uniform(seed, STREAM_PC, idx)


def dof_mask(mask_nodes: np.ndarray, dpn: int) -> np.ndarray:
    """Expand a per-node mask to interleaved DOFs (node*dpn + comp)."""
    return np.repeat(np.asarray(mask_nodes, dtype=np.uint8), dpn)


# ---------------------------------------------------------------------------
# The workloads: exact recipes used by tests and the benchmark.
# ---------------------------------------------------------------------------

def seed_for(cfg: int) -> int:
    return 2308 + cfg


def problem_laplace_jittered(n: int = 16, seed: int = 2308):
    """Scalar Laplace on n^3 jittered elements, k = exp(N(0,1)) iid per cell,
    Dirichlet on z=0 (16^3 is the small validation workload)."""
    xyz, conn = box_mesh(n, n, n, 1.0, 0.1, seed)
    k = field_lognormal(n ** 3, 0.0, 1.0, seed)
    mask = face_mask(n, n, n, "z0")
    return dict(physics=1, n=(n, n, n), xyz=xyz, conn=conn, coef=k[None, :], mask=mask)


def problem_laplace_layered(n: int = 128, seed: int = 2309):
    """Scalar Laplace on an undistorted n^3 grid with a layered lognormal
    coefficient (one lognormal(0,1.5) value per 4-cell z-layer times iid
    lognormal(0,0.5) per cell); no boundary condition."""
    xyz, conn = box_mesh(n, n, n, 1.0, 0.0, seed)
    k = field_layered(n, n, n, 4, 1.5, 0.5, seed)
    return dict(physics=1, n=(n, n, n), xyz=xyz, conn=conn, coef=k[None, :], mask=None)


def problem_vlaplace(n: int = 96, seed: int = 2313, jitter: float = 0.0):
    """Vector Laplace (3 DOF per node) on n^3 elements, k = exp(N(0,1)) iid
    per cell, Dirichlet (all components) on z=0."""
    xyz, conn = box_mesh(n, n, n, 1.0, jitter, seed)
    k = field_lognormal(n ** 3, 0.0, 1.0, seed)
    mask = face_mask(n, n, n, "z0")
    return dict(physics=2, n=(n, n, n), xyz=xyz, conn=conn, coef=k[None, :], mask=mask)


def problem_elasticity(n: int = 96, seed: int = 2310, jitter: float = 0.0):
    """Isotropic elasticity on n^3 elements, E = exp(N(ln 10,1)),
    nu ~ U(0.15,0.35) per cell, Dirichlet (all components) on z=0."""
    xyz, conn = box_mesh(n, n, n, 1.0, jitter, seed)
    E, nu = field_elastic(n ** 3, seed)
    lam, mu = lame_from_E_nu(E, nu)
    mask = face_mask(n, n, n, "z0")
    return dict(physics=3, n=(n, n, n), xyz=xyz, conn=conn, coef=np.stack([lam, mu]), mask=mask)
