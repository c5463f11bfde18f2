// Internal declarations of libq1mf (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <type_traits>
#include <vector>

#include "q1mf.h"

namespace q1 {

// Thread-local error text behind q1_last_error().
void set_error(const char *fmt, ...);
int fail(int code, const char *fmt, ...);

#define Q1_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return ::q1::fail(Q1_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                          \
  } while (0)

#define Q1_CHECK(cond, code, ...)                          \
  do {                                                     \
    if (!(cond)) return ::q1::fail((code), __VA_ARGS__);   \
  } while (0)

// Tiles of the LDS-tiled apply (built once at operator creation).
struct TileMap {
  int n_tiles = 0;
  int64_t n_steps = 0;            // steps of at most 64 elements (one wavefront)
  int max_nodes = 0;              // LDS accumulator entries per tile
  int32_t *node_ptr = nullptr;    // [n_tiles+1] node list of each tile
  uint32_t *nodes = nullptr;      // global node ids | shared bit 31 | Dirichlet bit 30
  int64_t n_entries = 0;          // entries of nodes (node_ptr[n_tiles])
  int32_t *tile_step = nullptr;   // [n_tiles+1] step range of each tile
  uint16_t *lconn = nullptr;      // [n_steps*64][8] corner indices into the tile list (0xffff: empty)
  void *coef_t = nullptr;         // cell coefficients in lane order [ncoef][n_steps*64]
  int64_t n_reset = 0;            // shared or Dirichlet nodes, reset before each apply
  int32_t *reset = nullptr;
  bool lds_atomic = false;        // corners collide within a step: accumulate with LDS atomics
  bool split = false;             // block variants: bitwise-reproducible split accumulation
  bool all_affine = false;        // every tile is a parallelepiped tile
  bool fixed = false;             // every tile is the default 16 x 8 x 4 scalar lattice tile
  // owner-computes tiles (scalar Laplace on a box lattice of parallelepipeds whose
  // element counts per direction are multiples of 16, 8, 4): the box size, or 0
  int own_nx = 0, own_ny = 0, own_nz = 0;
  int own_elem = 0;               // owner tiles' element: 0 parallelepiped, 1 general
                                  // hexahedron, 2 a cell's six Kuhn tetrahedra
  uint8_t *tile_affine = nullptr; // [n_tiles] 1: every element of the tile is a parallelepiped
  uint32_t *tile_lat = nullptr;   // [n_tiles] lattice tile A | B << 8 | steps-per-layer << 16 | C << 24, or 0
  uint32_t *tile_addr = nullptr;  // [n_tiles] lattice addressing: valid bit | shared-face bits, or 0
  int32_t *tile_g0 = nullptr;     // [n_tiles] global id of entry 0 of a lattice-addressed tile
  int64_t sy = 0, sz = 0;         // mesh strides of lattice addressing
  // block variant: partial sums of nodes shared between tiles go to halo slots
  // (no atomics), summed per node by a second kernel in a fixed order
  int64_t n_halo = 0;             // slots: 2 per reset node + one per further touching tile
  int32_t *slot = nullptr;        // [entries] halo slot of each node-list entry, -1 if none
  int32_t *hptr = nullptr;        // [n_reset+1] extra-slot range of each reset node
  int32_t *hnode = nullptr;       // [n_reset] node id, bit 31 set on Dirichlet nodes
  void *halo = nullptr;           // [n_halo][dpn] partial sums, overwritten by every apply
  void *qdata = nullptr;          // partial assembly: [48][n_steps*64] quadrature data
  size_t bytes = 0;
};

// Assembled CSR matrix of the matrix-based comparison.
struct CsrData {
  int64_t nrows = 0, nnz = 0;
  int32_t *rowptr = nullptr;  // [nrows+1]
  int32_t *col = nullptr;     // [nnz], sorted within each row
  void *val = nullptr;        // [nnz] of the operator's dtype
};

// Element colouring of the colour variant: elements of one colour share no node.
struct ColorMap {
  int n_colors = 0;
  std::vector<int64_t> ptr;     // [n_colors+1] element ranges in colour order
  int32_t *conn = nullptr;      // [8][n_elems] connectivity in colour order
  void *coef = nullptr;         // [ncoef][n_elems] coefficients in colour order
};

struct Op {
  int physics = 1;  // kind: 1 scalar Laplace, 2 vector Laplace, 3 elasticity
  int dpn() const { return physics == 1 ? 1 : 3; }  // DOF per node
  int elem = Q1_HEX8;  // element family; its value is the nodes per element
  int nloc() const { return elem; }
  int dtype = Q1_F64;
  int variant = Q1_V_ATOMIC;
  int64_t n_nodes = 0, n_elems = 0;
  const void *xyz = nullptr;
  const int32_t *conn = nullptr;
  const void *coef = nullptr;
  const uint8_t *mask = nullptr;
  int device = 0;
  int num_cus = 256;
  TileMap tiles;
  CsrData csr;
  ColorMap colors;
};

inline int xcd_count() { return 8; }

// Calls f(T{}, std::integral_constant<int, PH>{}) for the operator's dtype and
// physics kind (1 scalar Laplace, 2 vector Laplace, 3 elasticity).
template <typename F>
int dispatch_phys(const Op &op, F &&f) {
  if (op.dtype == Q1_F64) {
    switch (op.physics) {
      case 1: return f(double{}, std::integral_constant<int, 1>{});
      case 2: return f(double{}, std::integral_constant<int, 2>{});
      default: return f(double{}, std::integral_constant<int, 3>{});
    }
  }
  switch (op.physics) {
    case 1: return f(float{}, std::integral_constant<int, 1>{});
    case 2: return f(float{}, std::integral_constant<int, 2>{});
    default: return f(float{}, std::integral_constant<int, 3>{});
  }
}

// launchers (defined in the .hip files)
// stop: optional device flag; when it is non-zero at kernel start the launch does nothing
int launch_apply(Op &op, const void *x, void *y, hipStream_t s, const int *stop = nullptr);
int launch_diag(Op &op, void *d, hipStream_t s);
// linear tetrahedra and triquadratic hexahedra (q1_family.hip)
int launch_apply_family(Op &op, const void *x, void *y, hipStream_t s, const int *stop);
int launch_diag_family(Op &op, void *d, hipStream_t s);
// Q1_EINVAL unless every connectivity entry is in [0, n_nodes) (synchronises s).
int validate_conn(const Op &op, hipStream_t s);
int build_tiles(Op &op, hipStream_t s);
int launch_apply_tile(Op &op, const void *x, void *y, hipStream_t s, const int *stop);
// y = A x with the partial sums of x.y formed where y is written (per tile over its
// own nodes, per halo-sum workgroup over shared and Dirichlet nodes plus a fixed
// range of the tile partials): block and partial-assembly hexahedron operators.
// apply_dot_parts: doubles the launch needs at parts (0: not available) and, in
// *n_final, how many partials at parts[0..) make up x.y.
int64_t apply_dot_parts(const Op &op, int64_t *n_final);
int launch_apply_dot(Op &op, const void *x, void *y, hipStream_t s, const int *stop,
                     double *parts);
int launch_diag_tile(Op &op, void *d, hipStream_t s);
// The diagonal on owner-computes tiles of tetrahedra (bitwise reproducible).
int launch_diag_owner(Op &op, void *d, hipStream_t s);
void free_tiles(Op &op);
int build_colors(Op &op, hipStream_t s);
void free_colors(Op &op);
int csr_create(Op &op, hipStream_t s);
int launch_spmv(const Op &op, const void *x, void *y, hipStream_t s, const int *stop);
void free_csr(Op &op);

}  // namespace q1
