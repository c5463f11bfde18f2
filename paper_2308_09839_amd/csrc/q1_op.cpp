// Operator handles: creation, validation, dispatch and the byte/FLOP model.
#include <hip/hip_runtime.h>

#include <new>

#include "q1_internal.hpp"

namespace q1 {
namespace {

// Algorithmic FLOPs per element of the sum-factorised general-hexahedron apply
// (Jacobian at 8 points, adjugate and determinant, gradient, flux, transpose).
constexpr double kFlopsLaplace = 1070.0;
constexpr double kFlopsElasticity = 2070.0;
// vector Laplace: the geometry (Jacobians, adjugates, determinants: 780 of the
// scalar 1,070) once, the gradient, flux and transpose (290) per component
constexpr double kFlopsVLaplace = 780.0 + 3.0 * 290.0;
// linear tetrahedra: edges, the three cross products, det; then the gradient
// and the four flux products (Laplace) or H, S and S c_a (elasticity)
constexpr double kFlopsTetLaplace = 100.0;
constexpr double kFlopsTetElasticity = 220.0;
// triquadratic hexahedra, sum-factorised model: 1,296 FLOPs per field for the
// reference gradients at the 27 points (3 coordinates + the input components)
// and as many per component for the transposed evaluation, plus the per-point
// adjugate, determinant and flux (about 70 Laplace, 150 elasticity)
constexpr double kFlopsQ2Laplace = 4 * 1296.0 + 1296.0 + 27 * 70.0;
constexpr double kFlopsQ2Elasticity = 6 * 1296.0 + 3 * 1296.0 + 27 * 150.0;
// tricubic hexahedra, the same model with 4 points per direction: 16 x 4^4 =
// 4,096 FLOPs per field and pass, plus the per-point work at 64 points
constexpr double kFlopsQ3Laplace = 4 * 4096.0 + 4096.0 + 64 * 70.0;
constexpr double kFlopsQ3Elasticity = 6 * 4096.0 + 3 * 4096.0 + 64 * 150.0;

int check_device_ptr(const void *p, const char *what) {
  if (!p) return fail(Q1_EINVAL, "%s is NULL", what);
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(Q1_EINVAL, "%s is not a device pointer (%s)", what, hipGetErrorString(e));
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(Q1_EINVAL, "%s is not device memory", what);
  return Q1_OK;
}

}  // namespace
}  // namespace q1

using namespace q1;

struct q1_op : public q1::Op {};

extern "C" {

int q1_op_create(q1_op **out, int physics, int dtype, int variant, int64_t n_nodes,
                 int64_t n_elems, const void *xyz_d, const int32_t *conn_d, const void *coef_d,
                 const uint8_t *mask_d, void *stream) {
  return q1_op_create_elem(out, Q1_HEX8, physics, dtype, variant, n_nodes, n_elems, xyz_d, conn_d,
                           coef_d, mask_d, stream);
}

int q1_op_create_elem(q1_op **out, int elem, int physics, int dtype, int variant,
                      int64_t n_nodes, int64_t n_elems, const void *xyz_d, const int32_t *conn_d,
                      const void *coef_d, const uint8_t *mask_d, void *stream) {
  Q1_CHECK(out, Q1_EINVAL, "q1_op_create: NULL handle pointer");
  *out = nullptr;
  Q1_CHECK(elem == Q1_HEX8 || elem == Q1_TET4 || elem == Q1_HEX27 || elem == Q1_HEX64, Q1_EINVAL,
           "q1_op_create: element family must be 8, 4, 27 or 64, got %d", elem);
  Q1_CHECK(physics == Q1_LAPLACE || physics == Q1_VLAPLACE || physics == Q1_ELASTICITY,
           Q1_EINVAL,
           "q1_op_create: physics must be 1 (Laplace), 2 (vector Laplace) or 3 (elasticity), "
           "got %d", physics);
  Q1_CHECK(dtype == Q1_F64 || dtype == Q1_F32, Q1_EINVAL, "q1_op_create: bad dtype %d", dtype);
  Q1_CHECK(variant == Q1_V_AUTO || variant == Q1_V_ATOMIC || variant == Q1_V_COLOR ||
               variant == Q1_V_LDS_TILE || variant == Q1_V_BLOCK || variant == Q1_V_PA,
           Q1_EINVAL, "q1_op_create: bad variant %d", variant);
  Q1_CHECK(n_nodes > 0 && n_nodes < (int64_t(1) << 31) && n_elems >= 0 &&
               n_elems < (int64_t(1) << 31),
           Q1_EINVAL, "q1_op_create: bad sizes n_nodes=%lld n_elems=%lld", (long long)n_nodes,
           (long long)n_elems);
  if (elem != Q1_HEX8) {
    Q1_CHECK(physics == Q1_LAPLACE || physics == Q1_ELASTICITY, Q1_EUNSUPPORTED,
             "q1_op_create: element family %d supports scalar Laplace and elasticity", elem);
    Q1_CHECK(variant == Q1_V_AUTO || variant == Q1_V_ATOMIC ||
                 (elem == Q1_TET4 && variant == Q1_V_BLOCK),
             Q1_EUNSUPPORTED,
             "q1_op_create: element family %d supports the atomic-scatter apply (and "
             "tetrahedra the block tiles) only", elem);
  }
  int rc;
  if ((rc = check_device_ptr(xyz_d, "xyz"))) return rc;
  if (n_elems > 0) {
    if ((rc = check_device_ptr(conn_d, "conn"))) return rc;
    if ((rc = check_device_ptr(coef_d, "coef"))) return rc;
  }
  if (mask_d && (rc = check_device_ptr(mask_d, "mask"))) return rc;
  const size_t rb = dtype == Q1_F64 ? 8 : 4;
  Q1_CHECK(reinterpret_cast<uintptr_t>(xyz_d) % rb == 0 &&
               reinterpret_cast<uintptr_t>(coef_d) % rb == 0 &&
               reinterpret_cast<uintptr_t>(conn_d) % 4 == 0,
           Q1_EINVAL, "q1_op_create: misaligned array");
  q1_op *op = new (std::nothrow) q1_op();
  Q1_CHECK(op, Q1_ENOMEM, "q1_op_create: out of host memory");
  op->physics = physics;
  op->elem = elem;
  op->dtype = dtype;
  // AUTO: the block-staged tiles (fastest measured), else the one-wave tiles, else atomics
  op->variant = variant == Q1_V_AUTO
                    ? (n_elems > 0 && (elem == Q1_HEX8 || elem == Q1_TET4) ? Q1_V_BLOCK
                                                                           : Q1_V_ATOMIC)
                    : variant;
  op->n_nodes = n_nodes;
  op->n_elems = n_elems;
  op->xyz = xyz_d;
  op->conn = conn_d;
  op->coef = coef_d;
  op->mask = mask_d;
  hipError_t e = hipGetDevice(&op->device);
  if (e == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, op->device) == hipSuccess)
      op->num_cus = prop.multiProcessorCount;
  }
  if ((rc = validate_conn(*op, static_cast<hipStream_t>(stream)))) {
    delete op;
    return rc;
  }
  if (op->variant == Q1_V_PA && n_elems == 0) {
    delete op;
    return fail(Q1_EUNSUPPORTED, "q1_op_create: partial assembly needs elements");
  }
  if (op->variant == Q1_V_LDS_TILE || op->variant == Q1_V_BLOCK || op->variant == Q1_V_PA) {
    rc = build_tiles(*op, static_cast<hipStream_t>(stream));
    if (rc && variant == Q1_V_AUTO && rc == Q1_EUNSUPPORTED && op->variant == Q1_V_BLOCK &&
        elem == Q1_HEX8) {
      free_tiles(*op);  // tiles too large for LDS: one-wave tiles
      op->variant = Q1_V_LDS_TILE;
      rc = build_tiles(*op, static_cast<hipStream_t>(stream));
    }
    if (rc) {
      free_tiles(*op);
      if (variant == Q1_V_AUTO && rc == Q1_EUNSUPPORTED) {
        op->variant = Q1_V_ATOMIC;  // mesh the tiler does not handle
      } else {
        delete op;
        return rc;
      }
    }
  }
  if (op->variant == Q1_V_COLOR && n_elems > 0) {
    rc = build_colors(*op, static_cast<hipStream_t>(stream));
    if (rc) {
      free_colors(*op);
      delete op;
      return rc;
    }
  }
  *out = op;
  return Q1_OK;
}

int q1_op_apply(q1_op *op, const void *x_d, void *y_d, void *stream) {
  Q1_CHECK(op && x_d && y_d, Q1_EINVAL, "q1_op_apply: NULL argument");
  Q1_CHECK(x_d != y_d, Q1_EINVAL, "q1_op_apply: x and y must not alias");
  const size_t rb = op->dtype == Q1_F64 ? 8 : 4;
  Q1_CHECK(reinterpret_cast<uintptr_t>(x_d) % rb == 0 &&
               reinterpret_cast<uintptr_t>(y_d) % rb == 0,
           Q1_EINVAL, "q1_op_apply: misaligned vector");
  return launch_apply(*op, x_d, y_d, static_cast<hipStream_t>(stream));
}

int q1_op_diag(q1_op *op, void *d_d, void *stream) {
  Q1_CHECK(op && d_d, Q1_EINVAL, "q1_op_diag: NULL argument");
  return launch_diag(*op, d_d, static_cast<hipStream_t>(stream));
}

int q1_op_info(const q1_op *op, int *physics, int *dtype, int *variant, int64_t *n_nodes,
               int64_t *n_elems) {
  Q1_CHECK(op, Q1_EINVAL, "q1_op_info: NULL handle");
  if (physics) *physics = op->physics;
  if (dtype) *dtype = op->dtype;
  if (variant) *variant = op->variant;
  if (n_nodes) *n_nodes = op->n_nodes;
  if (n_elems) *n_elems = op->n_elems;
  return Q1_OK;
}

int q1_op_reproducible(const q1_op *op, int *reproducible) {
  Q1_CHECK(op && reproducible, Q1_EINVAL, "q1_op_reproducible: NULL argument");
  const bool block = op->variant == Q1_V_BLOCK || op->variant == Q1_V_PA;
  *reproducible = (op->elem == Q1_HEX8 && block && op->tiles.split) ||
                          (op->variant == Q1_V_BLOCK && op->tiles.own_nx > 0)
                      ? 1
                      : 0;
  return Q1_OK;
}

int q1_op_bytes(const q1_op *op, double *bytes, double *flops) {
  Q1_CHECK(op, Q1_EINVAL, "q1_op_bytes: NULL handle");
  const int rb = op->dtype == Q1_F64 ? 8 : 4;
  if (op->variant == Q1_V_CSR) {  // values + column indices + row pointers + x read + y write
    if (bytes)
      *bytes = double(op->csr.nnz) * (rb + 4) + double(op->csr.nrows) * (4 + 2 * rb);
    if (flops) *flops = 2.0 * double(op->csr.nnz);
    return Q1_OK;
  }
  const int coef_bytes = rb * (op->physics == Q1_ELASTICITY ? 2 : 1);
  if (op->elem != Q1_HEX8) {  // Table 2's convention with 4 B per node id of the element
    const double dpn = op->dpn();
    if (bytes)
      *bytes = double(op->n_elems) * (4.0 * op->nloc() + coef_bytes) +
               double(op->n_nodes) * (3.0 * rb + 3.0 * dpn * rb);
    const bool lap = op->physics == Q1_LAPLACE;
    if (flops)
      *flops = double(op->n_elems) * (op->elem == Q1_TET4
                                          ? (lap ? kFlopsTetLaplace : kFlopsTetElasticity)
                                          : op->elem == Q1_HEX27
                                                ? (lap ? kFlopsQ2Laplace : kFlopsQ2Elasticity)
                                                : (lap ? kFlopsQ3Laplace : kFlopsQ3Elasticity));
    return Q1_OK;
  }
  double b = 0.0;
  // partial assembly: Table 3's convention (node map, cell constant, stored point data,
  // three vector streams) with this library's stored data: 6 reals per point with k folded
  // in for the Laplace kinds, 9 per point plus (lambda, mu) per cell for elasticity;
  // otherwise Table 2
  int rc = Q1_OK;
  if (op->variant == Q1_V_PA && op->physics == Q1_ELASTICITY)
    b = double(op->n_elems) * (32.0 + coef_bytes + 8.0 * 9.0 * rb) +
        double(op->n_nodes) * 3.0 * 3.0 * rb;
  else if (op->variant == Q1_V_PA)
    rc = q1_model_bytes(2, op->physics, rb, 0, op->n_nodes, op->n_elems, 0, &b);
  else
    rc = q1_model_bytes(1, op->physics, rb, coef_bytes, op->n_nodes, op->n_elems, 0, &b);
  if (rc) return rc;
  if (bytes) *bytes = b;
  if (flops)
    *flops = double(op->n_elems) * (op->physics == Q1_LAPLACE     ? kFlopsLaplace
                                    : op->physics == Q1_VLAPLACE ? kFlopsVLaplace
                                                                 : kFlopsElasticity);
  return Q1_OK;
}

int q1_op_destroy(q1_op *op) {
  if (!op) return Q1_OK;
  free_tiles(*op);
  free_csr(*op);
  free_colors(*op);
  delete op;
  return Q1_OK;
}

int q1_csr_create(q1_op **out, const q1_op *like, void *stream) {
  Q1_CHECK(out && like, Q1_EINVAL, "q1_csr_create: NULL argument");
  *out = nullptr;
  Q1_CHECK(like->elem == Q1_HEX8, Q1_EUNSUPPORTED,
           "q1_csr_create: the CSR comparison is built for trilinear hexahedra");
  q1_op *op = new (std::nothrow) q1_op();
  Q1_CHECK(op, Q1_ENOMEM, "q1_csr_create: out of host memory");
  static_cast<Op &>(*op) = static_cast<const Op &>(*like);
  op->tiles = TileMap{};
  op->csr = CsrData{};
  op->colors = ColorMap{};
  op->variant = Q1_V_CSR;
  const int rc = csr_create(*op, static_cast<hipStream_t>(stream));
  if (rc) {
    free_csr(*op);
    delete op;
    return rc;
  }
  *out = op;
  return Q1_OK;
}

int q1_csr_info(const q1_op *op, int64_t *nrows, int64_t *nnz) {
  Q1_CHECK(op && op->variant == Q1_V_CSR, Q1_EINVAL, "q1_csr_info: not a CSR operator");
  if (nrows) *nrows = op->csr.nrows;
  if (nnz) *nnz = op->csr.nnz;
  return Q1_OK;
}

int q1_csr_export(const q1_op *op, int32_t *rowptr, int32_t *col, void *val) {
  Q1_CHECK(op && op->variant == Q1_V_CSR, Q1_EINVAL, "q1_csr_export: not a CSR operator");
  const CsrData &m = op->csr;
  const size_t rb = op->dtype == Q1_F64 ? 8 : 4;
  if (rowptr)
    Q1_HIP(hipMemcpy(rowptr, m.rowptr, size_t(m.nrows + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (col && m.nnz)
    Q1_HIP(hipMemcpy(col, m.col, size_t(m.nnz) * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (val && m.nnz) Q1_HIP(hipMemcpy(val, m.val, size_t(m.nnz) * rb, hipMemcpyDeviceToHost));
  return Q1_OK;
}

}  // extern "C"
