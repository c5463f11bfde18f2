// Matrix-free apply y = A x and diagonal of the Q1 operators: the three steps
// of Section 3 (gather u_e, local product v_e = A_e u_e, scatter-add v_e)
// with the element arithmetic of q1_elem.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "q1_elem.hpp"
#include "q1_internal.hpp"

namespace q1 {

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical blocks so that neighbouring elements (which
// share nodes) run behind the same L2.
__device__ __forceinline__ int xcd_block(int bid, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int x = bid & 7, local = bid >> 3;
  return x * q + min(x, r) + local;
}

// y = masked ? x : 0 (start of an accumulating apply)
template <typename T, int DPN>
__global__ void k_init_masked(int64_t n_nodes, const uint8_t *__restrict__ mask,
                              const T *__restrict__ x, T *__restrict__ y,
                              const int *__restrict__ stop) {
  if (stop && *stop) return;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_nodes * DPN) return;
  y[i] = (mask && mask[i / DPN]) ? x[i] : T(0);
}

template <typename T, int DPN>
__global__ void k_init_diag(int64_t n_nodes, const uint8_t *__restrict__ mask, T *__restrict__ d) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_nodes * DPN) return;
  d[i] = (mask && mask[i / DPN]) ? T(1) : T(0);
}

__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }

// One thread per element, global atomics for the scatter (the paper's
// one-thread-per-element strategy).
template <typename T, int PH, bool MASKED>
__global__ __launch_bounds__(256) void k_apply_atomic(
    int64_t ne, int64_t nn, const T *__restrict__ xyz, const int32_t *__restrict__ conn,
    const T *__restrict__ coef, const uint8_t *__restrict__ mask, const T *__restrict__ x,
    T *__restrict__ y, const int *__restrict__ stop) {
  constexpr int DPN = phys_dpn(PH);
  if (stop && *stop) return;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t e = int64_t(blk) * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  int32_t nid[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) nid[a] = conn[a * ne + e];
  T X[3][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int r = 0; r < 3; ++r) X[r][a] = xyz[r * nn + nid[a]];
  bool fixed[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) fixed[a] = MASKED ? (mask[nid[a]] != 0) : false;
  T u[DPN][8], v[DPN][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int j = 0; j < DPN; ++j) u[j][a] = fixed[a] ? T(0) : x[int64_t(nid[a]) * DPN + j];
  element_apply<T, PH>(X, u, coef[e], PH == 3 ? coef[ne + e] : T(0), v);
#pragma unroll
  for (int a = 0; a < 8; ++a)
    if (!fixed[a])
#pragma unroll
      for (int j = 0; j < DPN; ++j) atomic_add(&y[int64_t(nid[a]) * DPN + j], v[j][a]);
}

// One thread per element of one colour class [e0, e1) of the colour order: no
// two elements of a class share a node, so the scatter is a plain
// read-add-write; kernel boundaries order the classes.
template <typename T, int PH, bool MASKED>
__global__ __launch_bounds__(256) void k_apply_color(
    int64_t e0, int64_t e1, int64_t ne, int64_t nn, const T *__restrict__ xyz,
    const int32_t *__restrict__ conn, const T *__restrict__ coef,
    const uint8_t *__restrict__ mask, const T *__restrict__ x, T *__restrict__ y,
    const int *__restrict__ stop) {
  constexpr int DPN = phys_dpn(PH);
  if (stop && *stop) return;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t e = e0 + int64_t(blk) * blockDim.x + threadIdx.x;
  if (e >= e1) return;
  int32_t nid[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) nid[a] = conn[a * ne + e];
  T X[3][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int r = 0; r < 3; ++r) X[r][a] = xyz[r * nn + nid[a]];
  bool fixed[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) fixed[a] = MASKED ? (mask[nid[a]] != 0) : false;
  T u[DPN][8], v[DPN][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int j = 0; j < DPN; ++j) u[j][a] = fixed[a] ? T(0) : x[int64_t(nid[a]) * DPN + j];
  element_apply<T, PH>(X, u, coef[e], PH == 3 ? coef[ne + e] : T(0), v);
#pragma unroll
  for (int a = 0; a < 8; ++a)
    if (!fixed[a])
#pragma unroll
      for (int j = 0; j < DPN; ++j) y[int64_t(nid[a]) * DPN + j] += v[j][a];
}

// Diagonal of A: d_(a,i) += the element diagonal entries (element_diag),
// added with global atomics (order of additions varies between runs).
template <typename T, int PH, bool MASKED>
__global__ __launch_bounds__(256) void k_diag(int64_t ne, int64_t nn,
                                              const T *__restrict__ xyz,
                                              const int32_t *__restrict__ conn,
                                              const T *__restrict__ coef,
                                              const uint8_t *__restrict__ mask,
                                              T *__restrict__ d) {
  constexpr int DPN = phys_dpn(PH);
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  int32_t nid[8];
  T X[3][8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    nid[a] = conn[a * ne + e];
#pragma unroll
    for (int r = 0; r < 3; ++r) X[r][a] = xyz[r * nn + nid[a]];
  }
  T acc[DPN][8];
  element_diag<T, PH>(X, coef[e], PH == 3 ? coef[ne + e] : T(0), acc);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    if (MASKED && mask[nid[a]]) continue;
#pragma unroll
    for (int i = 0; i < DPN; ++i) atomic_add(&d[int64_t(nid[a]) * DPN + i], acc[i][a]);
  }
}

namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t n, int block) { return int((n + block - 1) / block); }

template <typename T, int PH>
int apply_atomic(Op &op, const void *xv, void *yv, hipStream_t s, const int *stop) {
  constexpr int DPN = phys_dpn(PH);
  const T *x = static_cast<const T *>(xv);
  T *y = static_cast<T *>(yv);
  const int64_t ndof = op.n_nodes * DPN;
  hipLaunchKernelGGL((k_init_masked<T, DPN>), dim3(grid_for(ndof, kBlock)), dim3(kBlock), 0, s,
                     op.n_nodes, op.mask, x, y, stop);
  if (op.n_elems == 0) return Q1_OK;
  const dim3 grid(grid_for(op.n_elems, kBlock));
  const T *xyz = static_cast<const T *>(op.xyz);
  const T *coef = static_cast<const T *>(op.coef);
  if (op.mask)
    hipLaunchKernelGGL((k_apply_atomic<T, PH, true>), grid, dim3(kBlock), 0, s, op.n_elems,
                       op.n_nodes, xyz, op.conn, coef, op.mask, x, y, stop);
  else
    hipLaunchKernelGGL((k_apply_atomic<T, PH, false>), grid, dim3(kBlock), 0, s, op.n_elems,
                       op.n_nodes, xyz, op.conn, coef, op.mask, x, y, stop);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

template <typename T, int PH>
int apply_color(Op &op, const void *xv, void *yv, hipStream_t s, const int *stop) {
  constexpr int DPN = phys_dpn(PH);
  const T *x = static_cast<const T *>(xv);
  T *y = static_cast<T *>(yv);
  const int64_t ndof = op.n_nodes * DPN;
  hipLaunchKernelGGL((k_init_masked<T, DPN>), dim3(grid_for(ndof, kBlock)), dim3(kBlock), 0, s,
                     op.n_nodes, op.mask, x, y, stop);
  const ColorMap &cm = op.colors;
  const T *xyz = static_cast<const T *>(op.xyz);
  const T *coef = static_cast<const T *>(cm.coef);
  for (int c = 0; c < cm.n_colors; ++c) {
    const int64_t e0 = cm.ptr[c], e1 = cm.ptr[c + 1];
    if (e1 <= e0) continue;
    const dim3 grid(grid_for(e1 - e0, kBlock));
    if (op.mask)
      hipLaunchKernelGGL((k_apply_color<T, PH, true>), grid, dim3(kBlock), 0, s, e0, e1,
                         op.n_elems, op.n_nodes, xyz, cm.conn, coef, op.mask, x, y, stop);
    else
      hipLaunchKernelGGL((k_apply_color<T, PH, false>), grid, dim3(kBlock), 0, s, e0, e1,
                         op.n_elems, op.n_nodes, xyz, cm.conn, coef, op.mask, x, y, stop);
  }
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

template <typename T, int PH>
int diag_impl(Op &op, void *dv, hipStream_t s) {
  constexpr int DPN = phys_dpn(PH);
  T *d = static_cast<T *>(dv);
  const int64_t ndof = op.n_nodes * DPN;
  hipLaunchKernelGGL((k_init_diag<T, DPN>), dim3(grid_for(ndof, kBlock)), dim3(kBlock), 0, s,
                     op.n_nodes, op.mask, d);
  if (op.n_elems > 0) {
    const dim3 grid(grid_for(op.n_elems, kBlock));
    const T *xyz = static_cast<const T *>(op.xyz);
    const T *coef = static_cast<const T *>(op.coef);
    if (op.mask)
      hipLaunchKernelGGL((k_diag<T, PH, true>), grid, dim3(kBlock), 0, s, op.n_elems,
                         op.n_nodes, xyz, op.conn, coef, op.mask, d);
    else
      hipLaunchKernelGGL((k_diag<T, PH, false>), grid, dim3(kBlock), 0, s, op.n_elems,
                         op.n_nodes, xyz, op.conn, coef, op.mask, d);
  }
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

}  // namespace

int launch_apply(Op &op, const void *x, void *y, hipStream_t s, const int *stop) {
  if (op.elem != Q1_HEX8) return launch_apply_family(op, x, y, s, stop);
  switch (op.variant) {
    case Q1_V_ATOMIC:
      return dispatch_phys(op, [&](auto t, auto ph) {
        return apply_atomic<decltype(t), decltype(ph)::value>(op, x, y, s, stop);
      });
    case Q1_V_COLOR:
      return dispatch_phys(op, [&](auto t, auto ph) {
        return apply_color<decltype(t), decltype(ph)::value>(op, x, y, s, stop);
      });
    case Q1_V_LDS_TILE:
    case Q1_V_BLOCK:
    case Q1_V_PA:
      return launch_apply_tile(op, x, y, s, stop);
    case Q1_V_CSR:
      return launch_spmv(op, x, y, s, stop);
    default:
      return fail(Q1_EUNSUPPORTED, "apply variant %d not available", op.variant);
  }
}

// Greedy first-fit colouring in element order: each element takes the lowest
// colour not yet used by an element sharing one of its nodes (per-node
// bitmasks of used colours).  On a lattice numbered lexicographically this
// gives the 8 parity classes.  Connectivity and coefficients are copied in
// colour order so that each class is read contiguously.
int build_colors(Op &op, hipStream_t s) {
  const int64_t ne = op.n_elems, nn = op.n_nodes;
  const int ncoef = phys_ncoef(op.physics);
  const size_t rb = op.dtype == Q1_F64 ? 8 : 4;
  Q1_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> conn(size_t(8) * ne);
  std::vector<unsigned char> coef(size_t(ncoef) * ne * rb);
  Q1_HIP(hipMemcpy(conn.data(), op.conn, conn.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  Q1_HIP(hipMemcpy(coef.data(), op.coef, coef.size(), hipMemcpyDeviceToHost));
  std::vector<uint64_t> used(nn, 0);
  std::vector<int> color(ne);
  int n_colors = 0;
  for (int64_t e = 0; e < ne; ++e) {
    uint64_t taken = 0;
    for (int a = 0; a < 8; ++a) {
      const int32_t g = conn[a * ne + e];
      Q1_CHECK(g >= 0 && g < nn, Q1_EINVAL, "colouring: node id %d of element %lld out of range",
               g, (long long)e);
      taken |= used[g];
    }
    Q1_CHECK(~taken != 0, Q1_EUNSUPPORTED, "colouring needs more than 64 colours");
    const int c = __builtin_ctzll(~taken);
    color[e] = c;
    n_colors = std::max(n_colors, c + 1);
    for (int a = 0; a < 8; ++a) used[conn[a * ne + e]] |= uint64_t(1) << c;
  }
  ColorMap &cm = op.colors;
  cm.n_colors = n_colors;
  cm.ptr.assign(n_colors + 1, 0);
  for (int64_t e = 0; e < ne; ++e) ++cm.ptr[color[e] + 1];
  for (int c = 0; c < n_colors; ++c) cm.ptr[c + 1] += cm.ptr[c];
  std::vector<int64_t> next(cm.ptr.begin(), cm.ptr.end() - 1);
  std::vector<int32_t> pconn(conn.size());
  std::vector<unsigned char> pcoef(coef.size());
  for (int64_t e = 0; e < ne; ++e) {
    const int64_t p = next[color[e]]++;
    for (int a = 0; a < 8; ++a) pconn[a * ne + p] = conn[a * ne + e];
    for (int k = 0; k < ncoef; ++k)
      std::memcpy(&pcoef[(size_t(k) * ne + p) * rb], &coef[(size_t(k) * ne + e) * rb], rb);
  }
  Q1_HIP(hipMalloc(&cm.conn, pconn.size() * sizeof(int32_t)));
  Q1_HIP(hipMalloc(&cm.coef, pcoef.size()));
  Q1_HIP(hipMemcpy(cm.conn, pconn.data(), pconn.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  Q1_HIP(hipMemcpy(cm.coef, pcoef.data(), pcoef.size(), hipMemcpyHostToDevice));
  return Q1_OK;
}

void free_colors(Op &op) {
  if (op.colors.conn) (void)hipFree(op.colors.conn);
  if (op.colors.coef) (void)hipFree(op.colors.coef);
  op.colors = ColorMap{};
}

// bad[0] = 1 when some connectivity entry is outside [0, nn)
__global__ void k_check_conn(int64_t n, const int32_t *__restrict__ conn, int64_t nn,
                             int *__restrict__ bad) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && (conn[i] < 0 || conn[i] >= nn)) bad[0] = 1;
}

int validate_conn(const Op &op, hipStream_t s) {
  if (op.n_elems == 0) return Q1_OK;
  int *bad = nullptr;
  Q1_HIP(hipMalloc(&bad, sizeof(int)));
  struct Free {
    int *p;
    ~Free() { (void)hipFree(p); }
  } fr{bad};
  const int64_t n = int64_t(op.nloc()) * op.n_elems;
  int h = 0;
  Q1_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_check_conn, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, n, op.conn,
                     op.n_nodes, bad);
  Q1_HIP(hipGetLastError());
  Q1_HIP(hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  Q1_HIP(hipStreamSynchronize(s));
  Q1_CHECK(h == 0, Q1_EINVAL, "connectivity holds a node id outside [0, %lld)",
           (long long)op.n_nodes);
  return Q1_OK;
}

int launch_diag(Op &op, void *d, hipStream_t s) {
  if (op.elem == Q1_TET4 && op.variant == Q1_V_BLOCK && op.tiles.own_nx > 0)
    return launch_diag_owner(op, d, s);
  if (op.elem != Q1_HEX8) return launch_diag_family(op, d, s);
  if ((op.variant == Q1_V_BLOCK || op.variant == Q1_V_PA) && op.tiles.split)
    return launch_diag_tile(op, d, s);
  return dispatch_phys(op, [&](auto t, auto ph) {
    return diag_impl<decltype(t), decltype(ph)::value>(op, d, s);
  });
}

}  // namespace q1
