// Matrix-based comparison: CSR assembly and SpMV of the same operator.
//
// Pattern (host, set-up): the columns of row (n, c) are all DOFs of the nodes
// sharing an element with node n, sorted.  Fill (device): one thread per
// element computes its element matrix column by column (the element product of
// q1_elem.hpp applied to unit vectors), finds each entry's column in the
// sorted row by binary search and adds it atomically -- the search-and-add
// assembly of Section 3.  Dirichlet rows and columns are then eliminated
// symmetrically (A_cc = 1).  SpMV: a group of lanes per row, each lane strides
// over the row's entries, and the group sums with cross-lane reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "q1_elem.hpp"
#include "q1_internal.hpp"

namespace q1 {

__device__ __forceinline__ void atomic_add_v(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_v(float *p, float v) { unsafeAtomicAdd(p, v); }

__device__ __forceinline__ int find_col(const int32_t *__restrict__ col, int lo, int hi,
                                        int32_t c) {
  // [lo, hi) sorted; returns position or -1
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int32_t v = col[mid];
    if (v == c) return mid;
    if (v < c) lo = mid + 1; else hi = mid;
  }
  return -1;
}

template <typename T, int PH>
__global__ __launch_bounds__(64) void k_csr_fill(int64_t ne, int64_t nn,
                                                 const T *__restrict__ xyz,
                                                 const int32_t *__restrict__ conn,
                                                 const T *__restrict__ coef,
                                                 const uint8_t *__restrict__ mask,
                                                 const int32_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ col,
                                                 T *__restrict__ val, int *__restrict__ missing) {
  constexpr int DPN = phys_dpn(PH);
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  int32_t nid[8];
  T X0[3][8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    nid[a] = conn[a * ne + e];
#pragma unroll
    for (int r = 0; r < 3; ++r) X0[r][a] = xyz[r * nn + nid[a]];
  }
  // column (b, j) of the element matrix = element product with a unit vector
  for (int b = 0; b < 8; ++b) {
    if (mask && mask[nid[b]]) continue;  // eliminated column
    for (int jb = 0; jb < DPN; ++jb) {
      T X[3][8];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int a = 0; a < 8; ++a) X[r][a] = X0[r][a];
      T colv[DPN][8], u[DPN][8];
#pragma unroll
      for (int j = 0; j < DPN; ++j)
#pragma unroll
        for (int a = 0; a < 8; ++a) u[j][a] = (a == b && j == jb) ? T(1) : T(0);
      element_apply<T, PH>(X, u, coef[e], PH == 3 ? coef[ne + e] : T(0), colv);
      const int32_t cidx = nid[b] * DPN + jb;
      for (int a = 0; a < 8; ++a) {
        if (mask && mask[nid[a]]) continue;  // eliminated row
        for (int ja = 0; ja < DPN; ++ja) {
          const int64_t row = int64_t(nid[a]) * DPN + ja;
          const int pos = find_col(col, rowptr[row], rowptr[row + 1], cidx);
          if (pos < 0) {
            atomicAdd(missing, 1);
            continue;
          }
          atomic_add_v(&val[pos], colv[ja][a]);
        }
      }
    }
  }
}

// Dirichlet rows: identity (the columns were never filled)
template <typename T, int DPN>
__global__ void k_csr_dirichlet(int64_t nn, const uint8_t *__restrict__ mask,
                                const int32_t *__restrict__ rowptr,
                                const int32_t *__restrict__ col, T *__restrict__ val) {
  const int64_t row = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (row >= nn * DPN || !mask[row / DPN]) return;
  for (int t = rowptr[row]; t < rowptr[row + 1]; ++t) val[t] = col[t] == row ? T(1) : T(0);
}

// y = A x with G lanes per row (G divides 64).
template <typename T, int G>
__global__ __launch_bounds__(256) void k_spmv(int64_t nrows, const int32_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ col,
                                              const T *__restrict__ val, const T *__restrict__ x,
                                              T *__restrict__ y, const int *__restrict__ stop) {
  if (stop && *stop) return;
  const int64_t gt = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t row = gt / G;
  const int sub = threadIdx.x % G;
  T s = T(0);
  if (row < nrows) {
    const int b = rowptr[row], e = rowptr[row + 1];
    for (int t = b + sub; t < e; t += G) s += val[t] * x[col[t]];
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
  if (row < nrows && sub == 0) y[row] = s;
}

namespace {

int build_pattern(int dpn, int64_t nn, int64_t ne, const std::vector<int32_t> &conn,
                  std::vector<int32_t> &rowptr, std::vector<int32_t> &col) {
  for (size_t i = 0; i < conn.size(); ++i)
    Q1_CHECK(conn[i] >= 0 && conn[i] < nn, Q1_EINVAL, "CSR pattern: connectivity entry %zu out of range", i);
  std::vector<int64_t> nptr(nn + 1, 0);
  for (int a = 0; a < 8; ++a)
    for (int64_t e = 0; e < ne; ++e) nptr[conn[a * ne + e] + 1]++;
  for (int64_t n = 0; n < nn; ++n) nptr[n + 1] += nptr[n];
  std::vector<int32_t> nel(nptr[nn]);
  std::vector<int64_t> fill(nptr.begin(), nptr.end() - 1);
  for (int64_t e = 0; e < ne; ++e)
    for (int a = 0; a < 8; ++a) nel[fill[conn[a * ne + e]]++] = int32_t(e);
  rowptr.assign(nn * dpn + 1, 0);
  std::vector<int32_t> nb;
  // count
  std::vector<int32_t> cnt(nn);
  for (int64_t n = 0; n < nn; ++n) {
    nb.assign(1, int32_t(n));  // the diagonal, also for a node no element references
    for (int64_t t = nptr[n]; t < nptr[n + 1]; ++t)
      for (int a = 0; a < 8; ++a) nb.push_back(conn[a * ne + nel[t]]);
    std::sort(nb.begin(), nb.end());
    cnt[n] = int32_t(std::unique(nb.begin(), nb.end()) - nb.begin());
  }
  int64_t nnz = 0;
  for (int64_t n = 0; n < nn; ++n)
    for (int c = 0; c < dpn; ++c) {
      nnz += int64_t(cnt[n]) * dpn;
      if (nnz >= (int64_t(1) << 31)) return fail(Q1_EUNSUPPORTED, "CSR with >= 2^31 non-zeros");
      rowptr[n * dpn + c + 1] = int32_t(nnz);
    }
  col.resize(nnz);
  for (int64_t n = 0; n < nn; ++n) {
    nb.assign(1, int32_t(n));  // the diagonal, also for a node no element references
    for (int64_t t = nptr[n]; t < nptr[n + 1]; ++t)
      for (int a = 0; a < 8; ++a) nb.push_back(conn[a * ne + nel[t]]);
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    for (int c = 0; c < dpn; ++c) {
      int32_t *dst = &col[rowptr[n * dpn + c]];
      for (size_t t = 0; t < nb.size(); ++t)
        for (int d = 0; d < dpn; ++d) *dst++ = nb[t] * dpn + d;
    }
  }
  return Q1_OK;
}

template <typename T>
int csr_create_t(Op &op, hipStream_t s) {
  CsrData &m = op.csr;
  const int dpn = op.dpn();
  const int64_t nn = op.n_nodes, ne = op.n_elems;
  std::vector<int32_t> conn(size_t(8) * ne), rowptr, col;
  Q1_HIP(hipStreamSynchronize(s));
  if (ne > 0)
    Q1_HIP(hipMemcpy(conn.data(), op.conn, conn.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  int rc = build_pattern(dpn, nn, ne, conn, rowptr, col);
  if (rc) return rc;
  m.nrows = nn * dpn;
  m.nnz = int64_t(col.size());
  Q1_HIP(hipMalloc(&m.rowptr, rowptr.size() * sizeof(int32_t)));
  Q1_HIP(hipMalloc(&m.col, std::max<size_t>(1, col.size()) * sizeof(int32_t)));
  Q1_HIP(hipMalloc(&m.val, std::max<size_t>(1, col.size()) * sizeof(T)));
  Q1_HIP(hipMemcpy(m.rowptr, rowptr.data(), rowptr.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  if (!col.empty())
    Q1_HIP(hipMemcpy(m.col, col.data(), col.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  Q1_HIP(hipMemsetAsync(m.val, 0, std::max<size_t>(1, col.size()) * sizeof(T), s));
  int *missing = nullptr;
  Q1_HIP(hipMalloc(&missing, sizeof(int)));
  Q1_HIP(hipMemsetAsync(missing, 0, sizeof(int), s));
  if (ne > 0) {
    const dim3 grid(unsigned((ne + 63) / 64));
    auto fill = op.physics == 1 ? k_csr_fill<T, 1> : op.physics == 2 ? k_csr_fill<T, 2>
                                                                      : k_csr_fill<T, 3>;
    hipLaunchKernelGGL(fill, grid, dim3(64), 0, s, ne, nn, static_cast<const T *>(op.xyz),
                       op.conn, static_cast<const T *>(op.coef), op.mask, m.rowptr, m.col,
                       static_cast<T *>(m.val), missing);
  }
  if (op.mask) {
    const dim3 grid(unsigned((m.nrows + 255) / 256));
    if (dpn == 1)
      hipLaunchKernelGGL((k_csr_dirichlet<T, 1>), grid, dim3(256), 0, s, nn, op.mask, m.rowptr,
                         m.col, static_cast<T *>(m.val));
    else
      hipLaunchKernelGGL((k_csr_dirichlet<T, 3>), grid, dim3(256), 0, s, nn, op.mask, m.rowptr,
                         m.col, static_cast<T *>(m.val));
  }
  Q1_HIP(hipGetLastError());
  int h_missing = 0;
  Q1_HIP(hipMemcpyAsync(&h_missing, missing, sizeof(int), hipMemcpyDeviceToHost, s));
  Q1_HIP(hipStreamSynchronize(s));
  (void)hipFree(missing);
  Q1_CHECK(h_missing == 0, Q1_EINVAL, "CSR fill: %d entries outside the pattern", h_missing);
  return Q1_OK;
}

template <typename T>
int spmv_t(const Op &op, const void *xv, void *yv, hipStream_t s, const int *stop) {
  const CsrData &m = op.csr;
  const T *x = static_cast<const T *>(xv);
  T *y = static_cast<T *>(yv);
  // 27 entries per row (scalar) -> 16 lanes; 81 (3 DOF per node) -> 32 lanes
  if (op.dpn() == 1) {
    const int64_t thr = m.nrows * 16;
    hipLaunchKernelGGL((k_spmv<T, 16>), dim3(unsigned((thr + 255) / 256)), dim3(256), 0, s,
                       m.nrows, m.rowptr, m.col, static_cast<const T *>(m.val), x, y, stop);
  } else {
    const int64_t thr = m.nrows * 32;
    hipLaunchKernelGGL((k_spmv<T, 32>), dim3(unsigned((thr + 255) / 256)), dim3(256), 0, s,
                       m.nrows, m.rowptr, m.col, static_cast<const T *>(m.val), x, y, stop);
  }
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

}  // namespace

int csr_create(Op &op, hipStream_t s) {
  return op.dtype == Q1_F64 ? csr_create_t<double>(op, s) : csr_create_t<float>(op, s);
}

int launch_spmv(const Op &op, const void *x, void *y, hipStream_t s, const int *stop) {
  return op.dtype == Q1_F64 ? spmv_t<double>(op, x, y, s, stop) : spmv_t<float>(op, x, y, s, stop);
}

void free_csr(Op &op) {
  CsrData &m = op.csr;
  if (m.rowptr) (void)hipFree(m.rowptr);
  if (m.col) (void)hipFree(m.col);
  if (m.val) (void)hipFree(m.val);
  m = CsrData{};
}

}  // namespace q1
