// Fused Jacobi-PCG for small problems: the whole solve in ONE workgroup of 8
// wavefronts and one launch.  The CG operations of Table 4 (apply, two dot
// products, three vector updates) run back to back with workgroup barriers in
// place of kernel boundaries (the paper names CG fusion as work it did not
// do); q = A p is accumulated in LDS (LDS atomics), so the DOF vector must fit
// in LDS.  Per iteration:
//   q = A p (element loop over all elements; Dirichlet rows q = p)
//   alpha = rho / p.q; x += alpha p; r -= alpha q; z = D^-1 r; rho' = r.z; r.r
//   stop when ||r|| <= rtol ||b||; beta = rho'/rho; p = z + beta p
// Every reduction is a fixed-order sum of the 8 wavefront partials, read by
// every thread, so all threads take the same branch.  After the loop the
// kernel applies A to x once more and returns the FP64 true residual.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>

#include "q1_elem.hpp"
#include "q1_internal.hpp"

namespace q1 {
namespace {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr size_t kLdsLimit = 64 * 1024;
constexpr size_t kRedBytes = 2 * kWaves * 2 * sizeof(double);

struct FusedArgs {
  int64_t nn, ne;
  const double *xyz;
  const int32_t *conn;
  const double *coef;
  const uint8_t *mask;
  const double *w;  // inverse diagonal, or NULL (no preconditioner)
  const double *b;
  double *x, *r, *p;
  double tol2;
  int maxit;
  int *out_iters, *out_status;
  double *out_rr, *out_bb, *out_true_rr;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// (a, b) summed over the workgroup in a fixed order; every thread gets the sums.
// Two buffers alternate, so a buffer is rewritten only after a later barrier.
__device__ __forceinline__ void block_sum2(double &a, double &b, double *red, int &phase) {
  a = wave_sum(a);
  b = wave_sum(b);
  double *buf = red + phase * 2 * kWaves;
  phase ^= 1;
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    buf[2 * w] = a;
    buf[2 * w + 1] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    sa += buf[2 * i];
    sb += buf[2 * i + 1];
  }
  a = sa;
  b = sb;
}

// q (LDS, zero on entry) += A_e src_e over all elements; Dirichlet corners read
// zero and receive nothing.  Ends with a barrier.
template <int PH>
__device__ __forceinline__ void apply_lds(const FusedArgs &A, const double *src, double *q) {
  constexpr int DPN = phys_dpn(PH);
  for (int64_t e = threadIdx.x; e < A.ne; e += kThreads) {
    int64_t g[8];
    bool fx[8];
    double X[3][8], u[DPN][8], v[DPN][8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      g[a] = A.conn[a * A.ne + e];
      fx[a] = A.mask && A.mask[g[a]];
#pragma unroll
      for (int d = 0; d < 3; ++d) X[d][a] = A.xyz[d * A.nn + g[a]];
#pragma unroll
      for (int j = 0; j < DPN; ++j) u[j][a] = fx[a] ? 0.0 : src[g[a] * DPN + j];
    }
    element_apply<double, PH>(X, u, A.coef[e], PH == 3 ? A.coef[A.ne + e] : 0.0, v);
#pragma unroll
    for (int a = 0; a < 8; ++a)
      if (!fx[a])
#pragma unroll
        for (int j = 0; j < DPN; ++j)
          __hip_atomic_fetch_add(&q[g[a] * DPN + j], v[j][a], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __syncthreads();
}

template <int PH>
__global__ __launch_bounds__(kThreads) void k_pcg_fused(FusedArgs A) {
  constexpr int DPN = phys_dpn(PH);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *red = reinterpret_cast<double *>(smem_raw);  // [2][kWaves][2]
  double *q = red + 4 * kWaves;                         // [n]
  const int64_t n = A.nn * DPN;
  const int tid = threadIdx.x;
  int phase = 0;
  auto fixed = [&](int64_t i) { return A.mask && A.mask[i / DPN]; };
  // x = 0, r = b, p = z = D^-1 b; rho = b.z, bb = b.b
  double rho = 0.0, bb = 0.0;
  for (int64_t i = tid; i < n; i += kThreads) {
    const double bi = A.b[i];
    const double zi = A.w ? A.w[i] * bi : bi;
    A.x[i] = 0.0;
    A.r[i] = bi;
    A.p[i] = zi;
    q[i] = 0.0;
    rho += bi * zi;
    bb += bi * bi;
  }
  block_sum2(rho, bb, red, phase);  // its barrier also publishes p and the zeroed q
  int it = 0, status = Q1_ENOCONV;
  double rr = bb;
  if (!(bb > 0.0)) status = Q1_OK;
  while (status == Q1_ENOCONV && it < A.maxit) {
    ++it;
    apply_lds<PH>(A, A.p, q);
    double pq = 0.0, unused = 0.0;
    for (int64_t i = tid; i < n; i += kThreads) {
      const double pi = A.p[i];
      const double qi = fixed(i) ? pi : q[i];  // Dirichlet rows: the entry itself
      q[i] = qi;
      pq += pi * qi;
    }
    block_sum2(pq, unused, red, phase);
    if (!(pq > 0.0) || !isfinite(pq)) {
      status = Q1_EBREAKDOWN;
      break;
    }
    const double alpha = rho / pq;
    double rho1 = 0.0;
    rr = 0.0;
    for (int64_t i = tid; i < n; i += kThreads) {
      A.x[i] += alpha * A.p[i];
      const double ri = A.r[i] - alpha * q[i];
      A.r[i] = ri;
      const double zi = A.w ? A.w[i] * ri : ri;
      rho1 += ri * zi;
      rr += ri * ri;
    }
    block_sum2(rho1, rr, red, phase);
    if (rr <= A.tol2 * bb) {
      status = Q1_OK;
      break;
    }
    if (!isfinite(rr)) {
      status = Q1_EBREAKDOWN;
      break;
    }
    const double beta = rho1 / rho;
    rho = rho1;
    for (int64_t i = tid; i < n; i += kThreads) {
      const double zi = A.w ? A.w[i] * A.r[i] : A.r[i];
      A.p[i] = zi + beta * A.p[i];
      q[i] = 0.0;
    }
    __syncthreads();  // p and the zeroed q before the next element loop
  }
  // true residual b - A x in FP64
  for (int64_t i = tid; i < n; i += kThreads) q[i] = 0.0;
  __syncthreads();
  apply_lds<PH>(A, A.x, q);
  double tr = 0.0, unused = 0.0;
  for (int64_t i = tid; i < n; i += kThreads) {
    const double ax = fixed(i) ? A.x[i] : q[i];
    const double d = A.b[i] - ax;
    tr += d * d;
  }
  block_sum2(tr, unused, red, phase);
  if (tid == 0) {
    *A.out_iters = it;
    *A.out_status = status;
    *A.out_rr = rr;
    *A.out_bb = bb;
    *A.out_true_rr = tr;
  }
}

__global__ void k_inv(int64_t n, double *__restrict__ d) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) d[i] = d[i] != 0.0 ? 1.0 / d[i] : 0.0;  // 0 on zero rows (unreferenced nodes)
}

}  // namespace
}  // namespace q1

using namespace q1;

extern "C" int q1_pcg_fused(q1_op *opv, int pc, const double *b_d, double *x_d, double rtol,
                            int maxit, q1_stats *st, void *stream) {
  Q1_CHECK(opv && b_d && x_d, Q1_EINVAL, "q1_pcg_fused: NULL argument");
  Q1_CHECK(pc == Q1_PC_NONE || pc == Q1_PC_JACOBI, Q1_EINVAL, "q1_pcg_fused: bad preconditioner");
  Q1_CHECK(rtol >= 0 && maxit >= 0, Q1_EINVAL, "q1_pcg_fused: need rtol >= 0 and maxit >= 0");
  Op &op = *reinterpret_cast<Op *>(opv);
  Q1_CHECK(op.dtype == Q1_F64, Q1_EUNSUPPORTED, "q1_pcg_fused: needs an FP64 operator");
  Q1_CHECK(op.elem == Q1_HEX8, Q1_EUNSUPPORTED, "q1_pcg_fused: needs trilinear hexahedra");
  const int64_t n = op.n_nodes * op.dpn();
  const size_t lds = kRedBytes + size_t(n) * sizeof(double);
  Q1_CHECK(lds <= kLdsLimit, Q1_EUNSUPPORTED,
           "q1_pcg_fused: %lld DOF do not fit in LDS (at most %zu)", (long long)n,
           (kLdsLimit - kRedBytes) / sizeof(double));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const auto t0 = std::chrono::steady_clock::now();
  // workspace: r, p, inverse diagonal, five result words
  double *ws = nullptr;
  const size_t nws = size_t(3 * n) + 8;
  Q1_HIP(hipMalloc(&ws, nws * sizeof(double)));
  struct Free {
    double *p;
    ~Free() { (void)hipFree(p); }
  } fr{ws};
  double *r = ws, *p = ws + n, *w = ws + 2 * n, *res = ws + 3 * n;
  if (pc == Q1_PC_JACOBI) {
    int rc = launch_diag(op, w, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_inv, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, n, w);
  }
  FusedArgs A;
  A.nn = op.n_nodes;
  A.ne = op.n_elems;
  A.xyz = static_cast<const double *>(op.xyz);
  A.conn = op.conn;
  A.coef = static_cast<const double *>(op.coef);
  A.mask = op.mask;
  A.w = pc == Q1_PC_JACOBI ? w : nullptr;
  A.b = b_d;
  A.x = x_d;
  A.r = r;
  A.p = p;
  A.tol2 = rtol * rtol;
  A.maxit = maxit;
  A.out_iters = reinterpret_cast<int *>(res);
  A.out_status = reinterpret_cast<int *>(res + 1);
  A.out_rr = res + 2;
  A.out_bb = res + 3;
  A.out_true_rr = res + 4;
  auto kern = op.physics == Q1_LAPLACE ? k_pcg_fused<1>
              : op.physics == Q1_VLAPLACE ? k_pcg_fused<2> : k_pcg_fused<3>;
  hipLaunchKernelGGL(kern, dim3(1), dim3(kThreads), lds, s, A);
  Q1_HIP(hipGetLastError());
  double h[5];
  Q1_HIP(hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, s));
  Q1_HIP(hipStreamSynchronize(s));
  int iters = 0, status = 0;
  std::memcpy(&iters, &h[0], sizeof(int));
  std::memcpy(&status, &h[1], sizeof(int));
  const auto t1 = std::chrono::steady_clock::now();
  if (st) {
    st->iters = iters;
    st->status = status;
    st->rel_res = h[3] > 0 ? std::sqrt(h[2] / h[3]) : 0.0;
    st->true_rel_res = h[3] > 0 ? std::sqrt(h[4] / h[3]) : 0.0;
    st->seconds = std::chrono::duration<double>(t1 - t0).count();
    st->fallback_at = -1;
    st->outer_iters = 0;
  }
  return status;
}
