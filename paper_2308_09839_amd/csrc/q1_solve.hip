// Krylov solvers on the device: Jacobi-preconditioned CG, flexible PCG and
// FP32/FP64 iterative refinement, built from the CG operations of Table 4
// (operator apply, the dot p^T A p, the axpys of x and r with the dot r^T r,
// the axpy of p).
//
// Reductions are deterministic and need no grid-wide fence: a kernel writes
// one partial sum per block (a fixed-order wave64 shuffle tree and a fixed
// combination of the block's waves), and every block of the NEXT kernel in
// stream order re-reduces the partials in the same fixed order, so all blocks
// see bit-identical scalars.  (A device-scope fence per block would write back
// and invalidate the whole L2 on this GPU.)  Iteration scalars never leave the
// device; the host reads a small status record every few iterations, and a
// device flag marks the solve finished, after which every queued kernel --
// the operator apply included -- returns at once.
//
// PCG iteration k (vectors x, r, p, q and the inverse diagonal w; z = w r is
// never stored):
//   apply      q = A p
//   dot        partials of p.q
//   update     alpha = rho_k / p.q; x += alpha p; r -= alpha q;
//              partials of rho_{k+1} = r.(w r) and of r.r
//   direction  convergence test on r.r; beta = rho_{k+1} / rho_k;
//              p = w r + beta p
// Vectors are of the operator's type T (double or float); every dot product
// accumulates in double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "q1_internal.hpp"

namespace q1 {

constexpr int kRT = 256;      // threads per reduction block
constexpr int kMaxRB = 1024;  // partial sums per reduction (4 blocks per compute unit)
// partials of p.q that a block apply may form (tile and halo-sum workgroups); an
// operator needing more takes the separate dot kernel
constexpr int kMaxDotParts = 32768;

// Device status record, read by the host every few iterations.
struct Status {
  int done, status, iter, pad;
  double rr, bb, rho, aux;
};

// Workspace of q1_pcg_noalloc: the status record, the reduction partials and
// the four solver vectors (r, p, q, w) of at most Q1_NOALLOC_MAX_DOF entries,
// in one static array that each GPU holds until the process ends.  Host code
// must not use the array's name as a device address: the per-device address
// comes from hipGetSymbolAddress (scratch_on).
constexpr int64_t kNoAllocMaxDof = Q1_NOALLOC_MAX_DOF;
constexpr size_t kNoAllocHead = 256;  // status record, padded
constexpr size_t kNoAllocPart = size_t(8) * kMaxRB * sizeof(double);
constexpr size_t kNoAllocDot = size_t(kMaxDotParts) * sizeof(double);
constexpr size_t kNoAllocVec = size_t(kNoAllocMaxDof) * sizeof(double);
constexpr size_t kNoAllocBytes = kNoAllocHead + kNoAllocPart + kNoAllocDot + 4 * kNoAllocVec;
static_assert(kNoAllocBytes == Q1_NOALLOC_BYTES, "header and workspace layout disagree");
static_assert(sizeof(Status) <= kNoAllocHead, "status record exceeds its slot");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// zero the status record (a kernel rather than a memset node, so that the
// stream work stays capturable)
__global__ void k_clear_status(Status *st) {
  static_assert(sizeof(Status) % sizeof(int) == 0, "status record of whole words");
  int *w = reinterpret_cast<int *>(st);
  for (int i = threadIdx.x; i < int(sizeof(Status) / sizeof(int)); i += blockDim.x) w[i] = 0;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Sum of N values over the block, returned to every thread (fixed order).
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N]) {
  __shared__ double sh[N][kRT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < N; ++i) sh[i][w] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double s = sh[i][0];
#pragma unroll
    for (int k = 1; k < kRT / 64; ++k) s += sh[i][k];
    v[i] = s;
  }
}

// Re-reduce the partials written by an earlier kernel, R rows of cnt[r] >= 1
// partials each: thread t adds partials t, t + 256, ... of each row in order,
// then the fixed block sum (the same value in every block).  The loads of four
// rounds are issued together, at clamped indices, before any of them is added.
template <int R>
__device__ __forceinline__ void sum_partials_nc(const double *const (&rows)[R],
                                                const int (&cnt)[R], double (&out)[R]) {
  constexpr int U = 4;
  int m = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    out[r] = 0.0;
    m = cnt[r] > m ? cnt[r] : m;
  }
  for (int j0 = int(threadIdx.x); j0 < m; j0 += U * kRT) {
    double a[U][R];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int r = 0; r < R; ++r) a[u][r] = rows[r][min(j0 + u * kRT, cnt[r] - 1)];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (j0 + u * kRT < cnt[r]) out[r] += a[u][r];
  }
  block_sum<R>(out);
}

// the same with one count for every row
template <int R>
__device__ __forceinline__ void sum_partials_n(const double *const (&rows)[R], int nb,
                                               double (&out)[R]) {
  int cnt[R];
#pragma unroll
  for (int r = 0; r < R; ++r) cnt[r] = nb;
  sum_partials_nc<R>(rows, cnt, out);
}

__device__ __forceinline__ double sum_partials(const double *__restrict__ part, int nb) {
  double out[1];
  sum_partials_n<1>({part}, nb, out);
  return out[0];
}

struct Range {
  int64_t i0, i1;
};
__device__ __forceinline__ Range block_range(int64_t n) {
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = int64_t(blockIdx.x) * chunk;
  return {i0, i0 + chunk < n ? i0 + chunk : n};
}

// ---- kernels ---------------------------------------------------------------

// w = 1/d (Jacobi) or 1; 0 on a zero row (a node that no element references)
template <typename T>
__global__ void k_inv_diag(int64_t n, const T *__restrict__ d, T *__restrict__ w, int jacobi) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) w[i] = jacobi ? (d[i] != T(0) ? T(1) / d[i] : T(0)) : T(1);
}

// x = 0, r = b, p = w b; partials rho_0 = b.(w b) and b.b
template <typename T>
__global__ __launch_bounds__(kRT) void k_pcg_init(int64_t n, const T *__restrict__ b,
                                                  const T *__restrict__ w, T *__restrict__ x,
                                                  T *__restrict__ r, T *__restrict__ p,
                                                  double *__restrict__ part_rho,
                                                  double *__restrict__ part_bb, int set_p) {
  const Range rg = block_range(n);
  double v[2] = {0.0, 0.0};
  for (int64_t i = rg.i0 + threadIdx.x; i < rg.i1; i += kRT) {
    const T bi = b[i];
    const T zi = w[i] * bi;
    x[i] = T(0);
    r[i] = bi;
    if (set_p) p[i] = zi;
    v[0] += double(bi) * double(zi);
    v[1] += double(bi) * double(bi);
  }
  block_sum<2>(v);
  if (threadIdx.x == 0) {
    part_rho[blockIdx.x] = v[0];
    part_bb[blockIdx.x] = v[1];
  }
}

// partials of a.c (skipped once the solve is done)
template <typename T>
__global__ __launch_bounds__(kRT) void k_dot(int64_t n, const T *__restrict__ a,
                                             const T *__restrict__ c, double *__restrict__ part,
                                             const Status *__restrict__ st) {
  if (st && st->done) return;
  const Range rg = block_range(n);
  double v[1] = {0.0};
  constexpr int U = 4;  // a round's loads together, the additions in the order i, i + 256, ...
  for (int64_t i0 = rg.i0 + threadIdx.x; i0 < rg.i1; i0 += U * kRT) {
    T av[U], cv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = min(i0 + u * kRT, rg.i1 - 1);
      av[u] = a[i];
      cv[u] = c[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u * kRT < rg.i1) v[0] += double(av[u]) * double(cv[u]);
  }
  block_sum<1>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// alpha = rho_k / p.q; x += alpha p; r -= alpha q; partials rho_{k+1}, r.r.
// FLEX (flexible PCG): keeps r_k in r_old and leaves rho_{k+1} to the
// preconditioner step.  TP, the type of p and q, is float in the mixed-precision
// solver (FP32 operator), whose x, r and w stay in double.
// npq: the number of p.q partials (the apply's when it forms them, else gridDim.x).
template <typename T, bool FLEX, typename TP = T>
__global__ __launch_bounds__(kRT) void k_pcg_update(
    int64_t n, const TP *__restrict__ p, const TP *__restrict__ q, const T *__restrict__ w,
    T *__restrict__ x, T *__restrict__ r, T *__restrict__ r_old,
    const double *__restrict__ part_pq, int npq, const double *__restrict__ part_rho_k,
    double *__restrict__ part_rho_k1, double *__restrict__ part_rr, Status *__restrict__ st) {
  if (st->done) return;
  const int nb = gridDim.x;
  double t[2];
  sum_partials_nc<2>({part_pq, part_rho_k}, {npq, nb}, t);
  const double pq = t[0], rho = t[1];
  if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rho)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->done = 1;
      st->status = Q1_EBREAKDOWN;
    }
    return;
  }
  const double alpha = rho / pq;
  const Range rg = block_range(n);
  double v[2] = {0.0, 0.0};
  // four elements per thread and round: all their loads (at clamped indices)
  // before any store; the additions keep the order i, i + 256, ...
  constexpr int U = 4;
  for (int64_t i0 = rg.i0 + threadIdx.x; i0 < rg.i1; i0 += U * kRT) {
    T rv[U], xv[U], wv[U];
    TP pv[U], qv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = min(i0 + u * kRT, rg.i1 - 1);
      rv[u] = r[i];
      xv[u] = x[i];
      pv[u] = p[i];
      qv[u] = q[i];
      if constexpr (!FLEX) wv[u] = w[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * kRT;
      if (i >= rg.i1) continue;
      if constexpr (FLEX) r_old[i] = rv[u];
      const T rn = T(double(rv[u]) - alpha * double(qv[u]));
      x[i] = T(double(xv[u]) + alpha * double(pv[u]));
      r[i] = rn;
      if constexpr (!FLEX) v[0] += double(rn) * double(wv[u] * rn);
      v[1] += double(rn) * double(rn);
    }
  }
  block_sum<2>(v);
  if (threadIdx.x == 0) {
    if constexpr (!FLEX) part_rho_k1[blockIdx.x] = v[0];
    part_rr[blockIdx.x] = v[1];
  }
}

// Convergence test after iteration `it`; beta = rho_{k+1} / rho_k;
// p = z + beta p with z = w r (PCG) or the stored z (flexible PCG); p of type TP
// (rounded to it).
template <typename T, typename TP = T>
__global__ __launch_bounds__(kRT) void k_pcg_direction(
    int64_t n, const T *__restrict__ r, const T *__restrict__ w, const T *__restrict__ z,
    TP *__restrict__ p, const double *__restrict__ part_num, const double *__restrict__ part_den,
    const double *__restrict__ part_rr, const double *__restrict__ part_bb, double tol2, int it,
    int maxit, Status *__restrict__ st) {
  if (st->done) return;
  const int nb = gridDim.x;
  double t[4];
  sum_partials_n<4>({part_num, part_den, part_rr, part_bb}, nb, t);
  const double num = t[0], den = t[1], rr = t[2], bb = t[3];
  const bool conv = rr <= tol2 * bb;
  const bool bad = !isfinite(rr);
  const bool stop = conv || bad || it >= maxit;
  if (!stop) {
    const double beta = num / den;
    const Range rg = block_range(n);
    constexpr int U = 4;  // as in k_pcg_update: a round's loads before its stores
    for (int64_t i0 = rg.i0 + threadIdx.x; i0 < rg.i1; i0 += U * kRT) {
      T zv[U];
      TP pv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = min(i0 + u * kRT, rg.i1 - 1);
        zv[u] = z ? z[i] : T(w[i] * r[i]);
        pv[u] = p[i];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + u * kRT;
        if (i < rg.i1) p[i] = TP(double(zv[u]) + beta * double(pv[u]));
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->iter = it;
    st->rr = rr;
    st->bb = bb;
    st->rho = num;
    if (stop) {
      st->done = 1;
      st->status = conv ? Q1_OK : (bad ? Q1_EBREAKDOWN : Q1_ENOCONV);
    }
  }
}

// Flexible PCG: partials of z.r (rho_{k+1}) and z.(r - r_old)
template <typename T>
__global__ __launch_bounds__(kRT) void k_fpcg_dots(int64_t n, const T *__restrict__ z,
                                                   const T *__restrict__ r,
                                                   const T *__restrict__ r_old,
                                                   double *__restrict__ part_rho,
                                                   double *__restrict__ part_num,
                                                   const Status *__restrict__ st) {
  if (st->done) return;
  const Range rg = block_range(n);
  double v[2] = {0.0, 0.0};
  for (int64_t i = rg.i0 + threadIdx.x; i < rg.i1; i += kRT) {
    const double zi = double(z[i]), ri = double(r[i]);
    v[0] += zi * ri;
    v[1] += zi * (ri - double(r_old[i]));
  }
  block_sum<2>(v);
  if (threadIdx.x == 0) {
    part_rho[blockIdx.x] = v[0];
    part_num[blockIdx.x] = v[1];
  }
}

// z = w r
template <typename T>
__global__ void k_jacobi(int64_t n, const T *__restrict__ w, const T *__restrict__ r,
                         T *__restrict__ z) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) z[i] = w[i] * r[i];
}

// y = b - y (residual from y = A x)
template <typename T>
__global__ void k_residual(int64_t n, const T *__restrict__ b, T *__restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = b[i] - y[i];
}

// single-block sum of partials into *out
__global__ __launch_bounds__(kRT) void k_finalize(const double *__restrict__ part, int nb,
                                                  double *__restrict__ out) {
  const double s = sum_partials(part, nb);
  if (threadIdx.x == 0) *out = s;
}

// the single-pass dot of the dot-product study: block partials added to *out
// with FP64 atomics (order, and so the last bits, vary from run to run)
template <typename T>
__global__ __launch_bounds__(kRT) void k_dot_atomic(int64_t n, const T *__restrict__ a,
                                                    const T *__restrict__ c,
                                                    double *__restrict__ out) {
  const Range rg = block_range(n);
  double v[1] = {0.0};
  for (int64_t i = rg.i0 + threadIdx.x; i < rg.i1; i += kRT) v[0] += double(a[i]) * double(c[i]);
  block_sum<1>(v);
  if (threadIdx.x == 0) unsafeAtomicAdd(out, v[0]);
}
__global__ void k_zero1(double *out) { *out = 0.0; }

// Iterative refinement helpers
// s = (float) (r / scale) with scale = sqrt(*nrm2)
__global__ void k_scale_to_f32(int64_t n, const double *__restrict__ r,
                               const double *__restrict__ nrm2, float *__restrict__ s) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) s[i] = float(r[i] / sqrt(*nrm2));
}
// x += sqrt(*nrm2) * d (FP64 update with the FP32 correction)
__global__ void k_ir_update(int64_t n, const float *__restrict__ d,
                            const double *__restrict__ nrm2, double *__restrict__ x) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] += sqrt(*nrm2) * double(d[i]);
}

// Mixed-precision PCG: p = (float) (w r) from the FP64 residual
__global__ void k_direction_start(int64_t n, const double *__restrict__ w,
                                  const double *__restrict__ r, float *__restrict__ p) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = float(w[i] * r[i]);
}
// partials of rho = r.(w r) and of r.r
__global__ __launch_bounds__(kRT) void k_rho_rr(int64_t n, const double *__restrict__ r,
                                                const double *__restrict__ w,
                                                double *__restrict__ part_rho,
                                                double *__restrict__ part_rr) {
  const Range rg = block_range(n);
  double v[2] = {0.0, 0.0};
  for (int64_t i = rg.i0 + threadIdx.x; i < rg.i1; i += kRT) {
    const double ri = r[i];
    v[0] += ri * (w[i] * ri);
    v[1] += ri * ri;
  }
  block_sum<2>(v);
  if (threadIdx.x == 0) {
    part_rho[blockIdx.x] = v[0];
    part_rr[blockIdx.x] = v[1];
  }
}
__global__ void k_clear_done(Status *st) { st->done = 0; st->status = 0; }


// ---- flexible CG with truncated orthogonalisation (FCG(m)) ------------------------
constexpr int kMaxTrunc = 8;

struct DirSet {  // window of previous directions p_j, q_j = A p_j and the partials of p_j.q_j
  const void *p[kMaxTrunc];
  const void *q[kMaxTrunc];
  const double *pq[kMaxTrunc];
};

// partials of z.q_j for the m directions of the window
template <typename T>
__global__ __launch_bounds__(kRT) void k_multi_dot(int64_t n, const T *__restrict__ z, DirSet d,
                                                   int m, double *__restrict__ part /*[m][kMaxRB]*/,
                                                   const Status *__restrict__ st) {
  if (st->done) return;
  const Range rg = block_range(n);
  double v[kMaxTrunc];
#pragma unroll
  for (int j = 0; j < kMaxTrunc; ++j) v[j] = 0.0;
  for (int64_t i = rg.i0 + threadIdx.x; i < rg.i1; i += kRT) {
    const double zi = double(z[i]);
#pragma unroll
    for (int j = 0; j < kMaxTrunc; ++j)
      if (j < m) v[j] += zi * double(static_cast<const T *>(d.q[j])[i]);
  }
  block_sum<kMaxTrunc>(v);
  if (threadIdx.x == 0)
    for (int j = 0; j < m; ++j) part[j * kMaxRB + blockIdx.x] = v[j];
}

// c_j = z.q_j / p_j.q_j for the m directions of the window, from the nz
// partials of z.q_j (k_multi_dot) and the np partials of p_j.q_j, in one
// block (a fixed-order reduction of all 2m rows)
__global__ __launch_bounds__(kRT) void k_fcg_coef(const double *__restrict__ part_zq, int nz,
                                                  DirSet d, int np, int m,
                                                  double *__restrict__ coef,
                                                  const Status *__restrict__ st) {
  if (st->done) return;
  // every load of the block is issued before the first addition (one memory
  // latency instead of one per round); the additions keep the order of
  // sum_partials: thread t adds partials t, t + 256, ... of each row
  constexpr int kRounds = kMaxRB / kRT;
  double a[kRounds][2 * kMaxTrunc];
#pragma unroll
  for (int k = 0; k < kRounds; ++k) {
    const int i = int(threadIdx.x) + k * kRT;
#pragma unroll
    for (int j = 0; j < kMaxTrunc; ++j) {
      a[k][j] = j < m && i < nz ? part_zq[j * kMaxRB + i] : 0.0;
      a[k][kMaxTrunc + j] = j < m && i < np ? d.pq[j][i] : 0.0;
    }
  }
  double v[2 * kMaxTrunc];
#pragma unroll
  for (int j = 0; j < 2 * kMaxTrunc; ++j) {
    v[j] = 0.0;
#pragma unroll
    for (int k = 0; k < kRounds; ++k) v[j] += a[k][j];
  }
  block_sum<2 * kMaxTrunc>(v);
  if (threadIdx.x < kMaxTrunc) {
    const int j = int(threadIdx.x);
    double c = 0.0;
#pragma unroll
    for (int t = 0; t < kMaxTrunc; ++t)
      if (t == j && t < m) c = v[kMaxTrunc + t] > 0.0 ? v[t] / v[kMaxTrunc + t] : 0.0;
    coef[j] = c;
  }
}

// p = z - sum_j c_j p_j with the coefficients of k_fcg_coef
template <typename T>
__global__ __launch_bounds__(kRT) void k_fcg_direction(int64_t n, const T *__restrict__ z,
                                                       DirSet d, int m,
                                                       const double *__restrict__ coef,
                                                       T *__restrict__ p,
                                                       const Status *__restrict__ st) {
  if (st->done) return;
  double c[kMaxTrunc];
#pragma unroll
  for (int j = 0; j < kMaxTrunc; ++j) c[j] = j < m ? coef[j] : 0.0;
  const Range rg = block_range(n);
  for (int64_t i = rg.i0 + threadIdx.x; i < rg.i1; i += kRT) {
    double v = double(z[i]);
#pragma unroll
    for (int j = 0; j < kMaxTrunc; ++j)
      if (j < m) v -= c[j] * double(static_cast<const T *>(d.p[j])[i]);
    p[i] = T(v);
  }
}

// partials of p.q and p.r
template <typename T>
__global__ __launch_bounds__(kRT) void k_dot_pq_pr(int64_t n, const T *__restrict__ p,
                                                   const T *__restrict__ q, const T *__restrict__ r,
                                                   double *__restrict__ part_pq,
                                                   double *__restrict__ part_pr,
                                                   const Status *__restrict__ st) {
  if (st->done) return;
  const Range rg = block_range(n);
  double v[2] = {0.0, 0.0};
  for (int64_t i = rg.i0 + threadIdx.x; i < rg.i1; i += kRT) {
    const double pi = double(p[i]);
    v[0] += pi * double(q[i]);
    v[1] += pi * double(r[i]);
  }
  block_sum<2>(v);
  if (threadIdx.x == 0) {
    part_pq[blockIdx.x] = v[0];
    part_pr[blockIdx.x] = v[1];
  }
}

// alpha = p.r / p.q; x += alpha p; r -= alpha q; partials of r.r
template <typename T>
__global__ __launch_bounds__(kRT) void k_fcg_update(int64_t n, const T *__restrict__ p,
                                                    const T *__restrict__ q, T *__restrict__ x,
                                                    T *__restrict__ r,
                                                    const double *__restrict__ part_pq,
                                                    const double *__restrict__ part_pr,
                                                    double *__restrict__ part_rr,
                                                    Status *__restrict__ st) {
  if (st->done) return;
  const int nb = gridDim.x;
  double t[2];
  sum_partials_n<2>({part_pq, part_pr}, nb, t);
  const double pq = t[0], pr = t[1];
  if (!(pq > 0.0) || !isfinite(pq) || !isfinite(pr)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->done = 1;
      st->status = Q1_EBREAKDOWN;
    }
    return;
  }
  const double alpha = pr / pq;
  const Range rg = block_range(n);
  double v[1] = {0.0};
  for (int64_t i = rg.i0 + threadIdx.x; i < rg.i1; i += kRT) {
    const T rn = T(double(r[i]) - alpha * double(q[i]));
    x[i] = T(double(x[i]) + alpha * double(p[i]));
    r[i] = rn;
    v[0] += double(rn) * double(rn);
  }
  block_sum<1>(v);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = v[0];
}

// Flexible CG guard: every block re-sums the z.r partials; when the sum is not
// positive and finite, or a fallback is recorded, z = D^-1 r (w r) on the
// block's range, and block 0 records the first fallback iteration.
template <typename T>
__global__ __launch_bounds__(kRT) void k_fcg_guard(int64_t n, const T *__restrict__ w,
                                                   const T *__restrict__ r, T *__restrict__ z,
                                                   const double *__restrict__ part_zr,
                                                   int *__restrict__ fb, int k,
                                                   const Status *__restrict__ st) {
  if (st->done) return;
  const double zr = sum_partials(part_zr, gridDim.x);
  const bool was = fb[0] != 0;
  if (was || (zr > 0.0 && isfinite(zr))) {
    if (!was) return;
  }
  const Range rg = block_range(n);
  for (int64_t i = rg.i0 + threadIdx.x; i < rg.i1; i += kRT) z[i] = w[i] * r[i];
  if (!was && blockIdx.x == 0 && threadIdx.x == 0) {
    fb[0] = 1;
    fb[1] = k;
  }
}

// fb = (flag, iteration)
__global__ void k_set_fallback(int *fb, int flag, int k) {
  if (fb[0] == 0 || flag == 0) {
    fb[0] = flag;
    fb[1] = k;
  }
}

// After iteration `it` of flexible CG: r.r from the partials into the history
// and the status; convergence, breakdown or the iteration limit end the solve.
__global__ __launch_bounds__(kRT) void k_fcg_check(const double *__restrict__ part_rr, int nb,
                                                   double *__restrict__ hist, double tol2, int it,
                                                   int maxit, Status *__restrict__ st) {
  if (st->done) return;
  const double rr = sum_partials(part_rr, nb);
  if (threadIdx.x == 0) {
    hist[it] = rr;
    st->rr = rr;
    st->iter = it;
    const bool conv = rr <= tol2 * st->bb, bad = !isfinite(rr);
    if (conv || bad || it >= maxit) {
      st->done = 1;
      st->status = conv ? Q1_OK : (bad ? Q1_EBREAKDOWN : Q1_ENOCONV);
    }
  }
}

// ---- host drivers ------------------------------------------------------------

namespace {

struct Work {
  void *r = nullptr, *p = nullptr, *q = nullptr, *w = nullptr, *r_old = nullptr,
       *z = nullptr;
  double *part = nullptr;  // [8][kMaxRB]
  double *dparts = nullptr;  // [kMaxDotParts]: p.q partials formed by the apply
  Status *st = nullptr;    // device
  Status *hst = nullptr;   // host mirror (pinned when owned)
  bool owned = true;       // false: the buffers live in the static scratch array
  Work() = default;
  Work(const Work &) = delete;
  ~Work() {
    if (!owned) return;
    void *d[] = {r, p, q, w, r_old, z, part, dparts, st};
    for (void *v : d)
      if (v) (void)hipFree(v);
    if (hst) (void)hipHostFree(hst);
  }
};

int nblocks_for(int64_t n) {
  const int64_t b = (n + int64_t(kRT) * 8 - 1) / (int64_t(kRT) * 8);
  return int(std::max<int64_t>(1, std::min<int64_t>(kMaxRB, b)));
}

inline dim3 grid1(int64_t n) { return dim3(unsigned((n + 255) / 256)); }

template <typename T>
int alloc_work(Work &W, int64_t n, bool flex) {
  const size_t b = size_t(std::max<int64_t>(n, 1)) * sizeof(T);
  Q1_HIP(hipMalloc(&W.r, b));
  Q1_HIP(hipMalloc(&W.p, b));
  Q1_HIP(hipMalloc(&W.q, b));
  Q1_HIP(hipMalloc(&W.w, b));
  if (flex) {
    Q1_HIP(hipMalloc(&W.r_old, b));
    Q1_HIP(hipMalloc(&W.z, b));
  }
  Q1_HIP(hipMalloc(&W.part, 8 * kMaxRB * sizeof(double)));
  Q1_HIP(hipMalloc(&W.dparts, kMaxDotParts * sizeof(double)));
  Q1_HIP(hipMalloc(&W.st, sizeof(Status)));
  Q1_HIP(hipHostMalloc(&W.hst, sizeof(Status), hipHostMallocDefault));
  return Q1_OK;
}

template <typename T>
int setup_diag(Op &op, Work &W, int pc, hipStream_t s) {
  const int64_t n = op.n_nodes * op.dpn();
  if (pc == Q1_PC_JACOBI) {
    const int rc = launch_diag(op, W.q, s);  // q as scratch
    if (rc) return rc;
  }
  hipLaunchKernelGGL((k_inv_diag<T>), grid1(n), dim3(256), 0, s, n, static_cast<const T *>(W.q),
                     static_cast<T *>(W.w), pc == Q1_PC_JACOBI ? 1 : 0);
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int read_status(Work &W, hipStream_t s) {
  Q1_HIP(hipMemcpyAsync(W.hst, W.st, sizeof(Status), hipMemcpyDeviceToHost, s));
  Q1_HIP(hipStreamSynchronize(s));
  return Q1_OK;
}

// ||b - A x||_2 / ||b||_2 with q and two partial rows as scratch (synchronises)
template <typename T>
int true_residual(Op &op, Work &W, const T *b, const T *x, double *out, hipStream_t s) {
  const int64_t n = op.n_nodes * op.dpn();
  const int nb = nblocks_for(n);
  T *q = static_cast<T *>(W.q);
  int rc = launch_apply(op, x, q, s);
  if (rc) return rc;
  hipLaunchKernelGGL((k_residual<T>), grid1(n), dim3(256), 0, s, n, b, q);
  hipLaunchKernelGGL((k_dot<T>), dim3(nb), dim3(kRT), 0, s, n, q, q, W.part + 6 * kMaxRB,
                     nullptr);
  hipLaunchKernelGGL((k_dot<T>), dim3(nb), dim3(kRT), 0, s, n, b, b, W.part + 7 * kMaxRB,
                     nullptr);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRT), 0, s, W.part + 6 * kMaxRB, nb, &W.st->aux);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRT), 0, s, W.part + 7 * kMaxRB, nb, &W.st->bb);
  Q1_HIP(hipGetLastError());
  if ((rc = read_status(W, s))) return rc;
  *out = W.hst->bb > 0 ? std::sqrt(W.hst->aux / W.hst->bb) : 0.0;
  return Q1_OK;
}

// Preconditioned CG on the operator's vector type T with x0 = 0.  Returns
// Q1_OK, Q1_ENOCONV (x = last iterate) or Q1_EBREAKDOWN.
// Snapshots of the iterate: after iteration iters[i] (counted from 1), x is
// copied to dst[i]; iters ascending.  A snapshot past the end of the solve
// receives the final iterate.
struct Snapshots {
  int n = 0;
  const int *iters = nullptr;
  void *const *dst = nullptr;
};

template <typename T>
int pcg_t(Op &op, int pc, const T *b, T *x, double rtol, int maxit, q1_stats *stats,
          hipStream_t s, bool true_res, const Snapshots &snap = Snapshots(),
          Work *given = nullptr) {
  const int64_t n = op.n_nodes * op.dpn();
  Work own;
  int rc;
  if (!given && (rc = alloc_work<T>(own, n, false))) return rc;
  Work &W = given ? *given : own;
  const auto t0 = std::chrono::steady_clock::now();
  if ((rc = setup_diag<T>(op, W, pc, s))) return rc;
  const int nb = nblocks_for(n);
  double *P = W.part;
  double *part_rho[2] = {P, P + kMaxRB};
  double *part_pq = P + 2 * kMaxRB, *part_rr = P + 3 * kMaxRB, *part_bb = P + 4 * kMaxRB;
  T *r = static_cast<T *>(W.r), *p = static_cast<T *>(W.p), *q = static_cast<T *>(W.q),
    *w = static_cast<T *>(W.w);
  // block operators form the partials of p.q while writing q (one pass less per
  // iteration); the decision depends on the operator alone, so the allocating and
  // the static-workspace entry points compute the same sums
  int64_t n_dot = 0;
  const int64_t need_dot = apply_dot_parts(op, &n_dot);
  const bool fused_dot = need_dot > 0 && need_dot <= kMaxDotParts && W.dparts;
  const int npq = fused_dot ? int(n_dot) : nb;
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, W.st);
  hipLaunchKernelGGL((k_pcg_init<T>), dim3(nb), dim3(kRT), 0, s, n, b, w, x, r, p, part_rho[0],
                     part_bb, 1);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRT), 0, s, part_bb, nb, &W.st->bb);
  Q1_HIP(hipGetLastError());
  if ((rc = read_status(W, s))) return rc;
  const double bb = W.hst->bb;
  int status = Q1_OK, iters = 0;
  double rr = bb;
  if (bb > 0.0) {
    const double tol2 = rtol * rtol;
    status = Q1_ENOCONV;
    int launched = 0, batch = 1, next_snap = 0;
    while (next_snap < snap.n && snap.iters[next_snap] <= 0)
      Q1_HIP(hipMemcpyAsync(snap.dst[next_snap++], x, size_t(n) * sizeof(T),
                            hipMemcpyDeviceToDevice, s));
    while (launched < maxit) {
      const int m = std::min(batch, maxit - launched);
      for (int j = 0; j < m; ++j) {
        const int k = launched + j;
        if (fused_dot) {  // p.q partials formed by the apply
          if ((rc = launch_apply_dot(op, p, q, s, &W.st->done, W.dparts))) return rc;
        } else {
          if ((rc = launch_apply(op, p, q, s, &W.st->done))) return rc;
          hipLaunchKernelGGL((k_dot<T>), dim3(nb), dim3(kRT), 0, s, n, p, q, part_pq, W.st);
        }
        hipLaunchKernelGGL((k_pcg_update<T, false>), dim3(nb), dim3(kRT), 0, s, n, p, q, w, x, r,
                           nullptr, fused_dot ? W.dparts : part_pq, npq, part_rho[k & 1],
                           part_rho[(k + 1) & 1], part_rr, W.st);
        hipLaunchKernelGGL((k_pcg_direction<T>), dim3(nb), dim3(kRT), 0, s, n, r, w, nullptr, p,
                           part_rho[(k + 1) & 1], part_rho[k & 1], part_rr, part_bb, tol2, k + 1,
                           maxit, W.st);
        while (next_snap < snap.n && snap.iters[next_snap] == k + 1)
          Q1_HIP(hipMemcpyAsync(snap.dst[next_snap++], x, size_t(n) * sizeof(T),
                                hipMemcpyDeviceToDevice, s));
      }
      Q1_HIP(hipGetLastError());
      launched += m;
      if ((rc = read_status(W, s))) return rc;
      if (W.hst->done) break;
      batch = std::min(batch * 2, 32);
    }
    iters = W.hst->iter;
    rr = W.hst->rr;
    if (W.hst->done) status = W.hst->status;
    while (next_snap < snap.n)
      Q1_HIP(hipMemcpyAsync(snap.dst[next_snap++], x, size_t(n) * sizeof(T),
                            hipMemcpyDeviceToDevice, s));
  }
  const auto t1 = std::chrono::steady_clock::now();
  if (stats) {
    stats->iters = iters;
    stats->status = status;
    stats->seconds = std::chrono::duration<double>(t1 - t0).count();
    stats->rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    stats->true_rel_res = stats->rel_res;
    stats->fallback_at = -1;
    stats->outer_iters = 0;
    if (true_res && bb > 0.0) {
      double t;
      if ((rc = true_residual<T>(op, W, b, x, &t, s))) return rc;
      stats->true_rel_res = t;
    }
  }
  return status;
}

// Flexible CG with a caller preconditioner z = M(r) and truncated
// orthogonalisation: the new direction is z made A-orthogonal to the last m
// directions (m = 1 is the Polak-Ribiere flexible PCG).  Falls back to Jacobi
// for the rest of the solve when M fails, gives z.r <= 0 or a non-finite
// value (both checked on the device, which then replaces z by D^-1 r), or when
// the residual has not dropped below its value safeguard_m iterations earlier
// (checked by the host at its status reads).  Like pcg_t the host reads the
// device status only every few iterations: each batch is sized from the
// observed convergence rate so that few iterations are queued past
// convergence (their kernels return at once, but the callback M still runs).
template <typename T>
int fpcg_t(Op &op, q1_precond_fn M, void *ctx, const T *b, T *x, double rtol, int maxit,
           int safeguard_m, int m, q1_stats *stats, hipStream_t s) {
  const int64_t n = op.n_nodes * op.dpn();
  Work W;
  int rc = alloc_work<T>(W, n, true);
  if (rc) return rc;
  // direction window: m slots of p and q, and the p.q partials of every slot;
  // the fallback record and the residual history
  void *dirs = nullptr;
  double *pq_parts = nullptr, *zq_parts = nullptr, *hist_d = nullptr;
  int *fb = nullptr;
  struct Free {
    void *p[5];
    ~Free() {
      for (void *v : p)
        if (v) (void)hipFree(v);
    }
  };
  const size_t vb = size_t(std::max<int64_t>(n, 1)) * sizeof(T);
  Q1_HIP(hipMalloc(&dirs, 2 * size_t(m) * vb));
  Free fr0{{dirs, nullptr, nullptr, nullptr, nullptr}};
  Q1_HIP(hipMalloc(&pq_parts, size_t(m) * kMaxRB * sizeof(double)));
  fr0.p[1] = pq_parts;
  Q1_HIP(hipMalloc(&zq_parts, size_t(kMaxTrunc + 1) * kMaxRB * sizeof(double)));
  double *coef_d = zq_parts + size_t(kMaxTrunc) * kMaxRB;  // the window's coefficients
  const int nbw = int(std::max<int64_t>(1, std::min<int64_t>(kMaxRB, (n + kRT - 1) / kRT)));
  fr0.p[2] = zq_parts;
  Q1_HIP(hipMalloc(&hist_d, size_t(maxit + 1) * sizeof(double)));
  fr0.p[3] = hist_d;
  Q1_HIP(hipMalloc(&fb, 2 * sizeof(int)));
  fr0.p[4] = fb;
  auto P = [&](int j) { return reinterpret_cast<T *>(static_cast<char *>(dirs) + size_t(j) * vb); };
  auto Qv = [&](int j) {
    return reinterpret_cast<T *>(static_cast<char *>(dirs) + size_t(m + j) * vb);
  };
  const auto t0 = std::chrono::steady_clock::now();
  if ((rc = setup_diag<T>(op, W, Q1_PC_JACOBI, s))) return rc;
  const int nb = nblocks_for(n);
  double *Pp = W.part;
  double *part_rho = Pp, *part_pr = Pp + kMaxRB, *part_rr = Pp + 3 * kMaxRB,
         *part_bb = Pp + 4 * kMaxRB;
  T *r = static_cast<T *>(W.r), *w = static_cast<T *>(W.w), *z = static_cast<T *>(W.z);
  Q1_HIP(hipMemsetAsync(W.st, 0, sizeof(Status), s));
  hipLaunchKernelGGL(k_set_fallback, dim3(1), dim3(1), 0, s, fb, 0, -1);
  hipLaunchKernelGGL((k_pcg_init<T>), dim3(nb), dim3(kRT), 0, s, n, b, w, x, r,
                     static_cast<T *>(W.p), part_rho, part_bb, 0);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRT), 0, s, part_bb, nb, &W.st->bb);
  Q1_HIP(hipGetLastError());
  if ((rc = read_status(W, s))) return rc;
  const double bb = W.hst->bb;
  int status = Q1_OK, iters = 0, fallback_at = -1;
  bool fallback = false;  // known to the host: M is no longer called
  double rr = bb;
  std::vector<double> hist(1, bb);
  auto start_fallback = [&](int k) -> int {
    fallback = true;
    fallback_at = k;
    hipLaunchKernelGGL(k_set_fallback, dim3(1), dim3(1), 0, s, fb, 1, k);
    Q1_HIP(hipGetLastError());
    return Q1_OK;
  };
  if (!M) {
    if ((rc = start_fallback(0))) return rc;
  }
  if (bb > 0.0) {
    const double tol2 = rtol * rtol;
    status = Q1_ENOCONV;
    int launched = 0, batch = 1;
    int hfb[2] = {0, -1};
    while (launched < maxit) {
      const int mm = std::min(batch, maxit - launched);
      for (int j = 0; j < mm; ++j) {
        const int k = launched + j;
        if (!fallback && M(ctx, r, z, s) != Q1_OK) {
          (void)hipGetLastError();
          if ((rc = start_fallback(k))) return rc;
        }
        // z.r > 0 and finite, else z = D^-1 r from here on (decided on the device)
        hipLaunchKernelGGL((k_dot<T>), dim3(nb), dim3(kRT), 0, s, n, z, r, part_rho, W.st);
        hipLaunchKernelGGL((k_fcg_guard<T>), dim3(nb), dim3(kRT), 0, s, n, w, r, z, part_rho, fb,
                           k, W.st);
        // window: the previous min(k, m) directions, oldest first
        const int cur = k % m, nwin = std::min(k, m);
        DirSet d{};
        for (int t = 0; t < nwin; ++t) {
          const int sl = (k - nwin + t) % m;
          d.p[t] = P(sl);
          d.q[t] = Qv(sl);
          d.pq[t] = pq_parts + size_t(sl) * kMaxRB;
        }
        if (nwin > 0) {
          // the window's dot products and the new direction: memory-bound passes
          // over m + 1 vectors, so launched on up to kMaxRB blocks; the
          // coefficients are reduced once, by one block
          hipLaunchKernelGGL((k_multi_dot<T>), dim3(nbw), dim3(kRT), 0, s, n, z, d, nwin,
                             zq_parts, W.st);
          hipLaunchKernelGGL(k_fcg_coef, dim3(1), dim3(kRT), 0, s, zq_parts, nbw, d, nb, nwin,
                             coef_d, W.st);
          hipLaunchKernelGGL((k_fcg_direction<T>), dim3(nbw), dim3(kRT), 0, s, n, z, d, nwin,
                             coef_d, P(cur), W.st);
        } else {
          Q1_HIP(hipMemcpyAsync(P(cur), z, size_t(n) * sizeof(T), hipMemcpyDeviceToDevice, s));
        }
        if ((rc = launch_apply(op, P(cur), Qv(cur), s, &W.st->done))) return rc;
        hipLaunchKernelGGL((k_dot_pq_pr<T>), dim3(nb), dim3(kRT), 0, s, n, P(cur), Qv(cur), r,
                           pq_parts + size_t(cur) * kMaxRB, part_pr, W.st);
        hipLaunchKernelGGL((k_fcg_update<T>), dim3(nb), dim3(kRT), 0, s, n, P(cur), Qv(cur), x, r,
                           pq_parts + size_t(cur) * kMaxRB, part_pr, part_rr, W.st);
        hipLaunchKernelGGL(k_fcg_check, dim3(1), dim3(kRT), 0, s, part_rr, nb, hist_d, tol2, k + 1,
                           maxit, W.st);
      }
      Q1_HIP(hipGetLastError());
      const int first = launched + 1;
      launched += mm;
      Q1_HIP(hipMemcpyAsync(hfb, fb, sizeof(hfb), hipMemcpyDeviceToHost, s));
      if ((rc = read_status(W, s))) return rc;
      const int done_it = W.hst->done ? W.hst->iter : launched;
      if (done_it >= first) {
        hist.resize(size_t(done_it) + 1);
        Q1_HIP(hipMemcpy(&hist[first], hist_d + first, size_t(done_it - first + 1) * sizeof(double),
                         hipMemcpyDeviceToHost));
      }
      if (!fallback && hfb[0]) {  // the device replaced z: stop calling M
        fallback = true;
        fallback_at = hfb[1];
      }
      if (W.hst->done) break;
      // stagnation: ||r|| not below its value safeguard_m iterations earlier
      if (safeguard_m > 0 && !fallback)
        for (int it = std::max(first, safeguard_m); it <= launched; ++it)
          if (!(hist[it] < hist[it - safeguard_m])) {
            if ((rc = start_fallback(launched))) return rc;
            break;
          }
      // next batch: about half the iterations the observed rate still needs
      int next = std::min(batch * 2, 32);
      const double now = hist[launched], before = hist[first - 1];
      if (now > 0.0 && before > now && launched >= first) {
        const double rate = std::log(now / before) / double(launched - first + 1);
        const double need = std::log(tol2 * bb / now) / rate;  // both logs negative
        if (std::isfinite(need)) next = std::max(1, std::min(next, int(need / 2)));
      }
      batch = next;
    }
    iters = W.hst->iter;
    rr = W.hst->rr;
    if (W.hst->done) status = W.hst->status;
  }
  const auto t1 = std::chrono::steady_clock::now();
  if (stats) {
    stats->iters = iters;
    stats->status = status;
    stats->seconds = std::chrono::duration<double>(t1 - t0).count();
    stats->rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    stats->fallback_at = fallback_at;
    stats->outer_iters = 0;
    stats->true_rel_res = stats->rel_res;
    if (bb > 0.0) {
      double t;
      if ((rc = true_residual<T>(op, W, b, x, &t, s))) return rc;
      stats->true_rel_res = t;
    }
  }
  return status;
}

// Mixed-precision PCG with reliable updates.  The search directions p and
// q = A p are FP32 and q comes from the FP32 operator; x, the residual r, the
// inverse diagonal and every dot product stay FP64, so the recurrences lose
// only what the FP32 apply and directions round away.  Whenever the recurrence
// residual has fallen by delta since the last refresh (or below rtol / sqrt 2),
// r = b - A64 x is recomputed with the FP64 operator and convergence is decided
// on it; otherwise the recurrences continue from it with the search direction
// kept (beta = rho(new r) / rho_{k-1}), so the Krylov history survives.
int mpcg_t(Op &A64, Op &A32, const double *b, double *x, double rtol, double delta, int maxit,
           q1_stats *stats, hipStream_t s) {
  const int64_t n = A64.n_nodes * A64.dpn();
  Work W;  // FP64 residual and inverse diagonal, partials and status
  int rc = alloc_work<double>(W, n, false);
  if (rc) return rc;
  float *p = nullptr, *q = nullptr;  // FP32 directions
  struct Free {
    float **a, **b;
    ~Free() {
      if (*a) (void)hipFree(*a);
      if (*b) (void)hipFree(*b);
    }
  } fr{&p, &q};
  Q1_HIP(hipMalloc(&p, size_t(n) * sizeof(float)));
  Q1_HIP(hipMalloc(&q, size_t(n) * sizeof(float)));
  const auto t0 = std::chrono::steady_clock::now();
  if ((rc = setup_diag<double>(A64, W, Q1_PC_JACOBI, s))) return rc;
  const int nb = nblocks_for(n);
  double *P = W.part;
  double *part_rho[2] = {P, P + kMaxRB};
  double *part_pq = P + 2 * kMaxRB, *part_rr = P + 3 * kMaxRB, *part_bb = P + 4 * kMaxRB;
  double *r = static_cast<double *>(W.r), *w = static_cast<double *>(W.w);
  // the FP32 block apply forms the partials of p.q (as in pcg_t)
  int64_t n_dot = 0;
  const int64_t need_dot = apply_dot_parts(A32, &n_dot);
  const bool fused_dot = need_dot > 0 && need_dot <= kMaxDotParts && W.dparts;
  const int npq = fused_dot ? int(n_dot) : nb;
  Q1_HIP(hipMemsetAsync(W.st, 0, sizeof(Status), s));
  // x = 0, r = b, partials of rho_0 = b.(w b) and b.b; p = (float) (w b)
  hipLaunchKernelGGL((k_pcg_init<double>), dim3(nb), dim3(kRT), 0, s, n, b, w, x, r, nullptr,
                     part_rho[0], part_bb, 0);
  hipLaunchKernelGGL(k_direction_start, grid1(n), dim3(256), 0, s, n, w, r, p);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRT), 0, s, part_bb, nb, &W.st->bb);
  Q1_HIP(hipGetLastError());
  if ((rc = read_status(W, s))) return rc;
  const double bb = W.hst->bb;
  double rr_true = bb, rr_ref = bb;
  int status = Q1_OK, k = 0, refreshes = 0;
  if (bb > 0.0) {
    const double tol2 = rtol * rtol;
    status = Q1_ENOCONV;
    while (k < maxit) {
      // recurrences until the residual fell by delta (or to the tolerance)
      const double thr = std::max(delta * delta * rr_ref, 0.5 * tol2 * bb);
      int batch = 1;
      bool stop = false;
      while (!stop && k < maxit) {
        const int m = std::min(batch, maxit - k);
        for (int j = 0; j < m; ++j, ++k) {
          if (fused_dot) {
            if ((rc = launch_apply_dot(A32, p, q, s, &W.st->done, W.dparts))) return rc;
          } else {
            if ((rc = launch_apply(A32, p, q, s, &W.st->done))) return rc;
            hipLaunchKernelGGL((k_dot<float>), dim3(nb), dim3(kRT), 0, s, n, p, q, part_pq,
                               W.st);
          }
          hipLaunchKernelGGL((k_pcg_update<double, false, float>), dim3(nb), dim3(kRT), 0, s, n,
                             p, q, w, x, r, nullptr, fused_dot ? W.dparts : part_pq, npq,
                             part_rho[k & 1], part_rho[(k + 1) & 1], part_rr, W.st);
          hipLaunchKernelGGL((k_pcg_direction<double, float>), dim3(nb), dim3(kRT), 0, s, n, r,
                             w, nullptr, p, part_rho[(k + 1) & 1], part_rho[k & 1], part_rr,
                             part_bb, thr / bb, k + 1, maxit, W.st);
        }
        Q1_HIP(hipGetLastError());
        if ((rc = read_status(W, s))) return rc;
        stop = W.hst->done != 0;
        batch = std::min(batch * 2, 32);
      }
      if (W.hst->done && W.hst->status == Q1_EBREAKDOWN) {
        status = Q1_EBREAKDOWN;
        break;
      }
      // the loop ran k iterations; the last direction step was skipped if it stopped early
      k = W.hst->iter;
      // reliable update: r = b - A64 x, with the partials of rho(r) and r.r
      if ((rc = launch_apply(A64, x, r, s))) return rc;
      hipLaunchKernelGGL((k_residual<double>), grid1(n), dim3(256), 0, s, n, b, r);
      hipLaunchKernelGGL(k_rho_rr, dim3(nb), dim3(kRT), 0, s, n, r, w, part_rho[k & 1], part_rr);
      hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRT), 0, s, part_rr, nb, &W.st->aux);
      Q1_HIP(hipGetLastError());
      if ((rc = read_status(W, s))) return rc;
      rr_true = W.hst->aux;
      ++refreshes;
      if (rr_true <= tol2 * bb) {
        status = Q1_OK;
        break;
      }
      if (k >= maxit) break;
      rr_ref = rr_true;
      // continue from the true residual, keeping p: beta = rho(new r) / rho_{k-1}
      hipLaunchKernelGGL(k_clear_done, dim3(1), dim3(1), 0, s, W.st);
      hipLaunchKernelGGL((k_pcg_direction<double, float>), dim3(nb), dim3(kRT), 0, s, n, r, w,
                         nullptr, p, part_rho[k & 1], part_rho[(k + 1) & 1], part_rr, part_bb,
                         0.0, k, maxit + 1, W.st);
      Q1_HIP(hipGetLastError());
    }
  }
  const auto t1 = std::chrono::steady_clock::now();
  if (stats) {
    stats->iters = k;
    stats->outer_iters = refreshes;
    stats->status = status;
    stats->seconds = std::chrono::duration<double>(t1 - t0).count();
    stats->rel_res = bb > 0 ? std::sqrt(rr_true / bb) : 0.0;
    stats->true_rel_res = stats->rel_res;
    stats->fallback_at = -1;
  }
  return status;
}

}  // namespace

// Jacobi preconditioner object usable as a q1_precond_fn context.
struct Jacobi {
  Op *op = nullptr;
  void *w = nullptr;
};

}  // namespace q1

namespace q1 {
namespace {

// Device address of `scratch` on device dev, looked up once per device with
// that device current (each GPU holds its own copy at its own address).
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
unsigned char *g_scratch[kMaxDevices] = {};

int scratch_on(int dev, unsigned char **out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  Q1_CHECK(dev >= 0 && dev < kMaxDevices, Q1_EUNSUPPORTED, "device %d beyond %d", dev,
           kMaxDevices);
  if (!g_scratch[dev]) {
    int cur = 0;
    Q1_HIP(hipGetDevice(&cur));
    if (cur != dev) Q1_HIP(hipSetDevice(dev));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      return fail(Q1_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch[dev] = static_cast<unsigned char *>(p);
  }
  *out = g_scratch[dev];
  return Q1_OK;
}

}  // namespace
}  // namespace q1

using namespace q1;

struct q1_jacobi : public q1::Jacobi {};

extern "C" {

int q1_pcg(q1_op *op, int pc, const void *b_d, void *x_d, double rtol, int maxit,
           q1_stats *st, void *stream) {
  Q1_CHECK(op && b_d && x_d, Q1_EINVAL, "q1_pcg: NULL argument");
  Q1_CHECK(pc == Q1_PC_NONE || pc == Q1_PC_JACOBI, Q1_EINVAL, "q1_pcg: bad preconditioner %d", pc);
  Q1_CHECK(rtol >= 0 && maxit >= 0, Q1_EINVAL, "q1_pcg: need rtol >= 0 and maxit >= 0");
  Op &o = *reinterpret_cast<Op *>(op);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (o.dtype == Q1_F64)
    return pcg_t<double>(o, pc, static_cast<const double *>(b_d), static_cast<double *>(x_d),
                         rtol, maxit, st, s, true);
  return pcg_t<float>(o, pc, static_cast<const float *>(b_d), static_cast<float *>(x_d), rtol,
                      maxit, st, s, true);
}

int q1_pcg_noalloc(q1_op *op, int pc, const void *b_d, void *x_d, double rtol, int maxit,
                   q1_stats *st, void *stream) {
  Q1_CHECK(op && b_d && x_d, Q1_EINVAL, "q1_pcg_noalloc: NULL argument");
  Q1_CHECK(pc == Q1_PC_NONE || pc == Q1_PC_JACOBI, Q1_EINVAL,
           "q1_pcg_noalloc: bad preconditioner %d", pc);
  Q1_CHECK(rtol >= 0 && maxit >= 0, Q1_EINVAL, "q1_pcg_noalloc: need rtol >= 0 and maxit >= 0");
  Op &o = *reinterpret_cast<Op *>(op);
  const int64_t n = o.n_nodes * o.dpn();
  Q1_CHECK(n <= kNoAllocMaxDof, Q1_EINVAL,
           "q1_pcg_noalloc: %lld DOFs exceed the static workspace's %lld (Q1_NOALLOC_MAX_DOF)",
           static_cast<long long>(n), static_cast<long long>(kNoAllocMaxDof));
  unsigned char *base = nullptr;
  int rc = scratch_on(o.device, &base);
  if (rc) return rc;
  thread_local Status host_status;  // pageable host mirror: no pinned allocation
  Work W;
  W.owned = false;
  W.st = reinterpret_cast<Status *>(base);
  W.part = reinterpret_cast<double *>(base + kNoAllocHead);
  W.dparts = reinterpret_cast<double *>(base + kNoAllocHead + kNoAllocPart);
  unsigned char *v = base + kNoAllocHead + kNoAllocPart + kNoAllocDot;
  W.r = v;
  W.p = v + kNoAllocVec;
  W.q = v + 2 * kNoAllocVec;
  W.w = v + 3 * kNoAllocVec;
  W.hst = &host_status;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (o.dtype == Q1_F64)
    return pcg_t<double>(o, pc, static_cast<const double *>(b_d), static_cast<double *>(x_d),
                         rtol, maxit, st, s, true, Snapshots(), &W);
  return pcg_t<float>(o, pc, static_cast<const float *>(b_d), static_cast<float *>(x_d), rtol,
                      maxit, st, s, true, Snapshots(), &W);
}

int q1_pcg_trace(q1_op *op, int pc, const void *b_d, void *x_d, double rtol, int maxit, int nsnap,
                 const int *snap_iters, void *const *snap_d, q1_stats *st, void *stream) {
  Q1_CHECK(op && b_d && x_d && nsnap >= 0 && (nsnap == 0 || (snap_iters && snap_d)), Q1_EINVAL,
           "q1_pcg_trace: NULL argument");
  Q1_CHECK(pc == Q1_PC_NONE || pc == Q1_PC_JACOBI, Q1_EINVAL, "q1_pcg_trace: bad preconditioner");
  Q1_CHECK(rtol >= 0 && maxit >= 0, Q1_EINVAL, "q1_pcg_trace: need rtol >= 0 and maxit >= 0");
  for (int i = 0; i < nsnap; ++i) {
    Q1_CHECK(snap_d[i], Q1_EINVAL, "q1_pcg_trace: NULL snapshot %d", i);
    Q1_CHECK(i == 0 || snap_iters[i] >= snap_iters[i - 1], Q1_EINVAL,
             "q1_pcg_trace: snapshot iterations must ascend");
  }
  Op &o = *reinterpret_cast<Op *>(op);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Snapshots sn;
  sn.n = nsnap;
  sn.iters = snap_iters;
  sn.dst = snap_d;
  if (o.dtype == Q1_F64)
    return pcg_t<double>(o, pc, static_cast<const double *>(b_d), static_cast<double *>(x_d), rtol,
                         maxit, st, s, true, sn);
  return pcg_t<float>(o, pc, static_cast<const float *>(b_d), static_cast<float *>(x_d), rtol,
                      maxit, st, s, true, sn);
}

int q1_fcg(q1_op *op, q1_precond_fn M, void *ctx, const void *b_d, void *x_d, double rtol,
           int maxit, int safeguard_m, int trunc_m, q1_stats *st, void *stream) {
  Q1_CHECK(op && b_d && x_d, Q1_EINVAL, "q1_fcg: NULL argument");
  Q1_CHECK(rtol >= 0 && maxit >= 0, Q1_EINVAL, "q1_fcg: need rtol >= 0 and maxit >= 0");
  Q1_CHECK(trunc_m >= 1 && trunc_m <= kMaxTrunc, Q1_EINVAL, "q1_fcg: trunc_m %d not in [1, %d]",
           trunc_m, kMaxTrunc);
  Op &o = *reinterpret_cast<Op *>(op);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (o.dtype == Q1_F64)
    return fpcg_t<double>(o, M, ctx, static_cast<const double *>(b_d), static_cast<double *>(x_d),
                          rtol, maxit, safeguard_m, trunc_m, st, s);
  return fpcg_t<float>(o, M, ctx, static_cast<const float *>(b_d), static_cast<float *>(x_d),
                       rtol, maxit, safeguard_m, trunc_m, st, s);
}

int q1_dot(int64_t n, int dtype, const void *a_d, const void *b_d, double *out_d, int variant,
           int nblocks, double *work_d, void *stream) {
  Q1_CHECK(a_d && b_d && out_d && n >= 0, Q1_EINVAL, "q1_dot: NULL argument or n < 0");
  Q1_CHECK(dtype == Q1_F64 || dtype == Q1_F32, Q1_EINVAL, "q1_dot: bad dtype %d", dtype);
  Q1_CHECK(variant == Q1_DOT_TWO_STAGE || variant == Q1_DOT_ATOMIC, Q1_EINVAL,
           "q1_dot: bad variant %d", variant);
  Q1_CHECK(nblocks >= 0 && nblocks <= kMaxRB, Q1_EINVAL, "q1_dot: nblocks %d not in [0, %d]",
           nblocks, kMaxRB);
  Q1_CHECK(variant != Q1_DOT_TWO_STAGE || work_d, Q1_EINVAL, "q1_dot: two-stage needs work_d");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nb = nblocks > 0 ? nblocks : nblocks_for(n);
  auto run = [&](auto t) -> int {
    using T = decltype(t);
    const T *a = static_cast<const T *>(a_d), *c = static_cast<const T *>(b_d);
    if (variant == Q1_DOT_TWO_STAGE) {
      hipLaunchKernelGGL((k_dot<T>), dim3(nb), dim3(kRT), 0, s, n, a, c, work_d, nullptr);
      hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRT), 0, s, work_d, nb, out_d);
    } else {
      hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, s, out_d);
      hipLaunchKernelGGL((k_dot_atomic<T>), dim3(nb), dim3(kRT), 0, s, n, a, c, out_d);
    }
    Q1_HIP(hipGetLastError());
    return Q1_OK;
  };
  return dtype == Q1_F64 ? run(double{}) : run(float{});
}

int q1_fpcg(q1_op *op, q1_precond_fn M, void *ctx, const void *b_d, void *x_d, double rtol,
            int maxit, int safeguard_m, q1_stats *st, void *stream) {
  return q1_fcg(op, M, ctx, b_d, x_d, rtol, maxit, safeguard_m, 1, st, stream);
}

int q1_jacobi_create(q1_jacobi **out, q1_op *op, void *stream) {
  Q1_CHECK(out && op, Q1_EINVAL, "q1_jacobi_create: NULL argument");
  *out = nullptr;
  Op &o = *reinterpret_cast<Op *>(op);
  q1_jacobi *J = new (std::nothrow) q1_jacobi();
  Q1_CHECK(J, Q1_ENOMEM, "q1_jacobi_create: out of host memory");
  J->op = &o;
  const int64_t n = o.n_nodes * o.dpn();
  const size_t rb = o.dtype == Q1_F64 ? 8 : 4;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipMalloc(&J->w, size_t(n) * rb) != hipSuccess) {
    delete J;
    return fail(Q1_ENOMEM, "q1_jacobi_create: device allocation failed");
  }
  int rc = launch_diag(o, J->w, s);
  if (!rc) {
    if (o.dtype == Q1_F64)
      hipLaunchKernelGGL((k_inv_diag<double>), grid1(n), dim3(256), 0, s, n,
                         static_cast<const double *>(J->w), static_cast<double *>(J->w), 1);
    else
      hipLaunchKernelGGL((k_inv_diag<float>), grid1(n), dim3(256), 0, s, n,
                         static_cast<const float *>(J->w), static_cast<float *>(J->w), 1);
    if (hipGetLastError() != hipSuccess) rc = fail(Q1_EHIP, "q1_jacobi_create: launch failed");
  }
  if (rc) {
    (void)hipFree(J->w);
    delete J;
    return rc;
  }
  *out = J;
  return Q1_OK;
}

int q1_precond_jacobi(void *ctx, const void *r_d, void *z_d, void *stream) {
  Q1_CHECK(ctx && r_d && z_d, Q1_EINVAL, "q1_precond_jacobi: NULL argument");
  q1_jacobi *J = static_cast<q1_jacobi *>(ctx);
  const int64_t n = J->op->n_nodes * J->op->dpn();
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (J->op->dtype == Q1_F64)
    hipLaunchKernelGGL((k_jacobi<double>), grid1(n), dim3(256), 0, s, n,
                       static_cast<const double *>(J->w), static_cast<const double *>(r_d),
                       static_cast<double *>(z_d));
  else
    hipLaunchKernelGGL((k_jacobi<float>), grid1(n), dim3(256), 0, s, n,
                       static_cast<const float *>(J->w), static_cast<const float *>(r_d),
                       static_cast<float *>(z_d));
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

int q1_jacobi_destroy(q1_jacobi *J) {
  if (!J) return Q1_OK;
  if (J->w) (void)hipFree(J->w);
  delete J;
  return Q1_OK;
}

int q1_mpcg(q1_op *op64, q1_op *op32, const double *b_d, double *x_d, double rtol,
            double delta, int maxit, q1_stats *st, void *stream) {
  Q1_CHECK(op64 && op32 && b_d && x_d, Q1_EINVAL, "q1_mpcg: NULL argument");
  Op &A64 = *reinterpret_cast<Op *>(op64);
  Op &A32 = *reinterpret_cast<Op *>(op32);
  Q1_CHECK(A64.dtype == Q1_F64 && A32.dtype == Q1_F32, Q1_EINVAL,
           "q1_mpcg: needs an FP64 and an FP32 operator");
  Q1_CHECK(A64.n_nodes == A32.n_nodes && A64.physics == A32.physics, Q1_EINVAL,
           "q1_mpcg: operators of different sizes");
  Q1_CHECK(rtol > 0 && delta > 0 && delta < 1 && maxit >= 0, Q1_EINVAL,
           "q1_mpcg: need rtol > 0, 0 < delta < 1, maxit >= 0");
  return mpcg_t(A64, A32, b_d, x_d, rtol, delta, maxit, st, static_cast<hipStream_t>(stream));
}

int q1_ir_solve(q1_op *op64, q1_op *op32, const double *b_d, double *x_d, double rtol,
                double inner_rtol, int max_outer, int max_inner, q1_stats *st, void *stream) {
  Q1_CHECK(op64 && op32 && b_d && x_d, Q1_EINVAL, "q1_ir_solve: NULL argument");
  Op &A64 = *reinterpret_cast<Op *>(op64);
  Op &A32 = *reinterpret_cast<Op *>(op32);
  Q1_CHECK(A64.dtype == Q1_F64 && A32.dtype == Q1_F32, Q1_EINVAL,
           "q1_ir_solve: needs an FP64 and an FP32 operator");
  Q1_CHECK(A64.n_nodes == A32.n_nodes && A64.physics == A32.physics, Q1_EINVAL,
           "q1_ir_solve: operators of different sizes");
  Q1_CHECK(rtol > 0 && inner_rtol > 0 && inner_rtol < 1 && max_outer > 0 && max_inner > 0,
           Q1_EINVAL, "q1_ir_solve: bad tolerances or limits");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = A64.n_nodes * A64.dpn();
  const auto t0 = std::chrono::steady_clock::now();
  Work W;  // FP64 residual, norms
  int rc = alloc_work<double>(W, n, false);
  if (rc) return rc;
  float *s32 = nullptr, *d32 = nullptr;
  struct Free {
    float **a, **b;
    ~Free() {
      if (*a) (void)hipFree(*a);
      if (*b) (void)hipFree(*b);
    }
  } fr{&s32, &d32};
  Q1_HIP(hipMalloc(&s32, size_t(n) * sizeof(float)));
  Q1_HIP(hipMalloc(&d32, size_t(n) * sizeof(float)));
  const int nb = nblocks_for(n);
  double *r = static_cast<double *>(W.r);
  double *part_bb = W.part + 4 * kMaxRB, *part_rr = W.part + 3 * kMaxRB;
  Q1_HIP(hipMemsetAsync(W.st, 0, sizeof(Status), s));
  Q1_HIP(hipMemsetAsync(x_d, 0, size_t(n) * sizeof(double), s));
  Q1_HIP(hipMemcpyAsync(r, b_d, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL((k_dot<double>), dim3(nb), dim3(kRT), 0, s, n, b_d, b_d, part_bb, nullptr);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRT), 0, s, part_bb, nb, &W.st->bb);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRT), 0, s, part_bb, nb, &W.st->rr);  // r_0 = b
  Q1_HIP(hipGetLastError());
  if ((rc = read_status(W, s))) return rc;
  const double bb = W.hst->bb;
  double rr = bb;
  int outer = 0, inner_total = 0, status = Q1_OK;
  double prev_rr = INFINITY;
  while (bb > 0.0 && rr > rtol * rtol * bb) {
    if (outer >= max_outer) {
      status = Q1_ENOCONV;
      break;
    }
    if (!(rr < prev_rr)) {  // no progress: refinement diverges or stagnates
      status = Q1_EBREAKDOWN;
      break;
    }
    prev_rr = rr;
    // s = r / ||r|| in FP32; solve A32 d = s to inner_rtol; x += ||r|| d
    hipLaunchKernelGGL(k_scale_to_f32, grid1(n), dim3(256), 0, s, n, r, &W.st->rr, s32);
    Q1_HIP(hipGetLastError());
    q1_stats ist{};
    rc = pcg_t<float>(A32, Q1_PC_JACOBI, s32, d32, inner_rtol, max_inner, &ist, s, false);
    if (rc != Q1_OK && rc != Q1_ENOCONV) return rc;
    inner_total += ist.iters;
    hipLaunchKernelGGL(k_ir_update, grid1(n), dim3(256), 0, s, n, d32, &W.st->rr, x_d);
    // r = b - A64 x in FP64
    if ((rc = launch_apply(A64, x_d, r, s))) return rc;
    hipLaunchKernelGGL((k_residual<double>), grid1(n), dim3(256), 0, s, n, b_d, r);
    hipLaunchKernelGGL((k_dot<double>), dim3(nb), dim3(kRT), 0, s, n, r, r, part_rr, nullptr);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRT), 0, s, part_rr, nb, &W.st->rr);
    Q1_HIP(hipGetLastError());
    if ((rc = read_status(W, s))) return rc;
    rr = W.hst->rr;
    ++outer;
  }
  const auto t1 = std::chrono::steady_clock::now();
  if (st) {
    st->iters = inner_total;
    st->outer_iters = outer;
    st->status = status;
    st->seconds = std::chrono::duration<double>(t1 - t0).count();
    st->rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    st->true_rel_res = st->rel_res;
    st->fallback_at = -1;
  }
  return status;
}

}  // extern "C"
