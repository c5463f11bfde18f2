// Element families beyond the trilinear hexahedron, named in the paper's
// conclusions (Section 7) as the next cases for its matrix-free algorithm:
// linear tetrahedra (simplicial elements) and triquadratic and tricubic
// hexahedra (higher-order elements).  The operators are the same scalar Laplace and
// isotropic elasticity with cell-wise coefficients (Section 2), applied
// without a matrix by the gather / local product / scatter-add of Section 3.
//
// Linear tetrahedra: one thread per element.  With E_c = X_c - X_0 (c = 1, 2,
// 3) the cross products c_1 = E_2 x E_3, c_2 = E_3 x E_1, c_3 = E_1 x E_2 and
// c_0 = -(c_1 + c_2 + c_3) are det J times the (constant) physical gradients
// of the four basis functions, det J = E_1 . c_1 and the volume det J / 6, so
//   Laplace      v_a = k (c_a . g) / (6 det J),  g = sum_b c_b u_b,
//   elasticity   v_a = S c_a / (6 det J),  S = lambda tr(H) I + mu (H + H^T),
//                H = sum_b u_b (x) c_b (= det J grad u).
// Hexahedra of order P = 2 (27 nodes) and 3 (64 nodes): (P+1)^3 threads per
// element (a block holds 9 or 4 elements).  Thread r stages node r
// (coordinates, input) in LDS, then evaluates quadrature point r of the
// (P+1)^3 Gauss rule: the Jacobian J, its adjugate A
// (rows the cross products of the columns, so J^-1 = A / det J) and the
// reference gradients g of the input; it leaves in LDS the reference flux f,
// with v_a = sum_q grad_hat phi_a(q) . f(q):
//   Laplace      f = k w A (sum_c g_c A_c) / det J,
//   elasticity   f_i = w S_i A^T / det J,  H = G A (det J grad u, rows of G
//                the reference gradients of the components), S as above;
// finally thread r gathers v_r for node r.  Both element kinds scatter with
// global atomics (the paper's one-thread-per-element strategy), after
// y = x on Dirichlet nodes and 0 elsewhere.
#include <hip/hip_runtime.h>

#include "q1_elem.hpp"
#include "q1_internal.hpp"

namespace q1 {
namespace {

constexpr int kFB = 256;  // threads per block

__device__ __forceinline__ void gadd(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void gadd(float *p, float v) { unsafeAtomicAdd(p, v); }

// y = x on Dirichlet nodes, 0 elsewhere (before the atomic scatter); the same
// with 1 for the diagonal
template <typename T, int DPN>
__global__ void k_fam_init(int64_t nn, const uint8_t *__restrict__ mask,
                           const T *__restrict__ x, T *__restrict__ y,
                           const int *__restrict__ stop) {
  if (stop && *stop) return;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nn * DPN) return;
  const bool fx = mask && mask[i / DPN];
  y[i] = fx ? (x ? x[i] : T(1)) : T(0);
}

// ---- linear tetrahedra -----------------------------------------------------

template <typename T>
struct TetGeom {
  T c[4][3];  // det J times the physical gradients
  T s;        // 1 / (6 det J)
};

template <typename T>
__device__ __forceinline__ TetGeom<T> tet_geom(const T X[3][4]) {
  TetGeom<T> G;
  const T E1[3] = {X[0][1] - X[0][0], X[1][1] - X[1][0], X[2][1] - X[2][0]};
  const T E2[3] = {X[0][2] - X[0][0], X[1][2] - X[1][0], X[2][2] - X[2][0]};
  const T E3[3] = {X[0][3] - X[0][0], X[1][3] - X[1][0], X[2][3] - X[2][0]};
  cross(E2, E3, G.c[1]);
  cross(E3, E1, G.c[2]);
  cross(E1, E2, G.c[3]);
#pragma unroll
  for (int r = 0; r < 3; ++r) G.c[0][r] = -(G.c[1][r] + G.c[2][r] + G.c[3][r]);
  G.s = rcp(T(6) * dot3(E1, G.c[1]));
  return G;
}

template <typename T, int PH, bool MASKED>
__global__ __launch_bounds__(kFB) void k_tet_apply(int64_t ne, int64_t nn,
                                                   const T *__restrict__ xyz,
                                                   const int32_t *__restrict__ conn,
                                                   const T *__restrict__ coef,
                                                   const uint8_t *__restrict__ mask,
                                                   const T *__restrict__ x, T *__restrict__ y,
                                                   const int *__restrict__ stop) {
  constexpr int DPN = phys_dpn(PH);
  if (stop && *stop) return;
  const int64_t e = int64_t(blockIdx.x) * kFB + threadIdx.x;
  if (e >= ne) return;
  int32_t nid[4];
  bool fixed[4];
  T X[3][4], u[DPN][4];
#pragma unroll
  for (int a = 0; a < 4; ++a) nid[a] = conn[a * ne + e];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    fixed[a] = MASKED && mask[nid[a]] != 0;
#pragma unroll
    for (int r = 0; r < 3; ++r) X[r][a] = xyz[r * nn + nid[a]];
#pragma unroll
    for (int j = 0; j < DPN; ++j) u[j][a] = fixed[a] ? T(0) : x[int64_t(nid[a]) * DPN + j];
  }
  T v[DPN][4];
  tet_element<T, PH>(X, u, coef[e], PH == 3 ? coef[ne + e] : T(0), v);
#pragma unroll
  for (int a = 0; a < 4; ++a)
    if (!fixed[a])
#pragma unroll
      for (int j = 0; j < DPN; ++j) gadd(&y[int64_t(nid[a]) * DPN + j], v[j][a]);
}

// diag: Laplace k |c_a|^2 / (6 det J); elasticity ((lambda + mu) c_ai^2 + mu |c_a|^2) / (6 det J)
template <typename T, int PH, bool MASKED>
__global__ __launch_bounds__(kFB) void k_tet_diag(int64_t ne, int64_t nn,
                                                  const T *__restrict__ xyz,
                                                  const int32_t *__restrict__ conn,
                                                  const T *__restrict__ coef,
                                                  const uint8_t *__restrict__ mask,
                                                  T *__restrict__ d) {
  constexpr int DPN = phys_dpn(PH);
  const int64_t e = int64_t(blockIdx.x) * kFB + threadIdx.x;
  if (e >= ne) return;
  int32_t nid[4];
  T X[3][4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    nid[a] = conn[a * ne + e];
#pragma unroll
    for (int r = 0; r < 3; ++r) X[r][a] = xyz[r * nn + nid[a]];
  }
  const TetGeom<T> G = tet_geom(X);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    if (MASKED && mask[nid[a]]) continue;
    const T cc = dot3(G.c[a], G.c[a]);
    if constexpr (PH == 1) {
      gadd(&d[nid[a]], coef[e] * G.s * cc);
    } else {
      const T lam = coef[e], mu = coef[ne + e];
#pragma unroll
      for (int i = 0; i < 3; ++i)
        gadd(&d[int64_t(nid[a]) * 3 + i], G.s * ((lam + mu) * G.c[a][i] * G.c[a][i] + mu * cc));
    }
  }
}

// ---- triquadratic and tricubic hexahedra ------------------------------------
//
// Order P = 2 (27 nodes) or 3 (64 nodes): nodes at t_m = -1 + 2m/P per
// direction, local node a = i + (P+1) j + (P+1)^2 k, P+1 Gauss points per
// direction.  A block holds 256 / (P+1)^3 elements, thread r of an element
// staging node r and then evaluating quadrature point r.

template <int P>
struct QP {
  static constexpr int N = P + 1;          // nodes (and Gauss points) per direction
  static constexpr int NPTS = N * N * N;   // nodes (and points) per element
  static constexpr int E = 256 / NPTS;     // elements per block
};

// 1-D Lagrange basis of order P on [-1, 1] and its derivative (quadratic: the
// closed forms; cubic: the product formula over the other nodes)
template <typename T, int P>
__device__ __forceinline__ T lag(int i, T t) {
  if constexpr (P == 2) {
    return i == 0 ? T(0.5) * t * (t - T(1)) : i == 1 ? T(1) - t * t : T(0.5) * t * (t + T(1));
  } else {
    T v = T(1);
#pragma unroll
    for (int m = 0; m <= P; ++m)
      if (m != i) v *= (t - (T(-1) + T(2 * m) / T(P))) / (T(2 * (i - m)) / T(P));
    return v;
  }
}
template <typename T, int P>
__device__ __forceinline__ T dlag(int i, T t) {
  if constexpr (P == 2) {
    return i == 0 ? t - T(0.5) : i == 1 ? T(-2) * t : t + T(0.5);
  } else {
    T d = T(0);
#pragma unroll
    for (int l = 0; l <= P; ++l) {
      if (l == i) continue;
      T v = T(1) / (T(2 * (i - l)) / T(P));
#pragma unroll
      for (int m = 0; m <= P; ++m)
        if (m != i && m != l) v *= (t - (T(-1) + T(2 * m) / T(P))) / (T(2 * (i - m)) / T(P));
      d += v;
    }
    return d;
  }
}
// Gauss-Legendre points and weights with P + 1 points
template <typename T, int P>
__device__ __forceinline__ T gpt(int q) {
  if constexpr (P == 2) {
    return q == 0 ? -T(0.77459666924148337703585307995648)
                  : q == 1 ? T(0) : T(0.77459666924148337703585307995648);
  } else {  // +-sqrt(3/7 +- (2/7) sqrt(6/5))
    const T a = T(0.33998104358485626480266575910324), b = T(0.86113631159405257522394648889281);
    return q == 0 ? -b : q == 1 ? -a : q == 2 ? a : b;
  }
}
template <typename T, int P>
__device__ __forceinline__ T gwt(int q) {
  if constexpr (P == 2) {
    return q == 1 ? T(8) / T(9) : T(5) / T(9);
  } else {  // (18 +- sqrt(30)) / 36
    const T wa = T(0.65214515486254614262693605077800), wb = T(0.34785484513745385737306394922200);
    return q == 0 || q == 3 ? wb : wa;
  }
}

// The per-thread 1-D tables: basis and derivative of the functions at one
// point (phase 2), or of one function at the points (phase 3).
template <typename T, int P>
struct Tab1 {
  T b[P + 1], d[P + 1];
};
template <typename T, int P>
__device__ __forceinline__ Tab1<T, P> at_point(int q) {
  Tab1<T, P> t;
  const T p = gpt<T, P>(q);
#pragma unroll
  for (int i = 0; i <= P; ++i) {
    t.b[i] = lag<T, P>(i, p);
    t.d[i] = dlag<T, P>(i, p);
  }
  return t;
}
template <typename T, int P>
__device__ __forceinline__ Tab1<T, P> of_function(int i) {
  Tab1<T, P> t;
#pragma unroll
  for (int q = 0; q <= P; ++q) {
    t.b[q] = lag<T, P>(i, gpt<T, P>(q));
    t.d[q] = dlag<T, P>(i, gpt<T, P>(q));
  }
  return t;
}

// Phase 2 at quadrature point r of a staged element: the Jacobian's
// adjugate rows A (A[0] = j1 x j2, A[1] = j2 x j0, A[2] = j0 x j1), det J, and
// the reference gradients G of NF staged fields.
template <typename T, int P, int NF>
__device__ __forceinline__ T qp_point(int r, const T (*sX)[QP<P>::NPTS],
                                      const T (*sU)[QP<P>::NPTS], T A[3][3], T G[NF][3]) {
  constexpr int N = QP<P>::N, NPTS = QP<P>::NPTS;
  const Tab1<T, P> tx = at_point<T, P>(r % N), ty = at_point<T, P>((r / N) % N),
                   tz = at_point<T, P>(r / (N * N));
  T J[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) J[c][d] = T(0);
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int d = 0; d < 3; ++d) G[f][d] = T(0);
#pragma unroll
  for (int a = 0; a < NPTS; ++a) {
    const int i = a % N, j = (a / N) % N, k = a / (N * N);
    const T d0 = tx.d[i] * ty.b[j] * tz.b[k];
    const T d1 = tx.b[i] * ty.d[j] * tz.b[k];
    const T d2 = tx.b[i] * ty.b[j] * tz.d[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T xc = sX[c][a];
      J[c][0] += xc * d0;
      J[c][1] += xc * d1;
      J[c][2] += xc * d2;
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const T uf = sU[f][a];
      G[f][0] += uf * d0;
      G[f][1] += uf * d1;
      G[f][2] += uf * d2;
    }
  }
  const T j0[3] = {J[0][0], J[1][0], J[2][0]};
  const T j1[3] = {J[0][1], J[1][1], J[2][1]};
  const T j2[3] = {J[0][2], J[1][2], J[2][2]};
  cross(j1, j2, A[0]);
  cross(j2, j0, A[1]);
  cross(j0, j1, A[2]);
  return dot3(j0, A[0]);
}

template <typename T, int PH, bool MASKED, int P>
__global__ __launch_bounds__(kFB) void k_qp_apply(int64_t ne, int64_t nn,
                                                  const T *__restrict__ xyz,
                                                  const int32_t *__restrict__ conn,
                                                  const T *__restrict__ coef,
                                                  const uint8_t *__restrict__ mask,
                                                  const T *__restrict__ x, T *__restrict__ y,
                                                  const int *__restrict__ stop) {
  constexpr int DPN = phys_dpn(PH);
  constexpr int N = QP<P>::N, NPTS = QP<P>::NPTS, E = QP<P>::E;
  if (stop && *stop) return;
  __shared__ T sX[E][3][NPTS];
  __shared__ T sU[E][DPN][NPTS];
  __shared__ T sF[E][DPN][3][NPTS];  // reference flux: [component][direction][point]
  const int le = int(threadIdx.x) / NPTS, r = int(threadIdx.x) - NPTS * le;
  const int64_t e = int64_t(blockIdx.x) * E + le;
  const bool active = le < E && e < ne;
  int64_t g = 0;
  bool fixed = true;
  if (active) {  // phase 1: node r
    g = conn[int64_t(r) * ne + e];
    fixed = MASKED && mask[g] != 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) sX[le][c][r] = xyz[c * nn + g];
#pragma unroll
    for (int j = 0; j < DPN; ++j) sU[le][j][r] = fixed ? T(0) : x[g * DPN + j];
  }
  __syncthreads();
  if (active) {  // phase 2: quadrature point r
    T A[3][3], G[DPN][3];
    const T det = qp_point<T, P, DPN>(r, sX[le], sU[le], A, G);
    const T s = gwt<T, P>(r % N) * gwt<T, P>((r / N) % N) * gwt<T, P>(r / (N * N)) * rcp(det);
    if constexpr (PH == 1) {
      T p[3];  // det J times the physical gradient
#pragma unroll
      for (int m = 0; m < 3; ++m) p[m] = G[0][0] * A[0][m] + G[0][1] * A[1][m] + G[0][2] * A[2][m];
      const T ks = coef[e] * s;
#pragma unroll
      for (int d = 0; d < 3; ++d) sF[le][0][d][r] = ks * dot3(A[d], p);
    } else {
      const T lam = coef[e], mu = coef[ne + e];
      T H[3][3];  // det J times the displacement gradient
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) H[i][j] = G[i][0] * A[0][j] + G[i][1] * A[1][j] + G[i][2] * A[2][j];
      const T ltr = lam * (H[0][0] + H[1][1] + H[2][2]);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        T Si[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) Si[j] = mu * (H[i][j] + H[j][i]) + (i == j ? ltr : T(0));
#pragma unroll
        for (int d = 0; d < 3; ++d) sF[le][i][d][r] = s * dot3(Si, A[d]);
      }
    }
  }
  __syncthreads();
  if (active && !fixed) {  // phase 3: node r gathers the test-function products
    const Tab1<T, P> fx = of_function<T, P>(r % N), fy = of_function<T, P>((r / N) % N),
                     fz = of_function<T, P>(r / (N * N));
    T v[DPN];
#pragma unroll
    for (int j = 0; j < DPN; ++j) v[j] = T(0);
#pragma unroll
    for (int q = 0; q < NPTS; ++q) {
      const int qx = q % N, qy = (q / N) % N, qz = q / (N * N);
      const T d0 = fx.d[qx] * fy.b[qy] * fz.b[qz];
      const T d1 = fx.b[qx] * fy.d[qy] * fz.b[qz];
      const T d2 = fx.b[qx] * fy.b[qy] * fz.d[qz];
#pragma unroll
      for (int j = 0; j < DPN; ++j)
        v[j] += d0 * sF[le][j][0][q] + d1 * sF[le][j][1][q] + d2 * sF[le][j][2][q];
    }
#pragma unroll
    for (int j = 0; j < DPN; ++j) gadd(&y[g * DPN + j], v[j]);
  }
}

// Sum-factorised apply of order P: the per-point reference gradients of the
// coordinates and the input, and the transposed evaluation of the flux, each
// in three 1-D passes through LDS (one thread per index triple of the
// element's N^3 nodes or points, N = P + 1):
//   A  T0[qx][j][k] = sum_i B[qx][i] f[i][j][k],  T1 = the same with D
//   B  from T0, T1 along y: f interpolated (T00), d/dxi (T10), d/deta (T01)
//   C  along z: g_xi = B T10, g_eta = B T01, g_zeta = D T00 at (qx, qy, qz)
// with B[q][i] = L_i(p_q) and D[q][i] = L_i'(p_q); then the flux at the point
// (as k_qp_apply), and the transpose of A-B-C on it:
//   v[i][j][k] = sum_q (D_i B_j B_k F_xi + B_i D_j B_k F_eta + B_i B_j D_k F_zeta).
// O(N^4) per field instead of O(N^6).  QPE<P, DPN, T>::E elements per block.
template <int P, int DPN, typename T>
struct QPE {
  static constexpr int NPTS = (P + 1) * (P + 1) * (P + 1);
  static constexpr int F = 3 + DPN;                       // coordinates and input fields
  static constexpr int RX = F > 3 * DPN ? F : 3 * DPN;    // node values, then the flux
  static constexpr int RY = 2 * F > 3 * DPN ? 2 * F : 3 * DPN;
  static constexpr int RZ = 3 * F > 2 * DPN ? 3 * F : 2 * DPN;
  static constexpr int BYTES = (RX + RY + RZ) * NPTS * int(sizeof(T));  // per element
  static constexpr int EMAX = 256 / NPTS;
  static constexpr int EL = (40 * 1024) / BYTES;
  static constexpr int E = EL < 1 ? 1 : (EL < EMAX ? EL : EMAX);
};

template <typename T, int PH, bool MASKED, int P>
__global__ __launch_bounds__(256) void k_qp_apply_sf(int64_t ne, int64_t nn,
                                                     const T *__restrict__ xyz,
                                                     const int32_t *__restrict__ conn,
                                                     const T *__restrict__ coef,
                                                     const uint8_t *__restrict__ mask,
                                                     const T *__restrict__ x, T *__restrict__ y,
                                                     const int *__restrict__ stop) {
  constexpr int DPN = phys_dpn(PH);
  using Q = QPE<P, DPN, T>;
  constexpr int N = P + 1, NPTS = Q::NPTS, E = Q::E, F = Q::F;
  if (stop && *stop) return;
  __shared__ T sX[E][Q::RX][NPTS];  // node values (F), then the flux (3 DPN)
  __shared__ T sY[E][Q::RY][NPTS];  // pass A (2F), then the transposed pass C (3 DPN)
  __shared__ T sZ[E][Q::RZ][NPTS];  // pass B (3F), then the transposed pass B (2 DPN)
  const int le = int(threadIdx.x) / NPTS, r = int(threadIdx.x) - NPTS * le;
  const int64_t e = int64_t(blockIdx.x) * E + le;
  const bool active = le < E && e < ne;
  const int a0 = r % N, a1 = (r / N) % N, a2 = r / (N * N);  // this thread's index triple
  // the 1-D tables B[q][i] and D[q][i] (N x N, constants of the rule)
  T Bt[N][N], Dt[N][N];
#pragma unroll
  for (int q = 0; q < N; ++q)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      Bt[q][i] = lag<T, P>(i, gpt<T, P>(q));
      Dt[q][i] = dlag<T, P>(i, gpt<T, P>(q));
    }
  int64_t g = 0;
  bool fixed = true;
  if (active) {  // node (a0, a1, a2) = r
    g = conn[int64_t(r) * ne + e];
    fixed = MASKED && mask[g] != 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) sX[le][c][r] = xyz[c * nn + g];
#pragma unroll
    for (int j = 0; j < DPN; ++j) sX[le][3 + j][r] = fixed ? T(0) : x[g * DPN + j];
  }
  __syncthreads();
  if (active) {  // pass A at (qx, j, k) = (a0, a1, a2): contract i
#pragma unroll
    for (int f = 0; f < F; ++f) {
      T t0 = T(0), t1 = T(0);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const T v = sX[le][f][i + N * (a1 + N * a2)];
        t0 += Bt[a0][i] * v;
        t1 += Dt[a0][i] * v;
      }
      sY[le][2 * f][r] = t0;
      sY[le][2 * f + 1][r] = t1;
    }
  }
  __syncthreads();
  if (active) {  // pass B at (qx, qy, k) = (a0, a1, a2): contract j
#pragma unroll
    for (int f = 0; f < F; ++f) {
      T u00 = T(0), u10 = T(0), u01 = T(0);
#pragma unroll
      for (int jj = 0; jj < N; ++jj) {
        const int s = a0 + N * (jj + N * a2);
        const T v0 = sY[le][2 * f][s], v1 = sY[le][2 * f + 1][s];
        u00 += Bt[a1][jj] * v0;
        u10 += Bt[a1][jj] * v1;
        u01 += Dt[a1][jj] * v0;
      }
      sZ[le][3 * f][r] = u00;
      sZ[le][3 * f + 1][r] = u10;
      sZ[le][3 * f + 2][r] = u01;
    }
  }
  __syncthreads();
  if (active) {  // pass C at (qx, qy, qz) = (a0, a1, a2): contract k, then the flux
    T Gr[F][3];
#pragma unroll
    for (int f = 0; f < F; ++f) {
      T gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
      for (int kk = 0; kk < N; ++kk) {
        const int s = a0 + N * (a1 + N * kk);
        gx += Bt[a2][kk] * sZ[le][3 * f + 1][s];
        gy += Bt[a2][kk] * sZ[le][3 * f + 2][s];
        gz += Dt[a2][kk] * sZ[le][3 * f][s];
      }
      Gr[f][0] = gx;
      Gr[f][1] = gy;
      Gr[f][2] = gz;
    }
    const T j0[3] = {Gr[0][0], Gr[1][0], Gr[2][0]};
    const T j1[3] = {Gr[0][1], Gr[1][1], Gr[2][1]};
    const T j2[3] = {Gr[0][2], Gr[1][2], Gr[2][2]};
    T A[3][3];
    cross(j1, j2, A[0]);
    cross(j2, j0, A[1]);
    cross(j0, j1, A[2]);
    const T det = dot3(j0, A[0]);
    const T s = gwt<T, P>(a0) * gwt<T, P>(a1) * gwt<T, P>(a2) * rcp(det);
    if constexpr (PH == 1) {
      T p[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) p[m] = Gr[3][0] * A[0][m] + Gr[3][1] * A[1][m] + Gr[3][2] * A[2][m];
      const T ks = coef[e] * s;
#pragma unroll
      for (int d = 0; d < 3; ++d) sX[le][d][r] = ks * dot3(A[d], p);
    } else {
      const T lam = coef[e], mu = coef[ne + e];
      T H[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
          H[i][jj] = Gr[3 + i][0] * A[0][jj] + Gr[3 + i][1] * A[1][jj] + Gr[3 + i][2] * A[2][jj];
      const T ltr = lam * (H[0][0] + H[1][1] + H[2][2]);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        T Si[3];
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) Si[jj] = mu * (H[i][jj] + H[jj][i]) + (i == jj ? ltr : T(0));
#pragma unroll
        for (int d = 0; d < 3; ++d) sX[le][3 * i + d][r] = s * dot3(Si, A[d]);
      }
    }
  }
  __syncthreads();  // the flux F[c][d] of component c, direction d, at sX[le][3c + d]
  if (active) {  // transposed pass C at (qx, qy, k) = (a0, a1, a2): contract qz
#pragma unroll
    for (int c = 0; c < DPN; ++c) {
      T u0 = T(0), u1 = T(0), u2 = T(0);
#pragma unroll
      for (int qz = 0; qz < N; ++qz) {
        const int s = a0 + N * (a1 + N * qz);
        u0 += Bt[qz][a2] * sX[le][3 * c][s];
        u1 += Bt[qz][a2] * sX[le][3 * c + 1][s];
        u2 += Dt[qz][a2] * sX[le][3 * c + 2][s];
      }
      sY[le][3 * c][r] = u0;
      sY[le][3 * c + 1][r] = u1;
      sY[le][3 * c + 2][r] = u2;
    }
  }
  __syncthreads();
  if (active) {  // transposed pass B at (qx, j, k) = (a0, a1, a2): contract qy
#pragma unroll
    for (int c = 0; c < DPN; ++c) {
      T w0 = T(0), w1 = T(0);
#pragma unroll
      for (int qy = 0; qy < N; ++qy) {
        const int s = a0 + N * (qy + N * a2);
        w0 += Bt[qy][a1] * sY[le][3 * c][s];
        w1 += Dt[qy][a1] * sY[le][3 * c + 1][s] + Bt[qy][a1] * sY[le][3 * c + 2][s];
      }
      sZ[le][2 * c][r] = w0;
      sZ[le][2 * c + 1][r] = w1;
    }
  }
  __syncthreads();
  if (active && !fixed) {  // transposed pass A at node (i, j, k) = (a0, a1, a2): contract qx
#pragma unroll
    for (int c = 0; c < DPN; ++c) {
      T v = T(0);
#pragma unroll
      for (int qx = 0; qx < N; ++qx) {
        const int s = qx + N * (a1 + N * a2);
        v += Dt[qx][a0] * sZ[le][2 * c][s] + Bt[qx][a0] * sZ[le][2 * c + 1][s];
      }
      gadd(&y[g * DPN + c], v);
    }
  }
}

// diag: Laplace sum_q k w |t|^2 / det J, elasticity
// sum_q w ((lambda + mu) t_i^2 + mu |t|^2) / det J, with t = sum_c dphi_c A[c]
// (det J times the physical gradient of the node's basis function)
template <typename T, int PH, bool MASKED, int P>
__global__ __launch_bounds__(kFB) void k_qp_diag(int64_t ne, int64_t nn,
                                                 const T *__restrict__ xyz,
                                                 const int32_t *__restrict__ conn,
                                                 const T *__restrict__ coef,
                                                 const uint8_t *__restrict__ mask,
                                                 T *__restrict__ dg) {
  constexpr int DPN = phys_dpn(PH);
  constexpr int N = QP<P>::N, NPTS = QP<P>::NPTS, E = QP<P>::E;
  __shared__ T sX[E][3][NPTS];
  __shared__ T sA[E][10][NPTS];  // adjugate rows and w / det J per point
  const int le = int(threadIdx.x) / NPTS, r = int(threadIdx.x) - NPTS * le;
  const int64_t e = int64_t(blockIdx.x) * E + le;
  const bool active = le < E && e < ne;
  int64_t g = 0;
  bool fixed = true;
  if (active) {
    g = conn[int64_t(r) * ne + e];
    fixed = MASKED && mask[g] != 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) sX[le][c][r] = xyz[c * nn + g];
  }
  __syncthreads();
  if (active) {
    T A[3][3], G[1][3];  // (the coordinate field stands in for the unused input)
    const T det = qp_point<T, P, 1>(r, sX[le], sX[le], A, G);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int m = 0; m < 3; ++m) sA[le][3 * c + m][r] = A[c][m];
    sA[le][9][r] = gwt<T, P>(r % N) * gwt<T, P>((r / N) % N) * gwt<T, P>(r / (N * N)) * rcp(det);
  }
  __syncthreads();
  if (active && !fixed) {
    const Tab1<T, P> fx = of_function<T, P>(r % N), fy = of_function<T, P>((r / N) % N),
                     fz = of_function<T, P>(r / (N * N));
    T acc[DPN];
#pragma unroll
    for (int j = 0; j < DPN; ++j) acc[j] = T(0);
    const T c0 = coef[e], c1 = PH == 3 ? coef[ne + e] : T(0);
#pragma unroll
    for (int q = 0; q < NPTS; ++q) {
      const int qx = q % N, qy = (q / N) % N, qz = q / (N * N);
      const T d0 = fx.d[qx] * fy.b[qy] * fz.b[qz];
      const T d1 = fx.b[qx] * fy.d[qy] * fz.b[qz];
      const T d2 = fx.b[qx] * fy.b[qy] * fz.d[qz];
      T t[3];
#pragma unroll
      for (int m = 0; m < 3; ++m)
        t[m] = d0 * sA[le][m][q] + d1 * sA[le][3 + m][q] + d2 * sA[le][6 + m][q];
      const T tt = dot3(t, t), s = sA[le][9][q];
      if constexpr (PH == 1) {
        acc[0] += c0 * s * tt;
      } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) acc[i] += s * ((c0 + c1) * t[i] * t[i] + c1 * tt);
      }
    }
#pragma unroll
    for (int j = 0; j < DPN; ++j) gadd(&dg[g * DPN + j], acc[j]);
  }
}

template <typename T, int PH>
int family_apply_t(Op &op, const void *xv, void *yv, hipStream_t s, const int *stop) {
  constexpr int DPN = phys_dpn(PH);
  const T *x = static_cast<const T *>(xv);
  T *y = static_cast<T *>(yv);
  const int64_t ndof = op.n_nodes * DPN;
  hipLaunchKernelGGL((k_fam_init<T, DPN>), dim3(unsigned((ndof + kFB - 1) / kFB)), dim3(kFB), 0,
                     s, op.n_nodes, op.mask, x, y, stop);
  if (op.n_elems > 0) {
    const T *xyz = static_cast<const T *>(op.xyz), *coef = static_cast<const T *>(op.coef);
    const bool m = op.mask != nullptr;
    if (op.elem == Q1_TET4) {
      const dim3 grid(unsigned((op.n_elems + kFB - 1) / kFB));
      hipLaunchKernelGGL((m ? k_tet_apply<T, PH, true> : k_tet_apply<T, PH, false>), grid,
                         dim3(kFB), 0, s, op.n_elems, op.n_nodes, xyz, op.conn, coef, op.mask,
                         x, y, stop);
    } else {
      auto run = [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        using Q = QPE<P, DPN, T>;
        const dim3 grid(unsigned((op.n_elems + Q::E - 1) / Q::E));
        hipLaunchKernelGGL((m ? k_qp_apply_sf<T, PH, true, P> : k_qp_apply_sf<T, PH, false, P>),
                           grid, dim3(Q::E * Q::NPTS), 0, s, op.n_elems, op.n_nodes, xyz,
                           op.conn, coef, op.mask, x, y, stop);
      };
      // triquadratic: the per-point form (measured on 64^3 FP64 9.0 GDOF/s against 8.1
      // sum-factorised); tricubic: the sum-factorised form (42^3 FP64 6.3 against 3.2)
      if (op.elem == Q1_HEX27) {
        const dim3 grid(unsigned((op.n_elems + QP<2>::E - 1) / QP<2>::E));
        hipLaunchKernelGGL((m ? k_qp_apply<T, PH, true, 2> : k_qp_apply<T, PH, false, 2>), grid,
                           dim3(kFB), 0, s, op.n_elems, op.n_nodes, xyz, op.conn, coef,
                           op.mask, x, y, stop);
      } else {
        run(std::integral_constant<int, 3>{});
      }
    }
  }
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

template <typename T, int PH>
int family_diag_t(Op &op, void *dv, hipStream_t s) {
  constexpr int DPN = phys_dpn(PH);
  T *d = static_cast<T *>(dv);
  const int64_t ndof = op.n_nodes * DPN;
  hipLaunchKernelGGL((k_fam_init<T, DPN>), dim3(unsigned((ndof + kFB - 1) / kFB)), dim3(kFB), 0,
                     s, op.n_nodes, op.mask, static_cast<const T *>(nullptr), d,
                     static_cast<const int *>(nullptr));
  if (op.n_elems > 0) {
    const T *xyz = static_cast<const T *>(op.xyz), *coef = static_cast<const T *>(op.coef);
    const bool m = op.mask != nullptr;
    if (op.elem == Q1_TET4) {
      const dim3 grid(unsigned((op.n_elems + kFB - 1) / kFB));
      hipLaunchKernelGGL((m ? k_tet_diag<T, PH, true> : k_tet_diag<T, PH, false>), grid,
                         dim3(kFB), 0, s, op.n_elems, op.n_nodes, xyz, op.conn, coef, op.mask, d);
    } else if (op.elem == Q1_HEX27) {
      const dim3 grid(unsigned((op.n_elems + QP<2>::E - 1) / QP<2>::E));
      hipLaunchKernelGGL((m ? k_qp_diag<T, PH, true, 2> : k_qp_diag<T, PH, false, 2>), grid,
                         dim3(kFB), 0, s, op.n_elems, op.n_nodes, xyz, op.conn, coef, op.mask, d);
    } else {
      const dim3 grid(unsigned((op.n_elems + QP<3>::E - 1) / QP<3>::E));
      hipLaunchKernelGGL((m ? k_qp_diag<T, PH, true, 3> : k_qp_diag<T, PH, false, 3>), grid,
                         dim3(kFB), 0, s, op.n_elems, op.n_nodes, xyz, op.conn, coef, op.mask, d);
    }
  }
  Q1_HIP(hipGetLastError());
  return Q1_OK;
}

}  // namespace

int launch_apply_family(Op &op, const void *x, void *y, hipStream_t s, const int *stop) {
  if (op.variant == Q1_V_BLOCK) return launch_apply_tile(op, x, y, s, stop);  // tetrahedra
  const bool f64 = op.dtype == Q1_F64;
  if (op.physics == Q1_LAPLACE)
    return f64 ? family_apply_t<double, 1>(op, x, y, s, stop)
               : family_apply_t<float, 1>(op, x, y, s, stop);
  if (op.physics == Q1_ELASTICITY)
    return f64 ? family_apply_t<double, 3>(op, x, y, s, stop)
               : family_apply_t<float, 3>(op, x, y, s, stop);
  return fail(Q1_EUNSUPPORTED, "element family %d: physics %d", op.elem, op.physics);
}

int launch_diag_family(Op &op, void *d, hipStream_t s) {
  const bool f64 = op.dtype == Q1_F64;
  if (op.physics == Q1_LAPLACE)
    return f64 ? family_diag_t<double, 1>(op, d, s) : family_diag_t<float, 1>(op, d, s);
  if (op.physics == Q1_ELASTICITY)
    return f64 ? family_diag_t<double, 3>(op, d, s) : family_diag_t<float, 3>(op, d, s);
  return fail(Q1_EUNSUPPORTED, "element family %d: physics %d", op.elem, op.physics);
}

}  // namespace q1
