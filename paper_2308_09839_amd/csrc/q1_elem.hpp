// Element-level arithmetic of the Q1 hexahedral operators (device code).
//
// Local node a = i + 2j + 4k sits at reference corner (2i-1, 2j-1, 2k-1).
// The Q1 space is spanned by the monomials psi_m = xi^mx eta^my zeta^mz,
// m = mx + 2my + 4mz.  Nodal values u_a and (unscaled) modal coefficients
// c_m = 8 * (coefficient of psi_m) are related by a 3-stage sum/difference
// butterfly (the tensor product of [[1,1],[-1,1]]), so the reference gradient
//   du/dxi = (c1 + c3 eta + c5 zeta + c7 eta zeta) / 8   (and cyclically)
// is read off the modes, and 2x2x2 Gauss points (+-1/sqrt(3)) are reached by
// 4-point evaluations.  This is the sum-factorised form of the per-quadrature
// -point work of Algorithm 1 (Jacobian, inverse and determinant, gradient of
// the input, flux, product with the test-function gradients).
//
// Scalings: with J' = 8J (columns from the coordinate modes), A' = adj(J'),
// det' = det J', the scalar-Laplace reference flux times 1/8 (which folds the
// inverse butterfly's factor) is  f = k / (512 det') A' A'^T g'  with g' the
// unscaled modal gradient; the elasticity flux is
// P = 1/(512 det') sigma'(H) A'^T with H = G' A' and
// sigma'(H) = lambda tr(H) I + mu (H + H^T).
#pragma once

#include <hip/hip_runtime.h>

namespace q1 {

template <typename T>
struct C {
  static constexpr T g = T(0.57735026918962576450914878050196);  // 1/sqrt(3)
  static constexpr T g2 = T(1.0) / T(3.0);
  static constexpr T third = T(1.0) / T(3.0);
  static constexpr T ninth = T(1.0) / T(9.0);
};

// Reciprocal: hardware estimate refined by Newton steps to full precision.
__device__ __forceinline__ double rcp(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-d, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float rcp(float d) {
  float r = __builtin_amdgcn_rcpf(d);
  float e = __builtin_fmaf(-d, r, 1.0f);
  return __builtin_fmaf(r, e, r);
}

// nodal -> unscaled modal (in place)
template <typename T>
__host__ __device__ __forceinline__ void butterfly_fwd(T v[8]) {
#pragma unroll
  for (int a = 0; a < 8; a += 2) {
    T s = v[a] + v[a + 1], d = v[a + 1] - v[a];
    v[a] = s; v[a + 1] = d;
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int a = (b & 1) | ((b & 2) << 1);  // 0,1,4,5
    T s = v[a] + v[a + 2], d = v[a + 2] - v[a];
    v[a] = s; v[a + 2] = d;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    T s = v[a] + v[a + 4], d = v[a + 4] - v[a];
    v[a] = s; v[a + 4] = d;
  }
}

// transpose of the inverse butterfly, unscaled: per dimension (w0, w1) -> (w0 - w1, w0 + w1)
template <typename T>
__device__ __forceinline__ void butterfly_bwd(T v[8]) {
#pragma unroll
  for (int a = 0; a < 8; a += 2) {
    T p = v[a], q = v[a + 1];
    v[a] = p - q; v[a + 1] = p + q;
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int a = (b & 1) | ((b & 2) << 1);
    T p = v[a], q = v[a + 2];
    v[a] = p - q; v[a + 2] = p + q;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    T p = v[a], q = v[a + 4];
    v[a] = p - q; v[a + 4] = p + q;
  }
}

// out[iA][iB] = p0 + sA g p1 + sB g p2 + sA sB g^2 p3 with s = 2i - 1
template <typename T>
__device__ __forceinline__ void eval4(T p0, T p1, T p2, T p3, T out[2][2]) {
  const T pp = p0 + C<T>::g2 * p3, pm = p0 - C<T>::g2 * p3;
  const T q1 = C<T>::g * (p1 + p2), q2 = C<T>::g * (p1 - p2);
  out[1][1] = pp + q1; out[0][0] = pp - q1;
  out[1][0] = pm + q2; out[0][1] = pm - q2;
}

// transpose of eval4: r0 = sum F, r1 = g sum sA F, r2 = g sum sB F, r3 = g^2 sum sA sB F
template <typename T>
__device__ __forceinline__ void eval4T(const T F[2][2], T &r0, T &r1, T &r2, T &r3) {
  const T spp = F[1][1] + F[0][0], smm = F[1][0] + F[0][1];
  const T d1 = F[1][1] - F[0][0], d2 = F[1][0] - F[0][1];
  r0 = spp + smm;
  r3 = C<T>::g2 * (spp - smm);
  r1 = C<T>::g * (d1 + d2);
  r2 = C<T>::g * (d1 - d2);
}

template <typename T>
__device__ __forceinline__ void cross(const T a[3], const T b[3], T c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
template <typename T>
__device__ __forceinline__ T dot3(const T a[3], const T b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Coordinates are affine images of the reference cube (a parallelepiped)
// exactly when the bilinear and trilinear coordinate modes vanish.
template <typename T>
__host__ __device__ __forceinline__ bool is_affine(const T X[3][8]) {
  bool z = true;
#pragma unroll
  for (int r = 0; r < 3; ++r)
    z = z && X[r][3] == T(0) && X[r][5] == T(0) && X[r][6] == T(0) && X[r][7] == T(0);
  return z;
}

// Geometry at one quadrature point from the modal coordinates:
// J' columns jx, jy, jz; adj rows a0 = jy x jz, a1 = jz x jx, a2 = jx x jy.
template <typename T>
struct QpGeom {
  T a0[3], a1[3], a2[3], det;
};

// ---------------------------------------------------------------------------
// Laplace on NC components sharing one coefficient: component c of the output
// is the scalar Laplace action on component c of the input (NC = 1 scalar
// Laplace, NC = 3 the vector Laplace, whose components do not couple).
// X [3][8] nodal coordinates (destroyed), u [NC][8] nodal input, k cell
// coefficient; v [NC][8] nodal output (v_e = A_e u_e).  The geometry is
// evaluated once for all components.
// ---------------------------------------------------------------------------
template <typename T, int NC>
__device__ __forceinline__ void laplace_element_n(T X[3][8], const T (*u_in)[8], T k,
                                                  T (*v)[8]) {
  T u[NC][8];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int a = 0; a < 8; ++a) u[c][a] = u_in[c][a];
    butterfly_fwd(u[c]);
  }
  butterfly_fwd(X[0]); butterfly_fwd(X[1]); butterfly_fwd(X[2]);
  T w[NC][8];
  if (is_affine(X)) {
    // constant Jacobian: exact modal integration of grad psi_m . D grad u
    const T C1[3] = {X[0][1], X[1][1], X[2][1]};
    const T C2[3] = {X[0][2], X[1][2], X[2][2]};
    const T C4[3] = {X[0][4], X[1][4], X[2][4]};
    T a0[3], a1[3], a2[3];
    cross(C2, C4, a0); cross(C4, C1, a1); cross(C1, C2, a2);
    const T det = dot3(C1, a0);
    const T s = k * rcp(T(64) * det);
    const T D00 = s * dot3(a0, a0), D01 = s * dot3(a0, a1), D02 = s * dot3(a0, a2);
    const T D11 = s * dot3(a1, a1), D12 = s * dot3(a1, a2), D22 = s * dot3(a2, a2);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const T *uc = u[c];
      T *wc = w[c];
      wc[0] = T(0);
      wc[1] = D00 * uc[1] + D01 * uc[2] + D02 * uc[4];
      wc[2] = D01 * uc[1] + D11 * uc[2] + D12 * uc[4];
      wc[4] = D02 * uc[1] + D12 * uc[2] + D22 * uc[4];
      wc[3] = C<T>::third * ((D00 + D11) * uc[3] + D02 * uc[6] + D12 * uc[5]);
      wc[5] = C<T>::third * ((D00 + D22) * uc[5] + D01 * uc[6] + D12 * uc[3]);
      wc[6] = C<T>::third * ((D11 + D22) * uc[6] + D01 * uc[5] + D02 * uc[3]);
      wc[7] = C<T>::ninth * (D00 + D11 + D22) * uc[7];
    }
  } else {
    T Jx[3][2][2], Jy[3][2][2], Jz[3][2][2];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      eval4(X[r][1], X[r][3], X[r][5], X[r][7], Jx[r]);  // [iy][iz]
      eval4(X[r][2], X[r][3], X[r][6], X[r][7], Jy[r]);  // [ix][iz]
      eval4(X[r][4], X[r][5], X[r][6], X[r][7], Jz[r]);  // [ix][iy]
    }
    T gx[NC][2][2], gy[NC][2][2], gz[NC][2][2];
    T Fx[NC][2][2], Fy[NC][2][2], Fz[NC][2][2];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      eval4(u[c][1], u[c][3], u[c][5], u[c][7], gx[c]);
      eval4(u[c][2], u[c][3], u[c][6], u[c][7], gy[c]);
      eval4(u[c][4], u[c][5], u[c][6], u[c][7], gz[c]);
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) Fx[c][p][q] = Fy[c][p][q] = Fz[c][p][q] = T(0);
    }
    const T ks = k * T(1.0 / 512.0);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int ix = q & 1, iy = (q >> 1) & 1, iz = (q >> 2) & 1;
      const T jx[3] = {Jx[0][iy][iz], Jx[1][iy][iz], Jx[2][iy][iz]};
      const T jy[3] = {Jy[0][ix][iz], Jy[1][ix][iz], Jy[2][ix][iz]};
      const T jz[3] = {Jz[0][ix][iy], Jz[1][ix][iy], Jz[2][ix][iy]};
      T a0[3], a1[3], a2[3];
      cross(jy, jz, a0); cross(jz, jx, a1); cross(jx, jy, a2);
      const T s = ks * rcp(dot3(jx, a0));
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const T g0 = gx[c][iy][iz], g1 = gy[c][ix][iz], g2 = gz[c][ix][iy];
        T t[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) t[d] = s * (g0 * a0[d] + g1 * a1[d] + g2 * a2[d]);
        Fx[c][iy][iz] += dot3(a0, t);
        Fy[c][ix][iz] += dot3(a1, t);
        Fz[c][ix][iy] += dot3(a2, t);
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      T *wc = w[c];
      T r0, r1, r2, r3;
      eval4T(Fx[c], r0, r1, r2, r3);
      wc[1] = r0; wc[3] = r1; wc[5] = r2; wc[7] = r3;
      eval4T(Fy[c], r0, r1, r2, r3);
      wc[2] = r0; wc[3] += r1; wc[6] = r2; wc[7] += r3;
      eval4T(Fz[c], r0, r1, r2, r3);
      wc[4] = r0; wc[5] += r1; wc[6] += r2; wc[7] += r3;
      wc[0] = T(0);
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    butterfly_bwd(w[c]);
#pragma unroll
    for (int a = 0; a < 8; ++a) v[c][a] = w[c][a];
  }
}

// Scalar Laplace: X [3][8] nodal coordinates (destroyed), u [8] nodal input,
// k cell coefficient; v [8] nodal output.
template <typename T>
__device__ __forceinline__ void laplace_element(T X[3][8], const T u_in[8], T k, T v[8]) {
  laplace_element_n<T, 1>(X, reinterpret_cast<const T(*)[8]>(u_in), k,
                          reinterpret_cast<T(*)[8]>(v));
}

// Laplace on NC components over an element already known to be a
// parallelepiped (the bilinear and trilinear coordinate modes vanish, checked
// once at set-up): the constant Jacobian comes from the three edges at corner
// 0, E_c = X_c - X_0 for c = 1, 2, 4 (J' = 4 E), so D = k / (16 det E) adj(E)
// adj(E)^T and the modal action is the closed form of the affine branch above.
// Reads corners 0, 1, 2, 4 of X only.
template <typename T, int NC>
__device__ __forceinline__ void laplace_element_parallelepiped_n(const T X[3][8],
                                                                 const T (*u_in)[8], T k,
                                                                 T (*v)[8]) {
  const T E1[3] = {X[0][1] - X[0][0], X[1][1] - X[1][0], X[2][1] - X[2][0]};
  const T E2[3] = {X[0][2] - X[0][0], X[1][2] - X[1][0], X[2][2] - X[2][0]};
  const T E4[3] = {X[0][4] - X[0][0], X[1][4] - X[1][0], X[2][4] - X[2][0]};
  T a0[3], a1[3], a2[3];
  cross(E2, E4, a0); cross(E4, E1, a1); cross(E1, E2, a2);
  const T s = k * rcp(T(16) * dot3(E1, a0));
  const T D00 = s * dot3(a0, a0), D01 = s * dot3(a0, a1), D02 = s * dot3(a0, a2);
  const T D11 = s * dot3(a1, a1), D12 = s * dot3(a1, a2), D22 = s * dot3(a2, a2);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    T u[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) u[a] = u_in[c][a];
    butterfly_fwd(u);
    T w[8];
    w[0] = T(0);
    w[1] = D00 * u[1] + D01 * u[2] + D02 * u[4];
    w[2] = D01 * u[1] + D11 * u[2] + D12 * u[4];
    w[4] = D02 * u[1] + D12 * u[2] + D22 * u[4];
    w[3] = C<T>::third * ((D00 + D11) * u[3] + D02 * u[6] + D12 * u[5]);
    w[5] = C<T>::third * ((D00 + D22) * u[5] + D01 * u[6] + D12 * u[3]);
    w[6] = C<T>::third * ((D11 + D22) * u[6] + D01 * u[5] + D02 * u[3]);
    w[7] = C<T>::ninth * (D00 + D11 + D22) * u[7];
    butterfly_bwd(w);
#pragma unroll
    for (int a = 0; a < 8; ++a) v[c][a] = w[a];
  }
}

template <typename T>
__device__ __forceinline__ void laplace_element_parallelepiped(const T X[3][8], const T u_in[8],
                                                               T k, T v[8]) {
  laplace_element_parallelepiped_n<T, 1>(X, reinterpret_cast<const T(*)[8]>(u_in), k,
                                         reinterpret_cast<T(*)[8]>(v));
}

// ---------------------------------------------------------------------------
// Isotropic elasticity: u [3][8] nodal displacement components (input),
// v [3][8] output, cell Lame constants lam, mu.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void elasticity_element(T X[3][8], const T u_in[3][8], T lam, T mu,
                                                   T v[3][8]) {
  T u[3][8];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int a = 0; a < 8; ++a) u[j][a] = u_in[j][a];
  butterfly_fwd(X[0]); butterfly_fwd(X[1]); butterfly_fwd(X[2]);
  butterfly_fwd(u[0]); butterfly_fwd(u[1]); butterfly_fwd(u[2]);
  const bool affine = is_affine(X);
  // gradient modes at the quadrature points: G[j][dir][iA][iB]
  T Gx[3][2][2], Gy[3][2][2], Gz[3][2][2];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    eval4(u[j][1], u[j][3], u[j][5], u[j][7], Gx[j]);
    eval4(u[j][2], u[j][3], u[j][6], u[j][7], Gy[j]);
    eval4(u[j][4], u[j][5], u[j][6], u[j][7], Gz[j]);
  }
  T Fx[3][2][2], Fy[3][2][2], Fz[3][2][2];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) Fx[j][p][q] = Fy[j][p][q] = Fz[j][p][q] = T(0);

  T Jx[3][2][2], Jy[3][2][2], Jz[3][2][2];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    eval4(X[r][1], X[r][3], X[r][5], X[r][7], Jx[r]);
    eval4(X[r][2], X[r][3], X[r][6], X[r][7], Jy[r]);
    eval4(X[r][4], X[r][5], X[r][6], X[r][7], Jz[r]);
  }
  // affine elements: one geometry for all points
  T ca0[3], ca1[3], ca2[3], cs = T(0);
  if (affine) {
    const T C1[3] = {X[0][1], X[1][1], X[2][1]};
    const T C2[3] = {X[0][2], X[1][2], X[2][2]};
    const T C4[3] = {X[0][4], X[1][4], X[2][4]};
    cross(C2, C4, ca0); cross(C4, C1, ca1); cross(C1, C2, ca2);
    cs = rcp(T(512) * dot3(C1, ca0));
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int ix = q & 1, iy = (q >> 1) & 1, iz = (q >> 2) & 1;
    T a0[3], a1[3], a2[3], s;
    if (affine) {
#pragma unroll
      for (int c = 0; c < 3; ++c) { a0[c] = ca0[c]; a1[c] = ca1[c]; a2[c] = ca2[c]; }
      s = cs;
    } else {
      const T jx[3] = {Jx[0][iy][iz], Jx[1][iy][iz], Jx[2][iy][iz]};
      const T jy[3] = {Jy[0][ix][iz], Jy[1][ix][iz], Jy[2][ix][iz]};
      const T jz[3] = {Jz[0][ix][iy], Jz[1][ix][iy], Jz[2][ix][iy]};
      cross(jy, jz, a0); cross(jz, jx, a1); cross(jx, jy, a2);
      s = rcp(T(512) * dot3(jx, a0));
    }
    // H = G' A'
    T H[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const T g0 = Gx[j][iy][iz], g1 = Gy[j][ix][iz], g2 = Gz[j][ix][iy];
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) H[j][kk] = g0 * a0[kk] + g1 * a1[kk] + g2 * a2[kk];
    }
    const T ls = lam * s, ms = mu * s;
    const T ltr = ls * (H[0][0] + H[1][1] + H[2][2]);
    T S[3][3];
    S[0][0] = ltr + T(2) * ms * H[0][0];
    S[1][1] = ltr + T(2) * ms * H[1][1];
    S[2][2] = ltr + T(2) * ms * H[2][2];
    S[0][1] = S[1][0] = ms * (H[0][1] + H[1][0]);
    S[0][2] = S[2][0] = ms * (H[0][2] + H[2][0]);
    S[1][2] = S[2][1] = ms * (H[1][2] + H[2][1]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Fx[i][iy][iz] += S[i][0] * a0[0] + S[i][1] * a0[1] + S[i][2] * a0[2];
      Fy[i][ix][iz] += S[i][0] * a1[0] + S[i][1] * a1[1] + S[i][2] * a1[2];
      Fz[i][ix][iy] += S[i][0] * a2[0] + S[i][1] * a2[1] + S[i][2] * a2[2];
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T w[8], r0, r1, r2, r3;
    eval4T(Fx[i], r0, r1, r2, r3);
    w[1] = r0; w[3] = r1; w[5] = r2; w[7] = r3;
    eval4T(Fy[i], r0, r1, r2, r3);
    w[2] = r0; w[3] += r1; w[6] = r2; w[7] += r3;
    eval4T(Fz[i], r0, r1, r2, r3);
    w[4] = r0; w[5] += r1; w[6] += r2; w[7] += r3;
    w[0] = T(0);
    butterfly_bwd(w);
#pragma unroll
    for (int a = 0; a < 8; ++a) v[i][a] = w[a];
  }
}

// ---------------------------------------------------------------------------
// Elasticity on an element known to be a parallelepiped.  With the constant
// Jacobian, the reference-gradient products of the modes integrate exactly to
// a block-sparse pattern: the linear modes (xi, eta, zeta) couple among
// themselves, the bilinear modes couple through the variable they share (xi*eta
// and xi*zeta through xi, ...), the trilinear mode only with itself.  For one
// such group with members (mode m, adjugate row a_m), H = sum_m u_m (x) a_m is
// the group's displacement gradient (up to scale), S = lambda tr(H) I +
// mu (H + H^T) its stress, and member m receives alpha S a_m, with alpha =
// 1/(16 det E), /3 for the bilinear groups and /9 for the trilinear one (the
// squared-variable integrals).  E_c = X_c - X_0 (c = 1, 2, 4) as in the Laplace
// parallelepiped path; reads corners 0, 1, 2, 4 of X only.
// ---------------------------------------------------------------------------
template <typename T, int NM>
__device__ __forceinline__ void elas_group(const T (&u)[3][8], T (&w)[3][8],
                                           const int (&mode)[NM], const T *const (&av)[NM],
                                           T lam, T mu, T alpha) {
  T H[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T h = T(0);
#pragma unroll
      for (int k = 0; k < NM; ++k) h += u[i][mode[k]] * av[k][j];
      H[i][j] = h;
    }
  const T lt = lam * (H[0][0] + H[1][1] + H[2][2]);
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    const T *a = av[k];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T si = lt * a[i];
#pragma unroll
      for (int j = 0; j < 3; ++j) si += mu * (H[i][j] + H[j][i]) * a[j];
      w[i][mode[k]] += alpha * si;
    }
  }
}

template <typename T>
__device__ __forceinline__ void elasticity_element_parallelepiped(const T X[3][8],
                                                                  const T (*u_in)[8], T lam,
                                                                  T mu, T (*v)[8]) {
  const T E1[3] = {X[0][1] - X[0][0], X[1][1] - X[1][0], X[2][1] - X[2][0]};
  const T E2[3] = {X[0][2] - X[0][0], X[1][2] - X[1][0], X[2][2] - X[2][0]};
  const T E4[3] = {X[0][4] - X[0][0], X[1][4] - X[1][0], X[2][4] - X[2][0]};
  T a0[3], a1[3], a2[3];
  cross(E2, E4, a0); cross(E4, E1, a1); cross(E1, E2, a2);
  const T r = rcp(T(16) * dot3(E1, a0));
  T u[3][8], w[3][8];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      u[c][a] = u_in[c][a];
      w[c][a] = T(0);
    }
    butterfly_fwd(u[c]);
  }
  const T r3 = r * C<T>::third, r9 = r * C<T>::ninth;
  {
    constexpr int m[3] = {1, 2, 4};
    const T *const a[3] = {a0, a1, a2};
    elas_group<T, 3>(u, w, m, a, lam, mu, r);
  }
  {
    constexpr int m[2] = {3, 6};  // through eta
    const T *const a[2] = {a0, a2};
    elas_group<T, 2>(u, w, m, a, lam, mu, r3);
  }
  {
    constexpr int m[2] = {3, 5};  // through xi
    const T *const a[2] = {a1, a2};
    elas_group<T, 2>(u, w, m, a, lam, mu, r3);
  }
  {
    constexpr int m[2] = {5, 6};  // through zeta
    const T *const a[2] = {a0, a1};
    elas_group<T, 2>(u, w, m, a, lam, mu, r3);
  }
  {
    constexpr int m[1] = {7};
    const T *const a_0[1] = {a0}, *const a_1[1] = {a1}, *const a_2[1] = {a2};
    elas_group<T, 1>(u, w, m, a_0, lam, mu, r9);
    elas_group<T, 1>(u, w, m, a_1, lam, mu, r9);
    elas_group<T, 1>(u, w, m, a_2, lam, mu, r9);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    butterfly_bwd(w[c]);
#pragma unroll
    for (int a = 0; a < 8; ++a) v[c][a] = w[c][a];
  }
}

// ---------------------------------------------------------------------------
// Partial assembly of the Laplace kinds: at each quadrature point q the
// symmetric factor D_q = k w det J J^-1 J^-T, in the units of the modal
// gradients above: D_q = (k/512) A A^T / det' with A the adjugate rows of the
// modal Jacobian J' (the quantity the general path forms on the fly).
// qd[q] = {D00, D01, D02, D11, D12, D22}.  X is destroyed.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void laplace_qdata(T X[3][8], T k, T qd[8][6]) {
  butterfly_fwd(X[0]); butterfly_fwd(X[1]); butterfly_fwd(X[2]);
  T Jx[3][2][2], Jy[3][2][2], Jz[3][2][2];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    eval4(X[r][1], X[r][3], X[r][5], X[r][7], Jx[r]);
    eval4(X[r][2], X[r][3], X[r][6], X[r][7], Jy[r]);
    eval4(X[r][4], X[r][5], X[r][6], X[r][7], Jz[r]);
  }
  const T ks = k * T(1.0 / 512.0);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int ix = q & 1, iy = (q >> 1) & 1, iz = (q >> 2) & 1;
    const T jx[3] = {Jx[0][iy][iz], Jx[1][iy][iz], Jx[2][iy][iz]};
    const T jy[3] = {Jy[0][ix][iz], Jy[1][ix][iz], Jy[2][ix][iz]};
    const T jz[3] = {Jz[0][ix][iy], Jz[1][ix][iy], Jz[2][ix][iy]};
    T a0[3], a1[3], a2[3];
    cross(jy, jz, a0); cross(jz, jx, a1); cross(jx, jy, a2);
    const T s = ks * rcp(dot3(jx, a0));
    qd[q][0] = s * dot3(a0, a0); qd[q][1] = s * dot3(a0, a1); qd[q][2] = s * dot3(a0, a2);
    qd[q][3] = s * dot3(a1, a1); qd[q][4] = s * dot3(a1, a2); qd[q][5] = s * dot3(a2, a2);
  }
}

// Laplace on NC components from stored quadrature data (no geometry).
template <typename T, int NC>
__device__ __forceinline__ void laplace_element_pa_n(const T (*qd)[6], const T (*u_in)[8],
                                                     T (*v)[8]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    T u[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) u[a] = u_in[c][a];
    butterfly_fwd(u);
    T gx[2][2], gy[2][2], gz[2][2];
    eval4(u[1], u[3], u[5], u[7], gx);
    eval4(u[2], u[3], u[6], u[7], gy);
    eval4(u[4], u[5], u[6], u[7], gz);
    T Fx[2][2], Fy[2][2], Fz[2][2];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int ix = q & 1, iy = (q >> 1) & 1, iz = (q >> 2) & 1;
      const T g0 = gx[iy][iz], g1 = gy[ix][iz], g2 = gz[ix][iy];
      const T *D = qd[q];
      const T f0 = D[0] * g0 + D[1] * g1 + D[2] * g2;
      const T f1 = D[1] * g0 + D[3] * g1 + D[4] * g2;
      const T f2 = D[2] * g0 + D[4] * g1 + D[5] * g2;
      // each (iy, iz) cell of Fx is reached by q with ix = 0 first, likewise below
      Fx[iy][iz] = ix == 0 ? f0 : Fx[iy][iz] + f0;
      Fy[ix][iz] = iy == 0 ? f1 : Fy[ix][iz] + f1;
      Fz[ix][iy] = iz == 0 ? f2 : Fz[ix][iy] + f2;
    }
    T w[8], r0, r1, r2, r3;
    eval4T(Fx, r0, r1, r2, r3);
    w[1] = r0; w[3] = r1; w[5] = r2; w[7] = r3;
    eval4T(Fy, r0, r1, r2, r3);
    w[2] = r0; w[3] += r1; w[6] = r2; w[7] += r3;
    eval4T(Fz, r0, r1, r2, r3);
    w[4] = r0; w[5] += r1; w[6] += r2; w[7] += r3;
    w[0] = T(0);
    butterfly_bwd(w);
#pragma unroll
    for (int a = 0; a < 8; ++a) v[c][a] = w[a];
  }
}

// ---------------------------------------------------------------------------
// Partial assembly of isotropic elasticity: at each quadrature point q the
// nine entries of B_q = sqrt(s) A' (A' the adjugate rows of the modal Jacobian
// J', s = 1/(512 det')), row-major.  With the cell's lambda, mu these give the
// flux exactly: H~ = G' B = sqrt(s) G' A', S~ = lambda tr(H~) I + mu (H~ + H~^T)
// = sqrt(s) sigma'(G' A'), and S~ B^T = s sigma'(G' A') A'^T, the flux of the
// general path.  X is destroyed.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void elasticity_qdata(T X[3][8], T qd[8][9]) {
  butterfly_fwd(X[0]); butterfly_fwd(X[1]); butterfly_fwd(X[2]);
  T Jx[3][2][2], Jy[3][2][2], Jz[3][2][2];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    eval4(X[r][1], X[r][3], X[r][5], X[r][7], Jx[r]);
    eval4(X[r][2], X[r][3], X[r][6], X[r][7], Jy[r]);
    eval4(X[r][4], X[r][5], X[r][6], X[r][7], Jz[r]);
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int ix = q & 1, iy = (q >> 1) & 1, iz = (q >> 2) & 1;
    const T jx[3] = {Jx[0][iy][iz], Jx[1][iy][iz], Jx[2][iy][iz]};
    const T jy[3] = {Jy[0][ix][iz], Jy[1][ix][iz], Jy[2][ix][iz]};
    const T jz[3] = {Jz[0][ix][iy], Jz[1][ix][iy], Jz[2][ix][iy]};
    T a0[3], a1[3], a2[3];
    cross(jy, jz, a0); cross(jz, jx, a1); cross(jx, jy, a2);
    const T r = sqrt(rcp(T(512) * dot3(jx, a0)));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      qd[q][c] = r * a0[c];
      qd[q][3 + c] = r * a1[c];
      qd[q][6 + c] = r * a2[c];
    }
  }
}

// Elasticity from stored quadrature data: qd(q, m) returns entry m of B_q
// (loaded where the point is reached).  The reference gradients are evaluated
// from the modes at each point and the point's flux is added straight into the
// output modes (the transposed evaluation), so only the input and output modes
// stay live across points.
template <typename T, typename QD>
__device__ __forceinline__ void elasticity_element_pa(QD qd, const T (*u_in)[8], T lam, T mu,
                                                      T (*v)[8]) {
  T u[3][8], w[3][8];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      u[j][a] = u_in[j][a];
      w[j][a] = T(0);
    }
    butterfly_fwd(u[j]);
  }
  const T g = C<T>::g, g2 = C<T>::g2;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const T sx = (q & 1) ? g : -g, sy = (q & 2) ? g : -g, sz = (q & 4) ? g : -g;
    const T sxy = (((q & 1) != 0) == ((q & 2) != 0)) ? g2 : -g2;
    const T sxz = (((q & 1) != 0) == ((q & 4) != 0)) ? g2 : -g2;
    const T syz = (((q & 2) != 0) == ((q & 4) != 0)) ? g2 : -g2;
    T B[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) B[m] = qd(q, m);
    T H[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const T g0 = u[j][1] + sy * u[j][3] + sz * u[j][5] + syz * u[j][7];
      const T g1 = u[j][2] + sx * u[j][3] + sz * u[j][6] + sxz * u[j][7];
      const T g4 = u[j][4] + sx * u[j][5] + sy * u[j][6] + sxy * u[j][7];
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) H[j][kk] = g0 * B[kk] + g1 * B[3 + kk] + g4 * B[6 + kk];
    }
    const T ltr = lam * (H[0][0] + H[1][1] + H[2][2]);
    T S[3][3];
    S[0][0] = ltr + T(2) * mu * H[0][0];
    S[1][1] = ltr + T(2) * mu * H[1][1];
    S[2][2] = ltr + T(2) * mu * H[2][2];
    S[0][1] = S[1][0] = mu * (H[0][1] + H[1][0]);
    S[0][2] = S[2][0] = mu * (H[0][2] + H[2][0]);
    S[1][2] = S[2][1] = mu * (H[1][2] + H[2][1]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T f0 = S[i][0] * B[0] + S[i][1] * B[1] + S[i][2] * B[2];
      const T f1 = S[i][0] * B[3] + S[i][1] * B[4] + S[i][2] * B[5];
      const T f2 = S[i][0] * B[6] + S[i][1] * B[7] + S[i][2] * B[8];
      w[i][1] += f0;
      w[i][2] += f1;
      w[i][4] += f2;
      w[i][3] += sy * f0 + sx * f1;
      w[i][5] += sz * f0 + sx * f2;
      w[i][6] += sz * f1 + sy * f2;
      w[i][7] += syz * f0 + sxz * f1 + sxy * f2;
    }
    // keep the next points' data loads below this point: hoisted together, the 72
    // loads alone would hold 144 registers
    if (q & 1) __asm__ volatile("" ::: "memory");
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    butterfly_bwd(w[i]);
#pragma unroll
    for (int a = 0; a < 8; ++a) v[i][a] = w[i][a];
  }
}

// ---------------------------------------------------------------------------
// Physics kinds (the values of the public enum): 1 scalar Laplace, 2 vector
// Laplace, 3 isotropic elasticity.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int phys_dpn(int ph) { return ph == 1 ? 1 : 3; }
__host__ __device__ constexpr int phys_ncoef(int ph) { return ph == 3 ? 2 : 1; }

// v_e = A_e u_e for kind PH: u, v [dpn][8]; c0 = k (Laplace kinds) or lambda,
// c1 = mu (elasticity).  X is destroyed.
template <typename T, int PH>
__device__ __forceinline__ void element_apply(T X[3][8], const T (*u)[8], T c0, T c1,
                                              T (*v)[8]) {
  if constexpr (PH == 1)
    laplace_element_n<T, 1>(X, u, c0, v);
  else if constexpr (PH == 2)
    laplace_element_n<T, 3>(X, u, c0, v);
  else
    elasticity_element<T>(X, u, c0, c1, v);
}

// Diagonal entries of the element matrix of kind PH, acc[i][a] for DOF i of
// node a: sum over the 8 Gauss points of, with t = A'^T g'_a (A' the adjugate
// of the scaled Jacobian, g'_a = 8 times the reference gradient of phi_a) and
// det' its determinant, Laplace kinds k |t|^2 / (512 det') (every component),
// elasticity ((lambda + mu) t_i^2 + mu |t|^2) / (512 det').  X is destroyed.
template <typename T, int PH>
__device__ __forceinline__ void element_diag(T X[3][8], T c0, T c1, T (*acc)[8]) {
  constexpr int DPN = phys_dpn(PH);
  butterfly_fwd(X[0]); butterfly_fwd(X[1]); butterfly_fwd(X[2]);
  T Jx[3][2][2], Jy[3][2][2], Jz[3][2][2];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    eval4(X[r][1], X[r][3], X[r][5], X[r][7], Jx[r]);
    eval4(X[r][2], X[r][3], X[r][6], X[r][7], Jy[r]);
    eval4(X[r][4], X[r][5], X[r][6], X[r][7], Jz[r]);
  }
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int i = 0; i < DPN; ++i) acc[i][a] = T(0);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int ix = q & 1, iy = (q >> 1) & 1, iz = (q >> 2) & 1;
    const T jx[3] = {Jx[0][iy][iz], Jx[1][iy][iz], Jx[2][iy][iz]};
    const T jy[3] = {Jy[0][ix][iz], Jy[1][ix][iz], Jy[2][ix][iz]};
    const T jz[3] = {Jz[0][ix][iy], Jz[1][ix][iy], Jz[2][ix][iy]};
    T a0[3], a1[3], a2[3];
    cross(jy, jz, a0); cross(jz, jx, a1); cross(jx, jy, a2);
    const T s = rcp(T(512) * dot3(jx, a0));
    const T xi = (2 * ix - 1) * C<T>::g, eta = (2 * iy - 1) * C<T>::g,
            zeta = (2 * iz - 1) * C<T>::g;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const T si = T(2 * (a & 1) - 1), sj = T(2 * ((a >> 1) & 1) - 1),
              sk = T(2 * ((a >> 2) & 1) - 1);
      const T g0 = si * (T(1) + sj * eta) * (T(1) + sk * zeta);
      const T g1 = sj * (T(1) + si * xi) * (T(1) + sk * zeta);
      const T g2 = sk * (T(1) + si * xi) * (T(1) + sj * eta);
      T t[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) t[c] = g0 * a0[c] + g1 * a1[c] + g2 * a2[c];
      const T tt = dot3(t, t);
      if constexpr (PH != 3) {
#pragma unroll
        for (int i = 0; i < DPN; ++i) acc[i][a] += c0 * s * tt;
      } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) acc[i][a] += s * ((c0 + c1) * t[i] * t[i] + c1 * tt);
      }
    }
  }
}

// Linear tetrahedron of kind PH (scalar Laplace or elasticity): X[3][4] the
// vertex coordinates, u[DPN][4] the input, v[DPN][4] the output.  With
// E_c = X_c - X_0 the cross products c_1 = E_2 x E_3, c_2 = E_3 x E_1,
// c_3 = E_1 x E_2, c_0 = -(c_1 + c_2 + c_3) are det J times the constant
// physical gradients, det J = E_1 . c_1, the volume det J / 6:
//   Laplace      v_a = k (c_a . g) / (6 det J),  g = sum_b c_b u_b,
//   elasticity   v_a = S c_a / (6 det J),  S = lambda tr(H) I + mu (H + H^T),
//                H = sum_b u_b (x) c_b.
template <typename T, int PH>
__device__ __forceinline__ void tet_element(const T X[3][4], const T (*u)[4], T c0, T c1,
                                            T (*v)[4]) {
  const T E1[3] = {X[0][1] - X[0][0], X[1][1] - X[1][0], X[2][1] - X[2][0]};
  const T E2[3] = {X[0][2] - X[0][0], X[1][2] - X[1][0], X[2][2] - X[2][0]};
  const T E3[3] = {X[0][3] - X[0][0], X[1][3] - X[1][0], X[2][3] - X[2][0]};
  T c[4][3];
  cross(E2, E3, c[1]);
  cross(E3, E1, c[2]);
  cross(E1, E2, c[3]);
#pragma unroll
  for (int r = 0; r < 3; ++r) c[0][r] = -(c[1][r] + c[2][r] + c[3][r]);
  const T s = rcp(T(6) * dot3(E1, c[1]));
  if constexpr (PH == 1) {
    T g[3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
      g[r] = c[0][r] * u[0][0] + c[1][r] * u[0][1] + c[2][r] * u[0][2] + c[3][r] * u[0][3];
    const T ks = c0 * s;
#pragma unroll
    for (int a = 0; a < 4; ++a) v[0][a] = ks * dot3(c[a], g);
  } else {
    T H[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        H[i][j] = u[i][0] * c[0][j] + u[i][1] * c[1][j] + u[i][2] * c[2][j] + u[i][3] * c[3][j];
    const T ltr = c0 * (H[0][0] + H[1][1] + H[2][2]);
    T S[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) S[i][j] = s * (c1 * (H[i][j] + H[j][i]) + (i == j ? ltr : T(0)));
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i) v[i][a] = dot3(S[i], c[a]);
  }
}

}  // namespace q1
