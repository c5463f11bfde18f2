/*
 * q1_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see
 * q1_oracle.h).  Every routine is the textbook definition written out with
 * plain loops: element matrices by quadrature (paper Section 2, element
 * matrix equations for scalar Laplace and linear elasticity), global assembly
 * by column search and addition (Section 3), CSR products and
 * Hestenes-Stiefel PCG (the CG operations of Table 4).
 */
#include "q1_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- reference element (Section 2: isoparametric map, Gaussian quadrature) */

void orc_quadrature(double pts[8][3], double w[8]) {
  const double g = 1.0 / sqrt(3.0);
  for (int q = 0; q < 8; ++q) {
    pts[q][0] = (q & 1) ? g : -g;
    pts[q][1] = (q & 2) ? g : -g;
    pts[q][2] = (q & 4) ? g : -g;
    w[q] = 1.0;
  }
}

/* phi_a(xi) = N_i(xi0) N_j(xi1) N_k(xi2), a = i + 2j + 4k,
 * N_0(t) = (1 - t)/2, N_1(t) = (1 + t)/2. */
static double n1d(int s, double t) { return s ? 0.5 * (1.0 + t) : 0.5 * (1.0 - t); }
static double dn1d(int s) { return s ? 0.5 : -0.5; }

void orc_ref_grad(const double xi[3], double dphi[8][3]) {
  for (int a = 0; a < 8; ++a) {
    int i = a & 1, j = (a >> 1) & 1, k = (a >> 2) & 1;
    dphi[a][0] = dn1d(i) * n1d(j, xi[1]) * n1d(k, xi[2]);
    dphi[a][1] = n1d(i, xi[0]) * dn1d(j) * n1d(k, xi[2]);
    dphi[a][2] = n1d(i, xi[0]) * n1d(j, xi[1]) * dn1d(k);
  }
}

/* J_rc = sum_a X[a][r] dphi[a][c]; inverse by cofactors; G[a][r] = sum_c
 * dphi[a][c] Jinv[c][r] is the physical gradient J^{-T} grad_hat phi_a.
 * Returns det J. */
static double physical_gradients(const double X[24], const double dphi[8][3],
                                 double G[8][3]) {
  double J[3][3] = {{0}};
  for (int a = 0; a < 8; ++a)
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) J[r][c] += X[3 * a + r] * dphi[a][c];
  double C[3][3]; /* cofactor matrix */
  C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  C[0][1] = -(J[1][0] * J[2][2] - J[1][2] * J[2][0]);
  C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  C[1][0] = -(J[0][1] * J[2][2] - J[0][2] * J[2][1]);
  C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  C[1][2] = -(J[0][0] * J[2][1] - J[0][1] * J[2][0]);
  C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  C[2][1] = -(J[0][0] * J[1][2] - J[0][2] * J[1][0]);
  C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
  double Jinv[3][3]; /* Jinv = adj(J)/det, adj = C^T */
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Jinv[r][c] = C[c][r] / det;
  for (int a = 0; a < 8; ++a)
    for (int r = 0; r < 3; ++r) {
      double s = 0.0;
      for (int c = 0; c < 3; ++c) s += dphi[a][c] * Jinv[c][r];
      G[a][r] = s;
    }
  return det;
}

/* [A^e]_ab = sum_q k w_q detJ (J^{-T} grad_hat phi_a) . (J^{-T} grad_hat phi_b)
 * (scalar Laplace element matrix, with the cell coefficient k). */
int orc_ke_laplace(const double X[24], double k, double Ke[64]) {
  double pts[8][3], w[8];
  orc_quadrature(pts, w);
  memset(Ke, 0, 64 * sizeof(double));
  for (int q = 0; q < 8; ++q) {
    double dphi[8][3], G[8][3];
    orc_ref_grad(pts[q], dphi);
    double det = physical_gradients(X, dphi, G);
    if (!(det > 0.0)) return -1;
    double s = k * w[q] * det;
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b)
        Ke[8 * a + b] += s * (G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2]);
  }
  return 0;
}

/* Vector Laplace (Section 2, the vector Laplace element matrix, with the cell
 * coefficient k): [A^e]_{3a+i,3b+j} = sum_q k w_q detJ (e_i (x) grad phi_a) :
 * (e_j (x) grad phi_b), the double contraction written out entry by entry. */
int orc_ke_vlaplace(const double X[24], double k, double Ke[576]) {
  double pts[8][3], w[8];
  orc_quadrature(pts, w);
  memset(Ke, 0, 576 * sizeof(double));
  for (int q = 0; q < 8; ++q) {
    double dphi[8][3], G[8][3];
    orc_ref_grad(pts[q], dphi);
    double det = physical_gradients(X, dphi, G);
    if (!(det > 0.0)) return -1;
    double s = k * w[q] * det;
    for (int a = 0; a < 8; ++a)
      for (int i = 0; i < 3; ++i)
        for (int b = 0; b < 8; ++b)
          for (int j = 0; j < 3; ++j) {
            double c = 0.0; /* sum_rs (e_i (x) G_a)_rs (e_j (x) G_b)_rs */
            for (int r = 0; r < 3; ++r)
              for (int t = 0; t < 3; ++t)
                c += (r == i ? G[a][t] : 0.0) * (r == j ? G[b][t] : 0.0);
            Ke[24 * (3 * a + i) + 3 * b + j] += s * c;
          }
  }
  return 0;
}

/* physics 1 scalar Laplace (1 DOF per node), 2 vector Laplace, 3 elasticity */
static int dpn_of(int physics) { return physics == 1 ? 1 : 3; }

static int element_matrix(int physics, const double X[24], const double *coef, int64_t ne,
                          int64_t e, double *Ke) {
  if (physics == 1) return orc_ke_laplace(X, coef[e], Ke);
  if (physics == 2) return orc_ke_vlaplace(X, coef[e], Ke);
  return orc_ke_elasticity(X, coef[e], coef[ne + e], Ke);
}

/* [A^e]_{3a+i,3b+j} = sum_q w_q detJ (e_i (x) grad phi_a) : sigma(e_j (x) grad phi_b)
 * with sigma(eps) = lambda tr(eps) I + 2 mu eps, which expands to
 * lambda G_ai G_bj + mu (delta_ij G_a.G_b + G_aj G_bi). */
int orc_ke_elasticity(const double X[24], double lam, double mu, double Ke[576]) {
  double pts[8][3], w[8];
  orc_quadrature(pts, w);
  memset(Ke, 0, 576 * sizeof(double));
  for (int q = 0; q < 8; ++q) {
    double dphi[8][3], G[8][3];
    orc_ref_grad(pts[q], dphi);
    double det = physical_gradients(X, dphi, G);
    if (!(det > 0.0)) return -1;
    double s = w[q] * det;
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b) {
        double gg = G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2];
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) {
            double v = lam * G[a][i] * G[b][j] + mu * ((i == j ? gg : 0.0) + G[a][j] * G[b][i]);
            Ke[24 * (3 * a + i) + 3 * b + j] += s * v;
          }
      }
  }
  return 0;
}

/* ---- linear tetrahedra (the paper's conclusions, Section 7: simplicial
 * elements) ------------------------------------------------------------- */

/* Reference tetrahedron with vertices (0,0,0), (1,0,0), (0,1,0), (0,0,1);
 * phi_0 = 1 - xi - eta - zeta, phi_a = xi_a (a = 1, 2, 3).  The gradients are
 * constant, so the stiffness integrand is constant and the one-point rule at
 * the centroid (weight 1/6, the reference volume) is exact.  Returns det J. */
static double tet_gradients(const double X[12], double G[4][3]) {
  static const double dphi[4][3] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  double J[3][3] = {{0}};
  for (int a = 0; a < 4; ++a)
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) J[r][c] += X[3 * a + r] * dphi[a][c];
  double C[3][3];
  C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  C[0][1] = -(J[1][0] * J[2][2] - J[1][2] * J[2][0]);
  C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  C[1][0] = -(J[0][1] * J[2][2] - J[0][2] * J[2][1]);
  C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  C[1][2] = -(J[0][0] * J[2][1] - J[0][1] * J[2][0]);
  C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  C[2][1] = -(J[0][0] * J[1][2] - J[0][2] * J[1][0]);
  C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
  for (int a = 0; a < 4; ++a)
    for (int r = 0; r < 3; ++r) {
      double v = 0.0; /* (J^{-T} grad_hat phi_a)_r = sum_c dphi[a][c] Jinv[c][r] */
      for (int c = 0; c < 3; ++c) v += dphi[a][c] * C[r][c] / det;
      G[a][r] = v;
    }
  return det;
}

/* [A^e]_ab = k |T| grad phi_a . grad phi_b with |T| = det J / 6. */
int orc_ke_tet_laplace(const double X[12], double k, double Ke[16]) {
  double G[4][3];
  const double det = tet_gradients(X, G);
  if (!(det > 0.0)) return -1;
  const double s = k * det / 6.0;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      Ke[4 * a + b] = s * (G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2]);
  return 0;
}

/* [A^e]_{3a+i,3b+j} = |T| (lambda G_ai G_bj + mu (delta_ij G_a.G_b + G_aj G_bi)). */
int orc_ke_tet_elasticity(const double X[12], double lam, double mu, double Ke[144]) {
  double G[4][3];
  const double det = tet_gradients(X, G);
  if (!(det > 0.0)) return -1;
  const double s = det / 6.0;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      const double gg = G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          Ke[12 * (3 * a + i) + 3 * b + j] =
              s * (lam * G[a][i] * G[b][j] + mu * ((i == j ? gg : 0.0) + G[a][j] * G[b][i]));
    }
  return 0;
}

/* ---- triquadratic (Q2) hexahedra (Section 7: quadratic elements) ------- */

/* Reference cube [-1,1]^3 with the 27 nodes at (t_i, t_j, t_k), t = (-1, 0, 1),
 * local node a = i + 3j + 9k; phi_a = L_i(xi) L_j(eta) L_k(zeta) with the 1-D
 * quadratic Lagrange basis L_0 = t(t-1)/2, L_1 = 1 - t^2, L_2 = t(t+1)/2.
 * Quadrature: 3x3x3 Gauss-Legendre, points 0, +-sqrt(3/5), weights 8/9, 5/9
 * (exact for the stiffness of elements with a trilinear geometry). */
static double lq(int i, double t) {
  return i == 0 ? 0.5 * t * (t - 1.0) : i == 1 ? 1.0 - t * t : 0.5 * t * (t + 1.0);
}
static double dlq(int i, double t) { return i == 0 ? t - 0.5 : i == 1 ? -2.0 * t : t + 0.5; }

void orc_q2_quadrature(double pts[27][3], double w[27]) {
  const double g = sqrt(0.6), gp[3] = {-g, 0.0, g}, gw[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
  for (int q = 0; q < 27; ++q) {
    const int i = q % 3, j = (q / 3) % 3, k = q / 9;
    pts[q][0] = gp[i]; pts[q][1] = gp[j]; pts[q][2] = gp[k];
    w[q] = gw[i] * gw[j] * gw[k];
  }
}

void orc_q2_ref_grad(const double xi[3], double dphi[27][3]) {
  for (int a = 0; a < 27; ++a) {
    const int i = a % 3, j = (a / 3) % 3, k = a / 9;
    dphi[a][0] = dlq(i, xi[0]) * lq(j, xi[1]) * lq(k, xi[2]);
    dphi[a][1] = lq(i, xi[0]) * dlq(j, xi[1]) * lq(k, xi[2]);
    dphi[a][2] = lq(i, xi[0]) * lq(j, xi[1]) * dlq(k, xi[2]);
  }
}

/* J, its cofactor inverse and the physical gradients of the 27 functions */
static double q2_gradients(const double X[81], const double dphi[27][3], double G[27][3]) {
  double J[3][3] = {{0}};
  for (int a = 0; a < 27; ++a)
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) J[r][c] += X[3 * a + r] * dphi[a][c];
  double C[3][3];
  C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  C[0][1] = -(J[1][0] * J[2][2] - J[1][2] * J[2][0]);
  C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  C[1][0] = -(J[0][1] * J[2][2] - J[0][2] * J[2][1]);
  C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  C[1][2] = -(J[0][0] * J[2][1] - J[0][1] * J[2][0]);
  C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  C[2][1] = -(J[0][0] * J[1][2] - J[0][2] * J[1][0]);
  C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
  for (int a = 0; a < 27; ++a)
    for (int r = 0; r < 3; ++r) {
      double v = 0.0;
      for (int c = 0; c < 3; ++c) v += dphi[a][c] * C[r][c] / det;
      G[a][r] = v;
    }
  return det;
}

int orc_ke_q2_laplace(const double X[81], double k, double Ke[729]) {
  double pts[27][3], w[27];
  orc_q2_quadrature(pts, w);
  memset(Ke, 0, 729 * sizeof(double));
  for (int q = 0; q < 27; ++q) {
    double dphi[27][3], G[27][3];
    orc_q2_ref_grad(pts[q], dphi);
    const double det = q2_gradients(X, dphi, G);
    if (!(det > 0.0)) return -1;
    const double s = k * w[q] * det;
    for (int a = 0; a < 27; ++a)
      for (int b = 0; b < 27; ++b)
        Ke[27 * a + b] += s * (G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2]);
  }
  return 0;
}

int orc_ke_q2_elasticity(const double X[81], double lam, double mu, double Ke[6561]) {
  double pts[27][3], w[27];
  orc_q2_quadrature(pts, w);
  memset(Ke, 0, 6561 * sizeof(double));
  for (int q = 0; q < 27; ++q) {
    double dphi[27][3], G[27][3];
    orc_q2_ref_grad(pts[q], dphi);
    const double det = q2_gradients(X, dphi, G);
    if (!(det > 0.0)) return -1;
    const double s = w[q] * det;
    for (int a = 0; a < 27; ++a)
      for (int b = 0; b < 27; ++b) {
        const double gg = G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2];
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            Ke[81 * (3 * a + i) + 3 * b + j] +=
                s * (lam * G[a][i] * G[b][j] + mu * ((i == j ? gg : 0.0) + G[a][j] * G[b][i]));
      }
  }
  return 0;
}

/* ---- tricubic (Q3) hexahedra (Section 7: higher-order elements) -------- */

/* Reference cube [-1,1]^3 with the 64 nodes at (t_i, t_j, t_k), t_m = -1 +
 * 2m/3, local node a = i + 4j + 16k; phi_a = L_i(xi) L_j(eta) L_k(zeta) with
 * the 1-D cubic Lagrange polynomials of those nodes, written as products.
 * Quadrature: 4x4x4 Gauss-Legendre, points +-sqrt(3/7 -+ (2/7) sqrt(6/5)),
 * weights (18 +- sqrt(30)) / 36 (exact for the stiffness of elements with a
 * trilinear geometry and for the polynomial degree of an affine element). */
static double lc_node(int m) { return -1.0 + 2.0 * m / 3.0; }
static double lc(int i, double t) {
  double v = 1.0;
  for (int m = 0; m < 4; ++m)
    if (m != i) v *= (t - lc_node(m)) / (lc_node(i) - lc_node(m));
  return v;
}
static double dlc(int i, double t) {
  double d = 0.0;
  for (int l = 0; l < 4; ++l) {
    if (l == i) continue;
    double v = 1.0 / (lc_node(i) - lc_node(l));
    for (int m = 0; m < 4; ++m)
      if (m != i && m != l) v *= (t - lc_node(m)) / (lc_node(i) - lc_node(m));
    d += v;
  }
  return d;
}

void orc_q3_quadrature(double pts[64][3], double w[64]) {
  const double a = sqrt(3.0 / 7.0 - 2.0 / 7.0 * sqrt(6.0 / 5.0));
  const double b = sqrt(3.0 / 7.0 + 2.0 / 7.0 * sqrt(6.0 / 5.0));
  const double wa = (18.0 + sqrt(30.0)) / 36.0, wb = (18.0 - sqrt(30.0)) / 36.0;
  const double gp[4] = {-b, -a, a, b}, gw[4] = {wb, wa, wa, wb};
  for (int q = 0; q < 64; ++q) {
    const int i = q % 4, j = (q / 4) % 4, k = q / 16;
    pts[q][0] = gp[i]; pts[q][1] = gp[j]; pts[q][2] = gp[k];
    w[q] = gw[i] * gw[j] * gw[k];
  }
}

void orc_q3_ref_grad(const double xi[3], double dphi[64][3]) {
  for (int a = 0; a < 64; ++a) {
    const int i = a % 4, j = (a / 4) % 4, k = a / 16;
    dphi[a][0] = dlc(i, xi[0]) * lc(j, xi[1]) * lc(k, xi[2]);
    dphi[a][1] = lc(i, xi[0]) * dlc(j, xi[1]) * lc(k, xi[2]);
    dphi[a][2] = lc(i, xi[0]) * lc(j, xi[1]) * dlc(k, xi[2]);
  }
}

/* J, its cofactor inverse and the physical gradients of the 64 functions */
static double q3_gradients(const double X[192], const double dphi[64][3], double G[64][3]) {
  double J[3][3] = {{0}};
  for (int a = 0; a < 64; ++a)
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) J[r][c] += X[3 * a + r] * dphi[a][c];
  double C[3][3];
  C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  C[0][1] = -(J[1][0] * J[2][2] - J[1][2] * J[2][0]);
  C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  C[1][0] = -(J[0][1] * J[2][2] - J[0][2] * J[2][1]);
  C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  C[1][2] = -(J[0][0] * J[2][1] - J[0][1] * J[2][0]);
  C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  C[2][1] = -(J[0][0] * J[1][2] - J[0][2] * J[1][0]);
  C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
  for (int a = 0; a < 64; ++a)
    for (int r = 0; r < 3; ++r) {
      double v = 0.0;
      for (int c = 0; c < 3; ++c) v += dphi[a][c] * C[r][c] / det;
      G[a][r] = v;
    }
  return det;
}

int orc_ke_q3_laplace(const double X[192], double k, double Ke[4096]) {
  double pts[64][3], w[64];
  orc_q3_quadrature(pts, w);
  memset(Ke, 0, 4096 * sizeof(double));
  for (int q = 0; q < 64; ++q) {
    double dphi[64][3], G[64][3];
    orc_q3_ref_grad(pts[q], dphi);
    const double det = q3_gradients(X, dphi, G);
    if (!(det > 0.0)) return -1;
    const double s = k * w[q] * det;
    for (int a = 0; a < 64; ++a)
      for (int b = 0; b < 64; ++b)
        Ke[64 * a + b] += s * (G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2]);
  }
  return 0;
}

int orc_ke_q3_elasticity(const double X[192], double lam, double mu, double Ke[36864]) {
  double pts[64][3], w[64];
  orc_q3_quadrature(pts, w);
  memset(Ke, 0, 36864 * sizeof(double));
  for (int q = 0; q < 64; ++q) {
    double dphi[64][3], G[64][3];
    orc_q3_ref_grad(pts[q], dphi);
    const double det = q3_gradients(X, dphi, G);
    if (!(det > 0.0)) return -1;
    const double s = w[q] * det;
    for (int a = 0; a < 64; ++a)
      for (int b = 0; b < 64; ++b) {
        const double gg = G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2];
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            Ke[192 * (3 * a + i) + 3 * b + j] +=
                s * (lam * G[a][i] * G[b][j] + mu * ((i == j ? gg : 0.0) + G[a][j] * G[b][i]));
      }
  }
  return 0;
}

static int element_matrix_n(int nloc, int physics, const double *X, const double *coef,
                            int64_t ne, int64_t e, double *Ke) {
  if (nloc == 8) return element_matrix(physics, X, coef, ne, e, Ke);
  const double c1 = physics == 3 ? coef[ne + e] : 0.0;
  if (nloc == 4)
    return physics == 1 ? orc_ke_tet_laplace(X, coef[e], Ke)
                        : orc_ke_tet_elasticity(X, coef[e], c1, Ke);
  if (nloc == 27)
    return physics == 1 ? orc_ke_q2_laplace(X, coef[e], Ke)
                        : orc_ke_q2_elasticity(X, coef[e], c1, Ke);
  return physics == 1 ? orc_ke_q3_laplace(X, coef[e], Ke)
                      : orc_ke_q3_elasticity(X, coef[e], c1, Ke);
}

/* ---- CSR pattern ------------------------------------------------------- */

static int cmp_i32(const void *p, const void *q) {
  int32_t a = *(const int32_t *)p, b = *(const int32_t *)q;
  return (a > b) - (a < b);
}

/* node -> element incidence lists */
static int node_elems(int nloc, int64_t nn, int64_t ne, const int32_t *conn, int64_t **ptr_out,
                      int64_t **lst_out) {
  int64_t *ptr = (int64_t *)calloc((size_t)nn + 1, sizeof(int64_t));
  int64_t *lst = (int64_t *)malloc((size_t)(nloc * ne + 1) * sizeof(int64_t));
  if (!ptr || !lst) { free(ptr); free(lst); return -1; }
  for (int a = 0; a < nloc; ++a)
    for (int64_t e = 0; e < ne; ++e) ptr[conn[a * ne + e] + 1]++;
  for (int64_t n = 0; n < nn; ++n) ptr[n + 1] += ptr[n];
  int64_t *fill = (int64_t *)malloc((size_t)nn * sizeof(int64_t));
  if (!fill) { free(ptr); free(lst); return -1; }
  memcpy(fill, ptr, (size_t)nn * sizeof(int64_t));
  for (int64_t e = 0; e < ne; ++e)
    for (int a = 0; a < nloc; ++a) {
      int32_t n = conn[a * ne + e];
      /* an element lists a node once even if (degenerately) repeated */
      int dup = 0;
      for (int b = 0; b < a; ++b) dup |= (conn[b * ne + e] == n);
      if (!dup) lst[fill[n]++] = e;
    }
  /* recompute ptr with the de-duplicated counts */
  int64_t *ptr2 = (int64_t *)calloc((size_t)nn + 1, sizeof(int64_t));
  if (!ptr2) { free(ptr); free(lst); free(fill); return -1; }
  int64_t w = 0;
  for (int64_t n = 0; n < nn; ++n) {
    ptr2[n] = w;
    for (int64_t t = ptr[n]; t < fill[n]; ++t) lst[w++] = lst[t];
  }
  ptr2[nn] = w;
  free(ptr); free(fill);
  *ptr_out = ptr2; *lst_out = lst;
  return 0;
}

int64_t orc_csr_pattern(int dpn, int64_t nn, int64_t ne, const int32_t *conn,
                        int64_t *rowptr, int32_t *col) {
  return orc_csr_pattern_n(dpn, 8, nn, ne, conn, rowptr, col);
}

int64_t orc_csr_pattern_n(int dpn, int nloc, int64_t nn, int64_t ne, const int32_t *conn,
                          int64_t *rowptr, int32_t *col) {
  int64_t *nptr, *nlst;
  if (node_elems(nloc, nn, ne, conn, &nptr, &nlst)) return -1;
  int64_t cap = 64;
  int32_t *buf = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
  if (!buf) { free(nptr); free(nlst); return -1; }
  int64_t nnz = 0;
  rowptr[0] = 0;
  for (int64_t n = 0; n < nn; ++n) {
    int64_t m = 0, need = nloc * (nptr[n + 1] - nptr[n]) + 1;
    if (need > cap) {
      cap = need;
      int32_t *nb = (int32_t *)realloc(buf, (size_t)cap * sizeof(int32_t));
      if (!nb) { free(buf); free(nptr); free(nlst); return -1; }
      buf = nb;
    }
    buf[m++] = (int32_t)n; /* the diagonal, also for a node no element references */
    for (int64_t t = nptr[n]; t < nptr[n + 1]; ++t)
      for (int a = 0; a < nloc; ++a) buf[m++] = conn[a * ne + nlst[t]];
    qsort(buf, (size_t)m, sizeof(int32_t), cmp_i32);
    int64_t u = 0;
    for (int64_t t = 0; t < m; ++t)
      if (t == 0 || buf[t] != buf[t - 1]) buf[u++] = buf[t];
    for (int c = 0; c < dpn; ++c) {
      int64_t row = n * dpn + c;
      if (col)
        for (int64_t t = 0; t < u; ++t)
          for (int d = 0; d < dpn; ++d) col[nnz + t * dpn + d] = buf[t] * dpn + d;
      nnz += u * dpn;
      rowptr[row + 1] = nnz;
    }
  }
  free(buf); free(nptr); free(nlst);
  return nnz;
}

static int64_t find_col(const int64_t *rowptr, const int32_t *col, int64_t row, int32_t c) {
  int64_t lo = rowptr[row], hi = rowptr[row + 1] - 1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (col[mid] == c) return mid;
    if (col[mid] < c) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

int orc_csr_assemble(int physics, int64_t nn, int64_t ne, const double *xyz,
                     const int32_t *conn, const double *coef, const uint8_t *mask,
                     const int64_t *rowptr, const int32_t *col, double *val) {
  return orc_csr_assemble_n(8, physics, nn, ne, xyz, conn, coef, mask, rowptr, col, val);
}

int orc_csr_assemble_n(int nloc, int physics, int64_t nn, int64_t ne, const double *xyz,
                       const int32_t *conn, const double *coef, const uint8_t *mask,
                       const int64_t *rowptr, const int32_t *col, double *val) {
  if (nloc != 8 && nloc != 4 && nloc != 27 && nloc != 64) return -3;
  if (nloc != 8 && physics == 2) return -3;
  const int dpn = dpn_of(physics);
  const int nd = nloc * dpn;
  const int64_t nrows = nn * dpn;
  memset(val, 0, (size_t)rowptr[nrows] * sizeof(double));
  double X[192];
  double *Ke = (double *)malloc((size_t)nd * nd * sizeof(double));
  if (!Ke) return -2;
  for (int64_t e = 0; e < ne; ++e) {
    for (int a = 0; a < nloc; ++a) {
      int32_t n = conn[a * ne + e];
      X[3 * a + 0] = xyz[0 * nn + n];
      X[3 * a + 1] = xyz[1 * nn + n];
      X[3 * a + 2] = xyz[2 * nn + n];
    }
    int rc = element_matrix_n(nloc, physics, X, coef, ne, e, Ke);
    if (rc) { free(Ke); return -1; }
    for (int p = 0; p < nd; ++p) {
      int64_t row = (int64_t)conn[(p / dpn) * ne + e] * dpn + p % dpn;
      for (int s = 0; s < nd; ++s) {
        int32_t c = conn[(s / dpn) * ne + e] * dpn + s % dpn;
        int64_t t = find_col(rowptr, col, row, c);
        if (t < 0) { free(Ke); return -2; }
        val[t] += Ke[nd * p + s];
      }
    }
  }
  free(Ke);
  if (mask) {
    for (int64_t row = 0; row < nrows; ++row) {
      int rfix = mask[row / dpn] != 0;
      for (int64_t t = rowptr[row]; t < rowptr[row + 1]; ++t) {
        int cfix = mask[col[t] / dpn] != 0;
        if (rfix || cfix) val[t] = (col[t] == row) ? 1.0 : 0.0;
      }
    }
  }
  return 0;
}

int orc_apply_rows(int physics, int64_t nn, int64_t ne, const double *xyz,
                   const int32_t *conn, const double *coef, const uint8_t *mask,
                   const double *x, int64_t n_rows, const int64_t *rows, double *y) {
  return orc_apply_rows_n(8, physics, nn, ne, xyz, conn, coef, mask, x, n_rows, rows, y);
}

int orc_apply_rows_n(int nloc, int physics, int64_t nn, int64_t ne, const double *xyz,
                     const int32_t *conn, const double *coef, const uint8_t *mask,
                     const double *x, int64_t n_rows, const int64_t *rows, double *y) {
  if (nloc != 8 && nloc != 4 && nloc != 27 && nloc != 64) return -3;
  if (nloc != 8 && physics == 2) return -3;
  const int dpn = dpn_of(physics), nd = nloc * dpn;
  /* slot[node] = 1 if any DOF of the node is selected */
  uint8_t *sel = (uint8_t *)calloc((size_t)nn, 1);
  int64_t *pos = (int64_t *)malloc((size_t)(nn * dpn) * sizeof(int64_t));
  if (!sel || !pos) { free(sel); free(pos); return -2; }
  for (int64_t i = 0; i < nn * dpn; ++i) pos[i] = -1;
  for (int64_t r = 0; r < n_rows; ++r) {
    sel[rows[r] / dpn] = 1;
    pos[rows[r]] = r;
    y[r] = 0.0;
  }
  double X[192];
  double *Ke = (double *)malloc((size_t)nd * nd * sizeof(double));
  if (!Ke) { free(sel); free(pos); return -2; }
  for (int64_t e = 0; e < ne; ++e) {
    int touch = 0;
    for (int a = 0; a < nloc; ++a) touch |= sel[conn[a * ne + e]];
    if (!touch) continue;
    for (int a = 0; a < nloc; ++a) {
      int32_t n = conn[a * ne + e];
      for (int c = 0; c < 3; ++c) X[3 * a + c] = xyz[c * nn + n];
    }
    int rc = element_matrix_n(nloc, physics, X, coef, ne, e, Ke);
    if (rc) { free(sel); free(pos); free(Ke); return -1; }
    for (int p = 0; p < nd; ++p) {
      int64_t row = (int64_t)conn[(p / dpn) * ne + e] * dpn + p % dpn;
      if (pos[row] < 0) continue;
      double s = 0.0;
      for (int q = 0; q < nd; ++q) {
        int32_t cn = conn[(q / dpn) * ne + e];
        if (mask && mask[cn]) continue; /* eliminated column */
        s += Ke[nd * p + q] * x[(int64_t)cn * dpn + q % dpn];
      }
      y[pos[row]] += s;
    }
  }
  if (mask)
    for (int64_t r = 0; r < n_rows; ++r)
      if (mask[rows[r] / dpn]) y[r] = x[rows[r]];
  free(sel); free(pos); free(Ke);
  return 0;
}

/* ---- products -------------------------------------------------------- */

void orc_spmv(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
              const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t t = rowptr[i]; t < rowptr[i + 1]; ++t) s += val[t] * x[col[t]];
    y[i] = s;
  }
}

void orc_diag(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
              double *d) {
  for (int64_t i = 0; i < n; ++i) {
    d[i] = 0.0;
    for (int64_t t = rowptr[i]; t < rowptr[i + 1]; ++t)
      if (col[t] == i) d[i] = val[t];
  }
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

static double dot(int64_t n, const double *a, const double *b) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* ---- Krylov solvers (CG operations of Table 4) ------------------------- */

int orc_pcg(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
            const double *b, double *x, double rtol, int maxit, int jacobi,
            int *iters, double *rel_res, double *res_hist) {
  double *r = (double *)malloc((size_t)n * sizeof(double));
  double *z = (double *)malloc((size_t)n * sizeof(double));
  double *p = (double *)malloc((size_t)n * sizeof(double));
  double *q = (double *)malloc((size_t)n * sizeof(double));
  double *d = (double *)malloc((size_t)n * sizeof(double));
  if (!r || !z || !p || !q || !d) { free(r); free(z); free(p); free(q); free(d); return -2; }
  orc_diag(n, rowptr, col, val, d);
  for (int64_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; }
  const double bnorm = sqrt(dot(n, b, b));
  int status = -4, k = 0;
  double rnorm = bnorm;
  if (res_hist) res_hist[0] = rnorm;
  if (bnorm == 0.0) { status = 0; goto done; }
  for (int64_t i = 0; i < n; ++i) z[i] = jacobi ? r[i] / d[i] : r[i];
  double rho = dot(n, r, z);
  memcpy(p, z, (size_t)n * sizeof(double));
  for (k = 0; k < maxit;) {
    orc_spmv(n, rowptr, col, val, p, q);
    double pq = dot(n, p, q);
    if (!(pq > 0.0) || !isfinite(pq)) { status = -5; break; }
    double alpha = rho / pq;
    for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
    ++k;
    rnorm = sqrt(dot(n, r, r));
    if (res_hist) res_hist[k] = rnorm;
    if (rnorm <= rtol * bnorm) { status = 0; break; }
    for (int64_t i = 0; i < n; ++i) z[i] = jacobi ? r[i] / d[i] : r[i];
    double rho_new = dot(n, r, z);
    double beta = rho_new / rho;
    for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    rho = rho_new;
  }
done:
  if (iters) *iters = k;
  if (rel_res) *rel_res = bnorm > 0.0 ? rnorm / bnorm : 0.0;
  free(r); free(z); free(p); free(q); free(d);
  return status;
}

int orc_fpcg(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
             const double *b, double *x, double rtol, int maxit, orc_precond_fn M, void *ctx,
             int *iters, double *rel_res, double *res_hist, double *x_hist) {
  double *r = (double *)malloc((size_t)n * sizeof(double));
  double *rold = (double *)malloc((size_t)n * sizeof(double));
  double *z = (double *)malloc((size_t)n * sizeof(double));
  double *p = (double *)malloc((size_t)n * sizeof(double));
  double *q = (double *)malloc((size_t)n * sizeof(double));
  if (!r || !rold || !z || !p || !q) {
    free(r); free(rold); free(z); free(p); free(q); return -2;
  }
  for (int64_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; }
  if (x_hist) memcpy(x_hist, x, (size_t)n * sizeof(double));
  const double bnorm = sqrt(dot(n, b, b));
  int status = -4, k = 0;
  double rnorm = bnorm;
  if (res_hist) res_hist[0] = rnorm;
  if (bnorm == 0.0) { status = 0; goto done; }
  if (M(ctx, n, r, z)) { status = -5; goto done; }
  double rho = dot(n, r, z);
  memcpy(p, z, (size_t)n * sizeof(double));
  for (k = 0; k < maxit;) {
    orc_spmv(n, rowptr, col, val, p, q);
    double pq = dot(n, p, q);
    if (!(pq > 0.0) || !isfinite(pq)) { status = -5; break; }
    double alpha = rho / pq;
    memcpy(rold, r, (size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
    ++k;
    rnorm = sqrt(dot(n, r, r));
    if (res_hist) res_hist[k] = rnorm;
    if (x_hist) memcpy(x_hist + (size_t)k * (size_t)n, x, (size_t)n * sizeof(double));
    if (rnorm <= rtol * bnorm) { status = 0; break; }
    if (M(ctx, n, r, z)) { status = -5; break; }
    double num = 0.0;
    for (int64_t i = 0; i < n; ++i) num += z[i] * (r[i] - rold[i]);
    double beta = num / rho;
    rho = dot(n, r, z);
    for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
done:
  if (iters) *iters = k;
  if (rel_res) *rel_res = bnorm > 0.0 ? rnorm / bnorm : 0.0;
  free(r); free(rold); free(z); free(p); free(q);
  return status;
}

/* Flexible CG with truncated orthogonalisation, FCG(m) (Notay, SIAM J. Sci.
 * Comput. 22, 2000).  Iteration k: z_k = M(r_k); the direction p_k is z_k
 * minus its A-projections on the previous min(k, m) directions,
 *   p_k = z_k - sum_j (z_k^T A p_j / p_j^T A p_j) p_j,
 * then alpha_k = p_k^T r_k / p_k^T A p_k, x += alpha_k p_k,
 * r -= alpha_k A p_k.  The directions p_j and their products A p_j are
 * kept, so no extra apply is needed. */
int orc_fcg(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
            const double *b, double *x, double rtol, int maxit, int m, orc_precond_fn M,
            void *ctx, int *iters, double *rel_res, double *res_hist, double *x_hist) {
  if (m < 1) return -1;
  double *r = (double *)malloc((size_t)n * sizeof(double));
  double *z = (double *)malloc((size_t)n * sizeof(double));
  double *P = (double *)malloc((size_t)m * (size_t)n * sizeof(double));
  double *Q = (double *)malloc((size_t)m * (size_t)n * sizeof(double));
  double *pAp = (double *)malloc((size_t)m * sizeof(double));
  double *c = (double *)malloc((size_t)m * sizeof(double));
  if (!r || !z || !P || !Q || !pAp || !c) {
    free(r); free(z); free(P); free(Q); free(pAp); free(c); return -2;
  }
  for (int64_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; }
  if (x_hist) memcpy(x_hist, x, (size_t)n * sizeof(double));
  const double bnorm = sqrt(dot(n, b, b));
  int status = -4, k = 0;
  double rnorm = bnorm;
  if (res_hist) res_hist[0] = rnorm;
  if (bnorm == 0.0) { status = 0; goto done; }
  for (k = 0; k < maxit;) {
    if (M(ctx, n, r, z)) { status = -5; break; }
    /* slot of direction j is j mod m; the window holds directions
     * k - nwin .. k - 1 */
    const int nwin = k < m ? k : m;
    for (int t = 0; t < nwin; ++t) {
      const int j = k - nwin + t;
      const double *qj = Q + (size_t)(j % m) * (size_t)n;
      c[t] = dot(n, z, qj) / pAp[j % m];
    }
    double *pk = P + (size_t)(k % m) * (size_t)n;
    double *qk = Q + (size_t)(k % m) * (size_t)n;
    for (int64_t i = 0; i < n; ++i) {
      double v = z[i];
      for (int t = 0; t < nwin; ++t) v -= c[t] * P[(size_t)((k - nwin + t) % m) * (size_t)n + i];
      pk[i] = v;
    }
    orc_spmv(n, rowptr, col, val, pk, qk);
    const double pq = dot(n, pk, qk);
    if (!(pq > 0.0) || !isfinite(pq)) { status = -5; break; }
    pAp[k % m] = pq;
    const double alpha = dot(n, pk, r) / pq;
    for (int64_t i = 0; i < n; ++i) { x[i] += alpha * pk[i]; r[i] -= alpha * qk[i]; }
    ++k;
    rnorm = sqrt(dot(n, r, r));
    if (res_hist) res_hist[k] = rnorm;
    if (x_hist) memcpy(x_hist + (size_t)k * (size_t)n, x, (size_t)n * sizeof(double));
    if (rnorm <= rtol * bnorm) { status = 0; break; }
  }
done:
  if (iters) *iters = k;
  if (rel_res) *rel_res = bnorm > 0.0 ? rnorm / bnorm : 0.0;
  free(r); free(z); free(P); free(Q); free(pAp); free(c);
  return status;
}
