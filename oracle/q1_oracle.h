/*
 * q1_oracle.h -- plain FP64 CPU oracle for the trilinear (Q1) hexahedral
 * scalar-Laplace and isotropic-elasticity operators.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may call it.  It shares no code with the GPU
 * library: it assembles element matrices by quadrature, sums them into a CSR
 * matrix and multiplies, which is the plain definition of the operator
 * (paper Section 2, the element matrices; Section 3, the remark on matrix
 * assembly by column search and addition).  It never performs a matrix-free
 * apply.
 *
 * Conventions (the paper leaves them open; the readings are listed with the
 * design notes of the repository):
 *   reference cube [-1,1]^3, local node a = i + 2j + 4k sits at
 *   (2i-1, 2j-1, 2k-1); 2x2x2 Gauss-Legendre quadrature, points +-1/sqrt(3),
 *   weights 1; J_rc = dx_r/dxi_c; DOF numbering node*dpn + component.
 *   Coordinates are [3][n_nodes] (structure of arrays), connectivity is
 *   [8][n_elems], cell coefficients are [ncoef][n_elems]: k for Laplace,
 *   (lambda, mu) for elasticity.  Dirichlet: a constrained DOF c gets row and
 *   column zeroed and A_cc = 1 (symmetric elimination).
 */
#ifndef Q1_ORACLE_H
#define Q1_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 2x2x2 Gauss-Legendre rule, q = qx + 2 qy + 4 qz. */
void orc_quadrature(double pts[8][3], double w[8]);
/* Reference gradients of the 8 trilinear basis functions at xi. */
void orc_ref_grad(const double xi[3], double dphi[8][3]);

/* Element matrices.  X is [8][3] (node-major).  Return 0, or -1 when
 * det J <= 0 at some quadrature point. */
int orc_ke_laplace(const double X[24], double k, double Ke[64]);
int orc_ke_elasticity(const double X[24], double lam, double mu, double Ke[576]);
int orc_ke_vlaplace(const double X[24], double k, double Ke[576]);

/* Linear tetrahedra: X is [4][3]; reference vertices (0,0,0), (1,0,0),
 * (0,1,0), (0,0,1).  Triquadratic hexahedra: X is [27][3], local node
 * a = i + 3j + 9k at (t_i, t_j, t_k), t = (-1, 0, 1); 3x3x3 Gauss rule.
 * Return 0, or -1 when det J <= 0 (at some quadrature point). */
int orc_ke_tet_laplace(const double X[12], double k, double Ke[16]);
int orc_ke_tet_elasticity(const double X[12], double lam, double mu, double Ke[144]);
void orc_q2_quadrature(double pts[27][3], double w[27]);
void orc_q2_ref_grad(const double xi[3], double dphi[27][3]);
int orc_ke_q2_laplace(const double X[81], double k, double Ke[729]);
int orc_ke_q2_elasticity(const double X[81], double lam, double mu, double Ke[6561]);
/* Tricubic hexahedra: X is [64][3], local node a = i + 4j + 16k at
 * (t_i, t_j, t_k), t_m = -1 + 2m/3; 4x4x4 Gauss rule. */
void orc_q3_quadrature(double pts[64][3], double w[64]);
void orc_q3_ref_grad(const double xi[3], double dphi[64][3]);
int orc_ke_q3_laplace(const double X[192], double k, double Ke[4096]);
int orc_ke_q3_elasticity(const double X[192], double lam, double mu, double Ke[36864]);

/* CSR pattern of the assembled operator, columns sorted.  rowptr has
 * n_nodes*dpn + 1 entries.  With col == NULL only rowptr is filled.
 * Returns nnz, or -1 on allocation failure. */
int64_t orc_csr_pattern(int dpn, int64_t n_nodes, int64_t n_elems, const int32_t *conn,
                        int64_t *rowptr, int32_t *col);
/* The same for elements of nloc nodes (connectivity [nloc][n_elems]).  Every
 * row holds its diagonal entry. */
int64_t orc_csr_pattern_n(int dpn, int nloc, int64_t n_nodes, int64_t n_elems,
                          const int32_t *conn, int64_t *rowptr, int32_t *col);

/* Fill values: element loop in element order, column found by binary search,
 * then Dirichlet elimination.  physics = 1 (Laplace) or 3 (elasticity).
 * Returns 0, -1 (bad element) or -2 (missing column). */
int orc_csr_assemble(int physics, int64_t n_nodes, int64_t n_elems, const double *xyz,
                     const int32_t *conn, const double *coef, const uint8_t *mask_nodes,
                     const int64_t *rowptr, const int32_t *col, double *val);
/* nloc = 8 (trilinear hexahedra), 4 (linear tetrahedra) or 27 (triquadratic
 * hexahedra; physics 1 or 3 for the last two).  -3 for other kinds. */
int orc_csr_assemble_n(int nloc, int physics, int64_t n_nodes, int64_t n_elems,
                       const double *xyz, const int32_t *conn, const double *coef,
                       const uint8_t *mask_nodes, const int64_t *rowptr, const int32_t *col,
                       double *val);

/* Selected rows of y = A x computed from element matrices without forming A:
 * for each element touching a selected node, its element matrix is computed
 * and the selected rows' products are added (element order), then the
 * Dirichlet elimination is applied.  rows are DOF indices (node*dpn + comp).
 * Returns 0, or -1 (bad element) / -2 (allocation). */
int orc_apply_rows(int physics, int64_t n_nodes, int64_t n_elems, const double *xyz,
                   const int32_t *conn, const double *coef, const uint8_t *mask_nodes,
                   const double *x, int64_t n_rows, const int64_t *rows, double *y_rows);
int orc_apply_rows_n(int nloc, int physics, int64_t n_nodes, int64_t n_elems,
                     const double *xyz, const int32_t *conn, const double *coef,
                     const uint8_t *mask_nodes, const double *x, int64_t n_rows,
                     const int64_t *rows, double *y_rows);

/* y = A x, rows in parallel (OpenMP), each row summed in column order. */
void orc_spmv(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
              const double *x, double *y);
void orc_diag(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
              double *d);
/* Number of threads the OpenMP regions use, and a way to set it. */
int orc_num_threads(void);
void orc_set_num_threads(int n);

/* Preconditioned CG (Hestenes-Stiefel), x0 = 0, stop when ||r||_2 <= rtol ||b||_2
 * on the recurrence residual.  jacobi != 0 uses z = D^{-1} r.  res_hist, if
 * not NULL, receives ||r_k||_2 for k = 0..iters.  Returns 0 (converged),
 * -4 (maxit reached, x holds the last iterate) or -5 (breakdown). */
int orc_pcg(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
            const double *b, double *x, double rtol, int maxit, int jacobi,
            int *iters, double *rel_res, double *res_hist);

/* Flexible PCG with a variable preconditioner z = M(r):
 * beta = z_{k+1}^T (r_{k+1} - r_k) / (r_k^T z_k) (Golub and Ye's inexact
 * PCG).  Same stopping rule and return codes as orc_pcg.  x_hist, if not
 * NULL, receives the iterates x_0 .. x_iters ([iters+1][n], maxit+1 rows
 * must fit). */
typedef int (*orc_precond_fn)(void *ctx, int64_t n, const double *r, double *z);
int orc_fpcg(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
             const double *b, double *x, double rtol, int maxit, orc_precond_fn M, void *ctx,
             int *iters, double *rel_res, double *res_hist, double *x_hist);

/* Flexible CG with truncated orthogonalisation FCG(m) (Notay 2000): the new
 * direction is z = M(r) made A-orthogonal to the previous min(k, m)
 * directions, alpha = p^T r / p^T A p.  m >= 1; with m >= maxit every
 * direction is A-orthogonalised against all earlier ones.  Same outputs and
 * return codes as orc_fpcg (-1 for m < 1). */
int orc_fcg(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
            const double *b, double *x, double rtol, int maxit, int m, orc_precond_fn M,
            void *ctx, int *iters, double *rel_res, double *res_hist, double *x_hist);

#ifdef __cplusplus
}
#endif
#endif
