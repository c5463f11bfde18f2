/*
 * q1mf.h -- C ABI of libq1mf, matrix-free trilinear (Q1) hexahedral finite
 * element operators for gfx950 (MI355X).
 *
 * The library applies y = A x without forming A for the scalar Laplace and
 * the isotropic linear-elasticity operators with cell-wise coefficients
 * (paper Section 2: element matrices of the scalar Laplace and elasticity
 * problems under the isoparametric map and Gaussian quadrature; Section 3:
 * the three-step gather / local product / scatter-add apply and Algorithm 1).
 *
 * Conventions shared by every entry point
 *   - Status: every function returns Q1_OK (0) or a negative Q1_E* code; the
 *     text of the last error of the calling thread is q1_last_error().
 *   - Pointers named *_d are DEVICE pointers owned by the caller (for example
 *     torch tensors' data_ptr()).  The library never frees or reallocates
 *     them.  Host pointers are named without the suffix.
 *   - stream is a hipStream_t (NULL = the null stream).  Device calls are
 *     asynchronous on that stream unless stated otherwise.
 *   - Reals are double for Q1_F64 operators and float for Q1_F32 operators:
 *     coordinates, coefficients and vectors all use the operator's dtype.
 *   - Indices are int32 (n_nodes < 2^31); counts are int64.
 *   - Mesh layout: coordinates structure-of-arrays [3][n_nodes]; connectivity
 *     [8][n_elems] with local node a = i + 2j + 4k at reference corner
 *     (2i-1, 2j-1, 2k-1) of [-1,1]^3; DOF numbering node*dpn + component
 *     (dpn = 1 scalar Laplace, 3 vector Laplace and elasticity); coefficients
 *     [ncoef][n_elems]: k for the Laplace kinds, (lambda, mu) for elasticity.
 *   - Quadrature: 2x2x2 Gauss-Legendre (points +-1/sqrt(3), weights 1).
 *   - Dirichlet mask (uint8 per node, or NULL for none): every DOF of a masked
 *     node is eliminated symmetrically, (A x)_c = x_c, and masked DOFs are
 *     left out of the gather and the scatter of all other rows.
 */
#ifndef Q1MF_H
#define Q1MF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status ------------------------------------------------------------ */
#define Q1_OK 0
#define Q1_EINVAL (-1)       /* bad size, NULL pointer, enum or alignment */
#define Q1_ENOMEM (-2)       /* device or host allocation failed */
#define Q1_EHIP (-3)         /* HIP runtime error; text in q1_last_error() */
#define Q1_ENOCONV (-4)      /* iteration limit reached; x holds the last iterate */
#define Q1_EBREAKDOWN (-5)   /* p^T A p <= 0, non-finite scalar, bad element */
#define Q1_EUNSUPPORTED (-6) /* valid request that the library does not support */

/* Text of the last error raised on the calling thread ("" if none). */
const char *q1_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int q1_version(void);

/* ---- host generators of the synthetic workloads --------------------------
 * Counter-based SplitMix64 (Steele, Lea & Flood 2014):
 *   draw(seed, stream, i) = splitmix64((seed ^ stream*0x9E3779B97F4A7C15) + i),
 *   U(0,1) = (draw >> 11) * 2^-53, N(0,1) = Box-Muller on U(2i), U(2i+1):
 *   sqrt(-2 log(1 - u1)) cos(2 pi u2).
 * All outputs are host arrays the caller allocates. */

/* Node and element counts of an nx*ny*nz box of hexahedra. */
int q1_box_sizes(int nx, int ny, int nz, int64_t *n_nodes, int64_t *n_elems);
/* Box mesh of spacing h: node id = i + (nx+1)(j + (ny+1)k), element
 * e = ex + nx(ey + ny ez).  Interior nodes move by U(-jitter_frac h,
 * jitter_frac h) per coordinate (stream 0, counter 3 id + c); surface nodes
 * stay on the box.  xyz [3][n_nodes], conn [8][n_elems]. */
int q1_box_mesh(int nx, int ny, int nz, double h, double jitter_frac, uint64_t seed,
                double *xyz, int32_t *conn);
/* mask[n] = 1 for nodes on one face (0:x=0 1:x=max 2:y=0 3:y=max 4:z=0 5:z=max). */
int q1_face_mask(int nx, int ny, int nz, int face, uint8_t *mask);
/* out[i] = exp(mu + sigma N_i) from the given stream. */
int q1_field_lognormal(int64_t n, double mu, double sigma, uint64_t seed, uint64_t stream,
                       double *out);
/* k_e = exp(s_layer N_1(ez / layer_cells)) * exp(s_cell N_2(e)) (streams 1 and 2). */
int q1_field_layered(int nx, int ny, int nz, int layer_cells, double s_layer, double s_cell,
                     uint64_t seed, double *k);
/* E = exp(N_1(ln 10, 1)), nu = 0.15 + 0.2 U_2 per cell. */
int q1_field_elastic(int64_t n, uint64_t seed, double *E, double *nu);
/* lambda = E nu / ((1+nu)(1-2nu)), mu = E / (2(1+nu)). */
int q1_lame_from_E_nu(int64_t n, const double *E, const double *nu, double *lam, double *mu);
/* out[i] = lo + (hi - lo) U_i from the given stream. */
int q1_vec_uniform(int64_t n, uint64_t seed, uint64_t stream, double lo, double hi,
                   double *out);

/* ---- operators ---------------------------------------------------------- */
typedef struct q1_op q1_op;

/* Physics kinds.  Q1_LAPLACE: scalar Laplace, 1 DOF per node, coefficient k.
 * Q1_VLAPLACE: vector Laplace (Section 2, the vector Laplace element matrix
 * with the cell coefficient k): 3 DOF per node, each component an independent
 * scalar Laplace; coefficient k.  Q1_ELASTICITY: isotropic elasticity, 3 DOF
 * per node, coefficients lambda and mu. */
enum { Q1_LAPLACE = 1, Q1_VLAPLACE = 2, Q1_ELASTICITY = 3 };
enum { Q1_F64 = 0, Q1_F32 = 1 };
/* Scatter strategies of the apply (Section 3, third step):
 *   ATOMIC   one thread per element, global atomic adds (the paper's
 *            one-thread-per-element strategy, Section 6);
 *   COLOR    one thread per element, elements split at set-up into colour
 *            classes that share no node (greedy first-fit; 8 classes on a
 *            lexicographic lattice); one launch per class with plain
 *            read-add-write scatter, no atomics; connectivity and
 *            coefficients are copied in class order (set-up synchronises);
 *            Q1_EUNSUPPORTED if more than 64 classes would be needed;
 *   LDS_TILE element tiles, one wavefront each: corners gathered from memory,
 *            accumulation in LDS, global atomics only for nodes shared with
 *            other tiles;
 *   BLOCK    larger tiles, one workgroup of four wavefronts each: the tile's
 *            node records (coordinates, input) are staged in LDS once,
 *            accumulation into one LDS copy with LDS atomics (FP64) or into
 *            per-wavefront copies added in a fixed order (FP32); nodes of one
 *            tile are stored directly, the partial sums of nodes shared
 *            between tiles go to halo slots owned by the operator and a
 *            second kernel adds each node's slots in tile order (no global
 *            atomics; each entry of y is written once).  Because the halo
 *            buffer belongs to the operator, two applies of one BLOCK
 *            operator must not run concurrently (issue them on one stream).
 *            The scalar Laplace kind on a box lattice in this header's
 *            numbering (element counts multiples of 16, 8 and 4; all elements
 *            parallelepipeds, or at most 131,072 general hexahedra; or the
 *            lattice's Kuhn split into tetrahedra, element 6e + t) takes
 *            owner-computes tiles instead: each workgroup computes the
 *            elements around a 16 x 8 x 4 box of nodes and stores those
 *            nodes of y once, in one kernel with no halo slots (the mesh
 *            checked entry by entry at creation; Q1_OWNER_TILE=0 in the
 *            environment at creation keeps the halo-slot tiles);
 *   PA       "partial assembly" (Section 3; the storage of Table 3): BLOCK's
 *            tiles and halo, but at set-up quadrature data of every element
 *            and point is computed and stored, and the apply reads it instead
 *            of the coordinates.  Laplace kinds: the symmetric factor
 *            k w det J J^-1 J^-T (6 reals per point, 48 per element).
 *            Elasticity: the 9 entries of sqrt(w det J) J^-1 per point (72
 *            per element; lambda and mu stay per cell), from which the flux
 *            w det J sigma J^-T follows exactly (Table 3 counts 21 values per
 *            point for isotropic elasticity without defining them);
 *   AUTO     the fastest measured strategy: BLOCK, else LDS_TILE when the tile
 *            does not fit in LDS, else ATOMIC;
 *   CSR      the assembled matrix (made by q1_csr_create only). */
enum { Q1_V_AUTO = 0, Q1_V_ATOMIC = 1, Q1_V_COLOR = 2, Q1_V_LDS_TILE = 3, Q1_V_CSR = 4,
       Q1_V_BLOCK = 5, Q1_V_PA = 6 };

/* Create an operator over caller-owned device arrays.  The arrays are
 * referenced, not copied: they must stay valid and unchanged until
 * q1_op_destroy.  coef_d holds k [n_elems] (Laplace) or lambda then mu
 * [2][n_elems] (elasticity).  mask_d may be NULL.  Every connectivity entry
 * is checked on the device to lie in [0, n_nodes) (Q1_EINVAL otherwise).
 * Set-up work (that check, tile maps) runs on `stream` and is complete when
 * the call returns.  A node that no element references has a zero row:
 * every variant writes y = 0 there (y = x when it is masked), its diagonal is
 * 0 (1 when masked) and the Jacobi weight of the solvers is 0 there. */
int q1_op_create(q1_op **op, int physics, int dtype, int variant, int64_t n_nodes,
                 int64_t n_elems, const void *xyz_d, const int32_t *conn_d, const void *coef_d,
                 const uint8_t *mask_d, void *stream);
/* Element families.  The paper's elements are trilinear hexahedra
 * (Q1_HEX8, the layout described at the top of this header); its conclusions
 * (Section 7) name simplicial and higher-order elements as the next cases for
 * the matrix-free algorithm, built here with the same physics:
 *   Q1_TET4   linear tetrahedra: connectivity [4][n_elems], reference vertices
 *             (0,0,0), (1,0,0), (0,1,0), (0,0,1) (positive orientation), the
 *             exact one-point rule (constant gradients);
 *   Q1_HEX27  triquadratic (Q2) hexahedra: connectivity [27][n_elems], local
 *             node a = i + 3j + 9k at (t_i, t_j, t_k) with t = (-1, 0, 1) of
 *             the reference cube, isoparametric geometry from the 27 nodes,
 *             3x3x3 Gauss-Legendre quadrature;
 *   Q1_HEX64  tricubic (Q3) hexahedra: connectivity [64][n_elems], local node
 *             a = i + 4j + 16k at (t_i, t_j, t_k) with t_m = -1 + 2m/3,
 *             isoparametric geometry from the 64 nodes, 4x4x4 Gauss-Legendre
 *             quadrature.
 * The enum values are the nodes per element. */
enum { Q1_HEX8 = 8, Q1_TET4 = 4, Q1_HEX27 = 27, Q1_HEX64 = 64 };
/* q1_op_create for an element family.  Q1_HEX8 is q1_op_create.  Q1_TET4,
 * Q1_HEX27 and Q1_HEX64: physics Q1_LAPLACE or Q1_ELASTICITY, variants
 * Q1_V_AUTO or Q1_V_ATOMIC (one thread per tetrahedron, one thread per node
 * and quadrature point of a triquadratic or tricubic element with the
 * element's nodes staged in LDS; global atomic scatter); other
 * variants and physics give Q1_EUNSUPPORTED.  The apply, diagonal, byte model
 * and the Krylov solvers accept these operators; q1_csr_create, the fused and
 * the batched solvers do not (Q1_EUNSUPPORTED). */
int q1_op_create_elem(q1_op **op, int elem, int physics, int dtype, int variant,
                      int64_t n_nodes, int64_t n_elems, const void *xyz_d, const int32_t *conn_d,
                      const void *coef_d, const uint8_t *mask_d, void *stream);
/* y = A x (overwrites y; x and y must not alias).  Both have n_nodes*dpn
 * entries of the operator's dtype. */
int q1_op_apply(q1_op *op, const void *x_d, void *y_d, void *stream);
/* d = diag(A), computed element by element without forming A; d_c = 1 on
 * Dirichlet DOFs. */
int q1_op_diag(q1_op *op, void *d_d, void *stream);
/* Properties: physics, dtype, variant actually used, n_nodes, n_elems. */
int q1_op_info(const q1_op *op, int *physics, int *dtype, int *variant, int64_t *n_nodes,
               int64_t *n_elems);
/* *reproducible = 1 when repeated applies and diagonals of this operator on
 * identical inputs give bitwise-identical results (the block and partial-
 * assembly variants on tiles that admit the split accumulation: every node
 * takes its LDS additions from one wavefront per pass, in a fixed order, and
 * shared nodes are summed in tile order; no global atomics; the owner-computes
 * tiles of the scalar kind on box lattices add with LDS atomics, one
 * wavefront per node and pass, in program order), else 0 (the atomic scatter
 * variants, and tiles that fall back to LDS atomics across wavefronts). */
int q1_op_reproducible(const q1_op *op, int *reproducible);
/* Algorithmic bytes and FLOPs of one apply under the Table 2 convention with
 * perfect caching: 32 B of node ids and the cell coefficients per element;
 * the coordinates plus three vector streams (x read, y read, y write) per
 * node.  FLOPs: the fixed per-element counts of the sum-factorised apply.
 * For a CSR operator: values and column indices per non-zero, row pointer,
 * x read and y write per row (Table 1 convention), 2 FLOPs per non-zero. */
int q1_op_bytes(const q1_op *op, double *algorithmic_bytes, double *algorithmic_flops);
/* Destroy the handle and its internal workspace (not the caller's arrays). */
int q1_op_destroy(q1_op *op);

/* ---- matrix-based comparison (Section 1 and Table 1: SpMV; Section 3: the
 *      fill by column search and atomic addition) ---------------------------
 * q1_csr_create assembles the operator `like` describes into CSR on the device
 * (pattern on the host from the connectivity, values by an element loop that
 * binary-searches each column and adds atomically, then the symmetric
 * Dirichlet elimination) and returns a new operator whose apply is the SpMV.
 * It references the same caller arrays as `like`.  Returns Q1_EUNSUPPORTED
 * for 2^31 or more non-zeros.  Synchronises `stream`. */
int q1_csr_create(q1_op **op_csr, const q1_op *like, void *stream);
/* Rows and non-zeros of a CSR operator. */
int q1_csr_info(const q1_op *op_csr, int64_t *nrows, int64_t *nnz);
/* Copy the matrix to caller HOST arrays rowptr [nrows+1], col [nnz], val [nnz]
 * (operator dtype); any of them may be NULL.  Synchronous. */
int q1_csr_export(const q1_op *op_csr, int32_t *rowptr, int32_t *col, void *val);

/* ---- Krylov solvers (the CG operations of Table 4) ------------------------
 * Vectors b_d and x_d have the operator's dtype; every dot product
 * accumulates in FP64 and is deterministic (fixed reduction order, no
 * atomics).  x0 = 0; convergence when ||r_k||_2 <= rtol ||b||_2 on the
 * recurrence residual.  The calls synchronise `stream` and return Q1_OK,
 * Q1_ENOCONV (x holds the last iterate) or Q1_EBREAKDOWN (p^T A p <= 0 or a
 * non-finite scalar); st (may be NULL) is filled in every case. */
typedef struct {
  int iters;           /* Krylov iterations (inner iterations summed for IR) */
  int status;          /* return code of the solve */
  double rel_res;      /* recurrence (or outer) residual ||r||/||b|| */
  double true_rel_res; /* ||b - A x||/||b|| recomputed at the end */
  double seconds;      /* host wall time of the solve, set-up included */
  int fallback_at;     /* flexible PCG: iteration of the switch to Jacobi, -1 if none */
  int outer_iters;     /* iterative refinement: outer steps */
} q1_stats;
enum { Q1_PC_NONE = 0, Q1_PC_JACOBI = 1 };

/* Dot product of two device vectors of n reals (dtype Q1_F64 or Q1_F32),
 * accumulated in FP64 and written to the device double out_d: the reduction of
 * Table 4's ddot operations, exposed so that implementations can be compared
 * (the paper's Section 6 finds the dot product's implementation decisive for CG
 * on AMD hardware).  Variants:
 *   Q1_DOT_TWO_STAGE  each block writes its partial (fixed-order wave64 and
 *                     block sums), then one block adds the partials in a fixed
 *                     order: bitwise reproducible; the reduction the solvers use;
 *   Q1_DOT_ATOMIC     one pass: each block adds its partial to out_d with an
 *                     FP64 atomic (out_d is cleared first by the call); the
 *                     order, and so the last bits, vary from run to run.
 * nblocks: blocks of 256 threads (1..1024; 0 = the solvers' choice, one block
 * per 2,048 entries up to 1024); work_d: device workspace of at least nblocks
 * (1024 for nblocks = 0) doubles for Q1_DOT_TWO_STAGE, may be NULL for
 * Q1_DOT_ATOMIC.  Asynchronous on `stream`. */
enum { Q1_DOT_TWO_STAGE = 0, Q1_DOT_ATOMIC = 1 };
int q1_dot(int64_t n, int dtype, const void *a_d, const void *b_d, double *out_d, int variant,
           int nblocks, double *work_d, void *stream);

/* Preconditioned CG (Hestenes-Stiefel) with z = D^{-1} r (Jacobi, D the
 * matrix-free diagonal) or z = r. */
int q1_pcg(q1_op *op, int pc, const void *b_d, void *x_d, double rtol, int maxit,
           q1_stats *st, void *stream);

/* For callers that cannot allocate device memory (code recorded under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): q1_pcg with
 * its whole workspace (the status record, the reduction partials and the four
 * solver vectors) in a static device array of Q1_NOALLOC_BYTES (about 96 MiB)
 * that each GPU the library runs on holds until the process ends.  Same
 * arguments, results and statuses as q1_pcg; Q1_EINVAL when n_nodes*dpn
 * exceeds Q1_NOALLOC_MAX_DOF (3,145,728: the 128^3 scalar and 96^3
 * elasticity problems fit).  Makes no device or pinned-host allocation (the
 * operator's own set-up already holds everything its apply and diagonal use).
 * All calls on one GPU share that GPU's array: calls that overlap in time on
 * one GPU race.  The array keeps the last call's contents; every call writes
 * each workspace entry before it reads it (the status record is cleared by a
 * kernel, not a memset).  Synchronises `stream`. */
#define Q1_NOALLOC_MAX_DOF 3145728
#define Q1_NOALLOC_BYTES (256 + 8 * 1024 * 8 + 32768 * 8 + 4 * (size_t)Q1_NOALLOC_MAX_DOF * 8)
int q1_pcg_noalloc(q1_op *op, int pc, const void *b_d, void *x_d, double rtol, int maxit,
                   q1_stats *st, void *stream);

/* A preconditioner callback: enqueue z = M(r) on `stream` (device vectors of
 * the operator's dtype) and return Q1_OK, or any other value to report
 * failure. */
/* q1_pcg that also records iterates: after iteration snap_iters[i] (counted
 * from 1, ascending; 0 = the initial x = 0) x is copied to the device vector
 * snap_d[i] (host array of nsnap device pointers, operator dtype); snapshots
 * past the last iteration receive the final x.  Used to harvest the
 * residual -> error pairs the learned preconditioner is trained on. */
int q1_pcg_trace(q1_op *op, int pc, const void *b_d, void *x_d, double rtol, int maxit, int nsnap,
                 const int *snap_iters, void *const *snap_d, q1_stats *st, void *stream);

typedef int (*q1_precond_fn)(void *ctx, const void *r_d, void *z_d, void *stream);
/* Flexible PCG (beta = z_{k+1}^T (r_{k+1} - r_k) / (r_k^T z_k)) with a
 * variable preconditioner M.  Safeguard: on a failing call, z^T r <= 0, a
 * non-finite value, or no decrease of ||r|| over safeguard_m iterations
 * (0 = off), the solve continues with Jacobi; st->fallback_at records when. */
int q1_fpcg(q1_op *op, q1_precond_fn M, void *ctx, const void *b_d, void *x_d, double rtol,
            int maxit, int safeguard_m, q1_stats *st, void *stream);
/* Flexible CG with truncated orthogonalisation, FCG(m) (Notay): the new
 * direction is z = M(r) made A-orthogonal to the last trunc_m directions
 * (1 <= trunc_m <= 8), and alpha = p^T r / p^T A p.  trunc_m = 1 is q1_fpcg.
 * A preconditioner that changes from one call to the next (a network, an
 * inner iteration) keeps the energy norm of the error decreasing; for a fixed
 * SPD M every trunc_m gives the PCG iterates.  Safeguards and stats as
 * q1_fpcg.  Keeps 2 * trunc_m extra vectors. */
int q1_fcg(q1_op *op, q1_precond_fn M, void *ctx, const void *b_d, void *x_d, double rtol,
           int maxit, int safeguard_m, int trunc_m, q1_stats *st, void *stream);

/* Jacobi preconditioner object, usable as the ctx of q1_precond_jacobi. */
typedef struct q1_jacobi q1_jacobi;
int q1_jacobi_create(q1_jacobi **J, q1_op *op, void *stream);
int q1_precond_jacobi(void *ctx, const void *r_d, void *z_d, void *stream);
int q1_jacobi_destroy(q1_jacobi *J);

/* Jacobi-PCG (pc as in q1_pcg) fused into ONE launch of one workgroup (8
 * wavefronts) for small problems: apply, dot products and vector updates of
 * every iteration (Table 4's CG operations) run back to back with workgroup
 * barriers; q = A p is accumulated in LDS, so n_nodes * dpn * 8 B plus 512 B
 * must fit in 64 KB (about 8,100 DOF), otherwise Q1_EUNSUPPORTED.  Same
 * iteration and stopping rule as q1_pcg; st->true_rel_res is computed in the
 * same launch.  FP64 operators of any variant (the kernel reads the caller's
 * coordinates, connectivity and coefficients); b_d, x_d FP64.  Allocates a
 * small workspace; synchronises `stream`. */
int q1_pcg_fused(q1_op *op, int pc, const double *b_d, double *x_d, double rtol, int maxit,
                 q1_stats *st, void *stream);

/* Mixed-precision iterative refinement: r = b - A64 x in FP64; s = r/||r||
 * rounded to FP32; Jacobi-PCG with the FP32 operator, FP32 vectors and FP64
 * dots solves A32 d = s to inner_rtol (at most max_inner iterations); then
 * x += ||r|| d in FP64; until ||r|| <= rtol ||b||.  op64 and op32 describe the
 * same operator (Q1_F64 and Q1_F32).  Returns Q1_EBREAKDOWN if an outer step
 * does not reduce ||r||, Q1_ENOCONV after max_outer steps.  b_d, x_d: FP64. */
int q1_ir_solve(q1_op *op64, q1_op *op32, const double *b_d, double *x_d, double rtol,
                double inner_rtol, int max_outer, int max_inner, q1_stats *st, void *stream);

/* Mixed-precision Jacobi-PCG with reliable updates: the search directions p
 * and q = A p are FP32 (q from the FP32 operator), while x, the residual r,
 * the inverse diagonal and every dot product are FP64.  Each time the
 * recurrence residual has fallen by the factor delta (0 < delta < 1, e.g. 0.1)
 * since the last refresh, or below rtol/sqrt(2) relative to ||b||, the true
 * residual r = b - A64 x is recomputed with the FP64 operator; convergence is
 * decided on it, and otherwise the recurrences continue from it with the
 * search direction kept.  Stops when the FP64 true residual satisfies
 * ||r|| <= rtol ||b||.  st->iters counts Krylov iterations, st->outer_iters
 * the refreshes.  b_d, x_d: FP64.  Workspace allocated and freed by the call. */
int q1_mpcg(q1_op *op64, q1_op *op32, const double *b_d, double *x_d, double rtol,
            double delta, int maxit, q1_stats *st, void *stream);

/* Batched persistent Jacobi-PCG: nprob independent scalar-Laplace problems
 * (FP64 operators created with Q1_V_LDS_TILE), each with nrhs
 * right-hand sides (1..4), solved by ONE cooperative kernel launch.  b_d and
 * x_d hold nprob*nrhs device vectors (problem-major, FP64); st, if not NULL,
 * nprob*nrhs records.  Each problem gets a share of the co-resident
 * wavefronts in proportion to its expected work (elements^(4/3)) and
 * synchronises them with its own barrier, two per iteration: the direction
 * update runs inside the apply and p^T A p comes from element energies.
 * Workspace (per problem: nrhs * 6 FP64 vectors, tile bookkeeping) is
 * allocated and freed by the call.  Returns the worst status over all solves;
 * Q1_EUNSUPPORTED for other operators or when more problems than co-resident
 * wavefronts are given.  Synchronises `stream`. */
int q1_batched_pcg(int nprob, q1_op *const *ops, int nrhs, const double *const *b_d,
                   double *const *x_d, double rtol, int maxit, q1_stats *st, void *stream);

/* Mixed-precision form of q1_batched_pcg (same operators, one launch; the
 * reliable-update scheme of q1_mpcg inside the persistent kernel).  Inside the one kernel the Krylov applies use FP32 copies of each
 * operator's coordinates and coefficients and FP32 search directions p, q,
 * while x, r and every dot product stay FP64.  When the recurrence residual
 * of a right-hand side has fallen by the factor delta (0 < delta < 1, e.g.
 * 0.1) since its last refresh, or below rtol/sqrt(2) relative to ||b||, or
 * at maxit, the kernel recomputes r = b - A x with the FP64 operator and
 * decides convergence on that true residual; otherwise the recurrences
 * continue from it with p kept.  st[k].outer_iters counts the refreshes and
 * st[k].rel_res is the true relative residual of the last refresh.  Device
 * memory per problem: FP32 copies of the geometry and coefficients, and per
 * right-hand side three FP32 vectors (two direction buffers, q) and four FP64
 * ones (b, x, r, the refresh apply's output), allocated and freed by the call.
 * Returns Q1_EINVAL for delta outside (0, 1); otherwise as q1_batched_pcg. */
int q1_batched_mpcg(int nprob, q1_op *const *ops, int nrhs, const double *const *b_d,
                    double *const *x_d, double rtol, double delta, int maxit, q1_stats *st,
                    void *stream);

/* ---- learned preconditioner --------------------------------------------------
 * The paper's conclusions (Section 7) name matrix-free preconditioners as
 * future work and say nothing of learned ones; the learned preconditioner is
 * this project's own addition, and this library defines its network: a 3-level 3-D convolutional U-Net on the node grid (16/32/64
 * channels; per level two 3x3x3 zero-padded convolutions with bias and ReLU;
 * 2x2x2 average pooling down; nearest 2x upsampling concatenated with the
 * skip tensor up; a 1x1 head), trained with Adam on residual -> error pairs,
 * and used as z = N(r) inside q1_fpcg, which falls back to Jacobi when z fails
 * (z.r <= 0, non-finite, stagnation).
 *
 * Tensors are channel-last [B][D][H][W][C] (z, y, x, channel), BF16 as
 * uint16_t bit patterns, C a multiple of 8.  Convolution weights are FP32
 * W[27][Cin][Cout] with tap t = 9 (dz+1) + 3 (dy+1) + (dx+1) and
 * y[v][co] = b[co] + sum_t sum_ci x[v + d_t][ci] W[t][ci][co] (zero outside
 * the grid).  Matrix-core operands are BF16, accumulation FP32. */

/* Single-layer primitives (synchronise `stream`; they allocate temporaries).
 * Forward: the input is the channel concatenation of a (ca channels; when
 * up_a, a lives on the half grid D/2 x H/2 x W/2 and is read at the parent
 * voxel, i.e. nearest 2x upsampling) and b (cb channels, may be 0 and NULL).
 * w_d is [27][ca+cb][cout]; bias_d may be NULL; relu != 0 applies max(0, .);
 * y_d is FP32 [B][D][H][W][cout].  cout is 16, 32, 48, 64 or 96 and ca + cb
 * is 8 or a multiple of 16 up to 96, otherwise Q1_EUNSUPPORTED. */
int q1_conv3d_forward(int B, int D, int H, int W, const uint16_t *a_d, int ca, int up_a,
                      const uint16_t *b_d, int cb, const float *w_d, const float *bias_d,
                      int cout, int relu, float *y_d, void *stream);
/* Backward-data: gx = adjoint of x -> conv(x, w) applied to gy (BF16
 * [V][cout]); w_d [27][cin][cout]; gx_d FP32 [V][cin]; cin as cout above. */
int q1_conv3d_backward_data(int B, int D, int H, int W, const uint16_t *gy_d, int cout,
                            const float *w_d, int cin, float *gx_d, void *stream);
/* Backward-weight: gw[t][ci][co] = sum_v x[v + d_t][ci] gy[v][co] and
 * gb[co] = sum_v gy[v][co], x read as in the forward; gw_d FP32
 * [27][ca+cb][cout], gb_d FP32 [cout]; cout a multiple of 16.  Deterministic. */
int q1_conv3d_backward_weight(int B, int D, int H, int W, const uint16_t *a_d, int ca, int up_a,
                              const uint16_t *b_d, int cb, const uint16_t *gy_d, int cout,
                              float *gw_d, float *gb_d, void *stream);

typedef struct q1_unet q1_unet;
/* Network for a D x H x W grid (multiples of 4) and up to `batch` samples
 * per pass.  Weights are He-normal from `seed` (SplitMix64), biases zero.
 * The handle owns its parameters, gradients, Adam moments and activations.
 * Synchronises `stream`. */
int q1_unet_create(q1_unet **net, int D, int H, int W, int batch, uint64_t seed, void *stream);
int q1_unet_destroy(q1_unet *net);
int q1_unet_info(const q1_unet *net, int64_t *nparams, int *D, int *H, int *W, int *batch);
/* Device pointers to the FP32 parameter and gradient vectors (nparams each).
 * Layout, in the layer order enc1a enc1b enc2a enc2b enc3a enc3b dec2a dec2b
 * dec1a dec1b: W[27][Cin][Cout] then b[Cout] (Cin 2, 16, 16, 32, 32, 64,
 * 64+32, 32, 32+16, 16; Cout 16, 16, 32, 32, 64, 64, 32, 32, 16, 16), then
 * the head w[16] and b.  After writing parameters call q1_unet_commit. */
int q1_unet_params(q1_unet *net, float **theta_d, float **grad_d);
/* Refresh the packed BF16 weights from the FP32 parameters. */
int q1_unet_commit(q1_unet *net, void *stream);
/* Copy the parameters (which = 0) or gradients (which = 1) to buf_d
 * (to_net = 0) or from buf_d into the network (to_net = 1; after writing
 * parameters call q1_unet_commit; writing gradients lets a caller apply Adam
 * to gradients it combined itself, e.g. summed over data-parallel ranks);
 * buf_d is a device FP32 [nparams]. */
int q1_unet_copy(q1_unet *net, int which, int to_net, float *buf_d, void *stream);
/* out = N(in) for the first nbatch samples: in_d BF16 [nbatch][D][H][W][8]
 * (channels 2..7 must be zero), out_d FP32 [nbatch][D][H][W].  Activations
 * stay in the handle for q1_unet_backward; in_d must stay unchanged until then. */
int q1_unet_forward(q1_unet *net, const uint16_t *in_d, float *out_d, int nbatch, void *stream);
/* Loss of the last forward: L = sum w (out - target)^2 / sum w and
 * dout = dL/dout (all FP32 [nbatch][D][H][W]); *loss_d (device, may be NULL). */
int q1_unet_mse(q1_unet *net, const float *out_d, const float *target_d, const float *weight_d,
                float *dout_d, float *loss_d, void *stream);
/* Gradient of the parameters for dL/dout = dout_d at the last forward's
 * activations, written to the gradient vector (overwritten, deterministic). */
int q1_unet_backward(q1_unet *net, const float *dout_d, void *stream);
/* One Adam step (Kingma and Ba) on the parameters with the current gradient;
 * step counts from 1; repacks the BF16 weights. */
int q1_unet_adam_step(q1_unet *net, float lr, float b1, float b2, float eps, int step,
                      void *stream);

typedef struct q1_unet_pc q1_unet_pc;
/* Preconditioner context for an nx x ny x nz-element box mesh (nodes
 * x-fastest, (nx+1)(ny+1)(nz+1) <= the grid) with cell coefficients k_d
 * (FP64 [nx*ny*nz], x-fastest) and optional Dirichlet node mask mask_d; the
 * node grid sits at the origin of the network grid.  The network handle, k_d
 * and mask_d must outlive the context.  Synchronises `stream`. */
int q1_unet_pc_create(q1_unet_pc **pc, q1_unet *net, int nx, int ny, int nz, const double *k_d,
                      const uint8_t *mask_d, void *stream);
/* Switch the context to the two-level form: with the FP64 scalar operator op
 * of the same mesh and w = 1 / diag(A),
 *   z1 = omega w r,  r1 = r - A z1,  d = N(encode(r1)),
 *   c = d.r1 / d.A d (0 if not positive), z = z1 + c d + omega w (r1 - c A d),
 * i.e. damped-Jacobi smoothing around the network acting as a coarse
 * correction, its scale chosen to minimise the energy norm of the error.
 * Costs two operator applies per use.  op must outlive the context. */
int q1_unet_pc_two_level(q1_unet_pc *pc, q1_op *op, double omega, void *stream);
/* Schedule of the network inside a solve: the network is evaluated on calls
 * 0, period, 2 period, ... counted from this call, and the plain Jacobi step
 * z = D^-1 r is taken on the others (a preconditioner that changes between
 * calls, for the flexible solvers).  period > 1 needs the two-level form (its
 * Jacobi weights).  Call it again before each solve to restart the count. */
int q1_unet_pc_schedule(q1_unet_pc *pc, int period);
/* Training pairs of the learned preconditioner from one Jacobi-PCG trajectory
 * of the FP64 scalar-Laplace operator op: for each recorded iterate x_k
 * (device FP64 vectors xk_d[i], host array of npairs pointers) and the
 * converged x*, the error e = x* - x_k and the residual r = A e; with
 * omega > 0 the pair is moved through one damped-Jacobi step as the two-level
 * preconditioner presents it to the network, e1 = e - omega D^-1 r, r1 = A e1.
 * Writes FP32 copies to e_d[i] and r_d[i] (n_nodes each).  Allocates three
 * FP64 vectors of workspace; synchronises `stream`. */
int q1_unet_pairs(q1_op *op, const double *xstar_d, int npairs, const double *const *xk_d,
                  double omega, float *const *e_d, float *const *r_d, void *stream);
int q1_unet_pc_destroy(q1_unet_pc *pc);
/* Network input of a nodal FP64 vector r: channel 0 = r on free nodes scaled
 * to unit RMS over them (0 on Dirichlet nodes), channel 1 = half the mean of
 * ln k over each node's cells, everything else 0; in_d BF16 [D][H][W][8]. */
int q1_unet_encode(q1_unet_pc *pc, const double *r_d, uint16_t *in_d, void *stream);
/* Training target of a nodal FP64 error e: e on free nodes scaled to unit
 * RMS, 0 elsewhere (FP32 [D][H][W]); weight_d (may be NULL) = 1 on free
 * nodes, 0 elsewhere. */
int q1_unet_encode_target(q1_unet_pc *pc, const double *e_d, float *target_d, float *weight_d,
                          void *stream);
/* q1_precond_fn for q1_fpcg with ctx = q1_unet_pc: z = N(encode(r)) on free
 * nodes, 0 on Dirichlet nodes (FP64 vectors).  Flexible PCG is invariant to a
 * positive scaling of z, so the output is not rescaled by ||r||. */
int q1_unet_precond(void *ctx, const void *r_d, void *z_d, void *stream);

/* Byte model of Section 4 (Tables 1-3) for n_elems hexahedra and n_nodes
 * nodes.  kind: 0 SpMV (Table 1: 12 B per non-zero with 27*dpn non-zeros per
 * row, two vectors), 1 matrix-free (Table 2), 2 partial assembly (Table 3).
 * cache: 0 perfect caching (nodal data read once), 1 no caching (nodal data
 * read once per element touching it).  real_bytes 8 or 4; coefficient bytes
 * per element coef_bytes (the paper counts 0 for Laplace, 16 for elasticity).
 * physics: a physics kind (1 DOF per node for Q1_LAPLACE, 3 otherwise). */
int q1_model_bytes(int kind, int physics, int real_bytes, int coef_bytes, int64_t n_nodes,
                   int64_t n_elems, int cache, double *bytes);

#ifdef __cplusplus
}
#endif
#endif /* Q1MF_H */
