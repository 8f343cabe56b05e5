/*
 * mgo.h -- FP64 CPU oracle for the all-at-once multigrid method of
 * S. Takacs, "Efficient smoothers for all-at-once multigrid methods for
 * Poisson and Stokes control problems" (arXiv 1502.03917).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this code: only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header, table or constant with
 * the HIP library; both sides only receive the same seeded input arrays.
 *
 * Everything is plain FP64, single-threaded, with explicitly assembled sparse
 * matrices, so that each step can be checked against the paper by eye.
 *
 * Discretisation (readings of passages the paper leaves open):
 *   - domain: unit square; level l has n = 2^l cells per side, h = 1/n,
 *     (n+1)^2 vertices, vertex (i,j) has index j*(n+1)+i;
 *   - every square is split by its diagonal from (i,j) to (i+1,j+1);
 *   - Courant (P1) elements, all vertices are unknowns (Neumann problem);
 *   - K_k is the matrix of the bilinear form of -Laplace(y)+y, i.e. the
 *     Laplacian stiffness matrix plus the mass matrix (section 1, the state
 *     equation); M_k the P1 mass matrix.
 */
#ifndef MGO_ORACLE_H
#define MGO_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* compressed sparse row matrix, 0-based, columns sorted within each row */
typedef struct {
  int nrows, ncols, nnz;
  int *rowptr; /* nrows+1 */
  int *col;    /* nnz */
  double *val; /* nnz */
} mgo_csr;

void mgo_csr_free(mgo_csr *A);

/* P1 mass matrix M and Laplacian stiffness matrix Klap on level with n cells
 * per side, by a loop over the 2 n^2 triangles. */
void mgo_assemble_p1(int n, mgo_csr *M, mgo_csr *Klap);

/* canonical embedding (P1 interpolation) from the grid with nc cells per side
 * to the grid with 2 nc cells per side; rows = fine vertices. */
void mgo_prolongation_p1(int nc, mgo_csr *P);

/* transpose */
void mgo_transpose(const mgo_csr *A, mgo_csr *At);

/* Taylor-Hood pieces (Stokes control, eq. mp3), n cells per side: scalar P2
 * mass M and Laplacian stiffness K, and the divergence blocks
 * D1 = -int q d_x phi, D2 = -int q d_y phi (rows: P1 vertices), over the
 * interior P2 nodes (full = 0; velocity vanishes on the boundary) or over
 * all (2n+1)^2 nodes (full = 1).  P2 node (a, b) of the half-step lattice,
 * at (a/(2n), b/(2n)), has index (b-1)(2n-1)+(a-1) (interior) or
 * b(2n+1)+a (full). */
void mgo_assemble_p2(int n, int full, mgo_csr *M, mgo_csr *K, mgo_csr *D1, mgo_csr *D2);
/* P2 interpolation from nc to 2 nc cells per side (interior or all nodes) */
void mgo_prolongation_p2(int nc, int full, mgo_csr *P);

/* opaque multigrid hierarchy */
typedef struct mgo_hier mgo_hier;

enum { MGO_NE = 0, MGO_LSGS = 1, MGO_SLSGS = 2, MGO_CGS = 3, MGO_VANKA = 4 };
enum { MGO_ORDER_LEX = 0, MGO_ORDER_COL7 = 1, MGO_ORDER_COL7SEQ = 2, MGO_ORDER_VLEX = 3, MGO_ORDER_COL3 = 4 };

/* Build levels coarse..fine (fine >= coarse+1 >= 2) of the Poisson control
 * KKT system for regularisation alpha > 0. problem 0 = Poisson control,
 * 1 = Stokes control (Taylor-Hood).  Returns NULL on invalid input. */
mgo_hier *mgo_create(int problem, int fine, int coarse, double alpha);
void mgo_destroy(mgo_hier *h);

/* number of unknowns on level l */
int mgo_ndof(const mgo_hier *h, int level);
/* copy out a matrix of level l: which = 0 A, 1 M, 2 Klap, 3 P (l-1 -> l),
 * 4 B (Stokes divergence block), 5 Mp (Stokes pressure mass).  With
 * rowptr == NULL only *nnz is returned. Returns nrows, or -1. */
int mgo_get_matrix(const mgo_hier *h, int level, int which, int *nrows, int *ncols, int *nnz,
                   int *rowptr, int *col, double *val);
/* diagonal L_k (which = 0) or diag(N_k) (which = 1) of level l */
int mgo_get_diag(const mgo_hier *h, int level, int which, double *out);

/* r = f - A_l x */
void mgo_residual(const mgo_hier *h, int level, const double *f, const double *x, double *r);

/* One smoothing step on level l keeping r = f - A x current (x, r in/out).
 * kind: MGO_NE (Alg. 1, damping tau), MGO_LSGS (Alg. 2 in ordering 'order'),
 * MGO_SLSGS (forward then reversed ordering), MGO_CGS (Poisson: collective
 * point GS over vertices: lexicographic, 7 colours for MGO_ORDER_COL7, 3
 * colours for MGO_ORDER_COL3), MGO_VANKA (Stokes: damped patch smoother over
 * the vertex patches, lexicographic for MGO_ORDER_LEX, else 9 colours).
 * Stokes orderings of Alg. 2: MGO_ORDER_LEX every unknown in index order;
 * MGO_ORDER_COL7 the colour order (25 P2-node colours (a mod 5)+5(b mod 5)
 * per velocity component with {v_c, lambda_c} grouped, then 9 vertex colours
 * (i mod 3)+3(j mod 3) with {p, mu} grouped); MGO_ORDER_COL7SEQ the same with
 * one unknown per group. */
void mgo_smooth(const mgo_hier *h, int level, int kind, int order, double tau, double *x, double *r);

/* Alg. 2 over a caller-given ordering: unknowns ord[gptr[g]..gptr[g+1]) form
 * group g and take their updates from one residual snapshot; groups are
 * visited in order (reverse = 0) or in reverse order (reverse = 1). */
void mgo_smooth_groups(const mgo_hier *h, int level, const int *ord, const int *gptr, int ngroup, int reverse,
                       double *x, double *r);

/* exact coarsest-level solve x = A^{-1} f by dense LU with partial pivoting */
void mgo_coarse_solve(const mgo_hier *h, const double *f, double *x);

/* Stokes: shift p and mu of a level-l vector to zero mean (weights Mp 1);
 * no-op for Poisson.  mgo_cycle and mgo_solve do this after every cycle. */
void mgo_project(const mgo_hier *h, int level, double *x);

/* one multigrid cycle (gamma = 1 V, 2 W) on level l, in place on x */
void mgo_cycle(const mgo_hier *h, int level, int kind, int order, double tau, int nu1, int nu2,
               int gamma, const double *f, double *x);

/* cycles until ||f - A x|| <= tol ||f|| (or max_cycles), in the Euclidean
 * norm (norm = 0) or the norm (v^T L_k^{-1} v)^{1/2} (norm = 1).  hist (may be
 * NULL) receives the relative residual before each cycle (max_cycles+1).
 * Returns the number of cycles done, or -1 when max_cycles was hit. */
int mgo_solve(const mgo_hier *h, int kind, int order, double tau, int nu1, int nu2, int gamma,
              const double *f, double *x, double tol, int max_cycles, int norm, double *hist);

#ifdef __cplusplus
}
#endif
/* threads used by the oracle's parallel loops (1 unless built with OpenMP) */
int mgo_threads(void);

#endif
