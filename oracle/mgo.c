/*
 * mgo.c -- FP64 CPU oracle for the all-at-once multigrid method of Takacs,
 * arXiv 1502.03917.  TEST INFRASTRUCTURE ONLY: used by the tests, the smoke
 * check and the CPU-baseline leg of the benchmark, never by the product path.
 *
 * Plain, slow, obviously correct: matrices are assembled element by element
 * into CSR, the smoothers are written from their defining formulas in
 * section 2 (whole-vector products for the normal-equation step, exact
 * coordinate descent for the Gauss-Seidel-like step), and the coarsest level
 * is solved by dense LU.
 * The Poisson-control parts are pinned by the tests in tests/test_oracle_*.py;
 * see the header mgo.h for the discretisation readings.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mgo.h"

#ifdef _OPENMP
#include <omp.h>
#endif

/* threads of the oracle's parallel loops: 1 in the default (single-threaded)
 * build, the OpenMP team size in the threaded build */
int mgo_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------ utils */

static void *xmalloc(size_t n) {
  void *p = malloc(n ? n : 1);
  if (!p) {
    fprintf(stderr, "mgo: out of memory (%zu bytes)\n", n);
    abort();
  }
  return p;
}
static void *xcalloc(size_t n, size_t s) {
  void *p = calloc(n ? n : 1, s ? s : 1);
  if (!p) {
    fprintf(stderr, "mgo: out of memory\n");
    abort();
  }
  return p;
}

void mgo_csr_free(mgo_csr *A) {
  if (!A) return;
  free(A->rowptr);
  free(A->col);
  free(A->val);
  memset(A, 0, sizeof(*A));
}

/* Row builder: every row keeps up to 'cap' (column, value) pairs; adding to an
 * existing column accumulates.  Turned into CSR with sorted columns. */
typedef struct {
  int nrows, ncols, cap;
  int *cnt, *col;
  double *val;
} rowbuild;

static void rb_init(rowbuild *b, int nrows, int ncols, int cap) {
  b->nrows = nrows;
  b->ncols = ncols;
  b->cap = cap;
  b->cnt = (int *)xcalloc((size_t)nrows, sizeof(int));
  b->col = (int *)xmalloc((size_t)nrows * cap * sizeof(int));
  b->val = (double *)xmalloc((size_t)nrows * cap * sizeof(double));
}

static void rb_add(rowbuild *b, int r, int c, double v) {
  int *cs = b->col + (size_t)r * b->cap;
  double *vs = b->val + (size_t)r * b->cap;
  for (int k = 0; k < b->cnt[r]; k++)
    if (cs[k] == c) {
      vs[k] += v;
      return;
    }
  if (b->cnt[r] == b->cap) {
    fprintf(stderr, "mgo: row %d exceeds capacity %d\n", r, b->cap);
    abort();
  }
  cs[b->cnt[r]] = c;
  vs[b->cnt[r]] = v;
  b->cnt[r]++;
}

static void rb_finish(rowbuild *b, mgo_csr *A) {
  A->nrows = b->nrows;
  A->ncols = b->ncols;
  A->rowptr = (int *)xmalloc(((size_t)b->nrows + 1) * sizeof(int));
  size_t nnz = 0;
  for (int r = 0; r < b->nrows; r++) nnz += b->cnt[r];
  A->nnz = (int)nnz;
  A->col = (int *)xmalloc(nnz * sizeof(int));
  A->val = (double *)xmalloc(nnz * sizeof(double));
  size_t at = 0;
  for (int r = 0; r < b->nrows; r++) {
    int *cs = b->col + (size_t)r * b->cap;
    double *vs = b->val + (size_t)r * b->cap;
    int m = b->cnt[r];
    /* insertion sort of the row by column */
    for (int a = 1; a < m; a++) {
      int c = cs[a];
      double v = vs[a];
      int q = a - 1;
      while (q >= 0 && cs[q] > c) {
        cs[q + 1] = cs[q];
        vs[q + 1] = vs[q];
        q--;
      }
      cs[q + 1] = c;
      vs[q + 1] = v;
    }
    A->rowptr[r] = (int)at;
    for (int a = 0; a < m; a++) {
      A->col[at] = cs[a];
      A->val[at] = vs[a];
      at++;
    }
  }
  A->rowptr[b->nrows] = (int)at;
  free(b->cnt);
  free(b->col);
  free(b->val);
}

void mgo_transpose(const mgo_csr *A, mgo_csr *At) {
  At->nrows = A->ncols;
  At->ncols = A->nrows;
  At->nnz = A->nnz;
  At->rowptr = (int *)xcalloc((size_t)A->ncols + 1, sizeof(int));
  At->col = (int *)xmalloc((size_t)A->nnz * sizeof(int));
  At->val = (double *)xmalloc((size_t)A->nnz * sizeof(double));
  for (int k = 0; k < A->nnz; k++) At->rowptr[A->col[k] + 1]++;
  for (int c = 0; c < A->ncols; c++) At->rowptr[c + 1] += At->rowptr[c];
  int *fill = (int *)xmalloc((size_t)A->ncols * sizeof(int));
  for (int c = 0; c < A->ncols; c++) fill[c] = At->rowptr[c];
  for (int r = 0; r < A->nrows; r++)
    for (int k = A->rowptr[r]; k < A->rowptr[r + 1]; k++) {
      int c = A->col[k];
      At->col[fill[c]] = r; /* rows visited in order: columns of At sorted */
      At->val[fill[c]] = A->val[k];
      fill[c]++;
    }
  free(fill);
}

static double csr_entry(const mgo_csr *A, int r, int c) {
  for (int k = A->rowptr[r]; k < A->rowptr[r + 1]; k++)
    if (A->col[k] == c) return A->val[k];
  return 0.0;
}

/* y = A x */
static void csr_mv(const mgo_csr *A, const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int r = 0; r < A->nrows; r++) {
    double s = 0.0;
    for (int k = A->rowptr[r]; k < A->rowptr[r + 1]; k++) s += A->val[k] * x[A->col[k]];
    y[r] = s;
  }
}

/* ------------------------------------------------------- P1 finite elements */

/* Local P1 matrices of the triangle with corners (px[a], py[a]):
 * Kl[a][b] = |T| grad(phi_a).grad(phi_b), Ml[a][b] = |T|/12 (1 + [a==b]). */
static void p1_local(const double px[3], const double py[3], double Kl[3][3], double Ml[3][3]) {
  double det = (px[1] - px[0]) * (py[2] - py[0]) - (px[2] - px[0]) * (py[1] - py[0]);
  double area = fabs(det) / 2.0;
  double gx[3], gy[3];
  for (int a = 0; a < 3; a++) {
    int b = (a + 1) % 3, c = (a + 2) % 3;
    gx[a] = (py[b] - py[c]) / det;
    gy[a] = (px[c] - px[b]) / det;
  }
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      Kl[a][b] = area * (gx[a] * gx[b] + gy[a] * gy[b]);
      Ml[a][b] = area / 12.0 * (a == b ? 2.0 : 1.0);
    }
}

/* the two triangles of square (i,j), split along its diagonal (i,j)-(i+1,j+1) */
static void square_triangles(int i, int j, int t, int vi[3], int vj[3]) {
  if (t == 0) {
    vi[0] = i; vj[0] = j;
    vi[1] = i + 1; vj[1] = j;
    vi[2] = i + 1; vj[2] = j + 1;
  } else {
    vi[0] = i; vj[0] = j;
    vi[1] = i + 1; vj[1] = j + 1;
    vi[2] = i; vj[2] = j + 1;
  }
}

void mgo_assemble_p1(int n, mgo_csr *M, mgo_csr *Klap) {
  int nv = (n + 1) * (n + 1);
  double h = 1.0 / n;
  rowbuild bm, bk;
  rb_init(&bm, nv, nv, 8);
  rb_init(&bk, nv, nv, 8);
  for (int j = 0; j < n; j++)
    for (int i = 0; i < n; i++)
      for (int t = 0; t < 2; t++) {
        int vi[3], vj[3], id[3];
        double px[3], py[3], Kl[3][3], Ml[3][3];
        square_triangles(i, j, t, vi, vj);
        for (int a = 0; a < 3; a++) {
          px[a] = vi[a] * h;
          py[a] = vj[a] * h;
          id[a] = vj[a] * (n + 1) + vi[a];
        }
        p1_local(px, py, Kl, Ml);
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) {
            rb_add(&bm, id[a], id[b], Ml[a][b]);
            rb_add(&bk, id[a], id[b], Kl[a][b]);
          }
      }
  rb_finish(&bm, M);
  rb_finish(&bk, Klap);
}

/* barycentric coordinates of (X,Y) in triangle (px,py) */
static void barycentric(const double px[3], const double py[3], double X, double Y, double lam[3]) {
  double det = (px[1] - px[0]) * (py[2] - py[0]) - (px[2] - px[0]) * (py[1] - py[0]);
  lam[1] = ((X - px[0]) * (py[2] - py[0]) - (px[2] - px[0]) * (Y - py[0])) / det;
  lam[2] = ((px[1] - px[0]) * (Y - py[0]) - (X - px[0]) * (py[1] - py[0])) / det;
  lam[0] = 1.0 - lam[1] - lam[2];
}

/* Canonical embedding of the coarse P1 space into the fine one: the fine
 * nodal value is the coarse function evaluated at the fine vertex. */
void mgo_prolongation_p1(int nc, mgo_csr *P) {
  int nf = 2 * nc, nvf = (nf + 1) * (nf + 1), nvc = (nc + 1) * (nc + 1);
  rowbuild b;
  rb_init(&b, nvf, nvc, 3);
  for (int bj = 0; bj <= nf; bj++)
    for (int ai = 0; ai <= nf; ai++) {
      double X = ai / 2.0, Y = bj / 2.0; /* in coarse grid units (exact) */
      int I = (int)floor(X), J = (int)floor(Y);
      if (I > nc - 1) I = nc - 1;
      if (J > nc - 1) J = nc - 1;
      int done = 0;
      for (int t = 0; t < 2 && !done; t++) {
        int vi[3], vj[3];
        double px[3], py[3], lam[3];
        square_triangles(I, J, t, vi, vj);
        for (int a = 0; a < 3; a++) {
          px[a] = vi[a];
          py[a] = vj[a];
        }
        barycentric(px, py, X, Y, lam);
        if (lam[0] >= 0.0 && lam[1] >= 0.0 && lam[2] >= 0.0) {
          for (int a = 0; a < 3; a++)
            if (lam[a] != 0.0) rb_add(&b, bj * (nf + 1) + ai, vj[a] * (nc + 1) + vi[a], lam[a]);
          done = 1;
        }
      }
      if (!done) {
        fprintf(stderr, "mgo: fine vertex outside the coarse mesh\n");
        abort();
      }
    }
  rb_finish(&b, P);
}

/* ------------------------------------------------------------- hierarchy */

typedef struct {
  int n;          /* cells per side */
  int ndof;       /* unknowns */
  int nfield;     /* number of solution fields */
  int foff[8];    /* field offsets */
  int fkind[8];   /* transfer of each field: index into Pk */
  int fdim[8];    /* field length */
  mgo_csr M, Klap, K, A, At;
  mgo_csr Pk[2], Rk[2]; /* transfers from the next coarser level */
  mgo_csr B, Mp;        /* Stokes only */
  double *L, *Nd;       /* diagonal L_k, diag(N_k) */
  double *x, *f, *r, *p;
  /* orderings for the Gauss-Seidel-like smoothers: order[] lists unknowns,
   * gptr[] delimits groups updated from one residual snapshot */
  int *ord[4], *gptr[4], ngroup[4];
  /* first group of each colour (and the end) in the COL7 order: the groups of
   * one colour share no residual entry, so their steps commute exactly */
  int cptr[8], ncolour;
  int *cgs_ord[3]; /* vertex orders for the collective smoother: lex, col7, col3 */
  int ncgs;
  /* coarsest level only: dense LU with partial pivoting (Stokes: of the
   * matrix bordered by the two mean-value constraints) */
  double *lu;
  int *piv;
  int nlu;
  /* Stokes: P2 nodes per velocity component, P1 vertices, the divergence
   * blocks of the two components, and the Vanka patches (one per vertex) */
  int nv, np;
  mgo_csr D1, D2;
  int *patch_ptr, *patch_dof;
  int *vanka_ord[2];
} mgo_level;

struct mgo_hier {
  int problem, fine, coarse;
  double alpha;
  mgo_level *lv; /* lv[l] for coarse <= l <= fine */
};

/* block 2x2 KKT matrix [[M, K], [K, -alpha^{-1} M]] (eq. mp2) */
static void build_kkt_poisson(mgo_level *L, double alpha) {
  int V = L->M.nrows;
  rowbuild b;
  rb_init(&b, 2 * V, 2 * V, 16);
  for (int r = 0; r < V; r++) {
    for (int k = L->M.rowptr[r]; k < L->M.rowptr[r + 1]; k++) {
      int c = L->M.col[k];
      double m = L->M.val[k];
      rb_add(&b, r, c, m);                      /* M          */
      rb_add(&b, V + r, V + c, -m / alpha);     /* -alpha^-1 M */
    }
    for (int k = L->K.rowptr[r]; k < L->K.rowptr[r + 1]; k++) {
      int c = L->K.col[k];
      rb_add(&b, r, V + c, L->K.val[k]); /* K */
      rb_add(&b, V + r, c, L->K.val[k]); /* K */
    }
  }
  rb_finish(&b, &L->A);
  mgo_transpose(&L->A, &L->At);
}

/* L_k = diag(Q_k) = blockdiag(diag(M + alpha^{1/2} K), diag(alpha^{-1} M + alpha^{-1/2} K)) */
static void build_L_poisson(mgo_level *L, double alpha) {
  int V = L->M.nrows;
  for (int v = 0; v < V; v++) {
    double m = csr_entry(&L->M, v, v), k = csr_entry(&L->K, v, v);
    L->L[v] = m + sqrt(alpha) * k;
    L->L[V + v] = m / alpha + k / sqrt(alpha);
  }
}

/* diagonal of N = A^T L^-1 A: N_ii = a_i^T L^-1 a_i over column a_i of A
 * (row i of A^T); computed once per level */
static void build_Ndiag(mgo_level *L) {
  const mgo_csr *At = &L->At;
  for (int i = 0; i < L->ndof; i++) {
    double s = 0.0;
    for (int k = At->rowptr[i]; k < At->rowptr[i + 1]; k++) s += At->val[k] * At->val[k] / L->L[At->col[k]];
    L->Nd[i] = s;
  }
}

static void build_orders_poisson(mgo_level *L) {
  int n = L->n, V = (n + 1) * (n + 1), N = 2 * V;
  /* lexicographic: all y in vertex order, then all lambda; one unknown per group */
  L->ord[MGO_ORDER_LEX] = (int *)xmalloc(N * sizeof(int));
  L->gptr[MGO_ORDER_LEX] = (int *)xmalloc((N + 1) * sizeof(int));
  for (int i = 0; i < N; i++) {
    L->ord[0][i] = i;
    L->gptr[0][i] = i;
  }
  L->gptr[0][N] = N;
  L->ngroup[0] = N;
  /* seven colours c(i,j) = (i + 2j) mod 7; a vertex's y and lambda form one group
   * (MGO_ORDER_COL7) or two consecutive groups (MGO_ORDER_COL7SEQ) */
  for (int o = 1; o <= 2; o++) {
    L->ord[o] = (int *)xmalloc(N * sizeof(int));
    L->gptr[o] = (int *)xmalloc((N + 1) * sizeof(int));
    int at = 0, g = 0;
    for (int c = 0; c < 7; c++)
      for (int j = 0; j <= n; j++)
        for (int i = 0; i <= n; i++) {
          if ((i + 2 * j) % 7 != c) continue;
          int v = j * (n + 1) + i;
          if (o == MGO_ORDER_COL7) {
            L->gptr[o][g++] = at;
            L->ord[o][at++] = v;
            L->ord[o][at++] = V + v;
          } else {
            L->gptr[o][g++] = at;
            L->ord[o][at++] = v;
            L->gptr[o][g++] = at;
            L->ord[o][at++] = V + v;
          }
        }
    L->gptr[o][g] = at;
    L->ngroup[o] = g;
  }
  {
    /* colour boundaries of COL7: one group per vertex, colours in order */
    int g = 0;
    L->ncolour = 7;
    for (int c = 0; c < 7; c++) {
      L->cptr[c] = g;
      for (int j = 0; j <= n; j++)
        for (int i = 0; i <= n; i++)
          if ((i + 2 * j) % 7 == c) g++;
    }
    L->cptr[7] = g;
  }
  /* vertex-interleaved lexicographic: y_v then lambda_v for v = 0, 1, ... */
  L->ord[MGO_ORDER_VLEX] = (int *)xmalloc(N * sizeof(int));
  L->gptr[MGO_ORDER_VLEX] = (int *)xmalloc((N + 1) * sizeof(int));
  for (int v = 0; v < V; v++) {
    L->ord[MGO_ORDER_VLEX][2 * v] = v;
    L->ord[MGO_ORDER_VLEX][2 * v + 1] = V + v;
  }
  for (int i = 0; i <= N; i++) L->gptr[MGO_ORDER_VLEX][i] = i;
  L->ngroup[MGO_ORDER_VLEX] = N;
  /* collective smoother: vertices in lexicographic order, by the seven colours
   * (i + 2j) mod 7, or by the three colours (i + j) mod 3 (no two neighbours
   * share a colour in either colouring) */
  L->ncgs = V;
  for (int o = 0; o < 3; o++) L->cgs_ord[o] = (int *)xmalloc(V * sizeof(int));
  for (int v = 0; v < V; v++) L->cgs_ord[0][v] = v;
  int at = 0;
  for (int c = 0; c < 7; c++)
    for (int j = 0; j <= n; j++)
      for (int i = 0; i <= n; i++)
        if ((i + 2 * j) % 7 == c) L->cgs_ord[1][at++] = j * (n + 1) + i;
  at = 0;
  for (int c = 0; c < 3; c++)
    for (int j = 0; j <= n; j++)
      for (int i = 0; i <= n; i++)
        if ((i + j) % 3 == c) L->cgs_ord[2][at++] = j * (n + 1) + i;
}

static void lu_factor(int n, double *a, int *piv) {
  for (int k = 0; k < n; k++) {
    int p = k;
    double best = fabs(a[(size_t)k * n + k]);
    for (int i = k + 1; i < n; i++)
      if (fabs(a[(size_t)i * n + k]) > best) {
        best = fabs(a[(size_t)i * n + k]);
        p = i;
      }
    piv[k] = p;
    if (p != k)
      for (int c = 0; c < n; c++) {
        double t = a[(size_t)k * n + c];
        a[(size_t)k * n + c] = a[(size_t)p * n + c];
        a[(size_t)p * n + c] = t;
      }
    double d = a[(size_t)k * n + k];
    if (d == 0.0) {
      fprintf(stderr, "mgo: singular coarsest matrix\n");
      abort();
    }
    for (int i = k + 1; i < n; i++) {
      double l = a[(size_t)i * n + k] / d;
      a[(size_t)i * n + k] = l;
      for (int c = k + 1; c < n; c++) a[(size_t)i * n + c] -= l * a[(size_t)k * n + c];
    }
  }
}

static void lu_solve(int n, const double *a, const int *piv, const double *b, double *x) {
  for (int i = 0; i < n; i++) x[i] = b[i];
  for (int k = 0; k < n; k++)
    if (piv[k] != k) {
      double t = x[k];
      x[k] = x[piv[k]];
      x[piv[k]] = t;
    }
  for (int i = 0; i < n; i++)
    for (int c = 0; c < i; c++) x[i] -= a[(size_t)i * n + c] * x[c];
  for (int i = n - 1; i >= 0; i--) {
    for (int c = i + 1; c < n; c++) x[i] -= a[(size_t)i * n + c] * x[c];
    x[i] /= a[(size_t)i * n + i];
  }
}

static void level_alloc_work(mgo_level *L) {
  L->L = (double *)xcalloc(L->ndof, sizeof(double));
  L->Nd = (double *)xcalloc(L->ndof, sizeof(double));
  L->x = (double *)xcalloc(L->ndof, sizeof(double));
  L->f = (double *)xcalloc(L->ndof, sizeof(double));
  L->r = (double *)xcalloc(L->ndof, sizeof(double));
  L->p = (double *)xcalloc(L->ndof, sizeof(double));
}

static int build_level_poisson(mgo_level *L, int n, double alpha) {
  L->n = n;
  int V = (n + 1) * (n + 1);
  L->ndof = 2 * V;
  L->nfield = 2;
  L->foff[0] = 0;
  L->foff[1] = V;
  L->fkind[0] = L->fkind[1] = 0;
  L->fdim[0] = L->fdim[1] = V;
  mgo_assemble_p1(n, &L->M, &L->Klap);
  /* K = Klap + M: stiffness matrix of the bilinear form of -Laplace(y) + y */
  rowbuild b;
  rb_init(&b, V, V, 8);
  for (int r = 0; r < V; r++) {
    for (int k = L->Klap.rowptr[r]; k < L->Klap.rowptr[r + 1]; k++) rb_add(&b, r, L->Klap.col[k], L->Klap.val[k]);
    for (int k = L->M.rowptr[r]; k < L->M.rowptr[r + 1]; k++) rb_add(&b, r, L->M.col[k], L->M.val[k]);
  }
  rb_finish(&b, &L->K);
  build_kkt_poisson(L, alpha);
  level_alloc_work(L);
  build_L_poisson(L, alpha);
  build_Ndiag(L);
  build_orders_poisson(L);
  return 0;
}

/* ------------------------------------------- Stokes control (Taylor-Hood) */
/*
 * Eq. mp3 with P2 velocity (v = 0 on the boundary: interior P2 nodes only)
 * and P1 pressure on the same mesh.  P2 nodes live on the half-step lattice
 * (a, b), 0 <= a, b <= 2n, at (a h/2, b h/2): vertices at even (a, b), edge
 * midpoints elsewhere.  Unknowns [v1 | v2 | p | lambda1 | lambda2 | mu],
 * interior P2 node (a, b) -> (b-1)(2n-1) + (a-1), vertex (i, j) -> j(n+1)+i.
 * Element matrices are integrated exactly in barycentric coordinates:
 *   int_T l1^a l2^b l3^c = 2 |T| a! b! c! / (a+b+c+2)!.
 */

/* polynomial in the barycentric coordinates, total degree <= 4 */
typedef struct {
  double c[5][5][5];
} bpoly;

static void bp_zero(bpoly *p) { memset(p, 0, sizeof(*p)); }

static void bp_mul(const bpoly *x, const bpoly *y, bpoly *out) {
  bp_zero(out);
  for (int a = 0; a <= 4; a++)
    for (int b = 0; a + b <= 4; b++)
      for (int c = 0; a + b + c <= 4; c++) {
        if (x->c[a][b][c] == 0.0) continue;
        for (int d = 0; a + d <= 4; d++)
          for (int e = 0; a + b + d + e <= 4; e++)
            for (int f = 0; a + b + c + d + e + f <= 4; f++)
              out->c[a + d][b + e][c + f] += x->c[a][b][c] * y->c[d][e][f];
      }
}

/* d/d l_k */
static void bp_diff(const bpoly *x, int k, bpoly *out) {
  bp_zero(out);
  for (int a = 0; a <= 4; a++)
    for (int b = 0; a + b <= 4; b++)
      for (int c = 0; a + b + c <= 4; c++) {
        double v = x->c[a][b][c];
        if (v == 0.0) continue;
        if (k == 0 && a > 0) out->c[a - 1][b][c] += a * v;
        if (k == 1 && b > 0) out->c[a][b - 1][c] += b * v;
        if (k == 2 && c > 0) out->c[a][b][c - 1] += c * v;
      }
}

static double fact(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; i++) f *= i;
  return f;
}

static double bp_int(const bpoly *x, double area) {
  double s = 0.0;
  for (int a = 0; a <= 4; a++)
    for (int b = 0; a + b <= 4; b++)
      for (int c = 0; a + b + c <= 4; c++)
        if (x->c[a][b][c] != 0.0) s += x->c[a][b][c] * 2.0 * area * fact(a) * fact(b) * fact(c) / fact(a + b + c + 2);
  return s;
}

/* P2 basis of a triangle: local nodes 0, 1, 2 (vertices), 3 = mid(0,1),
 * 4 = mid(1,2), 5 = mid(0,2); phi_k = l_k (2 l_k - 1), phi_ij = 4 l_i l_j */
static void p2_basis(bpoly phi[6]) {
  static const int e[3][2] = {{0, 1}, {1, 2}, {0, 2}};
  for (int k = 0; k < 6; k++) bp_zero(&phi[k]);
  phi[0].c[2][0][0] = 2.0, phi[0].c[1][0][0] = -1.0;
  phi[1].c[0][2][0] = 2.0, phi[1].c[0][1][0] = -1.0;
  phi[2].c[0][0][2] = 2.0, phi[2].c[0][0][1] = -1.0;
  for (int m = 0; m < 3; m++) {
    int pw[3] = {0, 0, 0};
    pw[e[m][0]] = 1;
    pw[e[m][1]] = 1;
    phi[3 + m].c[pw[0]][pw[1]][pw[2]] = 4.0;
  }
}

/* local P2 mass, stiffness, and divergence blocks -int q_i d_x phi_j, -int q_i d_y phi_j
 * (q_i = l_i, the P1 basis) of the triangle with vertices (px, py) */
static void p2_local(const double px[3], const double py[3], double Ml[6][6], double Kl[6][6], double Dx[3][6],
                     double Dy[3][6]) {
  double area2 = (px[1] - px[0]) * (py[2] - py[0]) - (px[2] - px[0]) * (py[1] - py[0]);
  double area = 0.5 * fabs(area2);
  double gx[3], gy[3]; /* gradients of the barycentric coordinates */
  for (int i = 0; i < 3; i++) {
    int j = (i + 1) % 3, k = (i + 2) % 3;
    gx[i] = (py[j] - py[k]) / area2;
    gy[i] = (px[k] - px[j]) / area2;
  }
  bpoly phi[6], dphi[6][3], t;
  p2_basis(phi);
  for (int a = 0; a < 6; a++)
    for (int k = 0; k < 3; k++) bp_diff(&phi[a], k, &dphi[a][k]);
  for (int a = 0; a < 6; a++)
    for (int b = 0; b < 6; b++) {
      bp_mul(&phi[a], &phi[b], &t);
      Ml[a][b] = bp_int(&t, area);
      double kab = 0.0;
      for (int k = 0; k < 3; k++)
        for (int m = 0; m < 3; m++) {
          bp_mul(&dphi[a][k], &dphi[b][m], &t);
          kab += (gx[k] * gx[m] + gy[k] * gy[m]) * bp_int(&t, area);
        }
      Kl[a][b] = kab;
    }
  for (int i = 0; i < 3; i++) {
    bpoly q;
    bp_zero(&q);
    if (i == 0) q.c[1][0][0] = 1.0;
    if (i == 1) q.c[0][1][0] = 1.0;
    if (i == 2) q.c[0][0][1] = 1.0;
    for (int b = 0; b < 6; b++) {
      double sx = 0.0, sy = 0.0;
      for (int k = 0; k < 3; k++) {
        bp_mul(&q, &dphi[b][k], &t);
        double v = bp_int(&t, area);
        sx += gx[k] * v;
        sy += gy[k] * v;
      }
      Dx[i][b] = -sx;
      Dy[i][b] = -sy;
    }
  }
}

/* half-lattice coordinates of the 6 P2 nodes of triangle t of square (i, j) */
static void p2_tri_nodes(int i, int j, int t, int na[6], int nb[6], int vi[3], int vj[3]) {
  square_triangles(i, j, t, vi, vj);
  for (int k = 0; k < 3; k++) {
    na[k] = 2 * vi[k];
    nb[k] = 2 * vj[k];
  }
  static const int e[3][2] = {{0, 1}, {1, 2}, {0, 2}};
  for (int m = 0; m < 3; m++) {
    na[3 + m] = vi[e[m][0]] + vi[e[m][1]];
    nb[3 + m] = vj[e[m][0]] + vj[e[m][1]];
  }
}

/* P2 node index: interior numbering (full = 0, boundary -> -1) or all (2n+1)^2 nodes */
static int p2_index(int n, int a, int b, int full) {
  if (full) return b * (2 * n + 1) + a;
  if (a < 1 || b < 1 || a > 2 * n - 1 || b > 2 * n - 1) return -1;
  return (b - 1) * (2 * n - 1) + (a - 1);
}

void mgo_assemble_p2(int n, int full, mgo_csr *M, mgo_csr *K, mgo_csr *D1, mgo_csr *D2) {
  int nv = full ? (2 * n + 1) * (2 * n + 1) : (2 * n - 1) * (2 * n - 1);
  int np = (n + 1) * (n + 1);
  double h = 1.0 / n;
  rowbuild bm, bk, b1, b2;
  rb_init(&bm, nv, nv, 25);
  rb_init(&bk, nv, nv, 25);
  rb_init(&b1, np, nv, 32);
  rb_init(&b2, np, nv, 32);
  for (int j = 0; j < n; j++)
    for (int i = 0; i < n; i++)
      for (int t = 0; t < 2; t++) {
        int na[6], nb[6], vi[3], vj[3];
        p2_tri_nodes(i, j, t, na, nb, vi, vj);
        double px[3], py[3];
        for (int k = 0; k < 3; k++) {
          px[k] = vi[k] * h;
          py[k] = vj[k] * h;
        }
        double Ml[6][6], Kl[6][6], Dx[3][6], Dy[3][6];
        p2_local(px, py, Ml, Kl, Dx, Dy);
        int g[6];
        for (int a = 0; a < 6; a++) g[a] = p2_index(n, na[a], nb[a], full);
        for (int a = 0; a < 6; a++) {
          if (g[a] < 0) continue;
          for (int b = 0; b < 6; b++) {
            if (g[b] < 0) continue;
            rb_add(&bm, g[a], g[b], Ml[a][b]);
            rb_add(&bk, g[a], g[b], Kl[a][b]);
          }
        }
        for (int q = 0; q < 3; q++) {
          int vq = vj[q] * (n + 1) + vi[q];
          for (int b = 0; b < 6; b++) {
            if (g[b] < 0) continue;
            rb_add(&b1, vq, g[b], Dx[q][b]);
            rb_add(&b2, vq, g[b], Dy[q][b]);
          }
        }
      }
  rb_finish(&bm, M);
  rb_finish(&bk, K);
  rb_finish(&b1, D1);
  rb_finish(&b2, D2);
}

/* P2 interpolation of the coarse P2 space (nc cells per side) at the fine P2
 * nodes (2 nc cells per side): the coarse basis functions evaluated at each
 * fine node.  Interior nodes only (full = 0) or all nodes. */
void mgo_prolongation_p2(int nc, int full, mgo_csr *P) {
  int nf = 2 * nc;
  int nrow = full ? (2 * nf + 1) * (2 * nf + 1) : (2 * nf - 1) * (2 * nf - 1);
  int ncol = full ? (2 * nc + 1) * (2 * nc + 1) : (2 * nc - 1) * (2 * nc - 1);
  rowbuild b;
  rb_init(&b, nrow, ncol, 6);
  double hc = 1.0 / nc;
  bpoly phi[6];
  p2_basis(phi);
  for (int fb = 0; fb <= 2 * nf; fb++)
    for (int fa = 0; fa <= 2 * nf; fa++) {
      int row = p2_index(nf, fa, fb, full);
      if (row < 0) continue;
      double X = fa / (2.0 * nf), Y = fb / (2.0 * nf);
      int i = (int)floor(X / hc), j = (int)floor(Y / hc);
      if (i > nc - 1) i = nc - 1;
      if (j > nc - 1) j = nc - 1;
      /* the "/" diagonal splits the square into x - i hc >= y - j hc (t = 0) and the rest */
      int t = (X - i * hc >= Y - j * hc) ? 0 : 1;
      int na[6], nb[6], vi[3], vj[3];
      p2_tri_nodes(i, j, t, na, nb, vi, vj);
      double px[3], py[3], lam[3];
      for (int k = 0; k < 3; k++) {
        px[k] = vi[k] * hc;
        py[k] = vj[k] * hc;
      }
      barycentric(px, py, X, Y, lam);
      for (int a = 0; a < 6; a++) {
        int col = p2_index(nc, na[a], nb[a], full);
        if (col < 0) continue;
        double w = 0.0;
        for (int aa = 0; aa <= 2; aa++)
          for (int bb = 0; aa + bb <= 2; bb++)
            for (int cc = 0; aa + bb + cc <= 2; cc++)
              if (phi[a].c[aa][bb][cc] != 0.0)
                w += phi[a].c[aa][bb][cc] * pow(lam[0], aa) * pow(lam[1], bb) * pow(lam[2], cc);
        if (fabs(w) > 1e-12) rb_add(&b, row, col, w);
      }
    }
  rb_finish(&b, P);
}

/* eq. mp3: rows/columns [v1 | v2 | p | lambda1 | lambda2 | mu] */
static void build_kkt_stokes(mgo_level *L, double alpha) {
  int nv = L->nv, np = L->np;
  int ov[2] = {0, nv}, op = 2 * nv, ol[2] = {2 * nv + np, 3 * nv + np}, om = 4 * nv + np;
  rowbuild b;
  rb_init(&b, L->ndof, L->ndof, 64);
  const mgo_csr *D[2] = {&L->D1, &L->D2};
  for (int c = 0; c < 2; c++) {
    for (int r = 0; r < nv; r++) {
      for (int k = L->M.rowptr[r]; k < L->M.rowptr[r + 1]; k++) {
        int cc = L->M.col[k];
        double m = L->M.val[k];
        rb_add(&b, ov[c] + r, ov[c] + cc, m);          /* M v            */
        rb_add(&b, ol[c] + r, ol[c] + cc, -m / alpha); /* -alpha^-1 M lambda */
      }
      for (int k = L->Klap.rowptr[r]; k < L->Klap.rowptr[r + 1]; k++) {
        int cc = L->Klap.col[k];
        rb_add(&b, ov[c] + r, ol[c] + cc, L->Klap.val[k]); /* K lambda */
        rb_add(&b, ol[c] + r, ov[c] + cc, L->Klap.val[k]); /* K v      */
      }
    }
    for (int q = 0; q < np; q++)
      for (int k = D[c]->rowptr[q]; k < D[c]->rowptr[q + 1]; k++) {
        int a = D[c]->col[k];
        double d = D[c]->val[k];
        rb_add(&b, op + q, ol[c] + a, d); /* D lambda   */
        rb_add(&b, om + q, ov[c] + a, d); /* D v        */
        rb_add(&b, ov[c] + a, om + q, d); /* D^T mu     */
        rb_add(&b, ol[c] + a, op + q, d); /* D^T p      */
      }
  }
  rb_finish(&b, &L->A);
  mgo_transpose(&L->A, &L->At);
}

/* L_k = blockdiag(W^, W^, P^, W^/alpha, W^/alpha, P^/alpha) with
 * W^ = diag(M + alpha^{1/2} K) and P^ = alpha diag(D W^-1 D^T) (section 2) */
static void build_L_stokes(mgo_level *L, double alpha) {
  int nv = L->nv, np = L->np;
  double *W = (double *)xmalloc((size_t)nv * sizeof(double));
  for (int a = 0; a < nv; a++) W[a] = csr_entry(&L->M, a, a) + sqrt(alpha) * csr_entry(&L->Klap, a, a);
  for (int a = 0; a < nv; a++) {
    L->L[a] = L->L[nv + a] = W[a];
    L->L[2 * nv + np + a] = L->L[3 * nv + np + a] = W[a] / alpha;
  }
  for (int q = 0; q < np; q++) {
    double s = 0.0;
    for (int k = L->D1.rowptr[q]; k < L->D1.rowptr[q + 1]; k++) s += L->D1.val[k] * L->D1.val[k] / W[L->D1.col[k]];
    for (int k = L->D2.rowptr[q]; k < L->D2.rowptr[q + 1]; k++) s += L->D2.val[k] * L->D2.val[k] / W[L->D2.col[k]];
    L->L[2 * nv + q] = alpha * s;
    L->L[4 * nv + np + q] = s;
  }
  free(W);
}

/* Orderings of Alg. 2 for Stokes.  LEX: every unknown in index order.
 * COL7 (the GPU order): for velocity component c = 1, 2 and the 25 colours
 * (a mod 5) + 5 (b mod 5) of the interior P2 nodes, groups {v_c, lambda_c} of
 * one node; then for the 9 colours (i mod 3) + 3 (j mod 3) of the vertices,
 * groups {p, mu} of one vertex.  COL7SEQ: the same with one unknown per group. */
static void build_orders_stokes(mgo_level *L) {
  int n = L->n, nv = L->nv, np = L->np, N = L->ndof, m = 2 * n - 1;
  for (int o = 0; o < 4; o++) {
    L->ord[o] = (int *)xmalloc((size_t)N * sizeof(int));
    L->gptr[o] = (int *)xmalloc(((size_t)N + 1) * sizeof(int));
  }
  for (int o = 0; o < 4; o += 3) { /* LEX and VLEX */
    for (int i = 0; i < N; i++) L->ord[o][i] = L->gptr[o][i] = i;
    L->gptr[o][N] = N;
    L->ngroup[o] = N;
  }
  for (int o = 1; o <= 2; o++) {
    int at = 0, g = 0;
    for (int c = 0; c < 2; c++)
      for (int col = 0; col < 25; col++)
        for (int b = 1; b <= m; b++)
          for (int a = 1; a <= m; a++) {
            if ((a % 5) + 5 * (b % 5) != col) continue;
            int node = (b - 1) * m + (a - 1);
            int iv = c * nv + node, il = 2 * nv + np + c * nv + node;
            L->gptr[o][g++] = at;
            L->ord[o][at++] = iv;
            if (o == 2) L->gptr[o][g++] = at;
            L->ord[o][at++] = il;
          }
    for (int col = 0; col < 9; col++)
      for (int j = 0; j <= n; j++)
        for (int i = 0; i <= n; i++) {
          if ((i % 3) + 3 * (j % 3) != col) continue;
          int q = j * (n + 1) + i;
          L->gptr[o][g++] = at;
          L->ord[o][at++] = 2 * nv + q;
          if (o == 2) L->gptr[o][g++] = at;
          L->ord[o][at++] = 4 * nv + np + q;
        }
    L->gptr[o][g] = at;
    L->ngroup[o] = g;
  }
}

/* Vanka patches (section 2, Stokes): for vertex (i, j) its p and mu, and
 * v1, v2, lambda1, lambda2 at the P2 node of the vertex and at the midpoints
 * of the (up to 6) mesh edges ending at it, where those nodes are interior
 * (two corners, whose edges all lie on the boundary, take the interior nodes
 * of their triangles instead).
 * Patch orders: lexicographic vertices, or 9 colours (i mod 3) + 3 (j mod 3). */
static void build_patches_stokes(mgo_level *L) {
  int n = L->n, nv = L->nv, np = L->np, m = 2 * n - 1;
  static const int di[7] = {0, 1, -1, 0, 0, 1, -1}, dj[7] = {0, 0, 0, 1, -1, 1, -1};
  L->patch_ptr = (int *)xmalloc(((size_t)np + 1) * sizeof(int));
  L->patch_dof = (int *)xmalloc((size_t)np * 30 * sizeof(int));
  int at = 0;
  for (int j = 0; j <= n; j++)
    for (int i = 0; i <= n; i++) {
      int q = j * (n + 1) + i;
      L->patch_ptr[q] = at;
      L->patch_dof[at++] = 2 * nv + q;
      L->patch_dof[at++] = 4 * nv + np + q;
      for (int d = 0; d < 7; d++) {
        int ii = i + di[d], jj = j + dj[d];
        if (ii < 0 || jj < 0 || ii > n || jj > n) continue;
        int a = i + ii, b = j + jj; /* vertex node (d = 0) or edge midpoint, half-lattice */
        if (a < 1 || b < 1 || a > m || b > m) continue;
        int node = (b - 1) * m + (a - 1);
        L->patch_dof[at++] = node;
        L->patch_dof[at++] = nv + node;
        L->patch_dof[at++] = 2 * nv + np + node;
        L->patch_dof[at++] = 3 * nv + np + node;
      }
      if (at - L->patch_ptr[q] == 2) {
        /* every edge at this vertex lies on the boundary (the corners (n, 0)
         * and (0, n)): the patch takes the interior P2 nodes of the triangles
         * that contain the vertex instead, so that its matrix is regular */
        for (int sj = j - 1; sj <= j; sj++)
          for (int si = i - 1; si <= i; si++) {
            if (si < 0 || sj < 0 || si >= n || sj >= n) continue;
            for (int t = 0; t < 2; t++) {
              int na[6], nb[6], vi[3], vj[3];
              p2_tri_nodes(si, sj, t, na, nb, vi, vj);
              int has = 0;
              for (int k = 0; k < 3; k++) has |= (vi[k] == i && vj[k] == j);
              if (!has) continue;
              for (int k = 0; k < 6; k++) {
                if (na[k] < 1 || nb[k] < 1 || na[k] > m || nb[k] > m) continue;
                int node = (nb[k] - 1) * m + (na[k] - 1), dup = 0;
                for (int u = L->patch_ptr[q]; u < at; u++) dup |= L->patch_dof[u] == node;
                if (dup) continue;
                L->patch_dof[at++] = node;
                L->patch_dof[at++] = nv + node;
                L->patch_dof[at++] = 2 * nv + np + node;
                L->patch_dof[at++] = 3 * nv + np + node;
              }
            }
          }
      }
    }
  L->patch_ptr[np] = at;
  L->vanka_ord[0] = (int *)xmalloc((size_t)np * sizeof(int));
  L->vanka_ord[1] = (int *)xmalloc((size_t)np * sizeof(int));
  for (int q = 0; q < np; q++) L->vanka_ord[0][q] = q;
  int k = 0;
  for (int col = 0; col < 9; col++)
    for (int j = 0; j <= n; j++)
      for (int i = 0; i <= n; i++)
        if ((i % 3) + 3 * (j % 3) == col) L->vanka_ord[1][k++] = j * (n + 1) + i;
}

static int build_level_stokes(mgo_level *L, int n, double alpha) {
  L->n = n;
  L->nv = (2 * n - 1) * (2 * n - 1);
  L->np = (n + 1) * (n + 1);
  int nv = L->nv, np = L->np;
  L->ndof = 4 * nv + 2 * np;
  L->nfield = 6;
  int off[6] = {0, nv, 2 * nv, 2 * nv + np, 3 * nv + np, 4 * nv + np};
  int kind[6] = {0, 0, 1, 0, 0, 1};
  for (int fl = 0; fl < 6; fl++) {
    L->foff[fl] = off[fl];
    L->fkind[fl] = kind[fl];
    L->fdim[fl] = kind[fl] ? np : nv;
  }
  /* scalar P2 mass (M) and Laplacian stiffness (Klap), divergence blocks,
   * and the P1 pressure mass (Mp) for the mean-value constraint */
  mgo_assemble_p2(n, 0, &L->M, &L->Klap, &L->D1, &L->D2);
  mgo_csr Kp1;
  mgo_assemble_p1(n, &L->Mp, &Kp1);
  mgo_csr_free(&Kp1);
  {
    /* B = [D1 D2] (np x 2 nv), for inspection */
    rowbuild b;
    rb_init(&b, np, 2 * nv, 48);
    for (int q = 0; q < np; q++) {
      for (int k = L->D1.rowptr[q]; k < L->D1.rowptr[q + 1]; k++) rb_add(&b, q, L->D1.col[k], L->D1.val[k]);
      for (int k = L->D2.rowptr[q]; k < L->D2.rowptr[q + 1]; k++) rb_add(&b, q, nv + L->D2.col[k], L->D2.val[k]);
    }
    rb_finish(&b, &L->B);
  }
  build_kkt_stokes(L, alpha);
  level_alloc_work(L);
  build_L_stokes(L, alpha);
  build_Ndiag(L);
  build_orders_stokes(L);
  build_patches_stokes(L);
  return 0;
}

/* weights of the pressure mean: w = Mp 1 (int of each P1 basis function) */
static void pressure_weights(const mgo_level *L, double *w) {
  for (int q = 0; q < L->np; q++) {
    double s = 0.0;
    for (int k = L->Mp.rowptr[q]; k < L->Mp.rowptr[q + 1]; k++) s += L->Mp.val[k];
    w[q] = s;
  }
}

/* p and mu with zero mean: v -= (w^T v / w^T 1) 1 */
static void project_means(const mgo_level *L, double *x) {
  double *w = (double *)xmalloc((size_t)L->np * sizeof(double));
  pressure_weights(L, w);
  double ww = 0.0;
  for (int q = 0; q < L->np; q++) ww += w[q];
  int offs[2] = {2 * L->nv, 4 * L->nv + L->np};
  for (int t = 0; t < 2; t++) {
    double s = 0.0;
    for (int q = 0; q < L->np; q++) s += w[q] * x[offs[t] + q];
    double c = s / ww;
    for (int q = 0; q < L->np; q++) x[offs[t] + q] -= c;
  }
  free(w);
}

/* ------------------------------------------------------ create / destroy */

mgo_hier *mgo_create(int problem, int fine, int coarse, double alpha) {
  if (problem != 0 && problem != 1) return NULL;
  if (!(alpha > 0.0) || !isfinite(alpha) || coarse < 1 || fine < coarse + 1 || fine > 12) return NULL;
  mgo_hier *h = (mgo_hier *)xcalloc(1, sizeof(mgo_hier));
  h->problem = problem;
  h->fine = fine;
  h->coarse = coarse;
  h->alpha = alpha;
  h->lv = (mgo_level *)xcalloc((size_t)fine + 1, sizeof(mgo_level));
  for (int l = coarse; l <= fine; l++) {
    mgo_level *L = &h->lv[l];
    if (problem == 0) {
      build_level_poisson(L, 1 << l, alpha);
    } else {
      build_level_stokes(L, 1 << l, alpha);
    }
    if (l > coarse) {
      if (problem == 0) {
        mgo_prolongation_p1(1 << (l - 1), &L->Pk[0]);
        mgo_transpose(&L->Pk[0], &L->Rk[0]); /* restriction = transpose, scale 1 */
      } else {
        mgo_prolongation_p2(1 << (l - 1), 0, &L->Pk[0]);
        mgo_transpose(&L->Pk[0], &L->Rk[0]);
        mgo_prolongation_p1(1 << (l - 1), &L->Pk[1]);
        mgo_transpose(&L->Pk[1], &L->Rk[1]);
      }
    }
  }
  /* coarsest level: dense LU with partial pivoting of A_{k0}; for Stokes of
   * [[A, C], [C^T, 0]] with C = the pressure-mean weights in the p and mu rows,
   * which removes the constant pressures from the kernel of A */
  mgo_level *C = &h->lv[coarse];
  int N = C->ndof, NB = problem == 0 ? N : N + 2;
  C->nlu = NB;
  C->lu = (double *)xcalloc((size_t)NB * NB, sizeof(double));
  C->piv = (int *)xcalloc(NB, sizeof(int));
  for (int r = 0; r < N; r++)
    for (int k = C->A.rowptr[r]; k < C->A.rowptr[r + 1]; k++) C->lu[(size_t)r * NB + C->A.col[k]] = C->A.val[k];
  if (problem == 1) {
    double *w = (double *)xmalloc((size_t)C->np * sizeof(double));
    pressure_weights(C, w);
    int offs[2] = {2 * C->nv, 4 * C->nv + C->np};
    for (int t = 0; t < 2; t++)
      for (int q = 0; q < C->np; q++) {
        C->lu[(size_t)(offs[t] + q) * NB + N + t] = w[q];
        C->lu[(size_t)(N + t) * NB + offs[t] + q] = w[q];
      }
    free(w);
  }
  lu_factor(NB, C->lu, C->piv);
  return h;
}

static void level_free(mgo_level *L) {
  mgo_csr_free(&L->M);
  mgo_csr_free(&L->Klap);
  mgo_csr_free(&L->K);
  mgo_csr_free(&L->A);
  mgo_csr_free(&L->At);
  for (int k = 0; k < 2; k++) {
    mgo_csr_free(&L->Pk[k]);
    mgo_csr_free(&L->Rk[k]);
  }
  mgo_csr_free(&L->B);
  mgo_csr_free(&L->Mp);
  free(L->L);
  free(L->Nd);
  free(L->x);
  free(L->f);
  free(L->r);
  free(L->p);
  for (int o = 0; o < 4; o++) {
    free(L->ord[o]);
    free(L->gptr[o]);
  }
  for (int o = 0; o < 3; o++) free(L->cgs_ord[o]);
  free(L->lu);
  free(L->piv);
  mgo_csr_free(&L->D1);
  mgo_csr_free(&L->D2);
  free(L->patch_ptr);
  free(L->patch_dof);
  free(L->vanka_ord[0]);
  free(L->vanka_ord[1]);
}

void mgo_destroy(mgo_hier *h) {
  if (!h) return;
  for (int l = h->coarse; l <= h->fine; l++) level_free(&h->lv[l]);
  free(h->lv);
  free(h);
}

int mgo_ndof(const mgo_hier *h, int level) {
  if (!h || level < h->coarse || level > h->fine) return -1;
  return h->lv[level].ndof;
}

int mgo_get_matrix(const mgo_hier *h, int level, int which, int *nrows, int *ncols, int *nnz, int *rowptr,
                   int *col, double *val) {
  if (!h || level < h->coarse || level > h->fine) return -1;
  const mgo_level *L = &h->lv[level];
  const mgo_csr *A = NULL;
  switch (which) {
    case 0: A = &L->A; break;
    case 1: A = &L->M; break;
    case 2: A = &L->Klap; break;
    case 3: A = level > h->coarse ? &L->Pk[0] : NULL; break;
    case 4: A = &L->B; break;
    case 5: A = &L->Mp; break;
    case 6: A = level > h->coarse ? &L->Pk[1] : NULL; break;
    default: return -1;
  }
  if (!A || !A->rowptr) return -1;
  *nrows = A->nrows;
  *ncols = A->ncols;
  *nnz = A->nnz;
  if (rowptr) {
    memcpy(rowptr, A->rowptr, ((size_t)A->nrows + 1) * sizeof(int));
    memcpy(col, A->col, (size_t)A->nnz * sizeof(int));
    memcpy(val, A->val, (size_t)A->nnz * sizeof(double));
  }
  return A->nrows;
}

int mgo_get_diag(const mgo_hier *h, int level, int which, double *out) {
  if (!h || level < h->coarse || level > h->fine) return -1;
  const mgo_level *L = &h->lv[level];
  memcpy(out, which == 0 ? L->L : L->Nd, (size_t)L->ndof * sizeof(double));
  return L->ndof;
}

/* ------------------------------------------------------------ operators */

void mgo_residual(const mgo_hier *h, int level, const double *f, const double *x, double *r) {
  const mgo_level *L = &h->lv[level];
  csr_mv(&L->A, x, r);
#pragma omp parallel for schedule(static)
  for (int i = 0; i < L->ndof; i++) r[i] = f[i] - r[i];
}

/* Normal-equation smoother (section 2): the damped Richardson step on the
 * normal equation A^T L^-1 A x = A^T L^-1 f with the preconditioner L,
 *   x <- x + tau L^-1 A^T L^-1 (f - A x),
 * written with whole-vector products: s = L^-1 r, t = A^T s, p = tau L^-1 t,
 * then x += p and r -= A p, so that r stays f - A x (the cost unit of Alg. 1:
 * one product with A^T and one with A per step). */
static void ne_step(const mgo_level *L, double tau, double *x, double *r) {
  int n = L->ndof;
  double *s = (double *)xmalloc((size_t)n * sizeof(double));
  double *t = (double *)xmalloc((size_t)n * sizeof(double));
  double *p = L->p;
  for (int i = 0; i < n; i++) s[i] = r[i] / L->L[i];
  csr_mv(&L->At, s, t);
  for (int i = 0; i < n; i++) p[i] = tau * t[i] / L->L[i];
  csr_mv(&L->A, p, t);
  for (int i = 0; i < n; i++) {
    x[i] += p[i];
    r[i] -= t[i];
  }
  free(s);
  free(t);
}

/* Least-squares Gauss-Seidel (section 2): Gauss-Seidel on the normal
 * equation N x = A^T L^-1 f, N = A^T L^-1 A, i.e. exact coordinate descent on
 * the functional 1/2 ||f - A x||^2_{L^-1}.  Along coordinate i (column a_i of
 * A, stored as row i of A^T) the functional is minimised by the step
 *   p = a_i^T L^-1 r / N_ii,  N_ii = a_i^T L^-1 a_i,
 * after which x_i += p and r -= p a_i.  The coordinates are taken in the
 * order `ord`; the coordinates of one group are stepped from the same
 * residual, which equals stepping them one after the other exactly when
 * their mutual entries of N vanish (the pair {y_v, lambda_v} in the Poisson
 * problem, a velocity component and its multiplier at one node or p and mu
 * at one vertex in the Stokes problem). */
static void lsgs_group(const mgo_level *L, const int *ord, const int *gptr, int g, double *x, double *r) {
  const mgo_csr *At = &L->At;
  double step[8];
  int first = gptr[g], count = gptr[g + 1] - gptr[g];
  /* the steps of the group, all from the current residual */
  for (int u = 0; u < count; u++) {
    int i = ord[first + u];
    double dot = 0.0;
    for (int k = At->rowptr[i]; k < At->rowptr[i + 1]; k++) dot += At->val[k] * (r[At->col[k]] / L->L[At->col[k]]);
    step[u] = dot / L->Nd[i];
  }
  /* then the coordinate moves and the residual update r -= p a_i */
  for (int u = 0; u < count; u++) {
    int i = ord[first + u];
    x[i] += step[u];
    for (int k = At->rowptr[i]; k < At->rowptr[i + 1]; k++) r[At->col[k]] -= step[u] * At->val[k];
  }
}

static void lsgs_groups(const mgo_level *L, const int *ord, const int *gptr, int ngroup, int reverse, double *x,
                        double *r) {
  for (int gg = 0; gg < ngroup; gg++) lsgs_group(L, ord, gptr, reverse ? ngroup - 1 - gg : gg, x, r);
}

/* the COL7 order colour by colour: the groups of one colour touch disjoint
 * residual entries, so they may be stepped in any order, or concurrently (the
 * threaded build of the oracle runs them with OpenMP; the result is the same
 * bit for bit) */
static void lsgs_colours(const mgo_level *L, int reverse, double *x, double *r) {
  const int *ord = L->ord[MGO_ORDER_COL7], *gptr = L->gptr[MGO_ORDER_COL7];
  for (int cc = 0; cc < L->ncolour; cc++) {
    int c = reverse ? L->ncolour - 1 - cc : cc;
#pragma omp parallel for schedule(static)
    for (int g = L->cptr[c]; g < L->cptr[c + 1]; g++) lsgs_group(L, ord, gptr, g, x, r);
  }
}

/* Collective Gauss-Seidel (point smoother): for each vertex v solve the 2x2
 * system of the unknowns (y_v, lambda_v) with the residual, update x, r. */
static void cgs_step(const mgo_level *L, const int *vord, int nvert, double *x, double *r) {
  const mgo_csr *A = &L->A, *At = &L->At;
  int V = nvert;
  for (int a = 0; a < nvert; a++) {
    int v = vord[a];
    int iy = v, il = V + v;
    double b11 = csr_entry(A, iy, iy), b12 = csr_entry(A, iy, il);
    double b21 = csr_entry(A, il, iy), b22 = csr_entry(A, il, il);
    double det = b11 * b22 - b12 * b21;
    double dy = (b22 * r[iy] - b12 * r[il]) / det;
    double dl = (b11 * r[il] - b21 * r[iy]) / det;
    x[iy] += dy;
    x[il] += dl;
    for (int k = At->rowptr[iy]; k < At->rowptr[iy + 1]; k++) r[At->col[k]] -= At->val[k] * dy;
    for (int k = At->rowptr[il]; k < At->rowptr[il + 1]; k++) r[At->col[k]] -= At->val[k] * dl;
  }
}

/* Patch (Vanka-type) smoother for Stokes (section 2): for each patch P_i in
 * turn, x += tau P_i (P_i^T A P_i)^{-1} P_i^T r, r -= tau A P_i (...)
 * (multiplicative, damped). */
static void vanka_step(const mgo_level *L, const int *vord, double tau, double *x, double *r) {
  const mgo_csr *A = &L->A, *At = &L->At;
  double a[30 * 30], rl[30], d[30];
  int piv[30];
  for (int t = 0; t < L->np; t++) {
    int q = vord[t];
    int b = L->patch_ptr[q], e = L->patch_ptr[q + 1], m = e - b;
    const int *dof = L->patch_dof + b;
    for (int u = 0; u < m; u++) {
      rl[u] = r[dof[u]];
      for (int w = 0; w < m; w++) a[u * m + w] = csr_entry(A, dof[u], dof[w]);
    }
    lu_factor(m, a, piv);
    lu_solve(m, a, piv, rl, d);
    for (int u = 0; u < m; u++) {
      double du = tau * d[u];
      x[dof[u]] += du;
      for (int k = At->rowptr[dof[u]]; k < At->rowptr[dof[u] + 1]; k++) r[At->col[k]] -= At->val[k] * du;
    }
  }
}

void mgo_smooth(const mgo_hier *h, int level, int kind, int order, double tau, double *x, double *r) {
  const mgo_level *L = &h->lv[level];
  if (order < 0 || order > 4) order = 0;
  switch (kind) {
    case MGO_NE: ne_step(L, tau, x, r); break;
    case MGO_LSGS:
      if (order == MGO_ORDER_COL3) order = MGO_ORDER_COL7;
      if (order == MGO_ORDER_COL7 && L->ncolour) {
        lsgs_colours(L, 0, x, r);
        break;
      }
      lsgs_groups(L, L->ord[order], L->gptr[order], L->ngroup[order], 0, x, r);
      break;
    case MGO_SLSGS:
      if (order == MGO_ORDER_COL3) order = MGO_ORDER_COL7;
      if (order == MGO_ORDER_COL7 && L->ncolour) {
        lsgs_colours(L, 0, x, r);
        lsgs_colours(L, 1, x, r);
        break;
      }
      lsgs_groups(L, L->ord[order], L->gptr[order], L->ngroup[order], 0, x, r);
      lsgs_groups(L, L->ord[order], L->gptr[order], L->ngroup[order], 1, x, r);
      break;
    case MGO_VANKA:
      if (L->patch_ptr) vanka_step(L, L->vanka_ord[order == MGO_ORDER_LEX ? 0 : 1], tau, x, r);
      break;
    case MGO_CGS: {
      if (!L->cgs_ord[0]) break; /* Poisson only */
      int which = 0; /* lexicographic for MGO_ORDER_LEX and MGO_ORDER_VLEX */
      if (order == MGO_ORDER_COL7 || order == MGO_ORDER_COL7SEQ) which = 1;
      if (order == MGO_ORDER_COL3) which = 2;
      cgs_step(L, L->cgs_ord[which], L->ncgs, x, r);
      break;
    }
    default: break;
  }
}

void mgo_smooth_groups(const mgo_hier *h, int level, const int *ord, const int *gptr, int ngroup, int reverse,
                       double *x, double *r) {
  lsgs_groups(&h->lv[level], ord, gptr, ngroup, reverse, x, r);
}

void mgo_coarse_solve(const mgo_hier *h, const double *f, double *x) {
  const mgo_level *C = &h->lv[h->coarse];
  if (C->nlu == C->ndof) {
    lu_solve(C->ndof, C->lu, C->piv, f, x);
    return;
  }
  /* bordered system: right-hand side (f; 0, 0), solution (x; multipliers) */
  double *fb = (double *)xcalloc(C->nlu, sizeof(double)), *xb = (double *)xcalloc(C->nlu, sizeof(double));
  memcpy(fb, f, (size_t)C->ndof * sizeof(double));
  lu_solve(C->nlu, C->lu, C->piv, fb, xb);
  memcpy(x, xb, (size_t)C->ndof * sizeof(double));
  free(fb);
  free(xb);
}

/* fine-level field-wise transfers: restriction with P^T, prolongation with P */
static void restrict_to(const mgo_level *Lf, const mgo_level *Lc, const double *rf, double *fc) {
  for (int fl = 0; fl < Lf->nfield; fl++) {
    const mgo_csr *R = &Lf->Rk[Lf->fkind[fl]];
    csr_mv(R, rf + Lf->foff[fl], fc + Lc->foff[fl]);
  }
}

static void prolong_add(const mgo_level *Lf, const mgo_level *Lc, const double *xc, double *xf) {
  for (int fl = 0; fl < Lf->nfield; fl++) {
    const mgo_csr *P = &Lf->Pk[Lf->fkind[fl]];
    const double *src = xc + Lc->foff[fl];
    double *dst = xf + Lf->foff[fl];
#pragma omp parallel for schedule(static)
    for (int rr = 0; rr < P->nrows; rr++) {
      double s = 0.0;
      for (int k = P->rowptr[rr]; k < P->rowptr[rr + 1]; k++) s += P->val[k] * src[P->col[k]];
      dst[rr] += s;
    }
  }
}

/* One multigrid iterate (section 2): nu1 smoothing steps, defect, restriction,
 * gamma recursive iterates on the coarse-grid problem from zero (exact solve on
 * the coarsest level), prolongation and correction, nu2 smoothing steps. */
static void cycle_rec(const mgo_hier *h, int l, int kind, int order, double tau, int nu1, int nu2, int gamma,
                      const double *f, double *x) {
  const mgo_level *L = &h->lv[l];
  if (l == h->coarse) {
    mgo_coarse_solve(h, f, x);
    return;
  }
  double *r = L->r;
  mgo_residual(h, l, f, x, r);
  for (int s = 0; s < nu1; s++) mgo_smooth(h, l, kind, order, tau, x, r);
  const mgo_level *C = &h->lv[l - 1];
  restrict_to(L, C, r, C->f);
  memset(C->x, 0, (size_t)C->ndof * sizeof(double));
  for (int g = 0; g < gamma; g++) cycle_rec(h, l - 1, kind, order, tau, nu1, nu2, gamma, C->f, C->x);
  prolong_add(L, C, C->x, x);
  mgo_residual(h, l, f, x, r);
  for (int s = 0; s < nu2; s++) mgo_smooth(h, l, kind, order, tau, x, r);
}

/* a cycle on the finest level of the call; for Stokes the pressure p and
 * the multiplier mu are then shifted to zero mean (the constants span the
 * kernel of A_k and leave every residual unchanged) */
static void top_cycle(const mgo_hier *h, int level, int kind, int order, double tau, int nu1, int nu2, int gamma,
                      const double *f, double *x) {
  cycle_rec(h, level, kind, order, tau, nu1, nu2, gamma, f, x);
  if (h->problem == 1) project_means(&h->lv[level], x);
}

void mgo_cycle(const mgo_hier *h, int level, int kind, int order, double tau, int nu1, int nu2, int gamma,
               const double *f, double *x) {
  top_cycle(h, level, kind, order, tau, nu1, nu2, gamma, f, x);
}

void mgo_project(const mgo_hier *h, int level, double *x) {
  if (h->problem == 1) project_means(&h->lv[level], x);
}

static double norm2(const double *v, int n) {
  double s = 0.0;
  for (int i = 0; i < n; i++) s += v[i] * v[i];
  return sqrt(s);
}

/* Euclidean norm (norm = 0) or (v^T L_k^{-1} v)^{1/2} (norm = 1) */
static double normL(const mgo_level *L, const double *v, int norm) {
  if (norm == 0) return norm2(v, L->ndof);
  double s = 0.0;
  for (int i = 0; i < L->ndof; i++) s += v[i] * v[i] / L->L[i];
  return sqrt(s);
}

int mgo_solve(const mgo_hier *h, int kind, int order, double tau, int nu1, int nu2, int gamma, const double *f,
              double *x, double tol, int max_cycles, int norm, double *hist) {
  const mgo_level *L = &h->lv[h->fine];
  double *r = (double *)xmalloc((size_t)L->ndof * sizeof(double));
  double nf = normL(L, f, norm);
  if (nf == 0.0) nf = 1.0;
  int it = 0;
  for (;; it++) {
    mgo_residual(h, h->fine, f, x, r);
    double rel = normL(L, r, norm) / nf;
    if (hist) hist[it] = rel;
    if (rel <= tol) break;
    if (it == max_cycles) {
      it = -1;
      break;
    }
    top_cycle(h, h->fine, kind, order, tau, nu1, nu2, gamma, f, x);
  }
  free(r);
  return it;
}
