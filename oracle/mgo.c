/*
 * mgo.c -- FP64 CPU oracle for the all-at-once multigrid method of Takacs,
 * arXiv 1502.03917.  TEST INFRASTRUCTURE ONLY: used by the tests, the smoke
 * check and the CPU-baseline leg of the benchmark, never by the product path.
 *
 * Plain, slow, obviously correct: matrices are assembled element by element
 * into CSR, the smoothers walk the sparse rows exactly as the paper's
 * algorithms describe, and the coarsest level is solved by dense LU.
 * The Poisson-control parts are pinned by the tests in tests/test_oracle_*.py;
 * see the header mgo.h for the discretisation readings.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mgo.h"

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
  int *cgs_ord[3]; /* vertex orders for the collective smoother: lex, col7, col3 */
  int ncgs;
  /* coarsest level only: dense LU with partial pivoting */
  double *lu;
  int *piv;
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

/* N_ii = sum_j A_ij^2 / L_jj (Alg. 2, prepared once) */
static void build_Ndiag(mgo_level *L) {
  for (int i = 0; i < L->ndof; i++) {
    double s = 0.0;
    for (int k = L->A.rowptr[i]; k < L->A.rowptr[i + 1]; k++) {
      double a = L->A.val[k];
      s += a * a / L->L[L->A.col[k]];
    }
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

/* ------------------------------------------------------ create / destroy */

mgo_hier *mgo_create(int problem, int fine, int coarse, double alpha) {
  if (problem != 0) return NULL;
  if (!(alpha > 0.0) || !isfinite(alpha) || coarse < 1 || fine < coarse + 1 || fine > 12) return NULL;
  mgo_hier *h = (mgo_hier *)xcalloc(1, sizeof(mgo_hier));
  h->problem = problem;
  h->fine = fine;
  h->coarse = coarse;
  h->alpha = alpha;
  h->lv = (mgo_level *)xcalloc((size_t)fine + 1, sizeof(mgo_level));
  for (int l = coarse; l <= fine; l++) {
    mgo_level *L = &h->lv[l];
    build_level_poisson(L, 1 << l, alpha);
    if (l > coarse) {
      mgo_prolongation_p1(1 << (l - 1), &L->Pk[0]);
      mgo_transpose(&L->Pk[0], &L->Rk[0]); /* restriction = transpose, scale 1 */
    }
  }
  /* coarsest level: dense LU with partial pivoting of A_{k0} */
  mgo_level *C = &h->lv[coarse];
  int N = C->ndof;
  C->lu = (double *)xcalloc((size_t)N * N, sizeof(double));
  C->piv = (int *)xcalloc(N, sizeof(int));
  for (int r = 0; r < N; r++)
    for (int k = C->A.rowptr[r]; k < C->A.rowptr[r + 1]; k++) C->lu[(size_t)r * N + C->A.col[k]] = C->A.val[k];
  lu_factor(N, C->lu, C->piv);
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
  for (int i = 0; i < L->ndof; i++) r[i] = f[i] - r[i];
}

/* Normal-equation smoother, Alg. 1: p_i = tau (sum_j A_ij r_j / L_jj) / L_ii
 * for all i from the old residual, then x_i += p_i and r_j -= A_ji p_i. */
static void ne_step(const mgo_level *L, double tau, double *x, double *r) {
  const mgo_csr *A = &L->A, *At = &L->At;
  double *p = L->p;
  for (int i = 0; i < L->ndof; i++) {
    double q = 0.0;
    for (int k = A->rowptr[i]; k < A->rowptr[i + 1]; k++) q += A->val[k] / L->L[A->col[k]] * r[A->col[k]];
    p[i] = tau * q / L->L[i];
  }
  for (int i = 0; i < L->ndof; i++) {
    x[i] += p[i];
    /* row i of At lists the entries A_ji of column i */
    for (int k = At->rowptr[i]; k < At->rowptr[i + 1]; k++) r[At->col[k]] -= At->val[k] * p[i];
  }
}

/* Least-squares Gauss-Seidel, Alg. 2, over the groups of an ordering: every
 * unknown i of a group takes q = sum_j A_ij r_j / L_jj from the same residual,
 * p = q / N_ii, x_i += p, r_j -= A_ji p.  Groups of one unknown are Alg. 2
 * verbatim; a group {y_v, lambda_v} is equivalent because the (y_v, lambda_v)
 * entry of N_k = A^T L^{-1} A is zero. */
static void lsgs_groups(const mgo_level *L, const int *ord, const int *gptr, int ngroup, int reverse, double *x,
                        double *r) {
  const mgo_csr *A = &L->A, *At = &L->At;
  double p[8];
  for (int gg = 0; gg < ngroup; gg++) {
    int g = reverse ? ngroup - 1 - gg : gg;
    int b = gptr[g], e = gptr[g + 1];
    for (int a = b; a < e; a++) {
      int i = ord[a];
      double q = 0.0;
      for (int k = A->rowptr[i]; k < A->rowptr[i + 1]; k++) q += A->val[k] / L->L[A->col[k]] * r[A->col[k]];
      p[a - b] = q / L->Nd[i];
    }
    for (int a = b; a < e; a++) {
      int i = ord[a];
      x[i] += p[a - b];
      for (int k = At->rowptr[i]; k < At->rowptr[i + 1]; k++) r[At->col[k]] -= At->val[k] * p[a - b];
    }
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

void mgo_smooth(const mgo_hier *h, int level, int kind, int order, double tau, double *x, double *r) {
  const mgo_level *L = &h->lv[level];
  if (order < 0 || order > 4) order = 0;
  switch (kind) {
    case MGO_NE: ne_step(L, tau, x, r); break;
    case MGO_LSGS:
      if (order == MGO_ORDER_COL3) order = MGO_ORDER_COL7;
      lsgs_groups(L, L->ord[order], L->gptr[order], L->ngroup[order], 0, x, r);
      break;
    case MGO_SLSGS:
      if (order == MGO_ORDER_COL3) order = MGO_ORDER_COL7;
      lsgs_groups(L, L->ord[order], L->gptr[order], L->ngroup[order], 0, x, r);
      lsgs_groups(L, L->ord[order], L->gptr[order], L->ngroup[order], 1, x, r);
      break;
    case MGO_CGS: {
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
  lu_solve(C->ndof, C->lu, C->piv, f, x);
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

void mgo_cycle(const mgo_hier *h, int level, int kind, int order, double tau, int nu1, int nu2, int gamma,
               const double *f, double *x) {
  cycle_rec(h, level, kind, order, tau, nu1, nu2, gamma, f, x);
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
    cycle_rec(h, h->fine, kind, order, tau, nu1, nu2, gamma, f, x);
  }
  free(r);
  return it;
}
