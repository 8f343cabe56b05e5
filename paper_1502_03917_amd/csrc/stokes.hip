// Stokes control (Takacs, arXiv 1502.03917, section 1 eq. mp3) on gfx950:
// Taylor-Hood P2 velocity (zero on the boundary) / P1 pressure on the
// uniform mesh of the unit square split along the (i,j)-(i+1,j+1)
// diagonals, the smoothers of section 2 and the multigrid cycle.
//
// Unknowns [v1 | v2 | p | lambda1 | lambda2 | mu]: v_c and lambda_c on the
// (2n-1)^2 interior nodes (a, b) of the half-step lattice (index
// (b-1)(2n-1)+(a-1)), p and mu on the (n+1)^2 vertices (index j(n+1)+i).
//
// The operator has six coupled fields and two element types.  It is
// assembled on the host (element matrices by Gauss quadrature) and kept on
// the device by stencil classes: the mesh is uniform, so rows that agree in
// column fields, lattice offsets and values share one entry list, and a
// level's matrix takes a few hundred classes instead of a CSR array.  The
// kernels walk rows through the classes: one thread per row for the
// residual and the prolongation, 16 lanes per row for the restriction and
// the normal-equation smoother; for a colour phase of the LSGS sweep
// (Alg. 2), 32 lanes per group of two unknowns with the two rows merged, the
// interior groups' records formed from their lattice index (on small levels,
// every phase of every step in one workgroup with the residual in LDS); a
// wave per patch for the patch (Vanka-type) smoother.
#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "mg_internal.hpp"

namespace mgk {

namespace {

constexpr int kSNT = 256;
constexpr int kMaxPatch = 30;

// ------------------------------------------------------------ host assembly

// Collapsed Gauss-Legendre rule on the reference triangle {xi, eta >= 0,
// xi + eta <= 1}: 3 x 3 points of the square mapped by eta = (1 - u) t; exact
// for polynomials of degree 4 (P2 x P2 products).
struct TriRule {
  double xi[9], eta[9], w[9];
  TriRule() {
    const double g[3] = {0.5 - std::sqrt(15.0) / 10.0, 0.5, 0.5 + std::sqrt(15.0) / 10.0};
    const double gw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    int k = 0;
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++, k++) {
        xi[k] = g[a];
        eta[k] = (1.0 - g[a]) * g[b];
        w[k] = gw[a] * gw[b] * (1.0 - g[a]);
      }
  }
};

// P2 shape functions on the reference triangle and their (xi, eta) gradients;
// nodes 0, 1, 2 = vertices (0,0), (1,0), (0,1); 3 = mid(0,1), 4 = mid(1,2), 5 = mid(0,2)
void p2_shape(double xi, double eta, double N[6], double dN[6][2]) {
  const double l[3] = {1.0 - xi - eta, xi, eta};
  const double dl[3][2] = {{-1.0, -1.0}, {1.0, 0.0}, {0.0, 1.0}};
  for (int k = 0; k < 3; k++) {
    N[k] = l[k] * (2.0 * l[k] - 1.0);
    for (int d = 0; d < 2; d++) dN[k][d] = (4.0 * l[k] - 1.0) * dl[k][d];
  }
  const int e[3][2] = {{0, 1}, {1, 2}, {0, 2}};
  for (int m = 0; m < 3; m++) {
    const int a = e[m][0], b = e[m][1];
    N[3 + m] = 4.0 * l[a] * l[b];
    for (int d = 0; d < 2; d++) dN[3 + m][d] = 4.0 * (dl[a][d] * l[b] + l[a] * dl[b][d]);
  }
}

// Element matrices of a triangle with corners c[3] (physical coordinates):
// P2 mass, P2 Laplacian stiffness, and Dc[q][a] = -int l_q d_c N_a.
void p2_element(const double cx[3], const double cy[3], double M[6][6], double K[6][6], double D[2][3][6]) {
  static const TriRule R;
  const double J00 = cx[1] - cx[0], J01 = cx[2] - cx[0], J10 = cy[1] - cy[0], J11 = cy[2] - cy[0];
  const double det = J00 * J11 - J01 * J10, adet = std::fabs(det);
  // inverse transpose: grad_x = J^-T grad_xi
  const double I00 = J11 / det, I01 = -J10 / det, I10 = -J01 / det, I11 = J00 / det;
  std::memset(M, 0, sizeof(double) * 36);
  std::memset(K, 0, sizeof(double) * 36);
  std::memset(D, 0, sizeof(double) * 36);
  for (int p = 0; p < 9; p++) {
    double N[6], dN[6][2], gx[6], gy[6];
    p2_shape(R.xi[p], R.eta[p], N, dN);
    for (int a = 0; a < 6; a++) {
      gx[a] = I00 * dN[a][0] + I01 * dN[a][1];
      gy[a] = I10 * dN[a][0] + I11 * dN[a][1];
    }
    const double w = R.w[p] * adet;
    const double l[3] = {1.0 - R.xi[p] - R.eta[p], R.xi[p], R.eta[p]};
    for (int a = 0; a < 6; a++) {
      for (int b = 0; b < 6; b++) {
        M[a][b] += w * N[a] * N[b];
        K[a][b] += w * (gx[a] * gx[b] + gy[a] * gy[b]);
      }
      for (int q = 0; q < 3; q++) {
        D[0][q][a] -= w * l[q] * gx[a];
        D[1][q][a] -= w * l[q] * gy[a];
      }
    }
  }
}

// The two triangles of a cell (unit cell corner at the origin), local nodes
// as offsets on the half-step lattice: vertices, then mid(0,1), mid(1,2), mid(0,2).
struct CellTri {
  int hu[6], hv[6];  // half-lattice offsets of the 6 nodes
  int vi[3], vj[3];  // vertex offsets (cells)
};
const CellTri kTri[2] = {
    // lower: (0,0), (1,0), (1,1)
    {{0, 2, 2, 1, 2, 1}, {0, 0, 2, 0, 1, 1}, {0, 1, 1}, {0, 0, 1}},
    // upper: (0,0), (1,1), (0,1)
    {{0, 2, 0, 1, 1, 0}, {0, 2, 2, 1, 2, 1}, {0, 1, 0}, {0, 1, 1}},
};

struct HCsr {
  int nrows = 0, ncols = 0;
  std::vector<int> rp, col;
  std::vector<double> val;
};

// row builder with a fixed capacity per row; duplicates accumulate
struct RowAcc {
  int nrows, ncols, cap;
  std::vector<int> cnt, col;
  std::vector<double> val;
  RowAcc(int nr, int nc, int c) : nrows(nr), ncols(nc), cap(c), cnt(nr, 0), col((size_t)nr * c), val((size_t)nr * c) {}
  bool add(int r, int c, double v) {
    int* cs = &col[(size_t)r * cap];
    double* vs = &val[(size_t)r * cap];
    for (int k = 0; k < cnt[r]; k++)
      if (cs[k] == c) {
        vs[k] += v;
        return true;
      }
    if (cnt[r] == cap) return false;
    cs[cnt[r]] = c;
    vs[cnt[r]] = v;
    cnt[r]++;
    return true;
  }
  HCsr finish() const {
    HCsr A;
    A.nrows = nrows;
    A.ncols = ncols;
    A.rp.assign(nrows + 1, 0);
    long long nnz = 0;
    for (int r = 0; r < nrows; r++) {
      nnz += cnt[r];
      if (nnz > INT_MAX) throw std::length_error("Stokes assembly: more than 2^31-1 nonzeros");
      A.rp[r + 1] = (int)nnz;
    }
    A.col.resize(A.rp[nrows]);
    A.val.resize(A.rp[nrows]);
    std::vector<std::pair<int, double>> row;
    for (int r = 0; r < nrows; r++) {
      row.clear();
      for (int k = 0; k < cnt[r]; k++) row.emplace_back(col[(size_t)r * cap + k], val[(size_t)r * cap + k]);
      std::sort(row.begin(), row.end(), [](const std::pair<int, double>& a, const std::pair<int, double>& b) {
        return a.first < b.first;
      });
      for (int k = 0; k < cnt[r]; k++) {
        A.col[A.rp[r] + k] = row[k].first;
        A.val[A.rp[r] + k] = row[k].second;
      }
    }
    return A;
  }
};

HCsr transpose(const HCsr& A) {
  HCsr T;
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.rp.assign(T.nrows + 1, 0);
  for (int c : A.col) T.rp[c + 1]++;
  for (int r = 0; r < T.nrows; r++) T.rp[r + 1] += T.rp[r];
  T.col.resize(A.col.size());
  T.val.resize(A.val.size());
  std::vector<int> at(T.rp.begin(), T.rp.end() - 1);
  for (int r = 0; r < A.nrows; r++)
    for (int k = A.rp[r]; k < A.rp[r + 1]; k++) {
      const int d = at[A.col[k]]++;
      T.col[d] = r;
      T.val[d] = A.val[k];
    }
  return T;
}

double entry(const HCsr& A, int r, int c) {
  const int* b = A.col.data() + A.rp[r];
  const int* e = A.col.data() + A.rp[r + 1];
  const int* it = std::lower_bound(b, e, c);
  return (it != e && *it == c) ? A.val[it - A.col.data()] : 0.0;
}

// interior P2 node index, -1 on the boundary
inline int node_of(int n, int a, int b) {
  const int m = 2 * n - 1;
  if (a < 1 || b < 1 || a > m || b > m) return -1;
  return (b - 1) * m + (a - 1);
}

// Position of an unknown on the half-step lattice.  Unknowns are field-major:
// v1, v2 (interior P2 nodes), p (P1 vertices), lambda1, lambda2, mu; a P2
// node (a, b) has index (b - 1) m + (a - 1), a vertex (2I, 2J) index J (n + 1) + I.
struct SGeo {
  int n, m, nv, np;
};
__host__ __device__ inline int sbase(const SGeo& g, int f) {
  return f == 0 ? 0 : f == 1 ? g.nv : f == 2 ? 2 * g.nv : f == 3 ? 2 * g.nv + g.np : f == 4 ? 3 * g.nv + g.np
                                                                                          : 4 * g.nv + g.np;
}
__host__ __device__ inline bool sp1(int f) { return f == 2 || f == 5; }
// field of unknown i and its lattice position
__host__ __device__ inline int sfield(const SGeo& g, int i) {
  return i < g.nv ? 0 : i < 2 * g.nv ? 1 : i < 2 * g.nv + g.np ? 2 : i < 3 * g.nv + g.np ? 3 : i < 4 * g.nv + g.np ? 4 : 5;
}
__host__ __device__ inline void spos(const SGeo& g, int i, int& hx, int& hy) {
  const int f = sfield(g, i), a = i - sbase(g, f);
  if (sp1(f)) {
    const int J = a / (g.n + 1);
    hx = 2 * (a - J * (g.n + 1));
    hy = 2 * J;
  } else {
    const int b = a / g.m;
    hx = a - b * g.m + 1;
    hy = b + 1;
  }
}
__host__ __device__ inline int sindex(const SGeo& g, int f, int hx, int hy) {
  return sbase(g, f) + (sp1(f) ? (hy >> 1) * (g.n + 1) + (hx >> 1) : (hy - 1) * g.m + (hx - 1));
}

// A with its rows grouped into stencil classes: rows whose entries agree in
// column field, lattice offset and value share one class (the mesh is
// uniform, so a level has a few hundred classes for millions of rows).  An
// entry packs the column field and its offset (dx, dy) from the row on the
// half-step lattice; the column is recomputed from the row's position.
struct ClassA {
  std::vector<int> row_cls, ptr, ent;
  std::vector<double> val;
};
constexpr int kEntOff = 16;  // offsets are stored + 16 in 8 bits
constexpr int kMaxRowEntries = 64;  // the one-workgroup LSGS kernel holds up to 64 entries of a row in registers
__host__ __device__ inline int sent_col(const SGeo& g, int e, int hx, int hy) {
  return sindex(g, e & 0xFF, hx + ((e >> 8) & 0xFF) - kEntOff, hy + ((e >> 16) & 0xFF) - kEntOff);
}

bool build_classes(const HCsr& A, const SGeo& g, ClassA& C, std::string* err) {
  // rows are looked up by a 64-bit hash of their entries and compared in
  // full with the class the hash points to
  std::unordered_map<unsigned long long, std::vector<int>> seen;
  C.row_cls.assign(A.nrows, 0);
  C.ptr.assign(1, 0);
  std::vector<int> ents;
  for (int i = 0; i < A.nrows; i++) {
    int hx, hy;
    spos(g, i, hx, hy);
    ents.clear();
    unsigned long long h = 0x243F6A8885A308D3ull;  // multiply-xorshift hash of the entries and value bits
    auto mix = [&](unsigned long long v) {
      h = (h ^ v) * 0x9E3779B97F4A7C15ull;
      h ^= h >> 29;
    };
    for (int k = A.rp[i]; k < A.rp[i + 1]; k++) {
      const int c = A.col[k], fc = sfield(g, c);
      int cx, cy;
      spos(g, c, cx, cy);
      const int dx = cx - hx, dy = cy - hy;
      if (dx < -kEntOff || dx >= 256 - kEntOff || dy < -kEntOff || dy >= 256 - kEntOff) {
        *err = "stokes: stencil offset out of range";
        return false;
      }
      const int e = fc | ((dx + kEntOff) << 8) | ((dy + kEntOff) << 16);
      if (sent_col(g, e, hx, hy) != c) {
        *err = "stokes: stencil class does not reproduce a column";
        return false;
      }
      ents.push_back(e);
      unsigned long long vb;
      std::memcpy(&vb, &A.val[k], sizeof(vb));
      mix((unsigned long long)(unsigned)e);
      mix(vb);
    }
    const int len = A.rp[i + 1] - A.rp[i];
    int id = -1;
    std::vector<int>& cand = seen[h];
    for (int c : cand) {
      if (C.ptr[c + 1] - C.ptr[c] != len) continue;
      bool same = true;
      for (int q = 0; q < len && same; q++)
        same = C.ent[C.ptr[c] + q] == ents[q] && C.val[C.ptr[c] + q] == A.val[A.rp[i] + q];
      if (same) {
        id = c;
        break;
      }
    }
    if (id < 0) {
      id = (int)C.ptr.size() - 1;
      cand.push_back(id);
      C.ent.insert(C.ent.end(), ents.begin(), ents.end());
      C.val.insert(C.val.end(), A.val.begin() + A.rp[i], A.val.begin() + A.rp[i + 1]);
      C.ptr.push_back((int)C.ent.size());
    }
    C.row_cls[i] = id;
  }
  for (size_t c = 0; c + 1 < C.ptr.size(); c++)
    if (C.ptr[c + 1] - C.ptr[c] > kMaxRowEntries) {
      *err = "stokes: a row has more entries than the one-workgroup LSGS kernel takes";
      return false;
    }
  return true;
}

struct Blocks {
  HCsr Ms, Ks, D[2];   // scalar P2 mass and stiffness (interior nodes); divergence rows over vertices
  std::vector<double> w;  // pressure-mean weights int(phi_q)
};

bool assemble_blocks(int n, Blocks& B) {
  const int m = 2 * n - 1, nv = m * m, np = (n + 1) * (n + 1);
  const double h = 1.0 / n;
  double Me[2][6][6], Ke[2][6][6], De[2][2][3][6];
  for (int t = 0; t < 2; t++) {
    double cx[3], cy[3];
    for (int k = 0; k < 3; k++) {
      cx[k] = kTri[t].vi[k] * h;
      cy[k] = kTri[t].vj[k] * h;
    }
    p2_element(cx, cy, Me[t], Ke[t], De[t]);
  }
  RowAcc M(nv, nv, 24), K(nv, nv, 24), D0(np, nv, 24), D1(np, nv, 24);
  B.w.assign(np, 0.0);
  for (int j = 0; j < n; j++)
    for (int i = 0; i < n; i++)
      for (int t = 0; t < 2; t++) {
        int g[6];
        for (int a = 0; a < 6; a++) g[a] = node_of(n, 2 * i + kTri[t].hu[a], 2 * j + kTri[t].hv[a]);
        for (int a = 0; a < 6; a++) {
          if (g[a] < 0) continue;
          for (int b = 0; b < 6; b++)
            if (g[b] >= 0 && !(M.add(g[a], g[b], Me[t][a][b]) && K.add(g[a], g[b], Ke[t][a][b]))) return false;
        }
        for (int q = 0; q < 3; q++) {
          const int vq = (j + kTri[t].vj[q]) * (n + 1) + i + kTri[t].vi[q];
          B.w[vq] += h * h / 6.0;  // int over the triangle of a P1 basis function: |T| / 3
          for (int a = 0; a < 6; a++)
            if (g[a] >= 0 && !(D0.add(vq, g[a], De[t][0][q][a]) && D1.add(vq, g[a], De[t][1][q][a]))) return false;
        }
      }
  B.Ms = M.finish();
  B.Ks = K.finish();
  B.D[0] = D0.finish();
  B.D[1] = D1.finish();
  return true;
}

// The operator of eq. mp3 as one CSR matrix (rows in field order; the
// sub-rows of each row are already sorted by column and lie in increasing
// column blocks).
HCsr assemble_kkt(int n, double alpha, const Blocks& B) {
  const int m = 2 * n - 1, nv = m * m, np = (n + 1) * (n + 1);
  const int ov[2] = {0, nv}, op = 2 * nv, ol[2] = {2 * nv + np, 3 * nv + np}, om = 4 * nv + np;
  const HCsr Dt[2] = {transpose(B.D[0]), transpose(B.D[1])};
  HCsr A;
  A.nrows = A.ncols = 4 * nv + 2 * np;
  A.rp.reserve(A.nrows + 1);
  A.rp.push_back(0);
  auto put = [&](const HCsr& S, int r, int off, double scale) {
    for (int k = S.rp[r]; k < S.rp[r + 1]; k++) {
      A.col.push_back(off + S.col[k]);
      A.val.push_back(scale * S.val[k]);
    }
  };
  auto endrow = [&]() {
    if (A.col.size() > (size_t)INT_MAX) throw std::length_error("Stokes KKT matrix: more than 2^31-1 nonzeros");
    A.rp.push_back((int)A.col.size());
  };
  for (int c = 0; c < 2; c++)  // v_c: M v_c + K lambda_c + D_c^T mu
    for (int a = 0; a < nv; a++) {
      put(B.Ms, a, ov[c], 1.0);
      put(B.Ks, a, ol[c], 1.0);
      put(Dt[c], a, om, 1.0);
      endrow();
    }
  for (int q = 0; q < np; q++) {  // p: D_1 lambda_1 + D_2 lambda_2
    put(B.D[0], q, ol[0], 1.0);
    put(B.D[1], q, ol[1], 1.0);
    endrow();
  }
  for (int c = 0; c < 2; c++)  // lambda_c: K v_c + D_c^T p - alpha^-1 M lambda_c
    for (int a = 0; a < nv; a++) {
      put(B.Ks, a, ov[c], 1.0);
      put(Dt[c], a, op, 1.0);
      put(B.Ms, a, ol[c], -1.0 / alpha);
      endrow();
    }
  for (int q = 0; q < np; q++) {  // mu: D_1 v_1 + D_2 v_2
    put(B.D[0], q, ov[0], 1.0);
    put(B.D[1], q, ov[1], 1.0);
    endrow();
  }
  return A;
}

// Prolongation from nc to 2 nc cells per side for the whole vector:
// P2 interpolation for v and lambda, P1 interpolation for p and mu.
HCsr assemble_prolongation(int nc) {
  const int nf = 2 * nc, mc = 2 * nc - 1, mf = 2 * nf - 1;
  const int nvc = mc * mc, nvf = mf * mf, npc = (nc + 1) * (nc + 1), npf = (nf + 1) * (nf + 1);
  // P2 block: the coarse basis evaluated at the fine interior nodes
  RowAcc P2(nvf, nvc, 6);
  for (int b = 1; b <= mf; b++)
    for (int a = 1; a <= mf; a++) {
      const int row = (b - 1) * mf + (a - 1);
      int I = a / 4, J = b / 4;
      if (I > nc - 1) I = nc - 1;
      if (J > nc - 1) J = nc - 1;
      const double s = a / 4.0 - I, t = b / 4.0 - J;
      const int tri = (s >= t) ? 0 : 1;
      const double xi = tri == 0 ? s - t : s, eta = tri == 0 ? t : t - s;
      double N[6], dN[6][2];
      p2_shape(xi, eta, N, dN);
      for (int k = 0; k < 6; k++) {
        const int col = node_of(nc, 2 * I + kTri[tri].hu[k], 2 * J + kTri[tri].hv[k]);
        if (col >= 0 && N[k] != 0.0) P2.add(row, col, N[k]);
      }
    }
  // P1 block: coarse vertices copied, fine vertices on coarse edges averaged
  RowAcc P1(npf, npc, 2);
  for (int j = 0; j <= nf; j++)
    for (int i = 0; i <= nf; i++) {
      const int row = j * (nf + 1) + i;
      const int i0 = i / 2, j0 = j / 2, i1 = (i + 1) / 2, j1 = (j + 1) / 2;
      if (i0 == i1 && j0 == j1) {
        P1.add(row, j0 * (nc + 1) + i0, 1.0);
      } else {
        P1.add(row, j0 * (nc + 1) + i0, 0.5);
        P1.add(row, j1 * (nc + 1) + i1, 0.5);
      }
    }
  const HCsr h2 = P2.finish(), h1 = P1.finish();
  HCsr P;
  P.nrows = 4 * nvf + 2 * npf;
  P.ncols = 4 * nvc + 2 * npc;
  P.rp.push_back(0);
  const int foff[6] = {0, nvc, 2 * nvc, 2 * nvc + npc, 3 * nvc + npc, 4 * nvc + npc};
  const bool p1[6] = {false, false, true, false, false, true};
  for (int fl = 0; fl < 6; fl++) {
    const HCsr& S = p1[fl] ? h1 : h2;
    for (int r = 0; r < S.nrows; r++) {
      for (int k = S.rp[r]; k < S.rp[r + 1]; k++) {
        P.col.push_back(foff[fl] + S.col[k]);
        P.val.push_back(S.val[k]);
      }
      P.rp.push_back((int)P.col.size());
    }
  }
  return P;
}

void lu_dense(int n, std::vector<double>& a, std::vector<int>& piv, bool& ok) {
  piv.resize(n);
  ok = true;
  for (int k = 0; k < n; k++) {
    int p = k;
    for (int i = k + 1; i < n; i++)
      if (std::fabs(a[(size_t)i * n + k]) > std::fabs(a[(size_t)p * n + k])) p = i;
    piv[k] = p;
    if (p != k)
      for (int c = 0; c < n; c++) std::swap(a[(size_t)k * n + c], a[(size_t)p * n + c]);
    const double d = a[(size_t)k * n + k];
    if (d == 0.0) {
      ok = false;
      return;
    }
    for (int i = k + 1; i < n; i++) {
      const double f = a[(size_t)i * n + k] / d;
      a[(size_t)i * n + k] = f;
      for (int c = k + 1; c < n; c++) a[(size_t)i * n + c] -= f * a[(size_t)k * n + c];
    }
  }
}

// Colour phases of Alg. 2 for the level with n cells per side: per velocity
// component c, 25 colours (a mod 5) + 5 (b mod 5) of the interior P2 nodes
// with groups {v_c, lambda_c} of one node; then 9 colours (i mod 3) + 3 (j mod 3)
// of the vertices with groups {p, mu}.  Phase k spans groups [ph[k], ph[k+1]).
void colour_groups(int n, std::vector<int2>& grp, std::vector<int>& ph) {
  const int m = 2 * n - 1, nv = m * m, np = (n + 1) * (n + 1);
  const int op = 2 * nv, ol = 2 * nv + np, om = 4 * nv + np;
  grp.clear();
  ph.assign(1, 0);
  for (int c = 0; c < 2; c++)
    for (int col = 0; col < 25; col++) {
      for (int b = 1; b <= m; b++)
        for (int a = 1; a <= m; a++)
          if (a % 5 + 5 * (b % 5) == col) {
            const int node = (b - 1) * m + (a - 1);
            grp.push_back(make_int2(c * nv + node, ol + c * nv + node));
          }
      ph.push_back((int)grp.size());
    }
  for (int col = 0; col < 9; col++) {
    for (int j = 0; j <= n; j++)
      for (int i = 0; i <= n; i++)
        if (i % 3 + 3 * (j % 3) == col) {
          const int q = j * (n + 1) + i;
          grp.push_back(make_int2(op + q, om + q));
        }
    ph.push_back((int)grp.size());
  }
}

// Patches of the patch smoother (one per vertex): the unknowns of patch q
// are dof[dptr[q] .. dptr[q+1]); patches listed by colour
// (i mod 3) + 3 (j mod 3), phase k spans order[ph[k] .. ph[k+1]).
bool build_patches(int n, std::vector<int>& dptr, std::vector<int>& dof, std::vector<int>& order,
                   std::vector<int>& ph, std::string* err) {
  const int m = 2 * n - 1, nv = m * m, np = (n + 1) * (n + 1);
  const int op = 2 * nv, ol = 2 * nv + np, om = 4 * nv + np;
  dptr.assign(np + 1, 0);
  dof.clear();
  order.clear();
  auto vel = [&](int node, std::vector<int>& d) {
    d.push_back(node);
    d.push_back(nv + node);
    d.push_back(ol + node);
    d.push_back(ol + nv + node);
  };
  const int di[7] = {0, 1, -1, 0, 0, 1, -1}, dj[7] = {0, 0, 0, 1, -1, 1, -1};
  for (int j = 0; j <= n; j++)
    for (int i = 0; i <= n; i++) {
      const int q = j * (n + 1) + i;
      std::vector<int> d = {op + q, om + q};
      for (int e = 0; e < 7; e++) {
        const int ii = i + di[e], jj = j + dj[e];
        if (ii < 0 || jj < 0 || ii > n || jj > n) continue;
        const int node = node_of(n, i + ii, j + jj);
        if (node >= 0) vel(node, d);
      }
      if (d.size() == 2) {
        // every edge at the vertex lies on the boundary: the interior nodes
        // of the triangles containing the vertex
        for (int cj = j - 1; cj <= j; cj++)
          for (int ci = i - 1; ci <= i; ci++) {
            if (ci < 0 || cj < 0 || ci >= n || cj >= n) continue;
            for (int t = 0; t < 2; t++) {
              bool has = false;
              for (int k = 0; k < 3; k++) has |= (ci + kTri[t].vi[k] == i && cj + kTri[t].vj[k] == j);
              if (!has) continue;
              for (int k = 0; k < 6; k++) {
                const int node = node_of(n, 2 * ci + kTri[t].hu[k], 2 * cj + kTri[t].hv[k]);
                if (node >= 0 && std::find(d.begin(), d.end(), node) == d.end()) vel(node, d);
              }
            }
          }
      }
      const int msz = (int)d.size();
      if (msz > kMaxPatch) {
        *err = "stokes: patch larger than 30 unknowns";
        return false;
      }
      dptr[q + 1] = dptr[q] + msz;
      dof.insert(dof.end(), d.begin(), d.end());
    }
  ph.assign(1, 0);
  for (int col = 0; col < 9; col++) {
    for (int j = 0; j <= n; j++)
      for (int i = 0; i <= n; i++)
        if (i % 3 + 3 * (j % 3) == col) order.push_back(j * (n + 1) + i);
    ph.push_back((int)order.size());
  }
  return true;
}

// ------------------------------------------------------------------ kernels

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

__device__ inline void block_store(double v, double* out) {
  __shared__ double sh[kSNT / 64];
  v = wsum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kSNT / 64; w++) s += sh[w];
    *out = s;
  }
}

// A read-only array seen through the constant address space: a load whose
// index is the same on every lane of the wave becomes one scalar load.
template <typename T>
__device__ inline const __attribute__((address_space(4))) T* cptr(const T* p) {
  return (const __attribute__((address_space(4))) T*)(p);
}

// Rows of a sparse operator: a CSR matrix (the transfers) or the stencil
// classes of A.  row() gives the entry range and the row's lattice position
// (classes) from which col_of() forms the column.
template <typename T>
struct CsrRows {
  const int* rp;
  const int* col;
  const T* val;
  __device__ void row(int i, int& kb, int& ke, int& pos) const {
    kb = rp[i];
    ke = rp[i + 1];
    pos = 0;
  }
  __device__ int col_of(int k, int) const { return col[k]; }
  __device__ T val_of(int k) const { return val[k]; }
  // the same for an entry index k common to the wave (loads from the
  // constant address space, i.e. scalar loads)
  __device__ int col_u(int k, int) const { return cptr(col)[k]; }
  __device__ T val_u(int k) const { return cptr(val)[k]; }
};
template <typename T>
struct ClassRows {
  const int* cls;
  const int* ptr;
  const int* ent;
  const T* val;
  SGeo g;
  __device__ void row(int i, int& kb, int& ke, int& pos) const {
    const int c = cls[i];
    kb = ptr[c];
    ke = ptr[c + 1];
    int hx, hy;
    spos(g, i, hx, hy);
    pos = hx | (hy << 16);
  }
  __device__ int col_of(int k, int pos) const { return sent_col(g, ent[k], pos & 0xFFFF, pos >> 16); }
  __device__ T val_of(int k) const { return val[k]; }
  __device__ int col_u(int k, int pos) const { return sent_col(g, cptr(ent)[k], pos & 0xFFFF, pos >> 16); }
  __device__ T val_u(int k) const { return cptr(val)[k]; }
};

// Row kernels with 16 lanes per row (16 rows per 256-thread block), each
// lane taking every 16th entry, partial sums combined by shuffles: the
// restriction (rows of 10 to 25 entries) and the normal-equation smoother.
constexpr int kRL = 16;
constexpr int kRows = kSNT / kRL;

template <typename T>
__device__ inline T row_sum(T v) {
#pragma unroll
  for (int o = kRL / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kRL);
  return v;
}

// r = f - A x, with per-block partial sums of ||r||_2^2 (MODE 1) or
// r^T L^-1 r (MODE 2); f == nullptr gives r = A x.  One thread per row,
// grid-stride over chunks of 128 rows, a pair of waves per chunk: the first
// wave takes the chunk's even rows, the second its odd rows.  Velocity nodes
// alternate in type along a lattice row, so a wave's rows then share one
// node type and, away from the boundary, one stencil class.  When every lane
// of the wave has the same class, the class's entries and values are read
// with scalar loads (one per entry for the whole wave) and only the x gathers
// are vector loads; otherwise each lane walks its own class.  The entries go
// in blocks of kResBlk, whose loads are issued together, and the products
// are summed in entry order either way.
constexpr int kResBlk = 8;
template <typename T, int MODE, typename AT>
__global__ __launch_bounds__(kSNT) void ks_resid(int n, AT A, const T* __restrict__ f, const T* __restrict__ x,
                                                 T* __restrict__ r, const double* __restrict__ Ldi,
                                                 double* __restrict__ part) {
  static_assert(kSNT % 128 == 0, "whole chunks of 128 rows per block");
  double s2 = 0.0;
  const int t = blockIdx.x * kSNT + threadIdx.x;
  const int i0 = (t & ~127) + 2 * (t & 63) + ((t >> 6) & 1);
  for (int i = i0; i < n; i += gridDim.x * kSNT) {
    int kb, ke, pos;
    A.row(i, kb, ke, pos);
    T s = 0;
    const int kb0 = __builtin_amdgcn_readfirstlane(kb), ke0 = __builtin_amdgcn_readfirstlane(ke);
    if (__builtin_amdgcn_ballot_w64(kb != kb0 || ke != ke0) == 0) {
      int k = kb0;
      for (; k + kResBlk <= ke0; k += kResBlk) {
        T av[kResBlk], xv[kResBlk];
#pragma unroll
        for (int u = 0; u < kResBlk; u++) {
          av[u] = A.val_u(k + u);
          xv[u] = x[A.col_u(k + u, pos)];
        }
#pragma unroll
        for (int u = 0; u < kResBlk; u++) s += av[u] * xv[u];
      }
      for (; k < ke0; k++) s += A.val_u(k) * x[A.col_u(k, pos)];
    } else {
      int k = kb;
      for (; k + kResBlk <= ke; k += kResBlk) {
        T av[kResBlk], xv[kResBlk];
#pragma unroll
        for (int u = 0; u < kResBlk; u++) {
          av[u] = A.val_of(k + u);
          xv[u] = x[A.col_of(k + u, pos)];
        }
#pragma unroll
        for (int u = 0; u < kResBlk; u++) s += av[u] * xv[u];
      }
      for (; k < ke; k++) s += A.val_of(k) * x[A.col_of(k, pos)];
    }
    const T ri = f ? f[i] - s : s;
    r[i] = ri;
    if (MODE == 1) s2 += (double)ri * (double)ri;
    if (MODE == 2) s2 += (double)ri * (double)ri * Ldi[i];
  }
  if (MODE) block_store(s2, &part[blockIdx.x]);
}

// per-block partial sums of ||v||^2 (MODE 1) or v^T L^-1 v (MODE 2), one thread per entry
template <int MODE>
__global__ __launch_bounds__(kSNT) void ks_vnorm(int n, const double* __restrict__ v, const double* __restrict__ Ldi,
                                                 double* __restrict__ part) {
  const int i = blockIdx.x * kSNT + threadIdx.x;
  double s2 = 0.0;
  if (i < n) s2 = MODE == 1 ? v[i] * v[i] : v[i] * v[i] * Ldi[i];
  block_store(s2, &part[blockIdx.x]);
}

// y += A x with one thread per row (grid-stride), for operators with a few
// entries per row (the prolongation: 1 to 3)
template <typename T, typename AT>
__global__ __launch_bounds__(kSNT) void ks_spmv_add1(int n, AT A, const T* __restrict__ x, T* __restrict__ y) {
  for (int i = blockIdx.x * kSNT + threadIdx.x; i < n; i += gridDim.x * kSNT) {
    int kb, ke, pos;
    A.row(i, kb, ke, pos);
    T s = 0;
    for (int k = kb; k < ke; k++) s += A.val_of(k) * x[A.col_of(k, pos)];
    y[i] += s;
  }
}

// y = A x (ADD 0) or y += A x (ADD 1); restriction variant also writes x_c = 0, r_c = f_c
template <typename T, int ADD, typename AT>
__global__ __launch_bounds__(kSNT) void ks_spmv(int n, AT A, const T* __restrict__ x, T* __restrict__ y,
                                                T* __restrict__ zero_out, T* __restrict__ copy_out) {
  const int ln = threadIdx.x % kRL;
  for (int i0 = blockIdx.x * kRows; i0 < n; i0 += gridDim.x * kRows) {
    const int i = i0 + threadIdx.x / kRL;
    T s = 0;
    if (i < n) {
      int kb, ke, pos;
      A.row(i, kb, ke, pos);
      for (int k = kb + ln; k < ke; k += kRL) s += A.val_of(k) * x[A.col_of(k, pos)];
    }
    s = row_sum(s);
    if (i >= n || ln != 0) continue;
    if (ADD) {
      y[i] += s;
    } else {
      y[i] = s;
      if (zero_out) zero_out[i] = (T)0;
      if (copy_out) copy_out[i] = s;
    }
  }
}

// Alg. 1, first loop with x += p: p_i = tau (sum_j A_ij r_j / L_jj) / L_ii
template <typename T, typename AT>
__global__ __launch_bounds__(kSNT) void ks_ne_p(int n, AT A, const T* __restrict__ Linv, T tau,
                                                const T* __restrict__ r, T* __restrict__ x, T* __restrict__ p) {
  const int ln = threadIdx.x % kRL;
  for (int i0 = blockIdx.x * kRows; i0 < n; i0 += gridDim.x * kRows) {
    const int i = i0 + threadIdx.x / kRL;
    T q = 0;
    if (i < n) {
      int kb, ke, pos;
      A.row(i, kb, ke, pos);
      for (int k = kb + ln; k < ke; k += kRL) {
        const int c = A.col_of(k, pos);
        q += A.val_of(k) * Linv[c] * r[c];
      }
    }
    q = row_sum(q);
    if (i >= n || ln != 0) continue;
    const T pi = tau * q * Linv[i];
    p[i] = pi;
    x[i] += pi;
  }
}

// Alg. 1, second loop: r -= A p (A symmetric: row i holds the column)
template <typename T, typename AT>
__global__ __launch_bounds__(kSNT) void ks_ne_r(int n, AT A, const T* __restrict__ p, T* __restrict__ r) {
  const int ln = threadIdx.x % kRL;
  for (int i0 = blockIdx.x * kRows; i0 < n; i0 += gridDim.x * kRows) {
    const int i = i0 + threadIdx.x / kRL;
    T s = 0;
    if (i < n) {
      int kb, ke, pos;
      A.row(i, kb, ke, pos);
      for (int k = kb + ln; k < ke; k += kRL) s += A.val_of(k) * p[A.col_of(k, pos)];
    }
    s = row_sum(s);
    if (i < n && ln == 0) r[i] -= s;
  }
}

// One colour phase of Alg. 2.  A group is two unknowns whose entry of
// N = A^T L^-1 A is zero (a velocity component and its multiplier at one
// node, or the pressure and its multiplier at one vertex), so both take q
// from the same residual; groups of a phase share no residual entry.  A group
// (i, j) keeps the union of its two rows' columns, each entry with both
// coefficients (A_ik, A_jk), in a group class (groups whose merged entries
// agree in field, lattice offset from row i and values share one).  One
// gather of L^-1 r over the union gives q_i and q_j; since no other group of
// the phase touches these residual entries, the gathered values are still
// current and each is written once, r_k - A_ik p_i - A_jk p_j.  The class
// also fixes L_kk^-1 of every merged column and N_ii^-1, N_jj^-1 (stored at
// the class's first entry), so the phase gathers nothing but r.  A group
// record is (i, j, first entry, end).
constexpr int kMaxGroupEntries = 96;

template <typename T>
struct T2of;
template <>
struct T2of<double> {
  typedef double2 type;
};
template <>
struct T2of<float> {
  typedef float2 type;
};

// A group per kGLR lanes, kGNE merged entries per lane in registers.  The
// phase's cost is the chain of dependent loads of each wave (record, entries,
// gathers), not bandwidth.
constexpr int kGLR = 32, kGNE = kMaxGroupEntries / kGLR;

constexpr int kGNT = 512;  // threads per workgroup (measured at 513^2: 64 slower by 14%, 256 and 512 alike in FP64, 512 2% faster in FP32)

// The groups of one wave, each on kGLR lanes (wave-uniform early exit).  The
// record of a group comes from rec(g) (false: no group): a load from the
// record list, or formed from the group's index on the lattice path.
template <typename T, typename Rec>
__device__ __forceinline__ void grp_wave_of(int wave, int ng, Rec rec, const int* __restrict__ gent,
                                            const typename T2of<T>::type* __restrict__ gval,
                                            const T* __restrict__ glinv,
                                            const typename T2of<T>::type* __restrict__ gninv, const SGeo& geo,
                                            T* __restrict__ x, T* __restrict__ r) {
  constexpr int LR = kGLR, G = 64 / LR, NE = kGNE;
  if (wave * G >= ng) return;  // uniform per wave
  const int lane = threadIdx.x % 64, ln = lane % LR;
  const int g = wave * G + lane / LR;
  const bool live = g < ng;
  int hx, hy;
  const int4 u = rec(live ? g : -1, hx, hy);
  int c[NE];
  typename T2of<T>::type a[NE];
  T l[NE], rc[NE];
#pragma unroll
  for (int e = 0; e < NE; e++) {
    const int k = u.z + ln + e * LR;
    const bool h = k < u.w;
    c[e] = h ? sent_col(geo, gent[k], hx, hy) : 0;
    if (h) {
      a[e] = gval[k];
      l[e] = glinv[k];
    } else {
      a[e].x = a[e].y = l[e] = 0;
    }
  }
  typename T2of<T>::type nn;
  if (live) nn = gninv[u.z];
  else nn.x = nn.y = 0;
  T qi = 0, qj = 0;
#pragma unroll
  for (int e = 0; e < NE; e++) {
    rc[e] = u.z + ln + e * LR < u.w ? r[c[e]] : (T)0;
    const T w = l[e] * rc[e];
    qi += a[e].x * w;
    qj += a[e].y * w;
  }
#pragma unroll
  for (int o = LR / 2; o > 0; o >>= 1) {
    qi += __shfl_xor(qi, o, LR);
    qj += __shfl_xor(qj, o, LR);
  }
  const T pi = qi * nn.x, pj = qj * nn.y;
  if (live && ln == 0) {
    x[u.x] += pi;
    x[u.y] += pj;
  }
#pragma unroll
  for (int e = 0; e < NE; e++)
    if (u.z + ln + e * LR < u.w) r[c[e]] = (rc[e] - a[e].x * pi) - a[e].y * pj;
}

template <typename T>
__device__ __forceinline__ void grp_wave(int wave, int g0, int ng, const int4* __restrict__ grp,
                                         const int* __restrict__ gent,
                                         const typename T2of<T>::type* __restrict__ gval,
                                         const T* __restrict__ glinv,
                                         const typename T2of<T>::type* __restrict__ gninv, const SGeo& geo,
                                         T* __restrict__ x, T* __restrict__ r) {
  auto rec = [&](int g, int& hx, int& hy) {
    const int4 u = g >= 0 ? grp[g0 + g] : make_int4(0, 0, 0, 0);
    spos(geo, u.x, hx, hy);
    return u;
  };
  grp_wave_of<T>(wave, ng, rec, gent, gval, glinv, gninv, geo, x, r);
}

template <typename T>
__global__ __launch_bounds__(kGNT) void ks_lsgs_grp(int g0, int ng, const int4* __restrict__ grp,
                                                    const int* __restrict__ gent,
                                                    const typename T2of<T>::type* __restrict__ gval,
                                                    const T* __restrict__ glinv,
                                                    const typename T2of<T>::type* __restrict__ gninv, SGeo geo,
                                                    T* __restrict__ x, T* __restrict__ r) {
  grp_wave<T>(blockIdx.x * (kGNT / 64) + threadIdx.x / 64, g0, ng, grp, gent, gval, glinv, gninv, geo, x, r);
}

// Every smoothing step of Alg. 2 on a small level in one workgroup.  On
// these levels a colour phase has few groups, so a launch per phase costs
// far more than the work: here the residual, x and L^-1 stay in LDS, phases
// are separated by workgroup barriers, and each lane's part of the matrix
// (which does not depend on the residual) comes from phase-ordered arrays
// built at setup, loaded one phase ahead of its use (the row and entry
// count two phases ahead).  Lane t of phase ph: meta[ph][t] = (row, count),
// entry e at col/val[ph][e][t]; row -1 and count 0 mark an idle lane.
constexpr int kWT = 1024, kWG = 4, kWLR = 32 / kWG, kWNE = 64 / kWLR;
constexpr int kWSlots = kWT / 64 * kWG;  // largest phase (in groups) the kernel takes
constexpr int kWLdsBytes = 150 * 1024;   // residual, x and L^-1 of the level
static_assert(kWLR * kWNE == kMaxRowEntries, "entries held per row");

template <typename T>
__device__ inline T wlr_sum(T v) {
#pragma unroll
  for (int o = kWLR / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWLR);
  return v;
}

// orders LDS accesses only: the kernel's global stores are its last act
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Global loads of the kernel below are buffer loads issued unconditionally:
// an unused one takes an offset past the end of its buffer, which the
// hardware answers with zero and no memory access.  With a fixed sequence of
// loads the compiler waits only for the data about to be used, so the loads
// for the next phase stay in flight through the current one.
constexpr unsigned kOff = 0x80000000u;  // past the end of every buffer (< 2 GiB each)

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, bytes, 0x00020000);
}
__device__ inline int bld_i(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}
__device__ inline double bld(__amdgpu_buffer_rsrc_t r, unsigned off, double*) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ inline float bld(__amdgpu_buffer_rsrc_t r, unsigned off, float*) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

template <typename T>
__global__ __launch_bounds__(kWT) void ks_lsgs_wg(int ndof, int nph, int nseq, int sweeps,
                                                  const int2* __restrict__ meta, const int* __restrict__ col,
                                                  const T* __restrict__ val, const T* __restrict__ Linv,
                                                  const T* __restrict__ Ninv, T* __restrict__ x, T* __restrict__ r) {
  __shared__ T lds[kWLdsBytes / sizeof(T)];
  T* rs = lds;
  T* ls = lds + ndof;
  T* xs = lds + 2 * ndof;
  const int t = threadIdx.x, ln = t % kWLR, half = (t / kWLR) & 1;
  for (int i = t; i < ndof; i += kWT) {
    rs[i] = r[i];
    ls[i] = Linv[i];
    xs[i] = x[i];
  }
  const int nent = nph * kWNE * kWT;
  const __amdgpu_buffer_rsrc_t Rm = rsrc(meta, nph * kWT * 8), Rc = rsrc(col, nent * 4),
                               Rv = rsrc(val, nent * (int)sizeof(T)), Rn = rsrc(Ninv, ndof * (int)sizeof(T));
  // phase of step s: sweeps alternate forward and backward colour order
  auto phase = [&](int s) {
    const int k = s % nph;
    return (s / nph) % sweeps ? nph - 1 - k : k;
  };
  // (row, count) of this lane at step s; steps past the end read (0, 0)
  auto ld_meta = [&](int s, int& row, int& cnt) {
    const unsigned o = s < nseq ? (unsigned)((phase(s) * kWT + t) * 8) : kOff;
    row = bld_i(Rm, o);
    cnt = bld_i(Rm, o + 4);
  };
  // entries (absent ones read column 0, value 0) and N_ii^-1 at step s
  auto ld_ent = [&](int s, int row, int cnt, int* c, T* v, T& ni) {
    const int ph = s < nseq ? phase(s) : 0;
#pragma unroll
    for (int e = 0; e < kWNE; e++) {
      const int i = (ph * kWNE + e) * kWT + t;
      c[e] = bld_i(Rc, e < cnt ? (unsigned)i * 4u : kOff);
      v[e] = bld(Rv, e < cnt ? (unsigned)(i * (int)sizeof(T)) : kOff, (T*)nullptr);
    }
    ni = bld(Rn, row >= 0 && cnt > 0 ? (unsigned)(row * (int)sizeof(T)) : kOff, (T*)nullptr);
  };
  // one step: q = sum_j A_ij L_jj^-1 r_j over each row of the group, then
  // x_i += p_i and r_j -= A_ji p_i
  auto step = [&](int row, int cnt, const int* c, const T* v, T ni) {
    T q = 0;
#pragma unroll
    for (int e = 0; e < kWNE; e++) q += v[e] * ls[c[e]] * rs[c[e]];
    q = wlr_sum(q);
    const T pv = q * ni;
    if (cnt > 0 && ln == 0) xs[row] += pv;
    // the group's two rows share residual entries: the second row's lanes
    // update after the first's (a wave's LDS accesses complete in order;
    // the empty asm keeps the compiler from reordering or reusing loads)
    if (half == 0) {
#pragma unroll
      for (int e = 0; e < kWNE; e++)
        if (e < cnt) rs[c[e]] -= v[e] * pv;
    }
    asm volatile("" ::: "memory");
    if (half == 1) {
#pragma unroll
      for (int e = 0; e < kWNE; e++)
        if (e < cnt) rs[c[e]] -= v[e] * pv;
    }
  };
  // two register sets, used in turn (unrolled by two so that neither is
  // copied into the other, which would wait for the loads in flight)
  int rowA, cntA, rowB, cntB, cA[kWNE], cB[kWNE];
  T vA[kWNE], vB[kWNE], nA, nB;
  ld_meta(0, rowA, cntA);
  ld_ent(0, rowA, cntA, cA, vA, nA);
  ld_meta(1, rowB, cntB);
  lds_barrier();
  for (int s = 0; s < nseq; s += 2) {
    ld_ent(s + 1, rowB, cntB, cB, vB, nB);
    step(rowA, cntA, cA, vA, nA);
    ld_meta(s + 2, rowA, cntA);
    lds_barrier();
    if (s + 1 == nseq) break;
    ld_ent(s + 2, rowA, cntA, cA, vA, nA);
    step(rowB, cntB, cB, vB, nB);
    ld_meta(s + 3, rowB, cntB);
    lds_barrier();
  }
  for (int i = t; i < ndof; i += kWT) {
    r[i] = rs[i];
    x[i] = xs[i];
  }
}

// The lattice path of an LSGS colour phase.  The groups of one colour lie on
// a lattice (every 5th P2 node in each direction, or every 3rd vertex), and
// on the uniform mesh every group more than a few half-steps from the
// boundary has the group class of its node type: the class depends only on
// the parities of the node's position (a P2 vertex node, or the midpoint of
// a horizontal, vertical or diagonal edge; one type for the vertex groups).
// There the group's record (its two unknowns and its class's entry range) is
// formed from its index, and the classes of the four node types are staged in
// LDS once per workgroup, so a wave's only global loads are the residual's
// gathers (no record, no class entries).  Groups are taken in the record
// path's order (row by row over the whole colour lattice, all node types
// interleaved), which keeps the residual lines that neighbouring groups share
// in cache; the groups near the boundary take the record path in the same
// launch.
struct LatPhase {
  int hx0, hy0;  // first interior group's position on the half-step lattice
  int nx, ny;    // interior groups per row, rows
  int step;      // lattice step between neighbouring groups (half-steps)
  int ent[4];    // class entry range per node type t = (hx & 1) + 2 (hy & 1)
  int len[4];
  int nblk;      // workgroups of the interior part; the record part follows
  int bi, bj;    // index bases of the fields of the group's two unknowns
  int p1;        // the groups sit at P1 vertices (pressure and its multiplier)
  int g0, ng;    // records [g0, g0 + ng) of the phase's remaining groups
};

template <typename T>
__global__ __launch_bounds__(kGNT) void ks_lsgs_lat(LatPhase P, const int4* __restrict__ grp,
                                                    const int* __restrict__ gent,
                                                    const typename T2of<T>::type* __restrict__ gval,
                                                    const T* __restrict__ glinv,
                                                    const typename T2of<T>::type* __restrict__ gninv, SGeo geo,
                                                    T* __restrict__ x, T* __restrict__ r) {
  constexpr int WPB = kGNT / 64;  // waves per workgroup
  const int blk = blockIdx.x, wave = (int)threadIdx.x / 64;
  if (blk >= P.nblk) {  // record part
    grp_wave<T>((blk - P.nblk) * WPB + wave, P.g0, P.ng, grp, gent, gval, glinv, gninv, geo, x, r);
    return;
  }
  // the classes of the four node types in LDS, read by every group of the
  // workgroup (type t's entries at [t * kMaxGroupEntries, + len), its N^-1
  // pair at the first), so that the phase's global accesses are the
  // residual's gathers and scatters
  using T2 = typename T2of<T>::type;
  constexpr int ME = kMaxGroupEntries;
  __shared__ int s_ent[4 * ME];
  __shared__ T2 s_val[4 * ME], s_ninv[4 * ME];
  __shared__ T s_linv[4 * ME];
  for (int q = (int)threadIdx.x; q < 4 * ME; q += kGNT) {
    const int t = q / ME, k = q - t * ME;
    // selects: no indexing of the argument by a thread value
    const int e0 = t == 0 ? P.ent[0] : t == 1 ? P.ent[1] : t == 2 ? P.ent[2] : P.ent[3];
    const int l0 = t == 0 ? P.len[0] : t == 1 ? P.len[1] : t == 2 ? P.len[2] : P.len[3];
    if (k < l0) {
      s_ent[q] = gent[e0 + k];
      s_val[q] = gval[e0 + k];
      s_linv[q] = glinv[e0 + k];
      if (k == 0) s_ninv[q] = gninv[e0];
    }
  }
  __syncthreads();
  auto rec = [&](int g, int& hx, int& hy) {
    const int gl = g >= 0 ? g : 0;
    const int gy = gl / P.nx, gx = gl - gy * P.nx;
    hx = P.hx0 + P.step * gx;
    hy = P.hy0 + P.step * gy;
    const int t = (hx & 1) + 2 * (hy & 1);
    const int l0 = t == 0 ? P.len[0] : t == 1 ? P.len[1] : t == 2 ? P.len[2] : P.len[3];
    const int b = P.p1 ? (hy >> 1) * (geo.n + 1) + (hx >> 1) : (hy - 1) * geo.m + (hx - 1);
    return g >= 0 ? make_int4(P.bi + b, P.bj + b, t * ME, t * ME + l0) : make_int4(0, 0, 0, 0);
  };
  grp_wave_of<T>(blk * WPB + wave, P.nx * P.ny, rec, s_ent, s_val, s_linv, s_ninv, geo, x, r);
}

// value of lane u (u uniform), read as scalars: independent of the exec mask
__device__ inline double bcast(double v, int u) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, u), hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), u);
  return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}
__device__ inline float bcast(float v, int u) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(unsigned, v), u));
}

// One colour phase of the patch smoother: x_P += tau A_PP^-1 r_P,
// r -= tau A_{:,P} A_PP^-1 r_P.  Patches (one per vertex) come in patch
// classes: patches whose unknowns sit at the same lattice offsets from the
// vertex and whose rows agree share the LU factors of A_PP (row-major, FP64,
// then the reciprocals of U's diagonal; the unknown codes also in the row
// order of the pivoting) and the union U of their rows'
// columns with the dense block A_{P,U} (stored [u][k]).  Class record:
// (m, first unknown code, first LU entry, first union code), (|U|, first
// coefficient).  Two patches per wave (a patch has at most 30 unknowns),
// one per half: lane c of a half keeps row c of the factors in registers and
// entry c of the vector; the substitutions go by columns, each finished
// entry broadcast by a scalar read.  Patches of one colour share no residual entry, so each lane gathers
// its union entries of r once and writes r_k - sum_u A_uk du_u once (du_u
// broadcast from lane u by a scalar read).
template <typename T>
__global__ __launch_bounds__(kSNT) void ks_vanka(int p0, int npatch, const int2* __restrict__ order,
                                                 const int4* __restrict__ cinfo, const int2* __restrict__ cun,
                                                 const int* __restrict__ pcode,
                                                 const int* __restrict__ pcodep, const double* __restrict__ lu,
                                                 const int* __restrict__ ucode, const T* __restrict__ coef,
                                                 SGeo geo, double tau, T* __restrict__ x, T* __restrict__ r) {
  const int w = blockIdx.x * (kSNT / 64) + threadIdx.x / 64;
  if (2 * w >= npatch) return;  // uniform per wave
  const int h = (threadIdx.x % 64) / 32, c = threadIdx.x % 32;  // half-wave h takes patch 2w + h
  const int t = 2 * w + h;
  const bool live = t < npatch;
  const int2 qc = live ? order[p0 + t] : make_int2(0, 0);  // (vertex, patch class)
  const int q = qc.x;
  const int4 ci = cinfo[qc.y];
  const int2 cu = cun[qc.y];
  const int m = live ? ci.x : 0, hx = 2 * (q % (geo.n + 1)), hy = 2 * (q / (geo.n + 1));
  const bool on = c < m;
  // entry j of this half's patch, broadcast from lane j of the half
  auto bc = [&](double v, int j) {
    const double v0 = bcast(v, j), v1 = bcast(v, 32 + j);
    return h ? v1 : v0;
  };
  const double* a = lu + ci.z;
  double arow[kMaxPatch];  // row c of the factors
#pragma unroll
  for (int j = 0; j < kMaxPatch; j++) arow[j] = (on && j < m) ? a[c * m + j] : 0.0;
  const double dinv = on ? a[m * m + c] : 0.0;  // 1 / u_cc
  // permuted right-hand side: entry c = r at the patch unknown in pivot position c
  double y = on ? (double)r[sent_col(geo, pcodep[ci.y + c], hx, hy)] : 0.0;
  // forward substitution with the unit lower factor, by columns: y_j is
  // final once columns < j are done; it is broadcast and the rows below
  // subtract L_cj y_j
#pragma unroll
  for (int j = 0; j + 1 < kMaxPatch; j++) {
    const double yj = bc(y, j);
    if (c > j && j + 1 < m) y -= arow[j] * yj;
  }
  // back substitution with the upper factor, by columns from the last
#pragma unroll
  for (int j = kMaxPatch - 1; j >= 0; j--) {
    if (c == j && j < m) y *= dinv;
    const double yj = bc(y, j);
    if (c < j && j < m) y -= arow[j] * yj;
  }
  const T du = on ? (T)(tau * y) : (T)0;
  if (on) x[sent_col(geo, pcode[ci.y + c], hx, hy)] += du;
  // union entries c, c + 32, c + 64 of U: loads at clamped indices (a lane
  // past |U| stores nothing), coefficients of unknowns u >= m meet du_u = 0
  const int nu = live ? cu.x : 1, mc = m > 0 ? m : 1;
  int col[3], kk[3];
  T rk[3], upd[3];
#pragma unroll
  for (int sl = 0; sl < 3; sl++) {
    const int k = c + 32 * sl;
    kk[sl] = k < nu ? k : nu - 1;
    col[sl] = sent_col(geo, ucode[ci.w + kk[sl]], hx, hy);
    rk[sl] = r[col[sl]];
    upd[sl] = 0;
  }
  // du_u broadcast once per u, used by the three slots (unrolled by 5: full
  // unrolling hoists all 90 coefficient loads and needs 258 registers)
#pragma unroll 5
  for (int u = 0; u < kMaxPatch; u++) {
    const T d0 = bcast(du, u), d1 = bcast(du, 32 + u), d = h ? d1 : d0;
    const int row = cu.y + (u < mc ? u : mc - 1) * nu;
#pragma unroll
    for (int sl = 0; sl < 3; sl++) upd[sl] += coef[row + kk[sl]] * d;
  }
#pragma unroll
  for (int sl = 0; sl < 3; sl++)
    if (live && c + 32 * sl < nu) r[col[sl]] = rk[sl] - upd[sl];
}

// pressure and multiplier means: per-block partial sums of w.p and w.mu
template <typename T>
__global__ __launch_bounds__(kSNT) void ks_wsum(int np, const double* __restrict__ w, const T* __restrict__ vp,
                                                const T* __restrict__ vm, double* __restrict__ part) {
  const int q = blockIdx.x * kSNT + threadIdx.x;
  const double a = q < np ? w[q] * (double)vp[q] : 0.0;
  const double b = q < np ? w[q] * (double)vm[q] : 0.0;
  block_store(a, &part[2 * blockIdx.x]);
  __syncthreads();
  block_store(b, &part[2 * blockIdx.x + 1]);
}

// s[0], s[1] = the two means (sums / wsum)
__global__ __launch_bounds__(kSNT) void ks_means(const double* __restrict__ part, int nb, double inv_w,
                                                 double* __restrict__ s) {
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nb; k += kSNT) {
    a += part[2 * k];
    b += part[2 * k + 1];
  }
  block_store(a, &s[0]);
  __syncthreads();
  block_store(b, &s[1]);
  __syncthreads();
  if (threadIdx.x == 0) {
    s[0] *= inv_w;
    s[1] *= inv_w;
  }
}

template <typename T>
__global__ __launch_bounds__(kSNT) void ks_shift(int np, const double* __restrict__ s, T* __restrict__ vp,
                                                 T* __restrict__ vm) {
  const int q = blockIdx.x * kSNT + threadIdx.x;
  if (q >= np) return;
  vp[q] = (T)((double)vp[q] - s[0]);
  vm[q] = (T)((double)vm[q] - s[1]);
}

// coarsest level: LU solve of the system bordered by the two mean constraints
template <typename T>
__global__ __launch_bounds__(256) void ks_coarse(int N, int NB, const double* __restrict__ lu,
                                                 const int* __restrict__ piv, const T* __restrict__ f,
                                                 T* __restrict__ x) {
  __shared__ double b[512];
  const int tid = threadIdx.x;
  for (int i = tid; i < NB; i += blockDim.x) b[i] = i < N ? (double)f[i] : 0.0;
  __syncthreads();
  if (tid == 0)
    for (int k = 0; k < NB; k++)
      if (piv[k] != k) {
        const double t = b[k];
        b[k] = b[piv[k]];
        b[piv[k]] = t;
      }
  __syncthreads();
  for (int k = 0; k < NB; k++) {
    const double bk = b[k];
    for (int i = k + 1 + tid; i < NB; i += blockDim.x) b[i] -= lu[(size_t)i * NB + k] * bk;
    __syncthreads();
  }
  for (int k = NB - 1; k >= 0; k--) {
    if (tid == 0) b[k] /= lu[(size_t)k * NB + k];
    __syncthreads();
    const double bk = b[k];
    for (int i = tid; i < k; i += blockDim.x) b[i] -= lu[(size_t)i * NB + k] * bk;
    __syncthreads();
  }
  for (int i = tid; i < N; i += blockDim.x) x[i] = (T)b[i];
}

// f = (M vd_1; M vd_2; 0; 0; 0; 0) with the scalar P2 mass M
__global__ __launch_bounds__(kSNT) void ks_rhs(int nv, int ndof, const int* __restrict__ rp,
                                               const int* __restrict__ col, const double* __restrict__ val,
                                               const double* __restrict__ vd, double* __restrict__ f) {
  const int i = blockIdx.x * kSNT + threadIdx.x;
  if (i >= ndof) return;
  double s = 0.0;
  if (i < 2 * nv) {
    const int c = i / nv, a = i - c * nv;
    for (int k = rp[a]; k < rp[a + 1]; k++) s += val[k] * vd[c * nv + col[k]];
  }
  f[i] = s;
}

inline int blocks_for(int n, int nt = kSNT) { return (n + nt - 1) / nt; }
// blocks of the row kernels (grid-stride over groups of kRows rows)
inline int row_blocks(int n) { return std::min(blocks_for(n, kRows), 4096); }
// blocks of the one-thread-per-row kernels (grid-stride over kSNT rows)
inline int thread_blocks(int n) { return std::min(blocks_for(n), 4096); }

template <typename T>
struct Dev {
  T* p = nullptr;
};

template <typename T>
hipError_t upload(T** d, const T* h, size_t n) {
  if (n == 0) {
    *d = nullptr;
    return hipSuccess;
  }
  hipError_t e = hipMalloc(d, n * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*d, h, n * sizeof(T), hipMemcpyHostToDevice);
}

}  // namespace

// ------------------------------------------------------------ solver object

struct StokesLevel {
  int l = 0, n = 0, nv = 0, np = 0, ndof = 0;
  SGeo geo{};
  // A by stencil classes: class of each row, entry range of each class,
  // packed (field, offset) entries and their values
  int *A_cls = nullptr, *A_ptr = nullptr, *A_ent = nullptr;
  double* A_val = nullptr;
  float* A_val32 = nullptr;
  int nclass = 0;
  double *Ld = nullptr, *Linv = nullptr, *Ninv = nullptr;
  float *Linv32 = nullptr, *Ninv32 = nullptr;
  // prolongation from level l-1 and restriction to it (its transpose)
  int *P_rp = nullptr, *P_col = nullptr, *R_rp = nullptr, *R_col = nullptr;
  double *P_val = nullptr, *R_val = nullptr;
  float *P_val32 = nullptr, *R_val32 = nullptr;
  // LSGS colour phases: groups of two unknowns, phase g spans groups [gph[g], gph[g+1])
  std::vector<int> gph;
  // merged groups: records (i, j, first entry, end), group-class entries and coefficient pairs
  int4* mgroups = nullptr;
  int* g_ent = nullptr;
  double2 *g_val = nullptr, *g_ninv = nullptr;
  double* g_linv = nullptr;
  float2 *g_val32 = nullptr, *g_ninv32 = nullptr;
  float* g_linv32 = nullptr;
  // the lattice path of the phases (see ks_lsgs_lat): per phase its
  // interior lattice, and the remaining groups' records (l_rec)
  std::vector<LatPhase> lph;
  int4* l_rec = nullptr;
  // the same phases laid out for the one-workgroup sweep (small levels only)
  int2* w_meta = nullptr;
  int* w_col = nullptr;
  double* w_val = nullptr;
  float* w_val32 = nullptr;
  // patch smoother: patches (one per vertex) ordered by colour, phase spans vph
  // patch smoother: patches (one per vertex) ordered by colour, phase spans vph;
  // patch classes (see ks_vanka)
  int2* v_order = nullptr;  // (vertex, patch class) in colour order
  int *v_code = nullptr, *v_pcodep = nullptr, *v_ucode = nullptr;
  int4* v_info = nullptr;
  int2* v_un = nullptr;
  double *v_lu = nullptr, *v_coef = nullptr;
  float* v_coef32 = nullptr;
  std::vector<int> vph;
  // pressure-mean weights
  double* w = nullptr;
  double wsum = 0.0;
  // workspace (the finest level takes the caller's x and f)
  double *x = nullptr, *f = nullptr, *r = nullptr, *p = nullptr;
  float *x32 = nullptr, *f32 = nullptr, *r32 = nullptr, *p32 = nullptr;
};

struct Stokes {
  int level = 0, k0 = 1, smoother = 1, nu1 = 2, nu2 = 2, gamma = 1;
  double alpha = 1.0, tau = 0.35;
  bool fp32 = false;
  bool wg_sweep = true;  // one-workgroup LSGS sweeps on small levels (MGKKT_NO_WG_SWEEP unset)
  bool lattice = true;   // lattice path of the LSGS phases (MGKKT_NO_STOKES_LATTICE unset)
  std::vector<StokesLevel> lv;  // lv[l - k0]
  int *M_rp = nullptr, *M_col = nullptr;  // scalar P2 mass of the finest level (right-hand side)
  double* M_val = nullptr;
  double* lu = nullptr;  // bordered coarsest LU
  int* piv = nullptr;
  int nlu = 0, ncoarse = 0;
  double* part = nullptr;  // partial sums of the mean projection
  double* means = nullptr;
  size_t npart = 0;
  std::vector<void*> owned;
  StokesLevel& L(int l) { return lv[l - k0]; }
};

namespace {

template <typename T>
hipError_t up(Stokes* S, T** d, const std::vector<T>& h) {
  hipError_t e = upload(d, h.data(), h.size());
  if (e == hipSuccess && *d) S->owned.push_back(*d);
  return e;
}

template <typename T>
hipError_t zalloc(Stokes* S, T** d, size_t n) {
  hipError_t e = hipMalloc(d, n * sizeof(T));
  if (e == hipSuccess) S->owned.push_back(*d);
  return e;
}

#define SCHK(expr)                          \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return e_;        \
  } while (0)

std::vector<float> to32(const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); }

// Patch classes (see ks_vanka): the class key is the unknown offsets, the
// union offsets and the coefficient block, looked up by hash and compared in
// full; A_PP is a sub-block of the block, so the LU factors (partial
// pivoting) are computed once per class.
struct PatchClasses {
  std::vector<int> cls, code, pcodep, ucode;  // pcodep: the unknown codes in pivot order
  std::vector<int4> info;
  std::vector<int2> un;
  std::vector<double> lu, coef;
};
bool build_patch_classes(const HCsr& A, const SGeo& g, const std::vector<int>& dptr, const std::vector<int>& dof,
                         PatchClasses& P, std::string* err) {
  const int np = (int)dptr.size() - 1;
  std::unordered_map<unsigned long long, std::vector<int>> seen;
  P.cls.assign(np, 0);
  std::vector<int> code, ucode;
  std::vector<double> coef;
  std::unordered_map<int, int> upos;
  auto enc = [&](int i, int hx, int hy, int& e) {
    int cx, cy;
    spos(g, i, cx, cy);
    const int dx = cx - hx, dy = cy - hy;
    if (dx < -kEntOff || dx >= 256 - kEntOff || dy < -kEntOff || dy >= 256 - kEntOff) return false;
    e = sfield(g, i) | ((dx + kEntOff) << 8) | ((dy + kEntOff) << 16);
    return sent_col(g, e, hx, hy) == i;
  };
  for (int q = 0; q < np; q++) {
    const int b = dptr[q], m = dptr[q + 1] - b;
    const int hx = 2 * (q % (g.n + 1)), hy = 2 * (q / (g.n + 1));
    code.resize(m);
    ucode.clear();
    upos.clear();
    bool ok = true;
    for (int u = 0; u < m && ok; u++) ok = enc(dof[b + u], hx, hy, code[u]);
    for (int u = 0; u < m && ok; u++)
      for (int k = A.rp[dof[b + u]]; k < A.rp[dof[b + u] + 1] && ok; k++)
        if (!upos.count(A.col[k])) {
          int e;
          ok = enc(A.col[k], hx, hy, e);
          upos[A.col[k]] = (int)ucode.size();
          ucode.push_back(e);
        }
    if (!ok) {
      *err = "stokes: a patch unknown or column is not a lattice offset of its vertex";
      return false;
    }
    const int nu = (int)ucode.size();
    if (nu > 96) {
      *err = "stokes: a patch couples to more than 96 unknowns";
      return false;
    }
    coef.assign((size_t)m * nu, 0.0);
    for (int u = 0; u < m; u++)
      for (int k = A.rp[dof[b + u]]; k < A.rp[dof[b + u] + 1]; k++) coef[(size_t)u * nu + upos[A.col[k]]] = A.val[k];
    unsigned long long h = 0x243F6A8885A308D3ull;
    auto mix = [&](unsigned long long v) {
      h = (h ^ v) * 0x9E3779B97F4A7C15ull;
      h ^= h >> 29;
    };
    auto mixd = [&](double v) {
      unsigned long long bb;
      std::memcpy(&bb, &v, 8);
      mix(bb);
    };
    mix((unsigned)m);
    mix((unsigned)nu);
    for (int u = 0; u < m; u++) mix((unsigned)code[u]);
    for (int k = 0; k < nu; k++) mix((unsigned)ucode[k]);
    for (double v : coef) mixd(v);
    int id = -1;
    for (int c : seen[h]) {
      const int4 ci = P.info[c];
      const int2 cu = P.un[c];
      if (ci.x != m || cu.x != nu) continue;
      bool same = std::equal(code.begin(), code.end(), P.code.begin() + ci.y) &&
                  std::equal(ucode.begin(), ucode.end(), P.ucode.begin() + ci.w) &&
                  std::equal(coef.begin(), coef.end(), P.coef.begin() + cu.y);
      if (same) {
        id = c;
        break;
      }
    }
    if (id < 0) {
      // A_PP from the block: A(d_u, d_v) is the coefficient at d_v's union
      // position (zero where d_v is no column of any patch row)
      std::vector<double> a((size_t)m * m, 0.0);
      for (int v = 0; v < m; v++) {
        auto it = upos.find(dof[b + v]);
        if (it == upos.end()) continue;
        for (int u = 0; u < m; u++) a[(size_t)u * m + v] = coef[(size_t)u * nu + it->second];
      }
      std::vector<int> pv;
      bool okf;
      lu_dense(m, a, pv, okf);
      if (!okf) {
        *err = "stokes: singular patch matrix";
        return false;
      }
      // the row swaps of the factorisation as one permutation: after them,
      // position k holds the entry that started at pm[k]
      std::vector<int> pm(m);
      for (int k = 0; k < m; k++) pm[k] = k;
      for (int k = 0; k < m; k++) std::swap(pm[k], pm[pv[k]]);
      id = (int)P.info.size();
      seen[h].push_back(id);
      P.info.push_back(make_int4(m, (int)P.code.size(), (int)P.lu.size(), (int)P.ucode.size()));
      P.un.push_back(make_int2(nu, (int)P.coef.size()));
      P.code.insert(P.code.end(), code.begin(), code.end());
      for (int k = 0; k < m; k++) P.pcodep.push_back(code[pm[k]]);
      P.lu.insert(P.lu.end(), a.begin(), a.end());
      for (int k = 0; k < m; k++) P.lu.push_back(1.0 / a[(size_t)k * m + k]);  // 1 / u_kk after the factors
      P.ucode.insert(P.ucode.end(), ucode.begin(), ucode.end());
      P.coef.insert(P.coef.end(), coef.begin(), coef.end());
    }
    P.cls[q] = id;
  }
  return true;
}

// Merged groups (see ks_lsgs_grp): entries of row i in its order, then those
// of row j that row i lacks.  Both unknowns of a group sit at one lattice
// position, so the merged entries follow from the two rows' stencil classes;
// the group class adds L^-1 of the merged columns and the two N^-1 (equal
// for all groups of the class, up to the hash's full comparison).
bool build_group_classes(const ClassA& C, const SGeo& g, const std::vector<int2>& grp,
                         const std::vector<double>& Linv, const std::vector<double>& Ninv, std::vector<int4>& rec,
                         std::vector<int>& ent, std::vector<double2>& val, std::vector<double>& lv,
                         std::vector<double2>& nv, std::string* err) {
  std::unordered_map<unsigned long long, std::vector<int>> pair_union;  // (class i, class j) -> merged entries
  std::unordered_map<unsigned long long, std::vector<int2>> seen;       // hash -> classes
  std::vector<std::vector<double2>> pair_vals;
  rec.resize(grp.size());
  ent.clear();
  val.clear();
  lv.clear();
  nv.clear();
  std::vector<double> lk;
  for (size_t q = 0; q < grp.size(); q++) {
    const int i = grp[q].x, j = grp[q].y;
    int hx, hy, jx, jy;
    spos(g, i, hx, hy);
    spos(g, j, jx, jy);
    if (jx != hx || jy != hy) {
      *err = "stokes: the two unknowns of a group sit at different lattice positions";
      return false;
    }
    const int ci = C.row_cls[i], cj = C.row_cls[j];
    const unsigned long long key = ((unsigned long long)(unsigned)ci << 32) | (unsigned)cj;
    auto pu = pair_union.find(key);
    if (pu == pair_union.end()) {
      std::vector<int> u;
      std::vector<double2> uv;
      for (int k = C.ptr[ci]; k < C.ptr[ci + 1]; k++) {
        u.push_back(C.ent[k]);
        uv.push_back(make_double2(C.val[k], 0.0));
      }
      for (int k = C.ptr[cj]; k < C.ptr[cj + 1]; k++) {
        size_t t = 0;
        while (t < u.size() && u[t] != C.ent[k]) t++;
        if (t == u.size()) {
          u.push_back(C.ent[k]);
          uv.push_back(make_double2(0.0, C.val[k]));
        } else {
          uv[t].y = C.val[k];
        }
      }
      if ((int)u.size() > kMaxGroupEntries) {
        *err = "stokes: a group has more entries than the LSGS kernel takes";
        return false;
      }
      u.push_back((int)pair_vals.size());  // index of the values, after the entries
      pair_vals.push_back(uv);
      pu = pair_union.emplace(key, u).first;
    }
    const std::vector<int>& u = pu->second;
    const int len = (int)u.size() - 1;
    const std::vector<double2>& uv = pair_vals[u[len]];
    lk.resize(len);
    unsigned long long h = key * 0x9E3779B97F4A7C15ull;
    auto mix = [&](double v) {
      unsigned long long b;
      std::memcpy(&b, &v, 8);
      h = (h ^ b) * 0x9E3779B97F4A7C15ull;
      h ^= h >> 29;
    };
    for (int t = 0; t < len; t++) {
      lk[t] = Linv[sent_col(g, u[t], hx, hy)];
      mix(lk[t]);
    }
    mix(Ninv[i]);
    mix(Ninv[j]);
    int id = -1;
    std::vector<int2>& cand = seen[h];  // (first entry, length) of the classes with this hash
    for (const int2 bl : cand) {
      const int b = bl.x;
      bool same = bl.y == len && nv[b].x == Ninv[i] && nv[b].y == Ninv[j];
      for (int t = 0; t < len && same; t++)
        same = ent[b + t] == u[t] && val[b + t].x == uv[t].x && val[b + t].y == uv[t].y && lv[b + t] == lk[t];
      if (same) {
        id = b;
        break;
      }
    }
    if (id < 0) {
      id = (int)ent.size();
      cand.push_back(make_int2(id, len));
      for (int t = 0; t < len; t++) {
        ent.push_back(u[t]);
        val.push_back(uv[t]);
        lv.push_back(lk[t]);
        nv.push_back(t == 0 ? make_double2(Ninv[i], Ninv[j]) : make_double2(0.0, 0.0));
      }
    }
    rec[q] = make_int4(i, j, id, id + len);
  }
  return true;
}

// The lattice path of the LSGS phases (see ks_lsgs_lat).  Per phase: for
// each node type the class of the group nearest the centre, and the largest
// boundary distance of a group of that type with another class; the groups
// farther from the boundary than all of these form the interior, which must
// be a full rectangle of the phase's lattice (checked), and each interior
// group's unknowns and class are checked against its record.  The other
// groups stay records, in phase order.
bool build_lattice(const SGeo& g, const std::vector<int4>& rec, const std::vector<int>& gph,
                   std::vector<LatPhase>& lph, std::vector<int4>& lrec, std::string* err) {
  const int n = g.n, m = g.m;
  lph.assign(gph.size() - 1, LatPhase{});
  lrec.clear();
  auto bdist = [&](int q) {
    int hx, hy;
    spos(g, rec[q].x, hx, hy);
    return std::min(std::min(hx, 2 * n - hx), std::min(hy, 2 * n - hy));
  };
  for (size_t p = 0; p + 1 < gph.size(); p++) {
    LatPhase& P = lph[p];
    const int q0 = gph[p], q1 = gph[p + 1];
    std::vector<char> inlat(q1 - q0, 0);
    P.g0 = (int)lrec.size();
    if (q1 > q0) {
      const int fi = sfield(g, rec[q0].x), fj = sfield(g, rec[q0].y);
      P.bi = sbase(g, fi);
      P.bj = sbase(g, fj);
      P.p1 = sp1(fi) ? 1 : 0;
      // per node type: the centre group's class
      int centre[4] = {-1, -1, -1, -1};
      long best[4] = {-1, -1, -1, -1};
      for (int q = q0; q < q1; q++) {
        int hx, hy;
        spos(g, rec[q].x, hx, hy);
        const int t = (hx & 1) + 2 * (hy & 1);
        const long d = (long)(hx - n) * (hx - n) + (long)(hy - n) * (hy - n);
        if (best[t] < 0 || d < best[t]) best[t] = d, centre[t] = q;
      }
      int margin = -1;
      for (int q = q0; q < q1; q++) {
        int hx, hy;
        spos(g, rec[q].x, hx, hy);
        const int t = (hx & 1) + 2 * (hy & 1);
        if (rec[q].z != rec[centre[t]].z) margin = std::max(margin, bdist(q));
      }
      int hx0 = 1 << 30, hy0 = 1 << 30, hx1 = -1, hy1 = -1, cnt = 0, step = 0;
      for (int q = q0; q < q1; q++)
        if (bdist(q) > margin) {
          int hx, hy;
          spos(g, rec[q].x, hx, hy);
          hx0 = std::min(hx0, hx), hx1 = std::max(hx1, hx), hy0 = std::min(hy0, hy), hy1 = std::max(hy1, hy);
          cnt++;
        }
      for (int q = q0; q < q1 && cnt > 1; q++)
        if (bdist(q) > margin) {
          int hx, hy;
          spos(g, rec[q].x, hx, hy);
          step = std::gcd(step, std::gcd(hx - hx0, hy - hy0));
        }
      if (cnt == 1) step = 1;
      const bool full = cnt > 0 && (long)((hx1 - hx0) / step + 1) * ((hy1 - hy0) / step + 1) == cnt;
      if (full) {
        P.hx0 = hx0, P.hy0 = hy0, P.step = step;
        P.nx = (hx1 - hx0) / step + 1, P.ny = (hy1 - hy0) / step + 1;
        for (int t = 0; t < 4; t++) {
          P.ent[t] = centre[t] >= 0 ? rec[centre[t]].z : 0;
          P.len[t] = centre[t] >= 0 ? rec[centre[t]].w - rec[centre[t]].z : 0;
        }
        for (int q = q0; q < q1; q++) {
          if (bdist(q) <= margin) continue;
          int hx, hy;
          spos(g, rec[q].x, hx, hy);
          const int t = (hx & 1) + 2 * (hy & 1);
          const int b = P.p1 ? (hy >> 1) * (n + 1) + (hx >> 1) : (hy - 1) * m + (hx - 1);
          if ((hx - hx0) % step || (hy - hy0) % step || rec[q].x != P.bi + b || rec[q].y != P.bj + b ||
              rec[q].z != P.ent[t] || rec[q].w != P.ent[t] + P.len[t]) {
            *err = "stokes: lattice group mismatch";
            return false;
          }
          inlat[q - q0] = 1;
        }
        P.nblk = (cnt + kGNT / kGLR - 1) / (kGNT / kGLR);
      }
      for (int q = q0; q < q1; q++)
        if (!inlat[q - q0]) lrec.push_back(rec[q]);
    }
    P.ng = (int)lrec.size() - P.g0;
  }
  return true;
}

// Lanes of the one-workgroup sweep: group slot k of a phase goes to wave
// k / kWG, its two rows to consecutive runs of kWLR lanes, and entry e of a
// row to lane e % kWLR, register e / kWLR.  Levels whose residual, x and
// L^-1 exceed the kernel's LDS, or with a phase of more than kWSlots groups,
// keep the launch per phase.
hipError_t build_wg_phases(Stokes* S, StokesLevel& L, const HCsr& A, const std::vector<int2>& grp) {
  const int nph = (int)L.gph.size() - 1;
  if (3 * (size_t)L.ndof * sizeof(double) > (size_t)kWLdsBytes) return hipSuccess;
  for (int ph = 0; ph < nph; ph++)
    if (L.gph[ph + 1] - L.gph[ph] > kWSlots) return hipSuccess;
  std::vector<int2> meta((size_t)nph * kWT, make_int2(-1, 0));
  std::vector<int> col((size_t)nph * kWNE * kWT, 0);
  std::vector<double> val(col.size(), 0.0);
  for (int ph = 0; ph < nph; ph++)
    for (int g = L.gph[ph]; g < L.gph[ph + 1]; g++) {
      const int k = g - L.gph[ph];
      for (int h = 0; h < 2; h++) {
        const int row = h ? grp[g].y : grp[g].x, kb = A.rp[row], len = A.rp[row + 1] - kb;
        for (int ln = 0; ln < kWLR; ln++) {
          const int t = (k / kWG) * 64 + (k % kWG) * 2 * kWLR + h * kWLR + ln;
          const int cnt = len > ln ? (len - ln + kWLR - 1) / kWLR : 0;
          meta[(size_t)ph * kWT + t] = make_int2(row, cnt);
          for (int e = 0; e < cnt; e++) {
            const size_t o = ((size_t)ph * kWNE + e) * kWT + t;
            col[o] = A.col[kb + ln + e * kWLR];
            val[o] = A.val[kb + ln + e * kWLR];
          }
        }
      }
    }
  SCHK(up(S, &L.w_meta, meta));
  SCHK(up(S, &L.w_col, col));
  SCHK(up(S, &L.w_val, val));
  if (S->fp32) SCHK(up(S, &L.w_val32, to32(val)));
  return hipSuccess;
}

hipError_t build_level(Stokes* S, int l, bool finest, std::string* err) {
  StokesLevel& L = S->L(l);
  const int n = 1 << l, m = 2 * n - 1;
  L.l = l;
  L.n = n;
  L.nv = m * m;
  L.np = (n + 1) * (n + 1);
  L.ndof = 4 * L.nv + 2 * L.np;
  Blocks B;
  if (!assemble_blocks(n, B)) {
    *err = "stokes: element assembly overflow";
    return hipErrorInvalidValue;
  }
  const HCsr A = assemble_kkt(n, S->alpha, B);
  L.geo = SGeo{n, m, L.nv, L.np};
  ClassA CA;
  if (!build_classes(A, L.geo, CA, err)) return hipErrorInvalidValue;
  L.nclass = (int)CA.ptr.size() - 1;
  SCHK(up(S, &L.A_cls, CA.row_cls));
  SCHK(up(S, &L.A_ptr, CA.ptr));
  SCHK(up(S, &L.A_ent, CA.ent));
  SCHK(up(S, &L.A_val, CA.val));
  // L = (W^, W^, P^, W^/alpha, W^/alpha, P^/alpha), W^ = diag(M + alpha^1/2 K), P^ = alpha diag(D W^-1 D^T)
  std::vector<double> Ld(L.ndof), W(L.nv);
  for (int a = 0; a < L.nv; a++) W[a] = entry(B.Ms, a, a) + std::sqrt(S->alpha) * entry(B.Ks, a, a);
  const int op = 2 * L.nv, ol = 2 * L.nv + L.np, om = 4 * L.nv + L.np;
  for (int a = 0; a < L.nv; a++) {
    Ld[a] = Ld[L.nv + a] = W[a];
    Ld[ol + a] = Ld[ol + L.nv + a] = W[a] / S->alpha;
  }
  for (int q = 0; q < L.np; q++) {
    double s = 0.0;
    for (int c = 0; c < 2; c++)
      for (int k = B.D[c].rp[q]; k < B.D[c].rp[q + 1]; k++) s += B.D[c].val[k] * B.D[c].val[k] / W[B.D[c].col[k]];
    Ld[op + q] = S->alpha * s;
    Ld[om + q] = s;
  }
  std::vector<double> Linv(L.ndof), Ninv(L.ndof);
  for (int i = 0; i < L.ndof; i++) Linv[i] = 1.0 / Ld[i];
  for (int i = 0; i < L.ndof; i++) {  // N_ii = sum_j A_ij^2 / L_jj (A symmetric)
    double s = 0.0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; k++) s += A.val[k] * A.val[k] * Linv[A.col[k]];
    Ninv[i] = 1.0 / s;
  }
  SCHK(up(S, &L.Ld, Ld));
  SCHK(up(S, &L.Linv, Linv));
  SCHK(up(S, &L.Ninv, Ninv));
  SCHK(up(S, &L.w, B.w));
  L.wsum = 0.0;
  for (double v : B.w) L.wsum += v;
  if (S->fp32) {
    SCHK(up(S, &L.A_val32, to32(CA.val)));
    SCHK(up(S, &L.Linv32, to32(Linv)));
    SCHK(up(S, &L.Ninv32, to32(Ninv)));
  }
  std::vector<int2> grp;
  colour_groups(n, grp, L.gph);
  {
    std::vector<int4> rec;
    std::vector<int> gent;
    std::vector<double2> gval, gni;
    std::vector<double> glv;
    if (!build_group_classes(CA, L.geo, grp, Linv, Ninv, rec, gent, gval, glv, gni, err)) return hipErrorInvalidValue;
    SCHK(up(S, &L.mgroups, rec));
    SCHK(up(S, &L.g_ent, gent));
    SCHK(up(S, &L.g_val, gval));
    SCHK(up(S, &L.g_linv, glv));
    SCHK(up(S, &L.g_ninv, gni));
    auto f2 = [](const std::vector<double2>& v) {
      std::vector<float2> o(v.size());
      for (size_t t = 0; t < v.size(); t++) o[t] = make_float2((float)v[t].x, (float)v[t].y);
      return o;
    };
    if (S->fp32) {
      SCHK(up(S, &L.g_val32, f2(gval)));
      SCHK(up(S, &L.g_ninv32, f2(gni)));
      SCHK(up(S, &L.g_linv32, to32(glv)));
    }
    if (S->lattice && (S->smoother == MG_LSGS || S->smoother == MG_SLSGS)) {
      std::vector<int4> lrec;
      if (!build_lattice(L.geo, rec, L.gph, L.lph, lrec, err)) return hipErrorInvalidValue;
      SCHK(up(S, &L.l_rec, lrec));
    }
  }
  if (S->wg_sweep && (S->smoother == MG_LSGS || S->smoother == MG_SLSGS)) SCHK(build_wg_phases(S, L, A, grp));
  // patches of the patch smoother
  if (S->smoother == MG_VANKA) {
    std::vector<int> dptr, dof, order;
    if (!build_patches(n, dptr, dof, order, L.vph, err)) return hipErrorInvalidValue;
    PatchClasses P;
    if (!build_patch_classes(A, L.geo, dptr, dof, P, err)) return hipErrorInvalidValue;
    std::vector<int2> oc(order.size());
    for (size_t t = 0; t < order.size(); t++) oc[t] = make_int2(order[t], P.cls[order[t]]);
    SCHK(up(S, &L.v_order, oc));
    SCHK(up(S, &L.v_info, P.info));
    SCHK(up(S, &L.v_un, P.un));
    SCHK(up(S, &L.v_code, P.code));
    SCHK(up(S, &L.v_pcodep, P.pcodep));
    SCHK(up(S, &L.v_lu, P.lu));
    SCHK(up(S, &L.v_ucode, P.ucode));
    SCHK(up(S, &L.v_coef, P.coef));
    if (S->fp32) SCHK(up(S, &L.v_coef32, to32(P.coef)));
  }
  // transfers from / to level l-1
  if (l > S->k0) {
    const HCsr P = assemble_prolongation(n / 2), R = transpose(P);
    SCHK(up(S, &L.P_rp, P.rp));
    SCHK(up(S, &L.P_col, P.col));
    SCHK(up(S, &L.P_val, P.val));
    SCHK(up(S, &L.R_rp, R.rp));
    SCHK(up(S, &L.R_col, R.col));
    SCHK(up(S, &L.R_val, R.val));
    if (S->fp32) {
      SCHK(up(S, &L.P_val32, to32(P.val)));
      SCHK(up(S, &L.R_val32, to32(R.val)));
    }
  }
  // workspace
  const size_t nd = L.ndof;
  if (!finest) {
    SCHK(zalloc(S, &L.x, nd));
    SCHK(zalloc(S, &L.f, nd));
  }
  SCHK(zalloc(S, &L.r, nd));
  SCHK(zalloc(S, &L.p, nd));
  if (S->fp32) {
    SCHK(zalloc(S, &L.x32, nd));
    SCHK(zalloc(S, &L.f32, nd));
    SCHK(zalloc(S, &L.r32, nd));
    SCHK(zalloc(S, &L.p32, nd));
  }
  if (finest) {
    SCHK(up(S, &S->M_rp, B.Ms.rp));
    SCHK(up(S, &S->M_col, B.Ms.col));
    SCHK(up(S, &S->M_val, B.Ms.val));
  }
  if (l == S->k0) {
    // bordered coarsest matrix [[A, C], [C^T, 0]], C = mean weights in the p and mu rows
    const int N = L.ndof, NB = N + 2;
    std::vector<double> a((size_t)NB * NB, 0.0);
    for (int r = 0; r < N; r++)
      for (int k = A.rp[r]; k < A.rp[r + 1]; k++) a[(size_t)r * NB + A.col[k]] = A.val[k];
    for (int q = 0; q < L.np; q++) {
      a[(size_t)(op + q) * NB + N] = a[(size_t)N * NB + op + q] = B.w[q];
      a[(size_t)(om + q) * NB + N + 1] = a[(size_t)(N + 1) * NB + om + q] = B.w[q];
    }
    std::vector<int> pv;
    bool ok;
    lu_dense(NB, a, pv, ok);
    if (!ok) {
      *err = "stokes: singular coarsest matrix";
      return hipErrorInvalidValue;
    }
    SCHK(up(S, &S->lu, a));
    SCHK(up(S, &S->piv, pv));
    S->nlu = NB;
    S->ncoarse = N;
  }
  return hipSuccess;
}

template <typename T>
struct SV;
template <>
struct SV<double> {
  static double* x(StokesLevel& L) { return L.x; }
  static double* f(StokesLevel& L) { return L.f; }
  static double* r(StokesLevel& L) { return L.r; }
  static double* p(StokesLevel& L) { return L.p; }
  static const double* A(StokesLevel& L) { return L.A_val; }
  static const double* P(StokesLevel& L) { return L.P_val; }
  static const double* R(StokesLevel& L) { return L.R_val; }
  static const double* Linv(StokesLevel& L) { return L.Linv; }
  static const double* Ninv(StokesLevel& L) { return L.Ninv; }
  static const double* W(StokesLevel& L) { return L.w_val; }
  static const double2* G(StokesLevel& L) { return L.g_val; }
  static const double* VC(StokesLevel& L) { return L.v_coef; }
  static const double* GL(StokesLevel& L) { return L.g_linv; }
  static const double2* GN(StokesLevel& L) { return L.g_ninv; }
};
template <>
struct SV<float> {
  static float* x(StokesLevel& L) { return L.x32; }
  static float* f(StokesLevel& L) { return L.f32; }
  static float* r(StokesLevel& L) { return L.r32; }
  static float* p(StokesLevel& L) { return L.p32; }
  static const float* A(StokesLevel& L) { return L.A_val32; }
  static const float* P(StokesLevel& L) { return L.P_val32; }
  static const float* R(StokesLevel& L) { return L.R_val32; }
  static const float* Linv(StokesLevel& L) { return L.Linv32; }
  static const float* Ninv(StokesLevel& L) { return L.Ninv32; }
  static const float* W(StokesLevel& L) { return L.w_val32; }
  static const float2* G(StokesLevel& L) { return L.g_val32; }
  static const float* VC(StokesLevel& L) { return L.v_coef32; }
  static const float* GL(StokesLevel& L) { return L.g_linv32; }
  static const float2* GN(StokesLevel& L) { return L.g_ninv32; }
};

// A of level L by stencil classes; the transfers P (from level l-1) and R (to it) as CSR
template <typename T>
ClassRows<T> a_rows(StokesLevel& L) {
  return ClassRows<T>{L.A_cls, L.A_ptr, L.A_ent, SV<T>::A(L), L.geo};
}
template <typename T>
CsrRows<T> p_rows(StokesLevel& L) {
  return CsrRows<T>{L.P_rp, L.P_col, SV<T>::P(L)};
}
template <typename T>
CsrRows<T> r_rows(StokesLevel& L) {
  return CsrRows<T>{L.R_rp, L.R_col, SV<T>::R(L)};
}

template <typename T>
hipError_t s_resid(StokesLevel& L, const T* f, const T* x, T* r, hipStream_t s) {
  hipLaunchKernelGGL((ks_resid<T, 0, ClassRows<T>>), dim3(thread_blocks(L.ndof)), dim3(kSNT), 0, s, L.ndof, a_rows<T>(L),
                     f, x, r, (const double*)nullptr, (double*)nullptr);
  return hipGetLastError();
}

template <typename T>
hipError_t s_smooth(Stokes* S, StokesLevel& L, T* x, T* r, int steps, hipStream_t s) {
  const ClassRows<T> A = a_rows<T>(L);
  for (int it = 0; it < steps; it++) {
    switch (S->smoother) {
      case MG_NE:
        hipLaunchKernelGGL((ks_ne_p<T, ClassRows<T>>), dim3(row_blocks(L.ndof)), dim3(kSNT), 0, s, L.ndof, A,
                           SV<T>::Linv(L), (T)S->tau, (const T*)r, x, SV<T>::p(L));
        hipLaunchKernelGGL((ks_ne_r<T, ClassRows<T>>), dim3(row_blocks(L.ndof)), dim3(kSNT), 0, s, L.ndof, A,
                           (const T*)SV<T>::p(L), r);
        break;
      case MG_LSGS:
      case MG_SLSGS: {
        const int nph = (int)L.gph.size() - 1;
        const int sweeps = S->smoother == MG_SLSGS ? 2 : 1;
        if (L.w_meta) {  // every step in one workgroup
          if (steps > 0)
            hipLaunchKernelGGL((ks_lsgs_wg<T>), dim3(1), dim3(kWT), 0, s, L.ndof, nph, steps * sweeps * nph, sweeps,
                               (const int2*)L.w_meta, (const int*)L.w_col, SV<T>::W(L), SV<T>::Linv(L),
                               SV<T>::Ninv(L), x, r);
          return hipGetLastError();
        }
        for (int sw = 0; sw < sweeps; sw++)
          for (int k = 0; k < nph; k++) {
            const int ph = sw == 0 ? k : nph - 1 - k;
            const int g0 = L.gph[ph], ng = L.gph[ph + 1] - g0;
            if (ng == 0) continue;  // a colour without nodes on a small level
            if (!L.lph.empty()) {
              const LatPhase& P = L.lph[ph];
              const int nb = P.nblk + (P.ng + kGNT / kGLR - 1) / (kGNT / kGLR);
              hipLaunchKernelGGL((ks_lsgs_lat<T>), dim3(nb), dim3(kGNT), 0, s, P, (const int4*)L.l_rec,
                                 (const int*)L.g_ent, SV<T>::G(L), SV<T>::GL(L), SV<T>::GN(L), L.geo, x, r);
              continue;
            }
            hipLaunchKernelGGL((ks_lsgs_grp<T>), dim3(blocks_for(ng, kGNT / kGLR)), dim3(kGNT), 0, s, g0, ng,
                               (const int4*)L.mgroups, (const int*)L.g_ent, SV<T>::G(L), SV<T>::GL(L), SV<T>::GN(L),
                               L.geo, x, r);
          }
        break;
      }
      case MG_VANKA:
        for (int ph = 0; ph + 1 < (int)L.vph.size(); ph++) {
          const int p0 = L.vph[ph], npch = L.vph[ph + 1] - p0;
          hipLaunchKernelGGL((ks_vanka<T>), dim3(blocks_for(npch, kSNT / 32)), dim3(kSNT), 0, s, p0, npch,
                             (const int2*)L.v_order, (const int4*)L.v_info, (const int2*)L.v_un,
                             (const int*)L.v_code, (const int*)L.v_pcodep, (const double*)L.v_lu,
                             (const int*)L.v_ucode, SV<T>::VC(L), L.geo, S->tau, x, r);
        }
        break;
    }
  }
  return hipGetLastError();
}

template <typename T>
hipError_t s_project(Stokes* S, StokesLevel& L, T* x, hipStream_t s) {
  const int nb = blocks_for(L.np);
  T* vp = x + 2 * L.nv;
  T* vm = x + 4 * L.nv + L.np;
  hipLaunchKernelGGL((ks_wsum<T>), dim3(nb), dim3(kSNT), 0, s, L.np, (const double*)L.w, (const T*)vp, (const T*)vm,
                     S->part);
  hipLaunchKernelGGL(ks_means, dim3(1), dim3(kSNT), 0, s, (const double*)S->part, nb, 1.0 / L.wsum, S->means);
  hipLaunchKernelGGL((ks_shift<T>), dim3(nb), dim3(kSNT), 0, s, L.np, (const double*)S->means, vp, vm);
  return hipGetLastError();
}

template <typename T>
hipError_t s_coarse(Stokes* S, const T* f, T* x, hipStream_t s) {
  hipLaunchKernelGGL((ks_coarse<T>), dim3(1), dim3(256), 0, s, S->ncoarse, S->nlu, (const double*)S->lu,
                     (const int*)S->piv, f, x);
  return hipGetLastError();
}

// one iterate on level l (section 2): smoothing, restriction of the defect,
// gamma coarse iterates from zero (exact bordered solve on k0), prolongation,
// residual, smoothing; r is current on entry when `current`
template <typename T>
hipError_t s_cycle(Stokes* S, int l, const T* f, T* x, T* r, bool current, hipStream_t s) {
  if (l == S->k0) return s_coarse<T>(S, f, x, s);
  StokesLevel& L = S->L(l);
  StokesLevel& C = S->L(l - 1);
  if (!current) SCHK(s_resid<T>(L, f, x, r, s));
  SCHK(s_smooth<T>(S, L, x, r, S->nu1, s));
  const bool to_k0 = (l - 1 == S->k0);
  hipLaunchKernelGGL((ks_spmv<T, 0, CsrRows<T>>), dim3(row_blocks(C.ndof)), dim3(kSNT), 0, s, C.ndof, r_rows<T>(L),
                     (const T*)r, SV<T>::f(C), to_k0 ? (T*)nullptr : SV<T>::x(C), to_k0 ? (T*)nullptr : SV<T>::r(C));
  SCHK(hipGetLastError());
  for (int g = 0; g < S->gamma; g++)
    SCHK(s_cycle<T>(S, l - 1, SV<T>::f(C), SV<T>::x(C), SV<T>::r(C), g == 0, s));
  hipLaunchKernelGGL((ks_spmv_add1<T, CsrRows<T>>), dim3(thread_blocks(L.ndof)), dim3(kSNT), 0, s, L.ndof,
                     p_rows<T>(L), (const T*)SV<T>::x(C), x);
  SCHK(hipGetLastError());
  SCHK(s_resid<T>(L, f, x, r, s));
  return s_smooth<T>(S, L, x, r, S->nu2, s);
}

}  // namespace

// ---------------------------------------------------------------- interface

static int stokes_create_body(Stokes* S, int level, int k0, double alpha, const mg_opts& o, Stokes** out, std::string* err);

// A host exception in the assembly (allocation, or a matrix too large for its
// 32-bit row pointers) releases the partly built solver and propagates to the
// C ABI's guard, which turns it into a status code.
int stokes_create(int level, int k0, double alpha, const mg_opts& o, Stokes** out, std::string* err) {
  Stokes* S = new Stokes;
  try {
    return stokes_create_body(S, level, k0, alpha, o, out, err);
  } catch (...) {
    stokes_destroy(S);
    throw;
  }
}

static int stokes_create_body(Stokes* S, int level, int k0, double alpha, const mg_opts& o, Stokes** out, std::string* err) {
  S->level = level;
  S->k0 = k0;
  S->alpha = alpha;
  S->smoother = o.smoother;
  S->nu1 = o.nu1;
  S->nu2 = o.nu2;
  S->gamma = o.gamma;
  S->tau = o.tau;
  S->fp32 = o.precision == MG_FP32_IR;
  S->wg_sweep = std::getenv("MGKKT_NO_WG_SWEEP") == nullptr;
  S->lattice = std::getenv("MGKKT_NO_STOKES_LATTICE") == nullptr;
  S->lv.resize(level - k0 + 1);
  for (int l = k0; l <= level; l++) {
    const hipError_t e = build_level(S, l, l == level, err);
    if (e != hipSuccess) {
      if (err->empty()) *err = std::string("stokes setup: ") + hipGetErrorString(e);
      stokes_destroy(S);
      return e == hipErrorOutOfMemory ? MG_ENOMEM : (e == hipErrorInvalidValue ? MG_EINVAL : MG_EHIP);
    }
  }
  S->npart = 2 * (size_t)blocks_for(S->L(level).np) + 2;
  if (zalloc(S, &S->part, S->npart) != hipSuccess || zalloc(S, &S->means, 2) != hipSuccess) {
    stokes_destroy(S);
    return MG_ENOMEM;
  }
  *out = S;
  return MG_OK;
}

void stokes_destroy(Stokes* S) {
  if (!S) return;
  for (void* p : S->owned) (void)hipFree(p);
  delete S;
}

size_t stokes_len(const Stokes* S, int level) {
  if (!S || level < S->k0 || level > S->level) return 0;
  return (size_t)S->lv[level - S->k0].ndof;
}

size_t stokes_partials(const Stokes* S) {
  const int n = S->lv.back().ndof;
  return (size_t)std::max(blocks_for(n), row_blocks(n));
}

void stokes_set(Stokes* S, const mg_opts& o) {
  S->nu1 = o.nu1;
  S->nu2 = o.nu2;
  S->gamma = o.gamma;
  S->tau = o.tau;
}

hipError_t stokes_rhs(Stokes* S, const double* vd, double* f, hipStream_t s) {
  StokesLevel& L = S->lv.back();
  hipLaunchKernelGGL(ks_rhs, dim3(blocks_for(L.ndof)), dim3(kSNT), 0, s, L.nv, L.ndof, (const int*)S->M_rp,
                     (const int*)S->M_col, (const double*)S->M_val, vd, f);
  return hipGetLastError();
}

hipError_t stokes_apply(Stokes* S, int l, const double* x, double* y, hipStream_t s) {
  StokesLevel& L = S->L(l);
  hipLaunchKernelGGL((ks_resid<double, 0, ClassRows<double>>), dim3(thread_blocks(L.ndof)), dim3(kSNT), 0, s, L.ndof,
                     a_rows<double>(L), (const double*)nullptr, x, y, (const double*)nullptr, (double*)nullptr);
  return hipGetLastError();
}

int stokes_residual_parts(const Stokes* S, int l) {
  if (!S || l < S->k0 || l > S->level) return 0;
  return thread_blocks(S->lv[l - S->k0].ndof);
}

hipError_t stokes_residual(Stokes* S, int l, const double* f, const double* x, double* r, double* part,
                           int norm_mode, int* nparts, hipStream_t s) {
  StokesLevel& L = S->L(l);
  const int nb = thread_blocks(L.ndof);
  if (nparts) *nparts = nb;
  const ClassRows<double> A = a_rows<double>(L);
  if (!part)
    hipLaunchKernelGGL((ks_resid<double, 0, ClassRows<double>>), dim3(nb), dim3(kSNT), 0, s, L.ndof, A, f, x, r,
                       (const double*)L.Linv, part);
  else if (norm_mode == 2)
    hipLaunchKernelGGL((ks_resid<double, 2, ClassRows<double>>), dim3(nb), dim3(kSNT), 0, s, L.ndof, A, f, x, r,
                       (const double*)L.Linv, part);
  else
    hipLaunchKernelGGL((ks_resid<double, 1, ClassRows<double>>), dim3(nb), dim3(kSNT), 0, s, L.ndof, A, f, x, r,
                       (const double*)L.Linv, part);
  return hipGetLastError();
}

hipError_t stokes_vnorm(Stokes* S, const double* v, double* part, int norm_mode, int* nparts, hipStream_t s) {
  StokesLevel& L = S->lv.back();
  const int nb = blocks_for(L.ndof);
  *nparts = nb;
  if (norm_mode == 2)
    hipLaunchKernelGGL((ks_vnorm<2>), dim3(nb), dim3(kSNT), 0, s, L.ndof, v, (const double*)L.Linv, part);
  else
    hipLaunchKernelGGL((ks_vnorm<1>), dim3(nb), dim3(kSNT), 0, s, L.ndof, v, (const double*)L.Linv, part);
  return hipGetLastError();
}

hipError_t stokes_smooth(Stokes* S, int l, double* x, double* r, int steps, hipStream_t s) {
  return s_smooth<double>(S, S->L(l), x, r, steps, s);
}

hipError_t stokes_restrict(Stokes* S, int l, const double* r, double* fc, hipStream_t s) {
  StokesLevel& L = S->L(l);
  StokesLevel& C = S->L(l - 1);
  hipLaunchKernelGGL((ks_spmv<double, 0, CsrRows<double>>), dim3(row_blocks(C.ndof)), dim3(kSNT), 0, s, C.ndof,
                     r_rows<double>(L), r, fc, (double*)nullptr, (double*)nullptr);
  return hipGetLastError();
}

hipError_t stokes_prolong_add(Stokes* S, int l, const double* xc, double* x, hipStream_t s) {
  StokesLevel& L = S->L(l);
  hipLaunchKernelGGL((ks_spmv_add1<double, CsrRows<double>>), dim3(thread_blocks(L.ndof)), dim3(kSNT), 0, s, L.ndof,
                     p_rows<double>(L), xc, x);
  return hipGetLastError();
}

hipError_t stokes_coarse_solve(Stokes* S, const double* f, double* x, hipStream_t s) {
  return s_coarse<double>(S, f, x, s);
}

hipError_t stokes_project(Stokes* S, int l, double* x, hipStream_t s) { return s_project<double>(S, S->L(l), x, s); }

// one FP64 cycle on the finest level with r current, then the mean projection
hipError_t stokes_cycle(Stokes* S, const double* f, double* x, double* r, bool current, hipStream_t s) {
  SCHK(s_cycle<double>(S, S->level, f, x, r, current, s));
  return s_project<double>(S, S->lv.back(), x, s);
}

double* stokes_fine_r(Stokes* S) { return S->lv.back().r; }

// one refinement step: FP32 cycle from zero on the scaled FP64 residual r
// (||r||^2 in nrm2 on the device), x += s c in FP64, then the mean
// projection of the FP64 iterate
hipError_t stokes_ir_step(Stokes* S, double* x, hipStream_t s, const double* nrm2, int inner) {
  StokesLevel& L = S->lv.back();
  const size_t n = L.ndof;
  SCHK(launch_to_f32_scaled(L.r, n, nrm2, L.f32, L.r32, s));
  SCHK(launch_zero_f32(L.x32, n, s));
  // inner_cycles FP32 cycles from zero; the residual is current for the first
  for (int k = 0; k < inner; k++) SCHK(s_cycle<float>(S, S->level, L.f32, L.x32, L.r32, k == 0, s));
  SCHK(launch_axpy_f32(L.x32, n, nrm2, x, s));
  return s_project<double>(S, L, x, s);
}

}  // namespace mgk
