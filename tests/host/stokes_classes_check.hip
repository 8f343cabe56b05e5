// Host-side check of the Stokes operator compression (no GPU needed):
//  - stencil classes: every row's columns and values come back exactly;
//  - merged LSGS groups: the union of a group's two rows, both coefficients,
//    L^-1 per entry and the two N^-1 come back exactly, and the groups of a
//    colour phase share no column;
//  - patch classes: every patch's unknowns, LU factors and pivots (computed
//    here from the CSR entries) and its coefficient block over the union of
//    its rows' columns come back exactly, and the patches of a colour share
//    no union column;
//  - the lattice path of the LSGS phases: with the smoother's own L^-1 and
//    N^-1, each phase's interior groups (their records formed from the
//    index as the kernel does) and its remaining records cover the phase's
//    groups exactly once, and each formed record equals the group's own.
// Prints one line per size and exits non-zero on any mismatch.
#include "../../paper_1502_03917_amd/csrc/stokes.hip"
#include <cstdio>
#include <map>
using namespace mgk;

static long check_rows(const HCsr& A, const SGeo& g, const ClassA& C) {
  long bad = 0;
  for (int i = 0; i < A.nrows; i++) {
    int hx, hy;
    spos(g, i, hx, hy);
    const int c = C.row_cls[i];
    if (C.ptr[c + 1] - C.ptr[c] != A.rp[i + 1] - A.rp[i]) { bad++; continue; }
    for (int k = 0; k < C.ptr[c + 1] - C.ptr[c]; k++)
      if (sent_col(g, C.ent[C.ptr[c] + k], hx, hy) != A.col[A.rp[i] + k] || C.val[C.ptr[c] + k] != A.val[A.rp[i] + k]) bad++;
  }
  return bad;
}

static long check_groups(int n, const HCsr& A, const SGeo& g, const ClassA& C) {
  std::vector<int2> grp;
  std::vector<int> ph;
  colour_groups(n, grp, ph);
  // any positive diagonal: a position-dependent one exercises the class key
  std::vector<double> Linv(A.nrows), Ninv(A.nrows);
  for (int i = 0; i < A.nrows; i++) Linv[i] = 1.0 + (i % 7 == 0 ? 0.5 : 0.0);
  for (int i = 0; i < A.nrows; i++) {
    double s = 0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; k++) s += A.val[k] * A.val[k] * Linv[A.col[k]];
    Ninv[i] = 1.0 / s;
  }
  std::vector<int4> rec;
  std::vector<int> ent;
  std::vector<double2> val, nv;
  std::vector<double> lv;
  std::string err;
  if (!build_group_classes(C, g, grp, Linv, Ninv, rec, ent, val, lv, nv, &err)) { printf("%s\n", err.c_str()); return 1; }
  long bad = 0;
  for (size_t q = 0; q < grp.size(); q++) {
    const int4 u = rec[q];
    if (u.x != grp[q].x || u.y != grp[q].y) bad++;
    int hx, hy;
    spos(g, u.x, hx, hy);
    std::map<int, double2> got, want;
    for (int k = u.z; k < u.w; k++) {
      const int c = sent_col(g, ent[k], hx, hy);
      if (got.count(c) || lv[k] != Linv[c]) bad++;
      got[c] = val[k];
    }
    if (nv[u.z].x != Ninv[u.x] || nv[u.z].y != Ninv[u.y]) bad++;
    for (int k = A.rp[u.x]; k < A.rp[u.x + 1]; k++) want[A.col[k]].x = A.val[k];
    for (int k = A.rp[u.y]; k < A.rp[u.y + 1]; k++) want[A.col[k]].y = A.val[k];
    if (got.size() != want.size()) { bad++; continue; }
    for (auto& kv : want) {
      auto it = got.find(kv.first);
      if (it == got.end() || it->second.x != kv.second.x || it->second.y != kv.second.y) bad++;
    }
  }
  for (size_t p = 0; p + 1 < ph.size(); p++) {
    std::map<int, int> owner;
    for (int q = ph[p]; q < ph[p + 1]; q++) {
      int hx, hy;
      spos(g, rec[q].x, hx, hy);
      for (int k = rec[q].z; k < rec[q].w; k++) {
        const int c = sent_col(g, ent[k], hx, hy);
        if (owner.count(c) && owner[c] != q) bad++;
        owner[c] = q;
      }
    }
  }
  return bad;
}

static long check_patches(int n, const HCsr& A, const SGeo& g) {
  std::vector<int> dptr, dof, order, ph;
  std::string err;
  if (!build_patches(n, dptr, dof, order, ph, &err)) { printf("%s\n", err.c_str()); return 1; }
  PatchClasses P;
  if (!build_patch_classes(A, g, dptr, dof, P, &err)) { printf("%s\n", err.c_str()); return 1; }
  long bad = 0;
  for (int q = 0; q + 1 < (int)dptr.size(); q++) {
    const int4 ci = P.info[P.cls[q]];
    const int2 cu = P.un[P.cls[q]];
    const int b = dptr[q], mm = dptr[q + 1] - b, hx = 2 * (q % (n + 1)), hy = 2 * (q / (n + 1));
    if (ci.x != mm) { bad++; continue; }
    std::vector<double> a((size_t)mm * mm);
    for (int u = 0; u < mm; u++)
      for (int v = 0; v < mm; v++) a[(size_t)u * mm + v] = entry(A, dof[b + u], dof[b + v]);
    std::vector<int> pv;
    bool okf;
    lu_dense(mm, a, pv, okf);
    std::vector<int> pm(mm);
    for (int k = 0; k < mm; k++) pm[k] = k;
    for (int k = 0; k < mm; k++) std::swap(pm[k], pm[pv[k]]);
    for (int u = 0; u < mm; u++)
      if (sent_col(g, P.code[ci.y + u], hx, hy) != dof[b + u] || sent_col(g, P.pcodep[ci.y + u], hx, hy) != dof[b + pm[u]]) bad++;
    for (int k = 0; k < mm * mm; k++)
      if (P.lu[ci.z + k] != a[k]) bad++;
    for (int k = 0; k < mm; k++)
      if (P.lu[ci.z + mm * mm + k] != 1.0 / a[(size_t)k * mm + k]) bad++;
    std::map<int, int> kofcol;
    for (int k = 0; k < cu.x; k++) {
      const int c = sent_col(g, P.ucode[ci.w + k], hx, hy);
      if (kofcol.count(c)) bad++;
      kofcol[c] = k;
    }
    for (int u = 0; u < mm; u++) {
      std::map<int, double> row;
      for (int k = A.rp[dof[b + u]]; k < A.rp[dof[b + u] + 1]; k++) row[A.col[k]] = A.val[k];
      for (auto& kc : kofcol) {
        const double want = row.count(kc.first) ? row[kc.first] : 0.0;
        if (P.coef[cu.y + (size_t)u * cu.x + kc.second] != want) bad++;
      }
      for (auto& rc : row)
        if (!kofcol.count(rc.first)) bad++;
    }
  }
  for (size_t p = 0; p + 1 < ph.size(); p++) {
    std::map<int, int> owner;
    for (int t = ph[p]; t < ph[p + 1]; t++) {
      const int q = order[t], hx = 2 * (q % (n + 1)), hy = 2 * (q / (n + 1));
      const int4 ci = P.info[P.cls[q]];
      for (int k = 0; k < P.un[P.cls[q]].x; k++) {
        const int c = sent_col(g, P.ucode[ci.w + k], hx, hy);
        if (owner.count(c) && owner[c] != q) bad++;
        owner[c] = q;
      }
    }
  }
  return bad;
}

static long check_lattice(int n, double alpha, const Blocks& B, const HCsr& A, const SGeo& g, const ClassA& C,
                          double* frac) {
  // L^-1 and N^-1 as the solver sets them up
  const int nv = g.nv, np = g.np, ndof = 4 * nv + 2 * np;
  std::vector<double> Ld(ndof), W(nv);
  for (int a = 0; a < nv; a++) W[a] = entry(B.Ms, a, a) + std::sqrt(alpha) * entry(B.Ks, a, a);
  const int op = 2 * nv, ol = 2 * nv + np, om = 4 * nv + np;
  for (int a = 0; a < nv; a++) {
    Ld[a] = Ld[nv + a] = W[a];
    Ld[ol + a] = Ld[ol + nv + a] = W[a] / alpha;
  }
  for (int q = 0; q < np; q++) {
    double s = 0.0;
    for (int c = 0; c < 2; c++)
      for (int k = B.D[c].rp[q]; k < B.D[c].rp[q + 1]; k++) s += B.D[c].val[k] * B.D[c].val[k] / W[B.D[c].col[k]];
    Ld[op + q] = alpha * s;
    Ld[om + q] = s;
  }
  std::vector<double> Linv(ndof), Ninv(ndof);
  for (int i = 0; i < ndof; i++) Linv[i] = 1.0 / Ld[i];
  for (int i = 0; i < ndof; i++) {
    double s = 0.0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; k++) s += A.val[k] * A.val[k] * Linv[A.col[k]];
    Ninv[i] = 1.0 / s;
  }
  std::vector<int2> grp;
  std::vector<int> ph;
  colour_groups(n, grp, ph);
  std::vector<int4> rec;
  std::vector<int> ent;
  std::vector<double2> val, nvv;
  std::vector<double> lv;
  std::string err;
  if (!build_group_classes(C, g, grp, Linv, Ninv, rec, ent, val, lv, nvv, &err)) { printf("%s\n", err.c_str()); return 1; }
  std::vector<LatPhase> lph;
  std::vector<int4> lrec;
  if (!build_lattice(g, rec, ph, lph, lrec, &err)) { printf("%s\n", err.c_str()); return 1; }
  if (lph.size() + 1 != ph.size()) return 1;
  long bad = 0, nlat = 0;
  for (size_t p = 0; p + 1 < ph.size(); p++) {
    const LatPhase& P = lph[p];
    std::map<std::pair<int, int>, int> own;  // (i, j) -> its record
    for (int t = ph[p]; t < ph[p + 1]; t++) own[{rec[t].x, rec[t].y}] = t;
    std::map<std::pair<int, int>, int> seen;  // (i, j) -> times covered
    if (P.nblk != (P.nx * P.ny + kGNT / kGLR - 1) / (kGNT / kGLR)) bad++;
    for (int gi = 0; gi < P.nx * P.ny; gi++) {
      // the record as the kernel forms it
      const int hx = P.hx0 + P.step * (gi % P.nx), hy = P.hy0 + P.step * (gi / P.nx);
      const int t = (hx & 1) + 2 * (hy & 1);
      const int b = P.p1 ? (hy >> 1) * (n + 1) + (hx >> 1) : (hy - 1) * g.m + (hx - 1);
      const int4 u = make_int4(P.bi + b, P.bj + b, P.ent[t], P.ent[t] + P.len[t]);
      seen[{u.x, u.y}]++;
      nlat++;
      auto it = own.find({u.x, u.y});
      if (it == own.end()) { bad++; continue; }
      const int4 v = rec[it->second];
      if (v.z != u.z || v.w != u.w) bad++;
      int vx, vy;
      spos(g, v.x, vx, vy);
      if (vx != hx || vy != hy) bad++;
    }
    for (int t = P.g0; t < P.g0 + P.ng; t++) seen[{lrec[t].x, lrec[t].y}]++;
    if ((int)seen.size() != ph[p + 1] - ph[p]) bad++;
    for (int t = ph[p]; t < ph[p + 1]; t++) {
      auto it = seen.find({rec[t].x, rec[t].y});
      if (it == seen.end() || it->second != 1) bad++;
    }
  }
  *frac = rec.empty() ? 0.0 : (double)nlat / rec.size();
  return bad;
}

int main() {
  for (int n : {2, 4, 8, 16, 64}) {
    Blocks B;
    if (!assemble_blocks(n, B)) { printf("assembly overflow\n"); return 1; }
    for (double alpha : {1.0, 1e-4}) {
      const HCsr A = assemble_kkt(n, alpha, B);
      const int m = 2 * n - 1;
      const SGeo g{n, m, m * m, (n + 1) * (n + 1)};
      ClassA C;
      std::string err;
      if (!build_classes(A, g, C, &err)) { printf("n=%d: %s\n", n, err.c_str()); return 1; }
      const long br = check_rows(A, g, C), bg = check_groups(n, A, g, C), bp = check_patches(n, A, g);
      double frac = 0.0;
      const long bl = check_lattice(n, alpha, B, A, g, C, &frac);
      printf("n=%d alpha=%g rows=%d bad rows=%ld groups=%ld patches=%ld lattice=%ld (%.3f of the groups)\n", n, alpha,
             A.nrows, br, bg, bp, bl, frac);
      if (br || bg || bp || bl) return 1;
    }
  }
  printf("ok\n");
  return 0;
}
