// HIP kernels of the all-at-once multigrid cycle for the Poisson-control KKT
// system (Takacs, arXiv 1502.03917, section 1 eq. mp2 and section 2) on gfx950.
//
// All kernels are matrix-free: the P1 mass matrix M and K = Klap + M act as
// 7-point stencils on the (n+1)x(n+1) vertex grid.  Vertices at least one
// (residual) or two (smoothers) rows away from the boundary use the constant
// interior coefficients held in the Lev struct (kernel arguments, scalar
// registers); the few boundary vertices read their coefficients from the small
// per-level class table.  The path is HBM-bound (about 2-4 flop per byte), so
// there is no MFMA: each lane owns one vertex and neighbouring lanes read
// neighbouring addresses.
#include "mg_internal.hpp"

namespace mgk {

namespace {

constexpr int kBX = 64;  // one wavefront along a grid row
constexpr int kBY = 4;
constexpr int kNT = kBX * kBY;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// deterministic block sum of one value per thread (256 threads), stored by thread 0
__device__ inline void block_sum_store(double v, double* out) {
  __shared__ double sh[kNT / 64];
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  v = wave_sum(v);
  if ((tid & 63) == 0) sh[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kNT / 64; w++) s += sh[w];
    *out = s;
  }
}

template <typename T>
__device__ inline void coef_MK(const Lev& L, int i, int j, T M[kNDir], T K[kNDir]) {
  const int c = cls3(i, L.n) * 3 + cls3(j, L.n);
#pragma unroll
  for (int d = 0; d < kNDir; d++) {
    M[d] = (T)L.tab->M[c][d];
    K[d] = (T)L.tab->K[c][d];
  }
}

__device__ inline bool inside(const Lev& L, int i, int j) { return i >= 0 && i <= L.n && j >= 0 && j <= L.n; }

// (A x)_v for both rows of vertex v = (i, j)
template <typename T>
__device__ inline void apply_at(const Lev& L, int i, int j, const T* __restrict__ x, T& ay, T& al) {
  const int v = j * L.ld + i;
  const T* xy = x;
  const T* xl = x + L.V;
  const T ai = (T)L.ainv;
  if (i >= 1 && i < L.n && j >= 1 && j < L.n) {
    const int ld = L.ld;
    const T yc = xy[v], lc = xl[v];
    const T ya = xy[v + 1] + xy[v - 1] + xy[v + ld] + xy[v - ld];
    const T yg = xy[v + ld + 1] + xy[v - ld - 1];
    const T la = xl[v + 1] + xl[v - 1] + xl[v + ld] + xl[v - ld];
    const T lg = xl[v + ld + 1] + xl[v - ld - 1];
    const T Mc = (T)L.Mc, Mo = (T)L.Mo, Kc = (T)L.Kc, Ka = (T)L.Ka, Kd = (T)L.Kd;
    ay = Mc * yc + Mo * (ya + yg) + (Kc * lc + Ka * la + Kd * lg);
    al = (Kc * yc + Ka * ya + Kd * yg) - ai * (Mc * lc + Mo * (la + lg));
  } else {
    T M[kNDir], K[kNDir];
    coef_MK(L, i, j, M, K);
    ay = 0;
    al = 0;
#pragma unroll
    for (int d = 0; d < kNDir; d++) {
      const int ii = i + kDI[d], jj = j + kDJ[d];
      if (!inside(L, ii, jj)) continue;
      const int m = jj * L.ld + ii;
      ay += M[d] * xy[m] + K[d] * xl[m];
      al += K[d] * xy[m] - ai * M[d] * xl[m];
    }
  }
}

// q = (A^T L^{-1} r) at the two unknowns of vertex (i, j):
//   q_y = sum_m (M_vm r^y_m + alpha K_vm r^l_m) / W_m
//   q_l = sum_m (K_vm r^y_m - M_vm r^l_m) / W_m
// (L = blockdiag(W, W / alpha)); also returns 1/W_v, 1/N_yy, 1/N_ll of v.
template <typename T>
__device__ inline void gather_q(const Lev& L, int i, int j, const T* __restrict__ r, T& qy, T& ql, T& wv, T& nyi,
                                T& nli) {
  const int v = j * L.ld + i;
  const T* ry = r;
  const T* rl = r + L.V;
  const T al = (T)L.alpha;
  if (i >= 2 && i <= L.n - 2 && j >= 2 && j <= L.n - 2) {
    const int ld = L.ld;
    const T yc = ry[v], lc = rl[v];
    const T ya = ry[v + 1] + ry[v - 1] + ry[v + ld] + ry[v - ld];
    const T yg = ry[v + ld + 1] + ry[v - ld - 1];
    const T la = rl[v + 1] + rl[v - 1] + rl[v + ld] + rl[v - ld];
    const T lg = rl[v + ld + 1] + rl[v - ld - 1];
    const T Mc = (T)L.Mc, Mo = (T)L.Mo, Kc = (T)L.Kc, Ka = (T)L.Ka, Kd = (T)L.Kd, Wi = (T)L.Winv;
    qy = Wi * (Mc * yc + Mo * (ya + yg) + al * (Kc * lc + Ka * la + Kd * lg));
    ql = Wi * ((Kc * yc + Ka * ya + Kd * yg) - (Mc * lc + Mo * (la + lg)));
    wv = Wi;
    nyi = (T)L.Nyi;
    nli = (T)L.Nli;
  } else {
    T M[kNDir], K[kNDir];
    coef_MK(L, i, j, M, K);
    qy = 0;
    ql = 0;
#pragma unroll
    for (int d = 0; d < kNDir; d++) {
      const int ii = i + kDI[d], jj = j + kDJ[d];
      if (!inside(L, ii, jj)) continue;
      const int m = jj * L.ld + ii;
      const T wi = (T)L.tab->Winv[cls3(ii, L.n) * 3 + cls3(jj, L.n)];
      const T a = ry[m], b = rl[m];
      qy += (M[d] * a + al * K[d] * b) * wi;
      ql += (K[d] * a - M[d] * b) * wi;
    }
    wv = (T)L.tab->Winv[cls3(i, L.n) * 3 + cls3(j, L.n)];
    const int c5 = cls5(i, L.n) * 5 + cls5(j, L.n);
    nyi = (T)L.tab->Nyi[c5];
    nli = (T)L.tab->Nli[c5];
  }
}

// r_m -= A_{m v} (py, pl) for the neighbours m of v (A symmetric: A_mv = A_vm)
template <typename T>
__device__ inline void scatter_r(const Lev& L, int i, int j, T py, T pl, T* __restrict__ r) {
  const int v = j * L.ld + i;
  T* ry = r;
  T* rl = r + L.V;
  const T ai = (T)L.ainv;
  if (i >= 1 && i < L.n && j >= 1 && j < L.n) {
    const int ld = L.ld;
    const T Mc = (T)L.Mc, Mo = (T)L.Mo, Kc = (T)L.Kc, Ka = (T)L.Ka, Kd = (T)L.Kd;
    const T dyc = Mc * py + Kc * pl, dya = Mo * py + Ka * pl, dyg = Mo * py + Kd * pl;
    const T dlc = Kc * py - ai * (Mc * pl), dla = Ka * py - ai * (Mo * pl), dlg = Kd * py - ai * (Mo * pl);
    ry[v] -= dyc;
    rl[v] -= dlc;
    ry[v + 1] -= dya;
    rl[v + 1] -= dla;
    ry[v - 1] -= dya;
    rl[v - 1] -= dla;
    ry[v + ld] -= dya;
    rl[v + ld] -= dla;
    ry[v - ld] -= dya;
    rl[v - ld] -= dla;
    ry[v + ld + 1] -= dyg;
    rl[v + ld + 1] -= dlg;
    ry[v - ld - 1] -= dyg;
    rl[v - ld - 1] -= dlg;
  } else {
    T M[kNDir], K[kNDir];
    coef_MK(L, i, j, M, K);
#pragma unroll
    for (int d = 0; d < kNDir; d++) {
      const int ii = i + kDI[d], jj = j + kDJ[d];
      if (!inside(L, ii, jj)) continue;
      const int m = jj * L.ld + ii;
      ry[m] -= M[d] * py + K[d] * pl;
      rl[m] -= K[d] * py - ai * (M[d] * pl);
    }
  }
}

// ------------------------------------------------------------------ kernels

// squared norm contribution of vertex (i, j): Euclidean (mode 1) or weighted
// by L^{-1} = blockdiag(W^{-1}, alpha W^{-1}) (mode 2)
template <int MODE>
__device__ inline double norm_term(const Lev& L, int i, int j, double ry, double rl) {
  if (MODE == 1) return ry * ry + rl * rl;
  const double wi = (i >= 1 && i < L.n && j >= 1 && j < L.n) ? L.Winv : L.tab->Winv[cls3(i, L.n) * 3 + cls3(j, L.n)];
  return wi * (ry * ry + L.alpha * (rl * rl));
}

// r = f - A x (HAS_F) or r = A x; MODE 1/2 also stores per-block partial sums
// of the squared Euclidean / L^{-1} norm of r
template <typename T, bool HAS_F, int MODE>
__device__ __forceinline__ void residual_body(Lev L, const T* __restrict__ f, const T* __restrict__ x,
                                                  T* __restrict__ r, double* __restrict__ part) {
  const int i = blockIdx.x * kBX + threadIdx.x;
  const int j = blockIdx.y * kBY + threadIdx.y;
  double s2 = 0.0;
  if (i <= L.n && j <= L.n) {
    const int v = j * L.ld + i;
    T ay, al;
    apply_at(L, i, j, x, ay, al);
    T ry, rl;
    if (HAS_F) {
      ry = f[v] - ay;
      rl = f[L.V + v] - al;
    } else {
      ry = ay;
      rl = al;
    }
    r[v] = ry;
    r[L.V + v] = rl;
    if (MODE) s2 = norm_term<MODE>(L, i, j, (double)ry, (double)rl);
  }
  if (MODE) block_sum_store(s2, &part[blockIdx.y * gridDim.x + blockIdx.x]);
}
template <typename T, bool HAS_F, int MODE>
__global__ __launch_bounds__(kNT) void k_residual(Lev L, const T* __restrict__ f, const T* __restrict__ x,
                                                  T* __restrict__ r, double* __restrict__ part) { residual_body<T, HAS_F, MODE>(L, f, x, r, part); }

// per-block partial sums of the squared norm of a level vector
template <int MODE>
__global__ __launch_bounds__(kNT) void k_vnorm(Lev L, const double* __restrict__ v, double* __restrict__ part) {
  const int i = blockIdx.x * kBX + threadIdx.x;
  const int j = blockIdx.y * kBY + threadIdx.y;
  double s2 = 0.0;
  if (i <= L.n && j <= L.n) {
    const int w = j * L.ld + i;
    s2 = norm_term<MODE>(L, i, j, v[w], v[L.V + w]);
  }
  block_sum_store(s2, &part[blockIdx.y * gridDim.x + blockIdx.x]);
}

template <typename T>
__device__ __forceinline__ void rhs_body(Lev L, const double* __restrict__ yd, T* __restrict__ f) {
  const int i = blockIdx.x * kBX + threadIdx.x;
  const int j = blockIdx.y * kBY + threadIdx.y;
  if (i > L.n || j > L.n) return;
  const int v = j * L.ld + i;
  double s = 0.0;
  if (i >= 1 && i < L.n && j >= 1 && j < L.n) {
    const int ld = L.ld;
    s = L.Mc * yd[v] + L.Mo * ((yd[v + 1] + yd[v - 1] + yd[v + ld] + yd[v - ld]) + (yd[v + ld + 1] + yd[v - ld - 1]));
  } else {
    double M[kNDir], K[kNDir];
    coef_MK(L, i, j, M, K);
#pragma unroll
    for (int d = 0; d < kNDir; d++) {
      const int ii = i + kDI[d], jj = j + kDJ[d];
      if (!inside(L, ii, jj)) continue;
      s += M[d] * yd[jj * L.ld + ii];
    }
  }
  f[v] = (T)s;
  f[L.V + v] = (T)0;
}
template <typename T>
__global__ __launch_bounds__(kNT) void k_rhs(Lev L, const double* __restrict__ yd, T* __restrict__ f) { rhs_body<T>(L, yd, f); }

// (M v)_w of one field at vertex (i, j)
__device__ inline double mass_at(const Lev& L, int i, int j, const double* __restrict__ v) {
  const int w = j * L.ld + i;
  if (i >= 1 && i < L.n && j >= 1 && j < L.n) {
    const int ld = L.ld;
    return L.Mc * v[w] + L.Mo * ((v[w + 1] + v[w - 1] + v[w + ld] + v[w - ld]) + (v[w + ld + 1] + v[w - ld - 1]));
  }
  double M[kNDir], K[kNDir];
  coef_MK(L, i, j, M, K);
  double s = 0.0;
#pragma unroll
  for (int d = 0; d < kNDir; d++) {
    const int ii = i + kDI[d], jj = j + kDJ[d];
    if (inside(L, ii, jj)) s += M[d] * v[jj * L.ld + ii];
  }
  return s;
}

// Gradient of a loss of the solution x of eq. mp2 through the adjoint x_a
// (A x_a = dLoss/dx, A symmetric): the right-hand side (M y_D; 0) gives
// dLoss/dy_D = M x_a^y, and dA/dalpha = blockdiag(0, alpha^-2 M) gives
// dLoss/dalpha = -alpha^-2 (x_a^lambda)^T M lambda; this kernel stores the
// first and per-block partial sums of (x_a^lambda)^T M lambda.
__global__ __launch_bounds__(kNT) void k_adjoint_grad(Lev L, const double* __restrict__ x,
                                                      const double* __restrict__ xa, double* __restrict__ gyd,
                                                      double* __restrict__ part) {
  const int i = blockIdx.x * kBX + threadIdx.x;
  const int j = blockIdx.y * kBY + threadIdx.y;
  double s = 0.0;
  if (i <= L.n && j <= L.n) {
    const int v = j * L.ld + i;
    gyd[v] = mass_at(L, i, j, xa);
    s = xa[L.V + v] * mass_at(L, i, j, x + L.V);
  }
  block_sum_store(s, &part[blockIdx.y * gridDim.x + blockIdx.x]);
}

// control u = alpha^-1 lambda (section 1)
__global__ __launch_bounds__(kNT) void k_control(Lev L, const double* __restrict__ x, double* __restrict__ u) {
  const int i = blockIdx.x * kBX + threadIdx.x;
  const int j = blockIdx.y * kBY + threadIdx.y;
  if (i > L.n || j > L.n) return;
  const int v = j * L.ld + i;
  u[v] = x[L.V + v] * L.ainv;
}

// Alg. 1, first loop, fused with x += p: p_i = tau (A^T L^{-1} r)_i / L_ii
template <typename T>
__device__ __forceinline__ void ne_p_body(Lev L, T* __restrict__ x, const T* __restrict__ r, T* __restrict__ p) {
  const int i = blockIdx.x * kBX + threadIdx.x;
  const int j = blockIdx.y * kBY + threadIdx.y;
  if (i > L.n || j > L.n) return;
  const int v = j * L.ld + i;
  T qy, ql, wv, nyi, nli;
  gather_q(L, i, j, r, qy, ql, wv, nyi, nli);
  const T tau = (T)L.tau;
  const T py = tau * qy * wv;
  const T pl = tau * ql * ((T)L.alpha * wv);
  p[v] = py;
  p[L.V + v] = pl;
  x[v] += py;
  x[L.V + v] += pl;
}
template <typename T>
__global__ __launch_bounds__(kNT) void k_ne_p(Lev L, T* __restrict__ x, const T* __restrict__ r, T* __restrict__ p) { ne_p_body<T>(L, x, r, p); }

// Alg. 1, second loop: r -= A p
template <typename T>
__device__ __forceinline__ void ne_r_body(Lev L, const T* __restrict__ p, T* __restrict__ r) {
  const int i = blockIdx.x * kBX + threadIdx.x;
  const int j = blockIdx.y * kBY + threadIdx.y;
  if (i > L.n || j > L.n) return;
  const int v = j * L.ld + i;
  T ay, al;
  apply_at(L, i, j, p, ay, al);
  r[v] -= ay;
  r[L.V + v] -= al;
}
template <typename T>
__global__ __launch_bounds__(kNT) void k_ne_r(Lev L, const T* __restrict__ p, T* __restrict__ r) { ne_r_body<T>(L, p, r); }

// One step of Alg. 1 in one pass over a tile of kNeTX x kNeTY vertices: r on
// the tile and a two-vertex ring is staged in LDS, p = tau L^-1 A^T L^-1 r is
// formed on the tile and a one-vertex ring (the expressions of gather_q), then
// x += p and r_out = r - A p (those of apply_at) on the tile.  Neighbouring
// tiles read r_in on their rings, so r_out is a second buffer; x is read and
// written per owned vertex.  The two-kernel form moves x, r and p through
// HBM twice (14 words per vertex); this one moves x and r once (8 words plus
// the ring's share of r).
constexpr int kNeTX = 64, kNeTY = 16;
static_assert(kNeTX * kNeTY % kNT == 0, "whole owned rows per pass");
template <typename T>
__global__ __launch_bounds__(kNT) void k_ne_tile(Lev L, T* __restrict__ x, const T* __restrict__ rin,
                                                 T* __restrict__ rout) {
  constexpr int RX = kNeTX + 4, RY = kNeTY + 4;  // r: tile + 2-vertex ring
  constexpr int PX = kNeTX + 2, PY = kNeTY + 2;  // p: tile + 1-vertex ring
  __shared__ T sry[RX * RY], srl[RX * RY], spy[PX * PY], spl[PX * PY];
  const int n = L.n, ld = L.ld, V = L.V;
  const int i0 = blockIdx.x * kNeTX, j0 = blockIdx.y * kNeTY;
  const int tid = threadIdx.y * kBX + threadIdx.x;
  const bool interior_tile = i0 >= 3 && i0 + kNeTX + 2 <= n - 1 && j0 >= 3 && j0 + kNeTY + 2 <= n - 1;
  // all loads of the staged r in flight before the first LDS store
  constexpr int NQ = (RX * RY + kNT - 1) / kNT;
  T ly[NQ], ll[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    const int e = tid + q * kNT;
    const int lj = e / RX, li = e - lj * RX;
    const int a = i0 - 2 + li, b = j0 - 2 + lj;
    const bool in = e < RX * RY && a >= 0 && a <= n && b >= 0 && b <= n;
    const int u = in ? b * ld + a : 0;
    ly[q] = in ? rin[u] : (T)0;
    ll[q] = in ? rin[V + u] : (T)0;
  }
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    const int e = tid + q * kNT;
    if (e < RX * RY) {
      sry[e] = ly[q];
      srl[e] = ll[q];
    }
  }
  __syncthreads();
  const T al = (T)L.alpha, ai = (T)L.ainv, tau = (T)L.tau;
  const T Mc = (T)L.Mc, Mo = (T)L.Mo, Kc = (T)L.Kc, Ka = (T)L.Ka, Kd = (T)L.Kd, Wi = (T)L.Winv;
  for (int e = tid; e < PX * PY; e += kNT) {
    const int lj = e / PX, li = e - lj * PX;
    const int i = i0 - 1 + li, j = j0 - 1 + lj;
    T py = 0, pl = 0;
    if (i >= 0 && i <= n && j >= 0 && j <= n) {
      const int c = (lj + 1) * RX + li + 1;  // (i, j) in the r array
      T qy, ql, wv;
      if (interior_tile || (i >= 2 && i <= n - 2 && j >= 2 && j <= n - 2)) {
        const T yc = sry[c], lc = srl[c];
        const T ya = sry[c + 1] + sry[c - 1] + sry[c + RX] + sry[c - RX];
        const T yg = sry[c + RX + 1] + sry[c - RX - 1];
        const T la = srl[c + 1] + srl[c - 1] + srl[c + RX] + srl[c - RX];
        const T lg = srl[c + RX + 1] + srl[c - RX - 1];
        qy = Wi * (Mc * yc + Mo * (ya + yg) + al * (Kc * lc + Ka * la + Kd * lg));
        ql = Wi * ((Kc * yc + Ka * ya + Kd * yg) - (Mc * lc + Mo * (la + lg)));
        wv = Wi;
      } else {
        T M[kNDir], K[kNDir];
        coef_MK(L, i, j, M, K);
        qy = 0;
        ql = 0;
#pragma unroll
        for (int d = 0; d < kNDir; d++) {
          const int ii = i + kDI[d], jj = j + kDJ[d];
          if (!inside(L, ii, jj)) continue;
          const int m = c + kDJ[d] * RX + kDI[d];
          const T wi = (T)L.tab->Winv[cls3(ii, n) * 3 + cls3(jj, n)];
          const T a = sry[m], b = srl[m];
          qy += (M[d] * a + al * K[d] * b) * wi;
          ql += (K[d] * a - M[d] * b) * wi;
        }
        wv = (T)L.tab->Winv[cls3(i, n) * 3 + cls3(j, n)];
      }
      py = tau * qy * wv;
      pl = tau * ql * (al * wv);
    }
    spy[e] = py;
    spl[e] = pl;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kNeTX * kNeTY / kNT; q++) {
    const int e = tid + q * kNT;
    const int lj = e / kNeTX, li = e - lj * kNeTX;
    const int i = i0 + li, j = j0 + lj;
    if (i > n || j > n) continue;
    const int c = (lj + 1) * PX + li + 1;  // (i, j) in the p array
    const int v = j * ld + i;
    const T yc = spy[c], lc = spl[c];
    T ay, aq;
    if (i >= 1 && i < n && j >= 1 && j < n) {
      const T ya = spy[c + 1] + spy[c - 1] + spy[c + PX] + spy[c - PX];
      const T yg = spy[c + PX + 1] + spy[c - PX - 1];
      const T la = spl[c + 1] + spl[c - 1] + spl[c + PX] + spl[c - PX];
      const T lg = spl[c + PX + 1] + spl[c - PX - 1];
      ay = Mc * yc + Mo * (ya + yg) + (Kc * lc + Ka * la + Kd * lg);
      aq = (Kc * yc + Ka * ya + Kd * yg) - ai * (Mc * lc + Mo * (la + lg));
    } else {
      T M[kNDir], K[kNDir];
      coef_MK(L, i, j, M, K);
      ay = 0;
      aq = 0;
#pragma unroll
      for (int d = 0; d < kNDir; d++) {
        const int ii = i + kDI[d], jj = j + kDJ[d];
        if (!inside(L, ii, jj)) continue;
        const int m = c + kDJ[d] * PX + kDI[d];
        ay += M[d] * spy[m] + K[d] * spl[m];
        aq += K[d] * spy[m] - ai * M[d] * spl[m];
      }
    }
    const int cr = (lj + 2) * RX + li + 2;  // (i, j) in the r array
    x[v] += yc;
    x[V + v] += lc;
    rout[v] = sry[cr] - ay;
    rout[V + v] = srl[cr] - aq;
  }
}

// first vertex of colour c in row j: (i + 2 j) mod 7 == c
__device__ inline int colour_start(int c, int j) { return ((c - 2 * j) % 7 + 7) % 7; }

// Alg. 2 restricted to the vertices of one colour.  Their closed
// neighbourhoods are disjoint, so every lane gathers, updates and scatters
// without conflicts; both unknowns of a vertex use one residual snapshot.
template <typename T>
__global__ __launch_bounds__(kNT) void k_lsgs_phase(Lev L, int c, T* __restrict__ x, T* __restrict__ r) {
  const int t = blockIdx.x * kBX + threadIdx.x;
  const int j = blockIdx.y * kBY + threadIdx.y;
  if (j > L.n) return;
  const int i = colour_start(c, j) + 7 * t;
  if (i > L.n) return;
  const int v = j * L.ld + i;
  T qy, ql, wv, nyi, nli;
  gather_q(L, i, j, r, qy, ql, wv, nyi, nli);
  const T py = qy * nyi, pl = ql * nli;
  x[v] += py;
  x[L.V + v] += pl;
  scatter_r(L, i, j, py, pl, r);
}

// collective point Gauss-Seidel on one colour: solve the 2x2 system
// [[M_vv, K_vv], [K_vv, -alpha^-1 M_vv]] d = (r^y_v, r^l_v), x += d, r -= A d
template <typename T>
__device__ __forceinline__ void cgs_phase_body(Lev L, int c, T* __restrict__ x, T* __restrict__ r) {
  const int t = blockIdx.x * kBX + threadIdx.x;
  const int j = blockIdx.y * kBY + threadIdx.y;
  if (j > L.n) return;
  const int i = colour_start(c, j) + 7 * t;
  if (i > L.n) return;
  const int v = j * L.ld + i;
  T mvv, kvv;
  if (i >= 1 && i < L.n && j >= 1 && j < L.n) {
    mvv = (T)L.Mc;
    kvv = (T)L.Kc;
  } else {
    const int cc = cls3(i, L.n) * 3 + cls3(j, L.n);
    mvv = (T)L.tab->M[cc][0];
    kvv = (T)L.tab->K[cc][0];
  }
  const T b11 = mvv, b12 = kvv, b21 = kvv, b22 = -(T)L.ainv * mvv;
  const T det = b11 * b22 - b12 * b21;
  const T ry = r[v], rl = r[L.V + v];
  const T dy = (b22 * ry - b12 * rl) / det;
  const T dl = (b11 * rl - b21 * ry) / det;
  x[v] += dy;
  x[L.V + v] += dl;
  scatter_r(L, i, j, dy, dl, r);
}
template <typename T>
__global__ __launch_bounds__(kNT) void k_cgs_phase(Lev L, int c, T* __restrict__ x, T* __restrict__ r) { cgs_phase_body<T>(L, c, x, r); }

// f_c = P^T r: coarse vertex (I, J) collects the fine residual at (2I, 2J)
// with weight 1 and at its six lattice neighbours with weight 1/2.
template <typename T>
__device__ __forceinline__ void restrict_body(Lev Lf, Lev Lc, const T* __restrict__ r, T* __restrict__ fc,
                                                  T* __restrict__ xc_zero, T* __restrict__ rc_copy) {
  const int I = blockIdx.x * kBX + threadIdx.x;
  const int J = blockIdx.y * kBY + threadIdx.y;
  if (I > Lc.n || J > Lc.n) return;
  const int a = 2 * I, b = 2 * J;
  const int u = b * Lf.ld + a;
  const T* ry = r;
  const T* rl = r + Lf.V;
  T hy = 0, hl = 0;
  if (a >= 1 && a < Lf.n && b >= 1 && b < Lf.n) {
    const int ld = Lf.ld;
    hy = (ry[u + 1] + ry[u - 1] + ry[u + ld] + ry[u - ld]) + (ry[u + ld + 1] + ry[u - ld - 1]);
    hl = (rl[u + 1] + rl[u - 1] + rl[u + ld] + rl[u - ld]) + (rl[u + ld + 1] + rl[u - ld - 1]);
  } else {
#pragma unroll
    for (int d = 1; d < kNDir; d++) {
      const int aa = a + kDI[d], bb = b + kDJ[d];
      if (!inside(Lf, aa, bb)) continue;
      hy += ry[bb * Lf.ld + aa];
      hl += rl[bb * Lf.ld + aa];
    }
  }
  const int w = J * Lc.ld + I;
  const T gy = ry[u] + (T)0.5 * hy, gl = rl[u] + (T)0.5 * hl;
  fc[w] = gy;
  fc[Lc.V + w] = gl;
  if (xc_zero) {
    xc_zero[w] = (T)0;
    xc_zero[Lc.V + w] = (T)0;
  }
  if (rc_copy) {
    rc_copy[w] = gy;
    rc_copy[Lc.V + w] = gl;
  }
}
template <typename T>
__global__ __launch_bounds__(kNT) void k_restrict(Lev Lf, Lev Lc, const T* __restrict__ r, T* __restrict__ fc,
                                                  T* __restrict__ xc_zero, T* __restrict__ rc_copy) { restrict_body<T>(Lf, Lc, r, fc, xc_zero, rc_copy); }

// x += P x_c: P1 interpolation; fine vertices on coarse edges (horizontal,
// vertical, or the (I,J)-(I+1,J+1) diagonal) take the mean of the endpoints.
template <typename T>
__device__ __forceinline__ void prolong_add_body(Lev Lf, Lev Lc, const T* __restrict__ xc, T* __restrict__ x) {
  const int a = blockIdx.x * kBX + threadIdx.x;
  const int b = blockIdx.y * kBY + threadIdx.y;
  if (a > Lf.n || b > Lf.n) return;
  const int I0 = a >> 1, J0 = b >> 1;
  const int I1 = (a + 1) >> 1, J1 = (b + 1) >> 1;
  const int w0 = J0 * Lc.ld + I0, w1 = J1 * Lc.ld + I1;
  const int u = b * Lf.ld + a;
  T vy, vl;
  if (w0 == w1) {
    vy = xc[w0];
    vl = xc[Lc.V + w0];
  } else {
    vy = (T)0.5 * (xc[w0] + xc[w1]);
    vl = (T)0.5 * (xc[Lc.V + w0] + xc[Lc.V + w1]);
  }
  x[u] += vy;
  x[Lf.V + u] += vl;
}
template <typename T>
__global__ __launch_bounds__(kNT) void k_prolong_add(Lev Lf, Lev Lc, const T* __restrict__ xc, T* __restrict__ x) { prolong_add_body<T>(Lf, Lc, xc, x); }

// (P x_c) at fine vertex (a, b): the coarse value at a coarse vertex, the mean
// of the endpoints on a coarse edge (same expression as prolong_add_body)
template <typename T>
__device__ __forceinline__ void prolong_at(const Lev& Lf, const Lev& Lc, const T* __restrict__ xc, int a, int b,
                                           T& vy, T& vl) {
  const int w0 = (b >> 1) * Lc.ld + (a >> 1), w1 = ((b + 1) >> 1) * Lc.ld + ((a + 1) >> 1);
  if (w0 == w1) {
    vy = xc[w0];
    vl = xc[Lc.V + w0];
  } else {
    vy = (T)0.5 * (xc[w0] + xc[w1]);
    vl = (T)0.5 * (xc[Lc.V + w0] + xc[Lc.V + w1]);
  }
  (void)Lf;
}

// x_out = x_in + P x_c and r = f - A x_out in one pass (section 2: coarse-grid
// correction followed by the fine residual).  The block first forms the
// corrected iterate on its vertices plus a one-vertex ring in LDS (one
// interpolation per vertex), then applies the stencil from there.  x_out must
// not alias x_in.  Same arithmetic as k_prolong_add followed by k_residual.
template <typename T>
__global__ __launch_bounds__(kNT) void k_prolong_residual(Lev Lf, Lev Lc, const T* __restrict__ xc,
                                                          const T* __restrict__ xin, const T* __restrict__ f,
                                                          T* __restrict__ xout, T* __restrict__ r) {
  constexpr int PX = kBX + 2, PY = kBY + 2;
  __shared__ T sy[PX * PY], sl[PX * PY];
  const int n = Lf.n, V = Lf.V, ld = Lf.ld;
  const int ib = blockIdx.x * kBX - 1, jb = blockIdx.y * kBY - 1;
  const int tid = threadIdx.y * kBX + threadIdx.x;
  for (int e = tid; e < PX * PY; e += kNT) {
    const int lj = e / PX, li = e - lj * PX;
    const int a = ib + li, b = jb + lj;
    T y = 0, l = 0;
    if (a >= 0 && a <= n && b >= 0 && b <= n) {
      T vy, vl;
      prolong_at(Lf, Lc, xc, a, b, vy, vl);
      const int u = b * ld + a;
      y = xin[u] + vy;
      l = xin[V + u] + vl;
    }
    sy[e] = y;
    sl[e] = l;
  }
  __syncthreads();
  const int i = blockIdx.x * kBX + threadIdx.x;
  const int j = blockIdx.y * kBY + threadIdx.y;
  if (i > n || j > n) return;
  const int c = (threadIdx.y + 1) * PX + threadIdx.x + 1;
  const T ai = (T)Lf.ainv;
  const T yc = sy[c], lc = sl[c];
  T ay, al;
  if (i >= 1 && i < n && j >= 1 && j < n) {
    const T ya = sy[c + 1] + sy[c - 1] + sy[c + PX] + sy[c - PX];
    const T yg = sy[c + PX + 1] + sy[c - PX - 1];
    const T la = sl[c + 1] + sl[c - 1] + sl[c + PX] + sl[c - PX];
    const T lg = sl[c + PX + 1] + sl[c - PX - 1];
    const T Mc = (T)Lf.Mc, Mo = (T)Lf.Mo, Kc = (T)Lf.Kc, Ka = (T)Lf.Ka, Kd = (T)Lf.Kd;
    ay = Mc * yc + Mo * (ya + yg) + (Kc * lc + Ka * la + Kd * lg);
    al = (Kc * yc + Ka * ya + Kd * yg) - ai * (Mc * lc + Mo * (la + lg));
  } else {
    T M[kNDir], K[kNDir];
    coef_MK(Lf, i, j, M, K);
    ay = 0;
    al = 0;
#pragma unroll
    for (int d = 0; d < kNDir; d++) {
      if (!inside(Lf, i + kDI[d], j + kDJ[d])) continue;
      const int m = c + kDJ[d] * PX + kDI[d];
      ay += M[d] * sy[m] + K[d] * sl[m];
      al += K[d] * sy[m] - ai * M[d] * sl[m];
    }
  }
  const int v = j * ld + i;
  xout[v] = yc;
  xout[V + v] = lc;
  r[v] = f[v] - ay;
  r[V + v] = f[V + v] - al;
}

// x = A_{k0}^{-1} f with the FP64 LU factors (row pivots piv) of A_{k0}
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_solve(int N, const double* __restrict__ lu, const int* __restrict__ piv,
                                                      const T* __restrict__ f, T* __restrict__ x) {
  __shared__ double b[512];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += blockDim.x) b[i] = (double)f[i];
  __syncthreads();
  if (tid == 0)
    for (int k = 0; k < N; k++)
      if (piv[k] != k) {
        const double t = b[k];
        b[k] = b[piv[k]];
        b[piv[k]] = t;
      }
  __syncthreads();
  for (int k = 0; k < N; k++) {  // unit lower triangular
    const double bk = b[k];
    for (int i = k + 1 + tid; i < N; i += blockDim.x) b[i] -= lu[(size_t)i * N + k] * bk;
    __syncthreads();
  }
  for (int k = N - 1; k >= 0; k--) {  // upper triangular
    if (tid == 0) b[k] /= lu[(size_t)k * N + k];
    __syncthreads();
    const double bk = b[k];
    for (int i = tid; i < k; i += blockDim.x) b[i] -= lu[(size_t)i * N + k] * bk;
    __syncthreads();
  }
  for (int i = tid; i < N; i += blockDim.x) x[i] = (T)b[i];
}

// *out = scale * sum of part[0..n) by one workgroup of NT threads, in a fixed
// order (four independent accumulators per thread keep loads in flight)
template <int NT, bool SQRT = false>
__device__ __forceinline__ void sum_body(const double* __restrict__ part, int n, double scale,
                                         double* __restrict__ out) {
  __shared__ double sh[NT / 64];
  const int tid = threadIdx.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int k = tid;
  for (; k + 3 * NT < n; k += 4 * NT) {
    a0 += part[k];
    a1 += part[k + NT];
    a2 += part[k + 2 * NT];
    a3 += part[k + 3 * NT];
  }
  for (; k < n; k += NT) a0 += part[k];
  double s = wave_sum((a0 + a1) + (a2 + a3));
  if ((tid & 63) == 0) sh[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; w++) t += sh[w];
    *out = SQRT ? sqrt(scale * t) : scale * t;
  }
}
__global__ __launch_bounds__(1024) void k_sum(const double* __restrict__ part, int n, double scale,
                                              double* __restrict__ out) {
  sum_body<1024>(part, n, scale, out);
}
// the same sum followed by its square root (a Euclidean norm from squared partials)
__global__ __launch_bounds__(1024) void k_sum_sqrt(const double* __restrict__ part, int n,
                                                   double* __restrict__ out) {
  sum_body<1024, true>(part, n, 1.0, out);
}

__global__ __launch_bounds__(256) void k_sumsq(const double* __restrict__ v, size_t n, double* __restrict__ part) {
  __shared__ double sh[4];
  double s = 0.0;
  for (size_t k = blockIdx.x * 256 + threadIdx.x; k < n; k += (size_t)gridDim.x * 256) s += v[k] * v[k];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// scale of a refinement step: s = ||r||_2 (from its square on the device), 1 if zero
__device__ inline double ir_scale(const double* nrm2) {
  const double q = *nrm2;
  return q > 0.0 ? sqrt(q) : 1.0;
}

__device__ __forceinline__ void to_f32_scaled_body(const double* __restrict__ r, size_t n, const double* __restrict__ nrm2,
                                float* __restrict__ out, float* __restrict__ out2) {
  const double inv = 1.0 / ir_scale(nrm2);
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const float v = (float)(r[k] * inv);
    out[k] = v;
    if (out2) out2[k] = v;
  }
}
__global__ void k_to_f32_scaled(const double* __restrict__ r, size_t n, const double* __restrict__ nrm2,
                                float* __restrict__ out, float* __restrict__ out2) { to_f32_scaled_body(r, n, nrm2, out, out2); }

// r = f - A x (FP64) with the norm partials of r (MODE 1 / 2), written as r / s
// in FP32 to out and out2 (s from its square at nrm2, 1 if zero) and not in
// FP64: the residual of a refinement step and the right-hand side of its
// FP32 cycles in one pass
template <int MODE>
__global__ __launch_bounds__(kNT) void k_residual_f32(Lev L, const double* __restrict__ f, const double* __restrict__ x,
                                                      const double* __restrict__ nrm2, float* __restrict__ out,
                                                      float* __restrict__ out2, double* __restrict__ part) {
  const int i = blockIdx.x * kBX + threadIdx.x;
  const int j = blockIdx.y * kBY + threadIdx.y;
  const double inv = 1.0 / ir_scale(nrm2);
  double s2 = 0.0;
  if (i <= L.n && j <= L.n) {
    const int v = j * L.ld + i;
    double ay, al;
    apply_at(L, i, j, x, ay, al);
    const double ry = f[v] - ay, rl = f[L.V + v] - al;
    const float vy = (float)(ry * inv), vl = (float)(rl * inv);
    out[v] = vy;
    out[L.V + v] = vl;
    out2[v] = vy;
    out2[L.V + v] = vl;
    s2 = norm_term<MODE>(L, i, j, ry, rl);
  }
  block_sum_store(s2, &part[blockIdx.y * gridDim.x + blockIdx.x]);
}

__device__ __forceinline__ void axpy_f32_body(const float* __restrict__ c, size_t n, const double* __restrict__ nrm2,
                           double* __restrict__ x) {
  const double scale = ir_scale(nrm2);
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    x[k] += scale * (double)c[k];
}
__global__ void k_axpy_f32(const float* __restrict__ c, size_t n, const double* __restrict__ nrm2,
                           double* __restrict__ x) { axpy_f32_body(c, n, nrm2, x); }

__device__ __forceinline__ void zero_f32_body(float* __restrict__ v, size_t n) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) v[k] = 0.f;
}
__global__ void k_zero_f32(float* __restrict__ v, size_t n) { zero_f32_body(v, n); }

// ---- batched wrappers: instance blockIdx.z (vertex grids) / blockIdx.y (1D)
template <typename T>
__device__ inline T* cur_r(const BInst<T>& a, int sel) { return sel ? a.r2 : a.r; }

template <typename T>
__global__ __launch_bounds__(kNT) void kb_residual(const BInst<T>* __restrict__ B, int sel) {
  const BInst<T>& a = B[blockIdx.z];
  if (!*a.active) return;
  residual_body<T, true, 0>(a.L, a.f, a.x, cur_r(a, sel), nullptr);
}

template <typename T>
__global__ __launch_bounds__(kNT) void kb_ne_p(const BInst<T>* __restrict__ B, int sel) {
  const BInst<T>& a = B[blockIdx.z];
  if (!*a.active) return;
  ne_p_body<T>(a.L, a.x, cur_r(a, sel), a.p);
}

template <typename T>
__global__ __launch_bounds__(kNT) void kb_ne_r(const BInst<T>* __restrict__ B, int sel) {
  const BInst<T>& a = B[blockIdx.z];
  if (!*a.active) return;
  ne_r_body<T>(a.L, a.p, cur_r(a, sel));
}

template <typename T>
__global__ __launch_bounds__(kNT) void kb_cgs_phase(const BInst<T>* __restrict__ B, int c, int sel) {
  const BInst<T>& a = B[blockIdx.z];
  if (!*a.active) return;
  cgs_phase_body<T>(a.L, c, a.x, cur_r(a, sel));
}

template <typename T>
__global__ __launch_bounds__(kNT) void kb_restrict(const BInst<T>* __restrict__ B, int sel, int zero_coarse) {
  const BInst<T>& a = B[blockIdx.z];
  if (!*a.active) return;
  restrict_body<T>(a.L, a.Lc, cur_r(a, sel), a.fc, zero_coarse ? a.xc : nullptr, zero_coarse ? a.rc : nullptr);
}

template <typename T>
__global__ __launch_bounds__(kNT) void kb_prolong_add(const BInst<T>* __restrict__ B) {
  const BInst<T>& a = B[blockIdx.z];
  if (!*a.active) return;
  prolong_add_body<T>(a.L, a.Lc, a.xc, a.x);
}

template <int MODE>
__global__ __launch_bounds__(kNT) void kb_residual_norm(const BFine* __restrict__ B) {
  const BFine& a = B[blockIdx.z];
  if (!*a.active) return;
  residual_body<double, true, MODE>(a.L, a.f, a.x, a.r, a.part);
}

template <int MODE>
__global__ __launch_bounds__(kNT) void kb_vnorm(const BFine* __restrict__ B) {
  const BFine& a = B[blockIdx.z];
  if (!*a.active) return;
  const Lev& L = a.L;
  const int i = blockIdx.x * kBX + threadIdx.x;
  const int j = blockIdx.y * kBY + threadIdx.y;
  double s2 = 0.0;
  if (i <= L.n && j <= L.n) {
    const int w = j * L.ld + i;
    s2 = norm_term<MODE>(L, i, j, a.f[w], a.f[L.V + w]);
  }
  block_sum_store(s2, &a.part[blockIdx.y * gridDim.x + blockIdx.x]);
}

__global__ __launch_bounds__(256) void kb_sum(const BFine* __restrict__ B, int nparts, int slot) {
  const BFine& a = B[blockIdx.x];
  if (!*a.active) return;
  sum_body<256>(a.part, nparts, 1.0, a.norm + slot);
}

__global__ void kb_to_f32_scaled(const BFine* __restrict__ B, size_t len) {
  const BFine& a = B[blockIdx.y];
  if (!*a.active) return;
  to_f32_scaled_body(a.r, len, a.norm, a.f32, a.r32);
}

__global__ void kb_zero_x32(const BFine* __restrict__ B, size_t len) {
  const BFine& a = B[blockIdx.y];
  if (!*a.active) return;
  zero_f32_body(a.x32, len);
}

__global__ void kb_axpy_f32(const BFine* __restrict__ B, size_t len) {
  const BFine& a = B[blockIdx.y];
  if (!*a.active) return;
  axpy_f32_body(a.x32, len, a.norm, a.x);
}

__global__ void kb_gather_norms(const double* const* __restrict__ norms, int count, double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= count) return;
  out[2 * b] = norms[b][0];
  out[2 * b + 1] = norms[b][1];
}

inline dim3 grid_vertices(int n) { return dim3((n + 1 + kBX - 1) / kBX, (n + 1 + kBY - 1) / kBY); }
inline dim3 grid_colour(int n) { return dim3(((n + 1 + 6) / 7 + kBX - 1) / kBX, (n + 1 + kBY - 1) / kBY); }
const dim3 kBlock(kBX, kBY);

}  // namespace

// ------------------------------------------------------------------ launchers

template <typename T>
hipError_t launch_residual(const Lev& L, const T* f, const T* x, T* r, double* part, int norm_mode, int* nblocks,
                           hipStream_t s) {
  const dim3 g = grid_vertices(L.n);
  if (nblocks) *nblocks = (int)(g.x * g.y);
  if (part && norm_mode == 2)
    hipLaunchKernelGGL((k_residual<T, true, 2>), g, kBlock, 0, s, L, f, x, r, part);
  else if (part)
    hipLaunchKernelGGL((k_residual<T, true, 1>), g, kBlock, 0, s, L, f, x, r, part);
  else
    hipLaunchKernelGGL((k_residual<T, true, 0>), g, kBlock, 0, s, L, f, x, r, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply(const Lev& L, const T* x, T* y, hipStream_t s) {
  hipLaunchKernelGGL((k_residual<T, false, 0>), grid_vertices(L.n), kBlock, 0, s, L, (const T*)nullptr, x, y,
                     (double*)nullptr);
  return hipGetLastError();
}

hipError_t launch_vnorm(const Lev& L, const double* v, double* part, int norm_mode, int* nblocks, hipStream_t s) {
  const dim3 g = grid_vertices(L.n);
  *nblocks = (int)(g.x * g.y);
  if (norm_mode == 2)
    hipLaunchKernelGGL((k_vnorm<2>), g, kBlock, 0, s, L, v, part);
  else
    hipLaunchKernelGGL((k_vnorm<1>), g, kBlock, 0, s, L, v, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rhs(const Lev& L, const double* yd, T* f, hipStream_t s) {
  hipLaunchKernelGGL((k_rhs<T>), grid_vertices(L.n), kBlock, 0, s, L, yd, f);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ne(const Lev& L, T* x, T* r, T* p, hipStream_t s) {
  hipLaunchKernelGGL((k_ne_p<T>), grid_vertices(L.n), kBlock, 0, s, L, x, (const T*)r, p);
  hipLaunchKernelGGL((k_ne_r<T>), grid_vertices(L.n), kBlock, 0, s, L, (const T*)p, r);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ne_tile(const Lev& L, T* x, const T* rin, T* rout, hipStream_t s) {
  const dim3 g((L.n + kNeTX) / kNeTX, (L.n + kNeTY) / kNeTY);
  hipLaunchKernelGGL((k_ne_tile<T>), g, kBlock, 0, s, L, x, rin, rout);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_lsgs_phase(const Lev& L, int colour, T* x, T* r, hipStream_t s) {
  hipLaunchKernelGGL((k_lsgs_phase<T>), grid_colour(L.n), kBlock, 0, s, L, colour, x, r);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cgs_phase(const Lev& L, int colour, T* x, T* r, hipStream_t s) {
  hipLaunchKernelGGL((k_cgs_phase<T>), grid_colour(L.n), kBlock, 0, s, L, colour, x, r);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(const Lev& Lf, const Lev& Lc, const T* r, T* fc, T* xc_zero, T* rc_copy, hipStream_t s) {
  hipLaunchKernelGGL((k_restrict<T>), grid_vertices(Lc.n), kBlock, 0, s, Lf, Lc, r, fc, xc_zero, rc_copy);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add(const Lev& Lf, const Lev& Lc, const T* xc, T* x, hipStream_t s) {
  hipLaunchKernelGGL((k_prolong_add<T>), grid_vertices(Lf.n), kBlock, 0, s, Lf, Lc, xc, x);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_residual(const Lev& Lf, const Lev& Lc, const T* xc, const T* xin, const T* f, T* xout, T* r,
                                   hipStream_t s) {
  if (xin == xout) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_prolong_residual<T>), grid_vertices(Lf.n), kBlock, 0, s, Lf, Lc, xc, xin, f, xout, r);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_solve(int N, const double* lu, const int* piv, const T* f, T* x, hipStream_t s) {
  if (N > 512) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_coarse_solve<T>), dim3(1), dim3(256), 0, s, N, lu, piv, f, x);
  return hipGetLastError();
}

hipError_t launch_sum(const double* part, int n, double* out, hipStream_t s, double scale) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, s, part, n, scale, out);
  return hipGetLastError();
}

hipError_t launch_sum_sqrt(const double* part, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_sqrt, dim3(1), dim3(1024), 0, s, part, n, out);
  return hipGetLastError();
}

hipError_t launch_adjoint_grad(const Lev& L, const double* x, const double* xa, double* gyd, double* part,
                               int* nblocks, hipStream_t s) {
  const dim3 g = grid_vertices(L.n);
  *nblocks = (int)(g.x * g.y);
  hipLaunchKernelGGL(k_adjoint_grad, g, kBlock, 0, s, L, x, xa, gyd, part);
  return hipGetLastError();
}

hipError_t launch_control(const Lev& L, const double* x, double* u, hipStream_t s) {
  hipLaunchKernelGGL(k_control, grid_vertices(L.n), kBlock, 0, s, L, x, u);
  return hipGetLastError();
}

hipError_t launch_sumsq(const double* v, size_t n, double* part, int* nblocks, hipStream_t s) {
  int nb = (int)((n + 255) / 256);
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  *nblocks = nb;
  hipLaunchKernelGGL(k_sumsq, dim3(nb), dim3(256), 0, s, v, n, part);
  return hipGetLastError();
}

static int grid1d(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  return g < 1 ? 1 : (int)g;
}

hipError_t launch_to_f32_scaled(const double* r, size_t n, const double* nrm2, float* out, float* out2, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f32_scaled, dim3(grid1d(n)), dim3(256), 0, s, r, n, nrm2, out, out2);
  return hipGetLastError();
}

hipError_t launch_residual_f32(const Lev& L, const double* f, const double* x, const double* nrm2, float* out,
                               float* out2, double* part, int norm_mode, int* nblocks, hipStream_t s) {
  if (!part || (norm_mode != 1 && norm_mode != 2)) return hipErrorInvalidValue;
  const dim3 g = grid_vertices(L.n);
  if (nblocks) *nblocks = (int)(g.x * g.y);
  if (norm_mode == 2)
    hipLaunchKernelGGL(k_residual_f32<2>, g, kBlock, 0, s, L, f, x, nrm2, out, out2, part);
  else
    hipLaunchKernelGGL(k_residual_f32<1>, g, kBlock, 0, s, L, f, x, nrm2, out, out2, part);
  return hipGetLastError();
}

hipError_t launch_axpy_f32(const float* c, size_t n, const double* nrm2, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_f32, dim3(grid1d(n)), dim3(256), 0, s, c, n, nrm2, x);
  return hipGetLastError();
}

hipError_t launch_zero_f32(float* v, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_f32, dim3(grid1d(n)), dim3(256), 0, s, v, n);
  return hipGetLastError();
}

int residual_blocks(int n) {
  const dim3 g = grid_vertices(n);
  return (int)(g.x * g.y);
}

static dim3 zgrid(dim3 g, int count) { return dim3(g.x, g.y, count); }

template <typename T>
hipError_t launch_b_residual(const BInst<T>* d, int count, int n, int sel, hipStream_t s) {
  hipLaunchKernelGGL((kb_residual<T>), zgrid(grid_vertices(n), count), kBlock, 0, s, d, sel);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_b_ne(const BInst<T>* d, int count, int n, int sel, hipStream_t s) {
  hipLaunchKernelGGL((kb_ne_p<T>), zgrid(grid_vertices(n), count), kBlock, 0, s, d, sel);
  hipLaunchKernelGGL((kb_ne_r<T>), zgrid(grid_vertices(n), count), kBlock, 0, s, d, sel);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_b_cgs_phase(const BInst<T>* d, int count, int n, int colour, int sel, hipStream_t s) {
  hipLaunchKernelGGL((kb_cgs_phase<T>), zgrid(grid_colour(n), count), kBlock, 0, s, d, colour, sel);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_b_restrict(const BInst<T>* d, int count, int nc, int sel, int zero_coarse, hipStream_t s) {
  hipLaunchKernelGGL((kb_restrict<T>), zgrid(grid_vertices(nc), count), kBlock, 0, s, d, sel, zero_coarse);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_b_prolong_add(const BInst<T>* d, int count, int nf, hipStream_t s) {
  hipLaunchKernelGGL((kb_prolong_add<T>), zgrid(grid_vertices(nf), count), kBlock, 0, s, d);
  return hipGetLastError();
}

hipError_t launch_b_residual_norm(const BFine* d, int count, int n, int norm_mode, hipStream_t s) {
  if (norm_mode == 2)
    hipLaunchKernelGGL((kb_residual_norm<2>), zgrid(grid_vertices(n), count), kBlock, 0, s, d);
  else
    hipLaunchKernelGGL((kb_residual_norm<1>), zgrid(grid_vertices(n), count), kBlock, 0, s, d);
  return hipGetLastError();
}

hipError_t launch_b_vnorm(const BFine* d, int count, int n, int norm_mode, hipStream_t s) {
  if (norm_mode == 2)
    hipLaunchKernelGGL((kb_vnorm<2>), zgrid(grid_vertices(n), count), kBlock, 0, s, d);
  else
    hipLaunchKernelGGL((kb_vnorm<1>), zgrid(grid_vertices(n), count), kBlock, 0, s, d);
  return hipGetLastError();
}

hipError_t launch_b_sum(const BFine* d, int count, int nparts, int slot, hipStream_t s) {
  hipLaunchKernelGGL(kb_sum, dim3(count), dim3(256), 0, s, d, nparts, slot);
  return hipGetLastError();
}

static dim3 ygrid(size_t len, int count) {
  size_t g = (len + 255) / 256;
  if (g > 1024) g = 1024;
  return dim3(g < 1 ? 1 : (unsigned)g, count);
}

hipError_t launch_b_to_f32_scaled(const BFine* d, int count, size_t len, hipStream_t s) {
  hipLaunchKernelGGL(kb_to_f32_scaled, ygrid(len, count), dim3(256), 0, s, d, len);
  return hipGetLastError();
}

hipError_t launch_b_zero_x32(const BFine* d, int count, size_t len, hipStream_t s) {
  hipLaunchKernelGGL(kb_zero_x32, ygrid(len, count), dim3(256), 0, s, d, len);
  return hipGetLastError();
}

hipError_t launch_b_axpy_f32(const BFine* d, int count, size_t len, hipStream_t s) {
  hipLaunchKernelGGL(kb_axpy_f32, ygrid(len, count), dim3(256), 0, s, d, len);
  return hipGetLastError();
}

hipError_t launch_b_gather_norms(const double* const* d, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(kb_gather_norms, dim3((count + 63) / 64), dim3(64), 0, s, d, count, out);
  return hipGetLastError();
}

// ---- dense coarse map: x = B r (accumulate 0) or x += B r (accumulate 1),
// B row-major N x N with N even.  Four waves share a row (two rows per
// 512-thread workgroup), so a wave keeps a quarter of the row's loads in
// flight and twice as many waves stream the matrix as with one wave per row;
// r is staged in LDS while those loads are in flight.  A lane reads pairs of
// entries (one 16- or 8-byte load); wave k of a row takes the 64-pair chunks
// k, k + 4, ...  Each wave sums its lanes in a fixed order, and the row's
// four partial sums are added in wave order.
namespace {
constexpr int kDenseWaves = 4;                                // waves per row
constexpr int kDenseThreads = 512;                            // threads per workgroup
constexpr int kDenseRows = kDenseThreads / 64 / kDenseWaves;  // rows per workgroup
template <typename T>
struct Pair2;
template <>
struct Pair2<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Pair2<float> {
  typedef float type __attribute__((ext_vector_type(2)));
};

template <typename T>
__global__ __launch_bounds__(kDenseThreads) void k_dense_map(const T* __restrict__ B, int N, const T* __restrict__ r,
                                                             T* __restrict__ x, int accumulate) {
  using T2 = typename Pair2<T>::type;
  __shared__ __align__(16) T rs[kDenseMapMaxN];
  __shared__ T part[kDenseThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row = blockIdx.x * kDenseRows + wave / kDenseWaves;
  const int wr = wave % kDenseWaves;
  const int np = N / 2;
  // loads in issue order: this thread's share of r, then its part of the row
  // (in flight while r is staged in LDS: the wait for r does not wait for them)
  constexpr int RU = (kDenseMapMaxN + kDenseThreads - 1) / kDenseThreads;
  T rv0[RU];
#pragma unroll
  for (int u = 0; u < RU; u++) {
    const int e = tid + u * kDenseThreads;
    rv0[u] = r[e < N ? e : N - 1];  // unconditional loads keep the wait counts exact
  }
  constexpr int U = (kDenseMapMaxN / 2 + 64 * kDenseWaves - 1) / (64 * kDenseWaves);  // pairs per lane
  T2 v[U];
  const T2* b2 = reinterpret_cast<const T2*>(B + (size_t)(row < N ? row : 0) * N);
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int q = lane + 64 * (wr + kDenseWaves * u);
    // clamped index and a zero weight past the row's end: the load itself
    // stays unconditional (a guarded load would be moved under a branch)
    const T w = q < np ? (T)1 : (T)0;
    v[u] = b2[q < np ? q : np - 1] * w;
  }
#pragma unroll
  for (int u = 0; u < RU; u++) {
    const int e = tid + u * kDenseThreads;
    if (e < N) rs[e] = rv0[u];
  }
  // a barrier that orders the LDS stores only (the row's loads stay in flight)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  const T2* r2 = reinterpret_cast<const T2*>(rs);
  T a0 = 0, a1 = 0;
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int q = lane + 64 * (wr + kDenseWaves * u);
    const T2 rv = r2[q < np ? q : 0];
    a0 += v[u].x * rv.x;
    a1 += v[u].y * rv.y;
  }
  T acc = a0 + a1;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) part[wave] = acc;
  __syncthreads();  // every wave gets here: a row past N only skips the store
  if (row < N && wr == 0 && lane == 0) {
    T sum = part[wave];
#pragma unroll
    for (int k = 1; k < kDenseWaves; k++) sum += part[wave + k];
    x[row] = accumulate ? x[row] + sum : sum;
  }
}
}  // namespace

template <typename T>
hipError_t launch_dense_map(const T* B, int N, const T* r, T* x, int accumulate, hipStream_t s) {
  if (N <= 0 || N > kDenseMapMaxN || (N & 1)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_dense_map<T>), dim3((N + kDenseRows - 1) / kDenseRows), dim3(kDenseThreads), 0, s, B, N, r,
                     x, accumulate);
  return hipGetLastError();
}
template hipError_t launch_dense_map<double>(const double*, int, const double*, double*, int, hipStream_t);
template hipError_t launch_dense_map<float>(const float*, int, const float*, float*, int, hipStream_t);

#define MGK_INSTANTIATE(T)                                                                                          \
  template hipError_t launch_residual<T>(const Lev&, const T*, const T*, T*, double*, int, int*, hipStream_t);         \
  template hipError_t launch_apply<T>(const Lev&, const T*, T*, hipStream_t);                                      \
  template hipError_t launch_rhs<T>(const Lev&, const double*, T*, hipStream_t);                                   \
  template hipError_t launch_ne<T>(const Lev&, T*, T*, T*, hipStream_t);                                           \
  template hipError_t launch_ne_tile<T>(const Lev&, T*, const T*, T*, hipStream_t);                                           \
  template hipError_t launch_lsgs_phase<T>(const Lev&, int, T*, T*, hipStream_t);                                  \
  template hipError_t launch_cgs_phase<T>(const Lev&, int, T*, T*, hipStream_t);                                   \
  template hipError_t launch_restrict<T>(const Lev&, const Lev&, const T*, T*, T*, T*, hipStream_t);              \
  template hipError_t launch_prolong_add<T>(const Lev&, const Lev&, const T*, T*, hipStream_t);                    \
  template hipError_t launch_prolong_residual<T>(const Lev&, const Lev&, const T*, const T*, const T*, T*, T*,      \
                                                 hipStream_t);                                                    \
  template hipError_t launch_coarse_solve<T>(int, const double*, const int*, const T*, T*, hipStream_t);         \
  template hipError_t launch_b_residual<T>(const BInst<T>*, int, int, int, hipStream_t);                          \
  template hipError_t launch_b_ne<T>(const BInst<T>*, int, int, int, hipStream_t);                                \
  template hipError_t launch_b_cgs_phase<T>(const BInst<T>*, int, int, int, int, hipStream_t);                    \
  template hipError_t launch_b_restrict<T>(const BInst<T>*, int, int, int, int, hipStream_t);                     \
  template hipError_t launch_b_prolong_add<T>(const BInst<T>*, int, int, hipStream_t);

MGK_INSTANTIATE(double)
MGK_INSTANTIATE(float)

}  // namespace mgk
