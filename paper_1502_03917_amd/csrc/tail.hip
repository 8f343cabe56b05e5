// Coarse-level tail of the multigrid cycle (section 2 of Takacs, arXiv
// 1502.03917) in one workgroup.
//
// On the coarse levels a cycle is a long chain of tiny dependent steps, so
// separate kernel launches cost far more than the arithmetic.  Here one
// workgroup keeps x, r and f of every level k0..T in LDS and runs the whole
// sub-cycle from a schedule of operations built by the host (smoothing,
// restriction, the FP64 LU solve on k0, prolongation + residual), reading f_T
// from global memory at the start and writing x_T back at the end.  All
// vertices use the per-class coefficient blocks of the level table, so
// boundary and interior vertices take the same path.
#include <cstring>
#include <type_traits>

#include "mg_internal.hpp"

namespace mgk {

namespace {

__device__ inline void bar() { __syncthreads(); }

// value of v in lane k of the wave (k uniform across the wave)
__device__ inline double lane_bcast(double v, int k) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, k);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), k);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// unknowns of the level that the coarse map covers, and the waves that split
// its columns
constexpr int kTailMapN = 2 * ((1 << kTailMapLevel) + 1) * ((1 << kTailMapLevel) + 1);
constexpr int kTailWaves = kTailThreads / 64;
static_assert(kTailMapN <= 3 * 64, "map rows: three per lane");

// bytes of the shared scratch: NE corrections of level T (2 V_T entries), the
// FP64 right-hand side of the coarsest solve, or the per-wave partial sums of
// the coarse map product (tails above the map level), whichever is largest
template <typename T>
__host__ __device__ inline size_t tail_scratch_bytes(int VT, int ncoarse, int Tl) {
  const size_t a = (size_t)2 * VT * sizeof(T), b = (size_t)ncoarse * sizeof(double);
  const size_t c = Tl > kTailMapLevel ? (size_t)kTailWaves * kTailMapN * sizeof(T) : 0;
  const size_t ab = a > b ? a : b;
  return ab > c ? ab : c;
}

struct TailLevel {
  int n, ld, V;
  int ox, or_, of;  // LDS offsets (elements) of x, r, f (2V each)
};

template <typename T>
struct TailArgs {
  TailLevel lv[kTailMaxLevels + 1];  // indexed by level
  Lev lev[kTailMaxLevels + 1];       // stencil constants and table pointer per level
  int k0, tlev, nops, smoother;  // tlev: the top level of the tail
  double tau;
  const int4* ops;       // device op list
  const double* lu;      // coarsest LU factors
  const int* piv;        // row interchanges (ncoarse), then the permutation they compose to (ncoarse)
  int ncoarse;
  const T* map;          // coarse map of level kTailMapLevel (column-major, nmap x nmap), or nullptr
  int nmap;
  int tab_lo;            // lowest level whose class blocks are used (below the map level: none)
  int use_lu;            // 0: no coarsest solve in the op list (the map covers it)
  const T* fT;           // f on level T (global)
  T* xT;                 // x on level T (global): in (if !first) / out
  int first;             // 1: x_T starts at zero and r_T = f_T
  const int* active;     // batched launches: 0 = skip this instance (nullptr: always run)
};

}  // namespace

template <typename T>
__device__ __forceinline__ void tail_body(const TailArgs<T>& A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int tid = threadIdx.x;
  constexpr int NT = kTailThreads;
  // shared layout after the level arrays: per-level class blocks, NE scratch p,
  // coarsest LU (double)
  const int Tl = A.tlev, k0 = A.k0;
  int off_end = 0;
  for (int l = k0; l <= Tl; l++) off_end = max(off_end, A.lv[l].of + 2 * A.lv[l].V);
  // All shared pointers are byte offsets from the LDS base: a pointer that
  // went through an integer would lose its address space and every access
  // through it would become a flat (generic) memory operation.
  auto align16 = [](size_t b) { return (b + 15) & ~size_t(15); };
  const size_t off_sp =
      align16((size_t)off_end * sizeof(T) + (size_t)(kTailMaxLevels + 1) * 25 * kC5 * sizeof(T));
  const size_t off_lu = align16(off_sp + tail_scratch_bytes<T>(A.lv[Tl].V, A.ncoarse, Tl));
  const int N0 = A.ncoarse;
  T* tC = sm + off_end;                                   // 25 * kC5 per level l in (k0, T]
  T* sp = reinterpret_cast<T*>(smem_raw + off_sp);        // NE scratch (2 V_T), also the coarse rhs in FP64
  double* slu = reinterpret_cast<double*>(smem_raw + off_lu);  // coarsest LU factors
  // two zero cells (one per field): neighbours outside the square are read
  // from and written to them, so every access of a vertex update is
  // unconditional (their coefficients are zero, so they stay zero)
  T* zs = reinterpret_cast<T*>(smem_raw + off_lu + (size_t)N0 * N0 * sizeof(double));

  // ---- load tables, LU, f_T and x_T.  Global loads are issued in unrolled
  // batches before the LDS stores that consume them, so a batch costs one
  // memory round trip (a loop of load-then-store would wait on every load).
  auto copy_in = [&](T* dst, const auto* src, int n) {  // dst[e] = (T)src[e], e < n
    constexpr int B = 8;
    for (int base = 0; base < n; base += B * NT) {
      T v[B];
#pragma unroll
      for (int u = 0; u < B; u++) {
        const int e = base + u * NT + tid;
        v[u] = e < n ? (T)src[e] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < B; u++) {
        const int e = base + u * NT + tid;
        if (e < n) dst[e] = v[u];
      }
    }
  };
  for (int l = A.tab_lo; l <= Tl; l++) copy_in(tC + l * 25 * kC5, &A.lev[l].tab->C5[0][0], 25 * kC5);
  if (A.use_lu) {
    // the LU stays FP64
    constexpr int B = 8;
    for (int base = 0; base < N0 * N0; base += B * NT) {
      double v[B];
#pragma unroll
      for (int u = 0; u < B; u++) {
        const int e = base + u * NT + tid;
        v[u] = e < N0 * N0 ? A.lu[e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < B; u++) {
        const int e = base + u * NT + tid;
        if (e < N0 * N0) slu[e] = v[u];
      }
    }
  }
  if (tid < 2) zs[tid] = (T)0;
  {
    const TailLevel& L = A.lv[Tl];
    copy_in(sm + L.of, A.fT, 2 * L.V);
    if (A.first) {
      for (int e = tid; e < 2 * L.V; e += NT) sm[L.ox + e] = (T)0;
    } else {
      copy_in(sm + L.ox, A.xT, 2 * L.V);
    }
  }
  bar();

  // Level parameters are copied into registers once per operation: read
  // from the argument block inside the vertex loops they would be fetched
  // again after every barrier, each fetch waiting for all LDS traffic.
  struct LP {
    int n, ld, V, ox, or_, of;
    T alpha, ainv;
    const T* cb0;  // the level's class blocks
  };
  auto level_params = [&](int l) {
    const TailLevel& g = A.lv[l];
    LP p;
    p.n = g.n;
    p.ld = g.ld;
    p.V = g.V;
    p.ox = g.ox;
    p.or_ = g.or_;
    p.of = g.of;
    p.alpha = (T)A.lev[l].alpha;
    p.ainv = (T)A.lev[l].ainv;
    p.cb0 = tC + l * 25 * kC5;
    return p;
  };

  // (A x) at vertex (i, j) from LDS array xa (both rows)
  auto apply_v = [&](const LP& L, const T* xa, int i, int j, T& ay, T& al) {
    const T* cb = L.cb0 + (cls5(i, L.n) * 5 + cls5(j, L.n)) * kC5;
    ay = 0;
    al = 0;
#pragma unroll
    for (int d = 0; d < kNDir; d++) {
      const int ii = i + kDI[d], jj = j + kDJ[d];
      const bool in = ii >= 0 && jj >= 0 && ii <= L.n && jj <= L.n;
      const int m = jj * L.ld + ii;
      const T a = *(in ? xa + m : zs), b = *(in ? xa + L.V + m : zs + 1);
      ay += cb[d] * a + cb[kNDir + d] * b;
      al += cb[kNDir + d] * a - L.ainv * cb[d] * b;
    }
  };
  // r = f - A x on one level
  auto residual = [&](const LP& L) {  // no barrier inside
    for (int v = tid; v < L.V; v += NT) {
      const int j = v / L.ld, i = v - j * L.ld;
      T ay, al;
      apply_v(L, sm + L.ox, i, j, ay, al);
      sm[L.or_ + v] = sm[L.of + v] - ay;
      sm[L.or_ + L.V + v] = sm[L.of + L.V + v] - al;
    }
  };
  // one vertex of a Gauss-Seidel-like phase: LSGS (Alg. 2) or collective GS
  auto gs_vertex = [&](const LP& L, int i, int j, bool collective) {
    const T* cb = L.cb0 + (cls5(i, L.n) * 5 + cls5(j, L.n)) * kC5;
    const T al = L.alpha, ainv = L.ainv;
    T* ry = sm + L.or_;
    T* rl = ry + L.V;
    // the class block in registers before any store: all shared arrays live
    // in one LDS block, so a store could alias it as far as the compiler knows
    T cm[kNDir], ck[kNDir], cw[kNDir];
#pragma unroll
    for (int d = 0; d < kNDir; d++) {
      cm[d] = cb[d];
      ck[d] = cb[kNDir + d];
      cw[d] = cb[2 * kNDir + d];
    }
    const T nyi = cb[3 * kNDir], nli = cb[3 * kNDir + 1];
    T* pa[kNDir];
    T* pb[kNDir];
    T va[kNDir], vb[kNDir];
#pragma unroll
    for (int d = 0; d < kNDir; d++) {
      const int ii = i + kDI[d], jj = j + kDJ[d];
      const bool in = ii >= 0 && jj >= 0 && ii <= L.n && jj <= L.n;
      const int m = jj * L.ld + ii;
      pa[d] = in ? ry + m : zs;
      pb[d] = in ? rl + m : zs + 1;
      va[d] = *pa[d];
      vb[d] = *pb[d];
    }
    // all 14 loads in flight before the first use (left to itself the
    // scheduler interleaves them with the sums, one LDS round trip per pair)
    __builtin_amdgcn_sched_barrier(0);
    T py, pl;
    if (!collective) {
      T qy = 0, ql = 0;
#pragma unroll
      for (int d = 0; d < kNDir; d++) {
        qy += (cm[d] * va[d] + al * ck[d] * vb[d]) * cw[d];
        ql += (ck[d] * va[d] - cm[d] * vb[d]) * cw[d];
      }
      py = qy * nyi;
      pl = ql * nli;
    } else {
      const T b11 = cm[0], b12 = ck[0], b21 = ck[0], b22 = -ainv * cm[0];
      const T det = b11 * b22 - b12 * b21;
      py = (b22 * va[0] - b12 * vb[0]) / det;
      pl = (b11 * vb[0] - b21 * va[0]) / det;
    }
    const int v = j * L.ld + i;
    T* xy = sm + L.ox + v;
    const T x0 = xy[0], x1 = xy[L.V];
#pragma unroll
    for (int d = 0; d < kNDir; d++) {
      *pa[d] = va[d] - (cm[d] * py + ck[d] * pl);
      *pb[d] = vb[d] - (ck[d] * py - ainv * (cm[d] * pl));
    }
    xy[0] = x0 + py;
    xy[L.V] = x1 + pl;
  };
  // one sweep in the colour order c = (i + 2j) mod 7 (reverse: c = 6..0);
  // work item k of a phase is slot t = k mod S of row j = k / S
  auto gs_sweep = [&](const LP& L, bool reverse, bool collective) {
    const int S = (L.ld + 6) / 7;
    const int nit = L.ld * S;
    for (int ph = 0; ph < 7; ph++) {
      const int c = reverse ? 6 - ph : ph;
      for (int k = tid; k < nit; k += NT) {
        const int j = k / S, t = k - j * S;
        const int i = ((c - 2 * j) % 7 + 7) % 7 + 7 * t;
        if (i <= L.n) gs_vertex(L, i, j, collective);
      }
      bar();
    }
  };
  // normal-equation step (Alg. 1): p = tau L^-1 A^T L^-1 r for all unknowns, x += p, r -= A p
  auto ne_step = [&](const LP& L) {
    const T al = L.alpha, tau = (T)A.tau;
    const T* ry = sm + L.or_;
    const T* rl = ry + L.V;
    for (int v = tid; v < L.V; v += NT) {
      const int j = v / L.ld, i = v - j * L.ld;
      const T* cb = L.cb0 + (cls5(i, L.n) * 5 + cls5(j, L.n)) * kC5;
      T qy = 0, ql = 0, wv = 0;
#pragma unroll
      for (int d = 0; d < kNDir; d++) {
        const int ii = i + kDI[d], jj = j + kDJ[d];
        const bool in = ii >= 0 && jj >= 0 && ii <= L.n && jj <= L.n;
        const int m = jj * L.ld + ii;
        const T a = *(in ? ry + m : zs), b = *(in ? rl + m : zs + 1);
        const T mm = cb[d], k = cb[kNDir + d], wi = cb[2 * kNDir + d];
        qy += (mm * a + al * k * b) * wi;
        ql += (k * a - mm * b) * wi;
        if (d == 0) wv = wi;
      }
      const T py = tau * qy * wv, pl = tau * ql * (al * wv);
      sp[v] = py;
      sp[L.V + v] = pl;
      sm[L.ox + v] += py;
      sm[L.ox + L.V + v] += pl;
    }
    bar();
    for (int v = tid; v < L.V; v += NT) {
      const int j = v / L.ld, i = v - j * L.ld;
      T ay, alv;
      apply_v(L, sp, i, j, ay, alv);
      sm[L.or_ + v] -= ay;
      sm[L.or_ + L.V + v] -= alv;
    }
    bar();
  };

  // level T starts from x_T = 0 (r_T = f_T) or from the given x_T (r_T = f_T - A x_T)
  if (A.first) {
    const TailLevel& L = A.lv[Tl];
    for (int e = tid; e < 2 * L.V; e += NT) sm[L.or_ + e] = sm[L.of + e];
  } else {
    residual(level_params(Tl));
  }
  bar();

  for (int o = 0; o < A.nops; o++) {
    const int4 op = A.ops[o];
    const int l = op.y;
    switch (op.x) {
      case kTailSmooth: {
        const LP P = level_params(l);
        const int sm_kind = A.smoother;
        for (int s = 0; s < op.z; s++) {
          if (sm_kind == MG_TAIL_NE)
            ne_step(P);
          else if (sm_kind == MG_TAIL_LSGS)
            gs_sweep(P, false, false);
          else if (sm_kind == MG_TAIL_SLSGS) {
            gs_sweep(P, false, false);
            gs_sweep(P, true, false);
          } else
            gs_sweep(P, false, true);
        }
        break;
      }
      case kTailResidual:
        residual(level_params(l));
        bar();
        break;
      case kTailRestrict: {  // f_{l-1} = P^T r_l; if l-1 > k0: x_{l-1} = 0, r_{l-1} = f_{l-1}
        const TailLevel Lf = A.lv[l];
        const TailLevel Lc = A.lv[l - 1];
        for (int w = tid; w < Lc.V; w += NT) {
          const int J = w / Lc.ld, I = w - J * Lc.ld;
          const int a = 2 * I, b = 2 * J;
          T gy = sm[Lf.or_ + b * Lf.ld + a], gl = sm[Lf.or_ + Lf.V + b * Lf.ld + a];
          T hy = 0, hl = 0;
#pragma unroll
          for (int d = 1; d < kNDir; d++) {
            const int aa = a + kDI[d], bb = b + kDJ[d];
            if (aa < 0 || bb < 0 || aa > Lf.n || bb > Lf.n) continue;
            hy += sm[Lf.or_ + bb * Lf.ld + aa];
            hl += sm[Lf.or_ + Lf.V + bb * Lf.ld + aa];
          }
          gy += (T)0.5 * hy;
          gl += (T)0.5 * hl;
          sm[Lc.of + w] = gy;
          sm[Lc.of + Lc.V + w] = gl;
          if (l - 1 > k0) {
            sm[Lc.ox + w] = 0;
            sm[Lc.ox + Lc.V + w] = 0;
            sm[Lc.or_ + w] = gy;
            sm[Lc.or_ + Lc.V + w] = gl;
          }
        }
        bar();
        break;
      }
      case kTailCoarse: {  // x_k0 = A_k0^{-1} f_k0, FP64 LU with row pivots
        // one wave, one row per lane (N0 <= 64): the permuted right-hand side,
        // then forward (unit lower) and back substitution with the pivot
        // entry of each step broadcast from its lane; no workgroup barriers
        const TailLevel Lc = A.lv[k0];
        if (tid < 64) {
          const int* perm = A.piv + N0;
          double v = tid < N0 ? (double)sm[Lc.of + perm[tid]] : 0.0;
          for (int k = 0; k + 1 < N0; k++) {
            const double bk = lane_bcast(v, k);
            if (tid > k && tid < N0) v -= slu[tid * N0 + k] * bk;
          }
          for (int k = N0 - 1; k >= 0; k--) {
            if (tid == k) v /= slu[k * N0 + k];
            const double bk = lane_bcast(v, k);
            if (tid < k) v -= slu[tid * N0 + k] * bk;
          }
          if (tid < N0) sm[Lc.ox + tid] = (T)v;
        }
        bar();
        break;
      }
      case kTailProlongResidual: {  // x_l += P x_{l-1}, then r_l = f_l - A x_l
        const TailLevel Lf = A.lv[l];
        const TailLevel Lc = A.lv[l - 1];
        for (int u = tid; u < Lf.V; u += NT) {
          const int b = u / Lf.ld, a = u - b * Lf.ld;
          const int w0 = (b >> 1) * Lc.ld + (a >> 1), w1 = ((b + 1) >> 1) * Lc.ld + ((a + 1) >> 1);
          T vy, vl;
          if (w0 == w1) {
            vy = sm[Lc.ox + w0];
            vl = sm[Lc.ox + Lc.V + w0];
          } else {
            vy = (T)0.5 * (sm[Lc.ox + w0] + sm[Lc.ox + w1]);
            vl = (T)0.5 * (sm[Lc.ox + Lc.V + w0] + sm[Lc.ox + Lc.V + w1]);
          }
          sm[Lf.ox + u] += vy;
          sm[Lf.ox + Lf.V + u] += vl;
        }
        bar();
        residual(level_params(l));
        bar();
        break;
      }
      case kTailApplyMap: {  // x_l += B r_l: the whole sub-cycle on level l and below, from zero
        // B is column-major: for one column, the lanes of a wave read
        // consecutive rows.  Each wave takes a quarter of the columns and each
        // lane three rows (lane, lane + 64, lane + 128), so a thread has
        // 3 x 14 loads in flight per batch; the per-wave partial sums meet in
        // the scratch and are added in wave order.
        const LP P = level_params(l);
        const int N = A.nmap;  // <= kTailMapN
        const int w = tid >> 6, lane = tid & 63;
        const int q = (N + kTailWaves - 1) / kTailWaves, cb0 = w * q, cb1 = min(N, cb0 + q);
        const T* rv = sm + P.or_;
        T acc[3] = {(T)0, (T)0, (T)0};
        constexpr int B = 14;
        for (int cb = cb0; cb < cb1; cb += B) {
          T v[3][B];
#pragma unroll
          for (int u = 0; u < B; u++)
#pragma unroll
            for (int k = 0; k < 3; k++) {
              const int row = lane + 64 * k, c = cb + u;
              v[k][u] = (c < cb1 && row < N) ? A.map[(size_t)c * N + row] : (T)0;
            }
#pragma unroll
          for (int u = 0; u < B; u++) {
            const T rc = cb + u < cb1 ? rv[cb + u] : (T)0;
#pragma unroll
            for (int k = 0; k < 3; k++) acc[k] += v[k][u] * rc;
          }
        }
#pragma unroll
        for (int k = 0; k < 3; k++)
          if (lane + 64 * k < N) sp[w * N + lane + 64 * k] = acc[k];
        bar();
        if (tid < N) {
          T sum = sp[tid];
          for (int ww = 1; ww < kTailWaves; ww++) sum += sp[ww * N + tid];
          sm[P.ox + tid] += sum;
        }
        bar();
        break;
      }
      default:
        break;
    }
  }

  // ---- x_T out
  {
    const TailLevel& L = A.lv[Tl];
    for (int e = tid; e < 2 * L.V; e += NT) A.xT[e] = sm[L.ox + e];
  }
}

template <typename T>
__global__ __launch_bounds__(kTailThreads) void k_tail(TailArgs<T> A) {
  tail_body<T>(A);
}

// one workgroup per instance of a batch
template <typename T>
__global__ __launch_bounds__(kTailThreads) void kb_tail(const TailArgs<T>* __restrict__ all) {
  const TailArgs<T>& A = all[blockIdx.x];
  if (A.active && !*A.active) return;
  tail_body<T>(A);
}

// host-side layout of the tail: LDS offsets and bytes
template <typename T>
size_t tail_layout(int k0, int Tl, TailLevel* lv) {
  int at = 0;
  for (int l = k0; l <= Tl; l++) {
    const int n = 1 << l;
    lv[l].n = n;
    lv[l].ld = n + 1;
    lv[l].V = (n + 1) * (n + 1);
    lv[l].ox = at;
    at += 2 * lv[l].V;
    lv[l].or_ = at;
    at += 2 * lv[l].V;
    lv[l].of = at;
    at += 2 * lv[l].V;
  }
  const int N0 = 2 * ((1 << k0) + 1) * ((1 << k0) + 1);
  return (size_t)at * sizeof(T) + (size_t)(kTailMaxLevels + 1) * 25 * kC5 * sizeof(T) + 16 +
         tail_scratch_bytes<T>(lv[Tl].V, N0, Tl) + 16 + (size_t)N0 * N0 * sizeof(double) + 2 * sizeof(T);
}

template <typename T>
size_t fill_tail_args(const TailLaunch& tl, const T* fT, T* xT, int first, const int* active, TailArgs<T>& a) {
  memset(&a, 0, sizeof(a));
  const size_t bytes = tail_layout<T>(tl.k0, tl.T, a.lv);
  for (int l = tl.k0; l <= tl.T; l++) a.lev[l] = tl.lev[l];
  a.k0 = tl.k0;
  a.tlev = tl.T;
  a.nops = tl.nops;
  a.ops = tl.ops;
  a.smoother = tl.smoother;
  a.tau = tl.tau;
  a.lu = tl.lu;
  a.piv = tl.piv;
  a.ncoarse = tl.ncoarse;
  if constexpr (std::is_same<T, double>::value)
    a.map = tl.map64;
  else
    a.map = tl.map32;
  a.nmap = tl.nmap;
  a.tab_lo = a.map ? kTailMapLevel : tl.k0 + 1;  // a W-cycle takes a residual on the map level
  a.use_lu = a.map ? 0 : 1;
  a.fT = fT;
  a.xT = xT;
  a.first = first;
  a.active = active;
  return bytes;
}

template <typename T>
hipError_t launch_tail(const TailLaunch& tl, const T* fT, T* xT, int first, hipStream_t s) {
  TailArgs<T> a;
  const size_t bytes = fill_tail_args<T>(tl, fT, xT, first, nullptr, a);
  if (bytes > tl.max_lds) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_tail<T>), dim3(1), dim3(kTailThreads), bytes, s, a);
  return hipGetLastError();
}

template <typename T>
size_t tail_args_bytes() {
  return sizeof(TailArgs<T>);
}

template <typename T>
void make_tail_args(const TailLaunch& tl, const T* fT, T* xT, int first, const int* active, void* out) {
  (void)fill_tail_args<T>(tl, fT, xT, first, active, *static_cast<TailArgs<T>*>(out));
}

template <typename T>
hipError_t launch_b_tail(const void* args, int count, size_t lds_bytes, hipStream_t s) {
  hipLaunchKernelGGL((kb_tail<T>), dim3(count), dim3(kTailThreads), lds_bytes, s,
                     static_cast<const TailArgs<T>*>(args));
  return hipGetLastError();
}

template <typename T>
size_t tail_lds_bytes(int k0, int Tl) {
  TailLevel lv[kTailMaxLevels + 1];
  return tail_layout<T>(k0, Tl, lv);
}

hipError_t tail_allow_lds(size_t bytes) {
  const void* fns[4] = {(const void*)k_tail<double>, (const void*)k_tail<float>, (const void*)kb_tail<double>,
                        (const void*)kb_tail<float>};
  for (const void* fn : fns) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t launch_tail<double>(const TailLaunch&, const double*, double*, int, hipStream_t);
template hipError_t launch_tail<float>(const TailLaunch&, const float*, float*, int, hipStream_t);
template size_t tail_lds_bytes<double>(int, int);
template size_t tail_lds_bytes<float>(int, int);
template size_t tail_args_bytes<double>();
template size_t tail_args_bytes<float>();
template void make_tail_args<double>(const TailLaunch&, const double*, double*, int, const int*, void*);
template void make_tail_args<float>(const TailLaunch&, const float*, float*, int, const int*, void*);
template hipError_t launch_b_tail<double>(const void*, int, size_t, hipStream_t);
template hipError_t launch_b_tail<float>(const void*, int, size_t, hipStream_t);

}  // namespace mgk
