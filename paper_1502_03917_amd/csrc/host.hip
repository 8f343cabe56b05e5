// Host side of libmgkkt: stencil tables, coarsest-level LU, level hierarchy,
// the multigrid cycle of section 2 (Takacs, arXiv 1502.03917) as a sequence of
// stream-ordered HIP launches, and the C ABI of include/mgkkt.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <algorithm>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/mgkkt.h"
#include "mg_internal.hpp"

using mgk::Lev;
using mgk::Tab;

namespace {

constexpr int kMaxLevel = 12;
// Stokes control: the host assembles the level's KKT matrix (eq. mp3) in CSR
// with 32-bit row pointers before compressing it into stencil classes; level
// 10 (1025^2 vertices, about 5.4e8 nonzeros) is the largest that fits them.
constexpr int kMaxStokesLevel = 10;
constexpr int kMaxCoarse = 3;  // coarsest LU of 2 (2^k0+1)^2 <= 162 unknowns
// mg_solve reports a stall when the best relative residual of the last 10
// iterates is not below half the best of the 10 before them
constexpr int kStallWindow = 10;
// batches: every instance needs the coarse-level tail on levels k0..5
constexpr int kMaxBatch = 1024;
constexpr int kBatchMinLevel = 6;

// ---------------------------------------------------------------- tables

int dir_of(int di, int dj) {
  for (int d = 0; d < mgk::kNDir; d++)
    if (mgk::kDI[d] == di && mgk::kDJ[d] == dj) return d;
  return -1;
}

// Row of vertex (i, j) of M and of the Laplacian stiffness matrix, from the
// triangles incident to it.  Square (p, q) is split into {(p,q), (p+1,q),
// (p+1,q+1)} with the right angle at (p+1,q) and {(p,q), (p+1,q+1), (p,q+1)}
// with the right angle at (p,q+1).  On a right isosceles P1 triangle the local
// mass matrix is |T|/12 (1 + delta) = h^2/24 (1 + delta); the local stiffness
// matrix has 1 at the right-angle vertex, 1/2 at the two others, -1/2 along
// the legs and 0 along the hypotenuse.
void row_coefs(int i, int j, int n, double M[mgk::kNDir], double Kl[mgk::kNDir]) {
  const double h2 = 1.0 / ((double)n * (double)n);
  for (int d = 0; d < mgk::kNDir; d++) M[d] = Kl[d] = 0.0;
  for (int q = j - 1; q <= j; q++)
    for (int p = i - 1; p <= i; p++) {
      if (p < 0 || q < 0 || p >= n || q >= n) continue;
      const int tri[2][3][2] = {{{p, q}, {p + 1, q}, {p + 1, q + 1}}, {{p, q}, {p + 1, q + 1}, {p, q + 1}}};
      const int right[2][2] = {{p + 1, q}, {p, q + 1}};
      for (int t = 0; t < 2; t++) {
        bool has_v = false;
        for (int a = 0; a < 3; a++) has_v |= (tri[t][a][0] == i && tri[t][a][1] == j);
        if (!has_v) continue;
        const bool v_right = (right[t][0] == i && right[t][1] == j);
        for (int a = 0; a < 3; a++) {
          const int wi = tri[t][a][0], wj = tri[t][a][1];
          const int d = dir_of(wi - i, wj - j);
          if (d == 0) {
            M[0] += 2.0 * h2 / 24.0;
            Kl[0] += v_right ? 1.0 : 0.5;
          } else {
            const bool w_right = (right[t][0] == wi && right[t][1] == wj);
            M[d] += h2 / 24.0;
            Kl[d] += (v_right || w_right) ? -0.5 : 0.0;
          }
        }
      }
    }
}

// representative index of a 3-class / 5-class along one axis (n >= 4)
int rep3(int c, int n) { return c == 0 ? 0 : (c == 2 ? n : n / 2); }
int rep5(int c, int n) { return c <= 1 ? c : (c == 2 ? n / 2 : (c == 3 ? n - 1 : n)); }

struct LevelTables {
  Tab tab;
  Lev lev;  // tab pointer filled in later
};

LevelTables make_tables(int level, double alpha, double tau) {
  const int n = 1 << level;
  LevelTables out;
  std::memset(&out, 0, sizeof(out));
  Tab& T = out.tab;
  const double sa = std::sqrt(alpha);
  double W9[9];
  for (int ci = 0; ci < 3; ci++)
    for (int cj = 0; cj < 3; cj++) {
      const int c = ci * 3 + cj;
      double M[mgk::kNDir], Kl[mgk::kNDir];
      row_coefs(rep3(ci, n), rep3(cj, n), n, M, Kl);
      for (int d = 0; d < mgk::kNDir; d++) {
        T.M[c][d] = M[d];
        T.K[c][d] = Kl[d] + M[d];
      }
      W9[c] = M[0] + sa * (Kl[0] + M[0]);  // diag(M + sqrt(alpha) K)
      T.Winv[c] = 1.0 / W9[c];
    }
  // N_ii = sum_j A_ij^2 / L_jj, L = blockdiag(W, W/alpha)
  for (int ci = 0; ci < 5; ci++)
    for (int cj = 0; cj < 5; cj++) {
      const int i = rep5(ci, n), j = rep5(cj, n);
      double M[mgk::kNDir], Kl[mgk::kNDir];
      row_coefs(i, j, n, M, Kl);
      double nyy = 0.0, nll = 0.0;
      for (int d = 0; d < mgk::kNDir; d++) {
        const int ii = i + mgk::kDI[d], jj = j + mgk::kDJ[d];
        if (ii < 0 || jj < 0 || ii > n || jj > n) continue;
        const double Wm = W9[mgk::cls3(ii, n) * 3 + mgk::cls3(jj, n)];
        const double m = M[d], k = Kl[d] + M[d];
        nyy += (m * m + alpha * k * k) / Wm;
        nll += (k * k + m * m / alpha) / Wm;
      }
      T.Nyi[ci * 5 + cj] = 1.0 / nyy;
      T.Nli[ci * 5 + cj] = 1.0 / nll;
      double* blk = T.C5[ci * 5 + cj];
      for (int d = 0; d < mgk::kNDir; d++) {
        const int ii = i + mgk::kDI[d], jj = j + mgk::kDJ[d];
        const bool in = !(ii < 0 || jj < 0 || ii > n || jj > n);
        blk[d] = in ? M[d] : 0.0;
        blk[mgk::kNDir + d] = in ? Kl[d] + M[d] : 0.0;
        blk[2 * mgk::kNDir + d] = in ? 1.0 / W9[mgk::cls3(ii, n) * 3 + mgk::cls3(jj, n)] : 0.0;
      }
      blk[3 * mgk::kNDir] = 1.0 / nyy;
      blk[3 * mgk::kNDir + 1] = 1.0 / nll;
      blk[3 * mgk::kNDir + 2] = 0.0;
    }
  Lev& L = out.lev;
  L.n = n;
  L.ld = n + 1;
  L.V = (n + 1) * (n + 1);
  L.alpha = alpha;
  L.ainv = 1.0 / alpha;
  L.tau = tau;
  const int mid = 1 * 3 + 1;  // inside class
  L.Mc = T.M[mid][0];
  L.Mo = T.M[mid][1];
  L.Kc = T.K[mid][0];
  L.Ka = T.K[mid][1];
  L.Kd = T.K[mid][5];
  L.Winv = T.Winv[mid];
  L.Nyi = T.Nyi[2 * 5 + 2];
  L.Nli = T.Nli[2 * 5 + 2];
  L.tab = nullptr;
  return out;
}

// dense KKT matrix of a (small) level, row-major, from the row stencils
std::vector<double> dense_kkt(int level, double alpha) {
  const int n = 1 << level, V = (n + 1) * (n + 1), N = 2 * V;
  std::vector<double> A((size_t)N * N, 0.0);
  for (int j = 0; j <= n; j++)
    for (int i = 0; i <= n; i++) {
      double M[mgk::kNDir], Kl[mgk::kNDir];
      row_coefs(i, j, n, M, Kl);
      const int v = j * (n + 1) + i;
      for (int d = 0; d < mgk::kNDir; d++) {
        const int ii = i + mgk::kDI[d], jj = j + mgk::kDJ[d];
        if (ii < 0 || jj < 0 || ii > n || jj > n) continue;
        const int m = jj * (n + 1) + ii;
        const double k = Kl[d] + M[d];
        A[(size_t)v * N + m] += M[d];
        A[(size_t)v * N + V + m] += k;
        A[(size_t)(V + v) * N + m] += k;
        A[(size_t)(V + v) * N + V + m] += -M[d] / alpha;
      }
    }
  return A;
}

// LU with partial (row) pivoting in place; returns false if singular
bool lu_factor(int N, std::vector<double>& a, std::vector<int>& piv) {
  piv.assign(N, 0);
  for (int k = 0; k < N; k++) {
    int p = k;
    for (int i = k + 1; i < N; i++)
      if (std::fabs(a[(size_t)i * N + k]) > std::fabs(a[(size_t)p * N + k])) p = i;
    piv[k] = p;
    if (p != k)
      for (int c = 0; c < N; c++) std::swap(a[(size_t)k * N + c], a[(size_t)p * N + c]);
    const double d = a[(size_t)k * N + k];
    if (d == 0.0 || !std::isfinite(d)) return false;
    for (int i = k + 1; i < N; i++) {
      const double l = a[(size_t)i * N + k] / d;
      a[(size_t)i * N + k] = l;
      for (int c = k + 1; c < N; c++) a[(size_t)i * N + c] -= l * a[(size_t)k * N + c];
    }
  }
  return true;
}

}  // namespace

// ------------------------------------------------- static scratch (no allocation)
//
// mg_residual_nalloc keeps its norm partial sums in this file-scope device
// array instead of the context's workspace: 32768 doubles (256 KiB), one copy
// per GPU, held until the process ends.  Host code never passes the array's
// name to a kernel (on the host it is only a stand-in symbol): mg_setup takes
// its device address once per device with hipGetSymbolAddress, with that
// device current, and the entry point uses that address.  Every call on a GPU
// shares the array, so calls that overlap on one GPU race.
constexpr int kScratchWords = 32768;
static __device__ __align__(256) double scratch[kScratchWords];

namespace {
constexpr int kScratchMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kScratchMaxDevices] = {};

// device address of `scratch` on device dev (which must be current), taken once
hipError_t scratch_init(int dev) {
  if (dev < 0 || dev >= kScratchMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[dev] = static_cast<double*>(ptr);
  return hipSuccess;
}

double* scratch_ptr(int dev) {
  if (dev < 0 || dev >= kScratchMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[dev];
}
}  // namespace

// -------------------------------------------------------------------- context

struct LevelBuf {
  int level = 0;
  Lev lev{};
  Tab* d_tab = nullptr;
  size_t len = 0;  // 2V
  // r2: second residual buffer; the fused LSGS sweep reads one and writes the other
  double *x = nullptr, *f = nullptr, *r = nullptr, *r2 = nullptr, *p = nullptr;
  float *x32 = nullptr, *f32 = nullptr, *r32 = nullptr, *r2_32 = nullptr, *p32 = nullptr;
};

struct mg_ctx {
  int problem = 0, level = 0, k0 = 1, device = 0;
  double alpha = 1.0;
  mg_opts o{};
  std::vector<LevelBuf> lv;  // lv[l - k0]
  int ncoarse = 0;
  double* d_lu = nullptr;
  int* d_piv = nullptr;
  double* d_part = nullptr;  // per-block partial sums
  size_t npart = 0;
  double* d_norm = nullptr;  // [0] = ||r||^2 of the latest residual, [1] = ||f||^2
  double* h_norm = nullptr;  // pinned host copy
  bool fp32_ready = false;
  bool fused = true;  // one kernel per LSGS sweep (else one kernel per colour phase)
  bool sweep2 = true;  // two sweeps per launch on small coarse levels (MGKKT_NO_SWEEP2 unset)
  // the restriction runs in the last pre-smoothing launch and the
  // prolongation with the new residual in the first post-smoothing launch
  // (MGKKT_NO_FUSED_TRANSFERS unset)
  bool xfer_allowed = true;
  // coarse-level tail: one workgroup runs the sub-cycle on levels k0..tail_T
  int tail_T = 0;       // 0: no tail
  bool tail_allowed = true;
  int4* d_tail_ops = nullptr;
  mgk::TailLaunch tail{};
  // precomputed coarse map of the tail (the sub-cycle on level kTailMapLevel
  // and below as a dense matrix); map_allowed: MGKKT_NO_MAP unset
  bool map_allowed = true;
  // the last post-smoothing sweep supplies the residual norm (MGKKT_NO_SWEEP_NORM unset)
  bool sweep_norm_allowed = true;
  double* d_map64 = nullptr;
  float* d_map32 = nullptr;
  // dense map of the tail's top level (kDenseMapLevel), row-major: one
  // matrix-vector product replaces the tail launch in single-instance cycles;
  // dmap_allowed: MGKKT_NO_DENSE_MAP unset
  bool dmap_allowed = true;
  int dmap_n = 0;  // 0: not built
  double* d_dmap64 = nullptr;
  float* d_dmap32 = nullptr;
  // HIP graph of one solver iterate (cycle + residual norm) for fixed f, x
  hipStream_t cap_stream = nullptr;  // capture stream (default priority)
  bool graphs = true;
  hipGraphExec_t gexec = nullptr;
  const double* g_f = nullptr;
  double* g_x = nullptr;
  bool capturing = false;
  unsigned long opts_gen = 0;  // bumped by mg_set_opts; caller graphs record it
  // timing of the finest-level smoothing sweeps
  bool timing = false;
  std::vector<hipEvent_t> ev;  // pairs
  size_t ev_used = 0;
  double t_ms = 0.0;
  long t_n = 0;
  std::string err;
  // Stokes control: the CSR-based solver of stokes.hip (nullptr for Poisson)
  mgk::Stokes* st = nullptr;
};

// caller-owned executable graph of one mg_cycle
struct mg_graph {
  hipGraphExec_t exec;
  mg_ctx* ctx;
  unsigned long gen;  // ctx->opts_gen at capture
};

namespace {

const char* kStatusText[] = {"success",
                             "invalid argument",
                             "HIP runtime error",
                             "device memory allocation failed",
                             "no convergence within max_cycles",
                             "non-finite residual norm",
                             "residual diverged",
                             "not supported by this build",
                             "residual stagnated at the precision floor"};

int fail(mg_ctx* c, int status, const std::string& msg) {
  if (c) c->err = msg;
  return status;
}

#define HIPCHK(ctx, expr)                                                                                  \
  do {                                                                                                     \
    hipError_t e_ = (expr);                                                                                \
    if (e_ != hipSuccess)                                                                                  \
      return fail((ctx), e_ == hipErrorOutOfMemory ? MG_ENOMEM : MG_EHIP,                                  \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                                      \
  } while (0)

LevelBuf& L_(mg_ctx* c, int l) { return c->lv[l - c->k0]; }

// paper defaults (section 3): NE 0.4 (Poisson) / 0.35 (Stokes), patch smoother 0.4
double default_tau(int problem, int smoother) {
  return (problem == MG_STOKES && smoother != MG_VANKA) ? 0.35 : 0.4;
}

// problem / smoother pairs that the build does not provide: the patch
// smoother is defined for Stokes only, the collective point smoother for
// Poisson only; Stokes solves the coarsest level k0 <= 2
bool unsupported_pair(int problem, const mg_opts& q) {
  if (problem == MG_POISSON && q.smoother == MG_VANKA) return true;
  if (problem == MG_STOKES && (q.smoother == MG_CGS || q.coarse_level > 2)) return true;
  return false;
}

bool valid_opts(const mg_opts* o, int level) {
  if (!o) return true;
  if (o->smoother < MG_NE || o->smoother > MG_VANKA) return false;
  if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 > 64 || o->nu2 > 64) return false;
  if (o->gamma < 1 || o->gamma > 2) return false;
  if (!std::isfinite(o->tau) || o->tau >= 2.0) return false;
  if (o->coarse_level < 1 || o->coarse_level > kMaxCoarse) return false;
  if (level >= 0 && level < o->coarse_level + 1) return false;
  if (o->precision != MG_FP64 && o->precision != MG_FP32_IR) return false;
  if (o->max_cycles < 0 || o->max_cycles > 100000) return false;
  if (o->inner_cycles < 1 || o->inner_cycles > 64) return false;
  if (o->norm != MG_NORM_L2 && o->norm != MG_NORM_LINV) return false;
  return true;
}

void destroy_impl(mg_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  for (auto& b : c->lv) {
    (void)hipFree(b.d_tab);
    (void)hipFree(b.x);
    (void)hipFree(b.f);
    (void)hipFree(b.r);
    (void)hipFree(b.r2);
    (void)hipFree(b.p);
    (void)hipFree(b.x32);
    (void)hipFree(b.f32);
    (void)hipFree(b.r32);
    (void)hipFree(b.r2_32);
    (void)hipFree(b.p32);
  }
  (void)hipFree(c->d_lu);
  (void)hipFree(c->d_piv);
  (void)hipFree(c->d_tail_ops);
  (void)hipFree(c->d_map64);
  (void)hipFree(c->d_map32);
  (void)hipFree(c->d_dmap64);
  (void)hipFree(c->d_dmap32);
  (void)hipFree(c->d_part);
  (void)hipFree(c->d_norm);
  if (c->h_norm) (void)hipHostFree(c->h_norm);
  for (auto e : c->ev) (void)hipEventDestroy(e);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  mgk::stokes_destroy(c->st);
  delete c;
}

int alloc_fp32(mg_ctx* c) {
  if (c->fp32_ready) return MG_OK;
  for (auto& b : c->lv) {
    const size_t bytes = b.len * sizeof(float);
    HIPCHK(c, hipMalloc(&b.x32, bytes));
    HIPCHK(c, hipMalloc(&b.f32, bytes));
    HIPCHK(c, hipMalloc(&b.r32, bytes));
    if (b.level > c->k0) {
      HIPCHK(c, hipMalloc(&b.p32, bytes));
      HIPCHK(c, hipMalloc(&b.r2_32, bytes));
    }
  }
  c->fp32_ready = true;
  return MG_OK;
}

// ------------------------------------------------------------- cycle (T = double / float)

template <typename T>
struct Work {
  T *x, *f, *r, *r2, *p;
};
Work<double> work(LevelBuf& b, double*) { return {b.x, b.f, b.r, b.r2, b.p}; }
Work<float> work(LevelBuf& b, float*) { return {b.x32, b.f32, b.r32, b.r2_32, b.p32}; }

// start a timed sweep with an event pair from the pool (folded into the
// running total when it fills up); timed solves run without graphs
hipEvent_t timing_begin(mg_ctx* c, hipStream_t s, size_t* slot) {
  if (c->ev_used + 2 > c->ev.size()) {
    // fold the recorded pairs into the running total before reusing them
    if (!c->ev.empty()) {
      (void)hipEventSynchronize(c->ev[c->ev_used - 1]);
      for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]) == hipSuccess) c->t_ms += ms;
      }
      c->ev_used = 0;
    }
    while (c->ev.size() < 2048) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) break;
      c->ev.push_back(e);
    }
  }
  *slot = c->ev_used;
  c->ev_used += 2;
  (void)hipEventRecord(c->ev[*slot], s);
  return c->ev[*slot + 1];
}

// `steps` smoothing steps on level l.  r holds f - A x on entry; the fused
// LSGS and collective-smoother sweeps alternate between r and alt, and r is
// updated to the buffer holding the current residual on return.
// Residual norm of the last sweep (FP64 tile sweeps only): when part is
// given, the last sweep also stores per-tile partial sums of ||r||^2 of the
// residual it leaves (norm mode `mode`) and *nb receives their number.
struct SweepNorm {
  double* part = nullptr;
  int mode = 0;
  int* nb = nullptr;
};

template <typename T>
hipError_t last_sweep(const Lev& L, int reverse, const T* xin, T* x, const T* rin, T* rout, const SweepNorm& sn,
                      hipStream_t s, bool cgs = false, const mgk::SweepIO<T>* io = nullptr) {
  if constexpr (std::is_same<T, double>::value) {
    if (sn.part)
      return cgs ? mgk::launch_cgs_sweep_norm(L, xin, x, rin, rout, sn.part, sn.mode, sn.nb, s, io)
                 : mgk::launch_lsgs_sweep_norm(L, reverse, xin, x, rin, rout, sn.part, sn.mode, sn.nb, s, io);
  }
  return cgs ? mgk::launch_cgs_sweep_from<T>(L, xin, x, rin, rout, s, io)
             : mgk::launch_lsgs_sweep_from<T>(L, reverse, xin, x, rin, rout, s, io);
}

// Grid transfers carried by the tile-sweep launches of one smooth_steps call:
// the first launch may form the prolongation with the new residual (first),
// the last may write the restriction (last) and its iterate to last_x.
// first_xzero: the first launch takes the iterate as zero (reads no x).
template <typename T>
struct SweepXfer {
  const mgk::SweepIO<T>* first = nullptr;
  const mgk::SweepIO<T>* last = nullptr;
  T* last_x = nullptr;
  bool first_xzero = false;
};

template <typename T>
int smooth_steps(mg_ctx* c, int l, T* x, T*& r, T* alt, T* p, int steps, hipStream_t s, const T* xin0 = nullptr,
                 const SweepNorm& sn = SweepNorm{}, const SweepXfer<T>& xf = SweepXfer<T>{}) {
  LevelBuf& b = L_(c, l);
  const Lev& L = b.lev;
  const bool timed = c->timing && l == c->level && !c->capturing;
  const bool fused = c->fused && alt != nullptr;
  // below the finest level, small levels run two sweeps per launch (an
  // LSGS or collective-smoother pair, or the forward and backward sweep of
  // an sLSGS step)
  const bool pairs = fused && c->sweep2 && l < c->level && L.n <= mgk::lsgs_sweep2_max_n();
  for (int it = 0; it < steps; it++) {
    // the first tile sweep may take the iterate from xin0 (fused prolongation)
    const T* xin = (it == 0 && xin0) ? xin0 : x;
    const SweepNorm none{};
    const SweepNorm& snl = (it == steps - 1) ? sn : none;
    // transfers of this step's launches: the prolongation on the first
    // launch of the call, the restriction (with the iterate written to
    // xf.last_x) on the last; a zero iterate on the first
    const bool first = it == 0;
    const bool last_single = it == steps - 1;          // a one-sweep launch ending the call
    const bool last_pair = pairs && it + 2 == steps;  // a two-sweep launch ending the call
    mgk::SweepIO<T> zio;
    auto io_for = [&](bool f, bool l) -> const mgk::SweepIO<T>* {
      const mgk::SweepIO<T>* a = (l && xf.last) ? xf.last : (f ? xf.first : nullptr);
      if (!(f && xf.first_xzero)) return a;
      if (a) zio = *a;
      zio.xin_zero = true;
      return &zio;
    };
    auto x_for = [&](bool l) { return (l && xf.last) ? xf.last_x : x; };
    size_t slot = 0;
    hipEvent_t stop = nullptr;
    if (timed) stop = timing_begin(c, s, &slot);
    switch (c->o.smoother) {
      case MG_NE:
        if (fused) {  // one pass over LDS tiles, r ping-pong
          HIPCHK(c, mgk::launch_ne_tile<T>(L, x, r, alt, s));
          std::swap(r, alt);
        } else {
          HIPCHK(c, mgk::launch_ne<T>(L, x, r, p, s));
        }
        break;
      case MG_LSGS:
        if (pairs && it + 1 < steps) {
          HIPCHK(c, mgk::launch_lsgs_sweep2<T>(L, 0, xin, x_for(last_pair), r, alt, s, io_for(first, last_pair)));
          std::swap(r, alt);
          it++;
        } else if (fused) {
          HIPCHK(c, last_sweep<T>(L, 0, xin, x_for(last_single), r, alt, snl, s, false, io_for(first, last_single)));
          std::swap(r, alt);
        } else {
          for (int col = 0; col < 7; col++) HIPCHK(c, mgk::launch_lsgs_phase<T>(L, col, x, r, s));
        }
        break;
      case MG_SLSGS:
        if (pairs) {
          HIPCHK(c, mgk::launch_lsgs_sweep2<T>(L, 2, xin, x_for(last_single), r, alt, s, io_for(first, last_single)));
          std::swap(r, alt);
        } else if (fused) {
          HIPCHK(c, mgk::launch_lsgs_sweep_from<T>(L, 0, xin, x, r, alt, s, io_for(first, false)));
          HIPCHK(c, last_sweep<T>(L, 1, x, x_for(last_single), alt, r, snl, s, false, io_for(false, last_single)));
        } else {
          for (int col = 0; col < 7; col++) HIPCHK(c, mgk::launch_lsgs_phase<T>(L, col, x, r, s));
          for (int col = 6; col >= 0; col--) HIPCHK(c, mgk::launch_lsgs_phase<T>(L, col, x, r, s));
        }
        break;
      case MG_CGS:
        if (pairs && it + 1 < steps) {
          HIPCHK(c, mgk::launch_cgs_sweep2<T>(L, xin, x_for(last_pair), r, alt, s, io_for(first, last_pair)));
          std::swap(r, alt);
          it++;
        } else if (fused) {
          HIPCHK(c, last_sweep<T>(L, 0, xin, x_for(last_single), r, alt, snl, s, true, io_for(first, last_single)));
          std::swap(r, alt);
        } else {
          for (int col = 0; col < 7; col++) HIPCHK(c, mgk::launch_cgs_phase<T>(L, col, x, r, s));
        }
        break;
      default:
        return fail(c, MG_EUNSUPPORTED, "smoother not provided for Poisson control");
    }
    if (timed && stop) {
      (void)hipEventRecord(stop, s);
      c->t_n++;
    }
  }
  return MG_OK;
}

template <typename T>
int coarse_solve_T(mg_ctx* c, const T* f, T* x, hipStream_t s) {
  HIPCHK(c, mgk::launch_coarse_solve<T>(c->ncoarse, c->d_lu, c->d_piv, f, x, s));
  return MG_OK;
}

// One iterate on level l for A_l x = f; r is level-l workspace.  If
// residual_current, r already holds f - A_l x.
// Op list of one iterate on level l of the tail (same steps as cycle_body):
// nu1 smoothing steps, restriction (x_{l-1} = 0, r_{l-1} = f_{l-1}), gamma
// coarse iterates (a fresh residual before the second), prolongation with the
// new residual, nu2 smoothing steps; the coarsest level is the LU solve.  On
// level map_level (0: none) an iterate is x += B r with the precomputed map B
// of the sub-cycle from zero (an iterate of a linear method from x equals
// x + B (f - A x)).
void tail_ops(const mg_ctx* c, int l, std::vector<int4>& ops, int map_level) {
  if (l == c->k0) {
    ops.push_back(make_int4(mgk::kTailCoarse, l, 0, 0));
    return;
  }
  if (l == map_level) {
    ops.push_back(make_int4(mgk::kTailApplyMap, l, 0, 0));
    return;
  }
  if (c->o.nu1) ops.push_back(make_int4(mgk::kTailSmooth, l, c->o.nu1, 0));
  ops.push_back(make_int4(mgk::kTailRestrict, l, 0, 0));
  for (int g = 0; g < c->o.gamma; g++) {
    if (g > 0 && l - 1 > c->k0) ops.push_back(make_int4(mgk::kTailResidual, l - 1, 0, 0));
    tail_ops(c, l - 1, ops, map_level);
  }
  ops.push_back(make_int4(mgk::kTailProlongResidual, l, 0, 0));
  if (c->o.nu2) ops.push_back(make_int4(mgk::kTailSmooth, l, c->o.nu2, 0));
}

// The coarse map B of level kTailMapLevel: column i is the tail's sub-cycle on
// that level (with everything below it) applied to the unit vector e_i, all
// columns computed by one batched tail launch.  Stored column-major in FP64
// and as an FP32 copy for the FP32 cycles.
int build_coarse_map(mg_ctx* c, const mgk::TailLaunch& base, size_t lds_bytes) {
  constexpr int ML = mgk::kTailMapLevel;
  const int N = 2 * ((1 << ML) + 1) * ((1 << ML) + 1);
  std::vector<int4> ops;
  tail_ops(c, ML, ops, 0);
  mgk::TailLaunch t = base;
  t.T = ML;
  t.nops = (int)ops.size();
  t.map64 = nullptr;
  t.map32 = nullptr;
  t.nmap = 0;
  int4* d_ops = nullptr;
  double* d_id = nullptr;
  void* d_args = nullptr;
  auto done = [&](int st) {
    (void)hipFree(d_ops);
    (void)hipFree(d_id);
    (void)hipFree(d_args);
    return st;
  };
  if (hipMalloc(&d_ops, ops.size() * sizeof(int4)) != hipSuccess ||
      hipMalloc(&d_id, (size_t)N * N * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->d_map64, (size_t)N * N * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->d_map32, (size_t)N * N * sizeof(float)) != hipSuccess)
    return done(fail(c, MG_ENOMEM, "coarse map: device allocation failed"));
  std::vector<double> id((size_t)N * N, 0.0);
  for (int i = 0; i < N; i++) id[(size_t)i * N + i] = 1.0;
  t.ops = d_ops;
  const size_t sz = mgk::tail_args_bytes<double>();
  std::vector<unsigned char> args((size_t)N * sz);
  for (int i = 0; i < N; i++)
    mgk::make_tail_args<double>(t, d_id + (size_t)i * N, c->d_map64 + (size_t)i * N, 1, nullptr, args.data() + i * sz);
  if (hipMalloc(&d_args, args.size()) != hipSuccess) return done(fail(c, MG_ENOMEM, "coarse map: device allocation failed"));
  hipError_t e = hipMemcpy(d_ops, ops.data(), ops.size() * sizeof(int4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_id, id.data(), id.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_args, args.data(), args.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = mgk::launch_b_tail<double>(d_args, N, lds_bytes, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  std::vector<double> m64((size_t)N * N);
  if (e == hipSuccess) e = hipMemcpy(m64.data(), c->d_map64, m64.size() * sizeof(double), hipMemcpyDeviceToHost);
  std::vector<float> m32(m64.begin(), m64.end());
  if (e == hipSuccess) e = hipMemcpy(c->d_map32, m32.data(), m32.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) return done(fail(c, MG_EHIP, std::string("coarse map: ") + hipGetErrorString(e)));
  for (double v : m64)
    if (!std::isfinite(v)) return done(fail(c, MG_EHIP, "coarse map: non-finite entry"));
  return done(MG_OK);
}

// The dense map B of the tail's top level T = kDenseMapLevel: from x_T = 0 the
// tail computes x_T = B f_T (every step is linear in f_T), so column i is the
// tail applied to the unit vector e_i.  All columns come from one batched tail
// launch; B is stored row-major (one row per wave in the product) in FP64 and
// as an FP32 copy for the FP32 cycles.
int build_dense_map(mg_ctx* c) {
  const int T = c->tail_T;
  const int N = 2 * ((1 << T) + 1) * ((1 << T) + 1);
  if (N > mgk::kDenseMapMaxN) return MG_OK;
  const size_t lds = mgk::tail_lds_bytes<double>(c->k0, T);
  double* d_id = nullptr;
  double* d_cols = nullptr;
  void* d_args = nullptr;
  auto done = [&](int st) {
    (void)hipFree(d_id);
    (void)hipFree(d_cols);
    (void)hipFree(d_args);
    return st;
  };
  const size_t nn = (size_t)N * N;
  if (hipMalloc(&d_id, nn * sizeof(double)) != hipSuccess || hipMalloc(&d_cols, nn * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->d_dmap64, nn * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->d_dmap32, nn * sizeof(float)) != hipSuccess)
    return done(fail(c, MG_ENOMEM, "dense map: device allocation failed"));
  std::vector<double> h(nn, 0.0);
  for (int i = 0; i < N; i++) h[(size_t)i * N + i] = 1.0;
  const size_t sz = mgk::tail_args_bytes<double>();
  std::vector<unsigned char> args((size_t)N * sz);
  for (int i = 0; i < N; i++)
    mgk::make_tail_args<double>(c->tail, d_id + (size_t)i * N, d_cols + (size_t)i * N, 1, nullptr, args.data() + i * sz);
  if (hipMalloc(&d_args, args.size()) != hipSuccess) return done(fail(c, MG_ENOMEM, "dense map: device allocation failed"));
  hipError_t e = hipMemcpy(d_id, h.data(), nn * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_args, args.data(), args.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = mgk::launch_b_tail<double>(d_args, N, lds, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  std::vector<double> cols(nn);
  if (e == hipSuccess) e = hipMemcpy(cols.data(), d_cols, nn * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return done(fail(c, MG_EHIP, std::string("dense map: ") + hipGetErrorString(e)));
  // column i (contiguous in cols) becomes column i of the row-major matrix
  std::vector<float> h32(nn);
  for (int i = 0; i < N; i++)
    for (int r = 0; r < N; r++) {
      const double v = cols[(size_t)i * N + r];
      if (!std::isfinite(v)) return done(fail(c, MG_EHIP, "dense map: non-finite entry"));
      h[(size_t)r * N + i] = v;
      h32[(size_t)r * N + i] = (float)v;
    }
  e = hipMemcpy(c->d_dmap64, h.data(), nn * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_dmap32, h32.data(), nn * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) return done(fail(c, MG_EHIP, std::string("dense map: ") + hipGetErrorString(e)));
  c->dmap_n = N;
  return done(MG_OK);
}

// (Re)build the tail for the context's options; tail level min(5, level - 1).
// k0 <= 2: the tail solves the coarsest system with one lane per unknown
// (2 (2^k0 + 1)^2 <= 64).
int setup_tail(mg_ctx* c) {
  (void)hipFree(c->d_tail_ops);
  (void)hipFree(c->d_map64);
  (void)hipFree(c->d_map32);
  c->d_tail_ops = nullptr;
  c->d_map64 = nullptr;
  c->d_map32 = nullptr;
  (void)hipFree(c->d_dmap64);
  (void)hipFree(c->d_dmap32);
  c->d_dmap64 = nullptr;
  c->d_dmap32 = nullptr;
  c->dmap_n = 0;
  c->tail_T = 0;
  const int T = c->level - 1 < 5 ? c->level - 1 : 5;
  if (!c->tail_allowed || T <= c->k0 || c->k0 > 2 || c->problem != MG_POISSON) return MG_OK;
  mgk::TailLaunch& t = c->tail;
  t = mgk::TailLaunch{};
  t.k0 = c->k0;
  t.T = T;
  static const int map[4] = {mgk::MG_TAIL_NE, mgk::MG_TAIL_LSGS, mgk::MG_TAIL_SLSGS, mgk::MG_TAIL_CGS};
  if (c->o.smoother < MG_NE || c->o.smoother > MG_CGS)
    return fail(c, MG_EUNSUPPORTED, "coarse tail: smoother not provided for Poisson control");
  t.smoother = map[c->o.smoother];
  t.tau = c->o.tau;
  t.lu = c->d_lu;
  t.piv = c->d_piv;
  t.ncoarse = c->ncoarse;
  for (int l = c->k0; l <= T; l++) t.lev[l] = L_(c, l).lev;
  const size_t need = mgk::tail_lds_bytes<double>(c->k0, T);
  int dev = 0, maxlds = 0;
  HIPCHK(c, hipGetDevice(&dev));
  HIPCHK(c, hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  t.max_lds = (size_t)maxlds;
  if (need > t.max_lds) return MG_OK;  // does not fit: no tail
  HIPCHK(c, mgk::tail_allow_lds(need));
  // the coarse map replaces the sub-cycle on level kTailMapLevel when the
  // tail reaches above it
  int map_level = 0;
  if (c->map_allowed && T > mgk::kTailMapLevel && c->k0 < mgk::kTailMapLevel) {
    int st = build_coarse_map(c, t, mgk::tail_lds_bytes<double>(c->k0, mgk::kTailMapLevel));
    if (st != MG_OK) return st;
    map_level = mgk::kTailMapLevel;
    t.map64 = c->d_map64;
    t.map32 = c->d_map32;
    t.nmap = 2 * ((1 << map_level) + 1) * ((1 << map_level) + 1);
  }
  std::vector<int4> ops;
  tail_ops(c, T, ops, map_level);
  HIPCHK(c, hipMalloc(&c->d_tail_ops, ops.size() * sizeof(int4)));
  HIPCHK(c, hipMemcpy(c->d_tail_ops, ops.data(), ops.size() * sizeof(int4), hipMemcpyHostToDevice));
  t.nops = (int)ops.size();
  t.ops = c->d_tail_ops;
  c->tail_T = T;
  if (c->dmap_allowed && T == mgk::kDenseMapLevel) return build_dense_map(c);
  return MG_OK;
}

// set while mg_batch_setup creates its instances: batched cycles launch the
// tail for all instances at once and never use a dense map
thread_local bool t_batch_instance = false;

const double* dmap(const mg_ctx* c, double*) { return c->d_dmap64; }
const float* dmap(const mg_ctx* c, float*) { return c->d_dmap32; }

// One iterate on level l for A_l x = f; r is level-l workspace (one of the
// level's two residual buffers).  If residual_current, r already holds f - A_l x.
template <typename T>
int cycle_body(mg_ctx* c, int l, const T* f, T* x, T* r, bool residual_current, hipStream_t s,
               const SweepNorm& sn = SweepNorm{}, bool x_zero = false) {
  if (l == c->k0) return coarse_solve_T<T>(c, f, x, s);
  LevelBuf& b = L_(c, l);
  LevelBuf& bc = L_(c, l - 1);
  Work<T> wb = work(b, (T*)nullptr);
  Work<T> wc = work(bc, (T*)nullptr);
  T* alt = (r == wb.r) ? wb.r2 : wb.r;
  int st;
  if (!residual_current) HIPCHK(c, mgk::launch_residual<T>(b.lev, f, x, r, nullptr, 0, nullptr, s));
  // defect restriction; the coarse iterate starts from zero with r_c = f_c
  const bool coarse_is_k0 = (l - 1 == c->k0);
  const bool tail = (l - 1 == c->tail_T);
  T* xc0 = (coarse_is_k0 || tail) ? nullptr : wc.x;
  T* rc = (coarse_is_k0 || tail) ? nullptr : wc.r;
  // With tile-sweep smoothers on both sides the restriction runs in the last
  // pre-smoothing launch, which writes the smoothed iterate to the level's
  // scratch p; the post-smoothing then starts from p (x + P x_c and its
  // residual formed by the first sweep launch, or by the separate kernel
  // reading p and writing x).
  // Timed solves (mg_timing_enable) keep the transfers apart, so that every
  // timed finest-level step is a plain smoothing step.
  const bool tile_smoother =
      c->fused && (c->o.smoother == MG_LSGS || c->o.smoother == MG_SLSGS || c->o.smoother == MG_CGS);
  const bool xfer = tile_smoother && c->xfer_allowed && !c->timing && c->o.nu1 > 0 && c->o.nu2 > 0;
  if (xfer) {
    mgk::SweepIO<T> rio;
    rio.fc = wc.f;
    rio.xc0 = xc0;
    rio.rc = rc;
    rio.Lc = bc.lev;
    SweepXfer<T> xf;
    xf.last = &rio;
    xf.last_x = wb.p;
    xf.first_xzero = x_zero;
    if ((st = smooth_steps<T>(c, l, x, r, alt, wb.p, c->o.nu1, s, nullptr, SweepNorm{}, xf)) != MG_OK) return st;
  } else {
    SweepXfer<T> xf;
    xf.first_xzero = x_zero;
    if ((st = smooth_steps<T>(c, l, x, r, alt, wb.p, c->o.nu1, s, nullptr, SweepNorm{}, xf)) != MG_OK) return st;
    HIPCHK(c, mgk::launch_restrict<T>(b.lev, bc.lev, r, wc.f, xc0, rc, s));
  }
  alt = (r == wb.r) ? wb.r2 : wb.r;
  for (int g = 0; g < c->o.gamma; g++) {
    if (tail && c->dmap_n) {
      // x_c = B f_c from zero; a further iterate x_c += B (f_c - A x_c)
      if (g == 0) {
        HIPCHK(c, mgk::launch_dense_map<T>(dmap(c, (T*)nullptr), c->dmap_n, wc.f, wc.x, 0, s));
      } else {
        HIPCHK(c, mgk::launch_residual<T>(bc.lev, wc.f, wc.x, wc.r, nullptr, 0, nullptr, s));
        HIPCHK(c, mgk::launch_dense_map<T>(dmap(c, (T*)nullptr), c->dmap_n, wc.r, wc.x, 1, s));
      }
    } else if (tail)
      HIPCHK(c, mgk::launch_tail<T>(c->tail, wc.f, wc.x, g == 0 ? 1 : 0, s));
    else if ((st = cycle_body<T>(c, l - 1, wc.f, wc.x, wc.r, g == 0, s)) != MG_OK)
      return st;
  }
  // the prolongation with the residual pays inside the first post-smoothing
  // launch only on the levels swept one sweep per launch (above 513^2): it
  // reads the iterate and f on the whole tile region, where the separate
  // kernel reads each vertex once; on the two-sweep levels the launch of its
  // own is cheaper
  if (xfer && b.lev.n > mgk::lsgs_sweep2_max_n()) {
    mgk::SweepIO<T> pio;
    pio.xc = wc.x;
    pio.f = f;
    pio.Lc = bc.lev;
    SweepXfer<T> xf;
    xf.first = &pio;
    return smooth_steps<T>(c, l, x, r, alt, wb.p, c->o.nu2, s, wb.p, sn, xf);
  }
  // x += P x_c and r = f - A x.  Before a tile-sweep post-smoother both go in
  // one kernel that writes the corrected iterate to the level's scratch p
  // (unused by LSGS); the first sweep reads it from there and writes x.
  const bool fuse = tile_smoother && c->o.nu2 > 0;
  if (fuse && xfer) {
    // the pre-smoothed iterate is in p
    HIPCHK(c, mgk::launch_prolong_residual<T>(b.lev, bc.lev, wc.x, wb.p, f, x, r, s));
    return smooth_steps<T>(c, l, x, r, alt, wb.p, c->o.nu2, s, nullptr, sn);
  }
  if (fuse) {
    HIPCHK(c, mgk::launch_prolong_residual<T>(b.lev, bc.lev, wc.x, x, f, wb.p, r, s));
    return smooth_steps<T>(c, l, x, r, alt, wb.p, c->o.nu2, s, wb.p, sn);
  }
  HIPCHK(c, mgk::launch_prolong_add<T>(b.lev, bc.lev, wc.x, x, s));
  HIPCHK(c, mgk::launch_residual<T>(b.lev, f, x, r, nullptr, 0, nullptr, s));
  return smooth_steps<T>(c, l, x, r, alt, wb.p, c->o.nu2, s);
}

int norm_mode(const mg_ctx* c) { return c->o.norm == MG_NORM_LINV ? 2 : 1; }

// Stopping rule of the solve loop, applied after every iterate (it = number
// of iterates so far) to ||r||^2 and ||f||^2: returns kContinue or the final
// status with a message.
constexpr int kContinue = 1;
struct Monitor {
  double nf = -1.0, rel0 = -1.0, rel = 0.0;
  std::vector<double> hist;
  int check(double r2, double f2, double tol, int it, int max_cycles, const char** why) {
    if (nf < 0.0) nf = std::sqrt(f2) > 0.0 ? std::sqrt(f2) : 1.0;
    rel = std::sqrt(r2) / nf;
    if (rel0 < 0.0) rel0 = rel;
    if (!std::isfinite(rel)) return *why = "non-finite residual norm", MG_ENAN;
    if (rel <= tol) return MG_OK;
    if (rel > 1e3 * rel0 && rel0 > 0.0) return *why = "residual grew above 1e3 x initial", MG_EDIVERGE;
    hist.push_back(rel);
    if (it + 1 >= 2 * kStallWindow) {
      double best_new = hist[it], best_old = hist[it - kStallWindow];
      for (int k = 1; k < kStallWindow; k++) {
        best_new = std::fmin(best_new, hist[it - k]);
        best_old = std::fmin(best_old, hist[it - kStallWindow - k]);
      }
      if (best_new > 0.5 * best_old)
        return *why = "residual stagnated: no factor 2 gained over the last 10 iterates", MG_ESTALL;
    }
    if (it >= max_cycles) return *why = "max_cycles reached", MG_ENOTCONV;
    return kContinue;
  }
};

// ||r||^2 of the fine residual into d_norm[slot] (stream-ordered)
int residual_norm(mg_ctx* c, const double* f, const double* x, double* r, int slot, hipStream_t s) {
  int nb = 0;
  if (c->st)
    HIPCHK(c, mgk::stokes_residual(c->st, c->level, f, x, r, c->d_part, norm_mode(c), &nb, s));
  else
    HIPCHK(c, mgk::launch_residual<double>(L_(c, c->level).lev, f, x, r, c->d_part, norm_mode(c), &nb, s));
  HIPCHK(c, mgk::launch_sum(c->d_part, nb, c->d_norm + slot, s));
  return MG_OK;
}

// one refinement step: FP32 cycles from zero on the scaled FP64 residual held
// in the fine r buffer (with ||r||^2 in d_norm[0]), then x += s c in FP64
int ir_step(mg_ctx* c, double* x, hipStream_t s) {
  LevelBuf& b = L_(c, c->level);
  HIPCHK(c, mgk::launch_to_f32_scaled(b.r, b.len, c->d_norm, b.f32, b.r32, s));
  HIPCHK(c, mgk::launch_zero_f32(b.x32, b.len, s));
  int st;
  for (int k = 0; k < c->o.inner_cycles; k++)
    if ((st = cycle_body<float>(c, c->level, b.f32, b.x32, b.r32, k == 0, s)) != MG_OK) return st;
  HIPCHK(c, mgk::launch_axpy_f32(b.x32, b.len, c->d_norm, x, s));
  return MG_OK;
}

// Poisson solves with FP32 refinement keep the fine residual only as the
// right-hand side of the next step's FP32 cycles, r / ||f|| in FP32 (its
// squared norm from the same pass into d_norm[0]; ||f||^2 in d_norm[1]), and
// the step's update is x += ||f|| c.  Any fixed scale keeps the FP32 values
// in range, and the FP32 arithmetic is relative to them.
bool ir_fused(const mg_ctx* c) { return !c->st && c->o.precision == MG_FP32_IR; }

int residual_norm_f32(mg_ctx* c, const double* f, const double* x, hipStream_t s) {
  LevelBuf& b = L_(c, c->level);
  int nb = 0;
  HIPCHK(c, mgk::launch_residual_f32(b.lev, f, x, c->d_norm + 1, b.f32, b.r32, c->d_part, norm_mode(c), &nb, s));
  HIPCHK(c, mgk::launch_sum(c->d_part, nb, c->d_norm, s));
  return MG_OK;
}

// the refinement step of a solve: FP32 cycles from zero on the right-hand
// side left by residual_norm_f32, then x += ||f|| c.  With a tile-sweep
// pre-smoother the first launch takes the zero iterate as zero (and writes
// every vertex of x32), so x32 is not cleared.
int ir_step_solve(mg_ctx* c, double* x, hipStream_t s) {
  LevelBuf& b = L_(c, c->level);
  const bool xz = c->fused && c->o.nu1 > 0 &&
                  (c->o.smoother == MG_LSGS || c->o.smoother == MG_SLSGS || c->o.smoother == MG_CGS);
  if (!xz) HIPCHK(c, mgk::launch_zero_f32(b.x32, b.len, s));
  int st;
  for (int k = 0; k < c->o.inner_cycles; k++)
    if ((st = cycle_body<float>(c, c->level, b.f32, b.x32, b.r32, k == 0, s, SweepNorm{}, xz && k == 0)) != MG_OK)
      return st;
  HIPCHK(c, mgk::launch_axpy_f32(b.x32, b.len, c->d_norm + 1, x, s));
  return MG_OK;
}

// one solver iterate for fixed (f, x): cycle (FP64) or refinement step
// (FP32 cycles), then the fine residual and its squared norm in d_norm[0]
// the residual buffer of the finest level
double* fine_r(mg_ctx* c) { return c->st ? mgk::stokes_fine_r(c->st) : L_(c, c->level).r; }

// FP64 Poisson iterates whose last post-smoothing step is a tile sweep that
// leaves the residual in the finest level's first buffer (an even number of
// LSGS or collective-smoother sweeps per cycle, or sLSGS) take the residual
// norm from that sweep.
bool sweep_norm(const mg_ctx* c) {
  if (c->st || !c->sweep_norm_allowed || c->o.precision != MG_FP64 || !c->fused || c->o.nu2 < 1 || c->timing)
    return false;
  if (c->o.smoother == MG_SLSGS) return true;
  return (c->o.smoother == MG_LSGS || c->o.smoother == MG_CGS) && (c->o.nu1 + c->o.nu2) % 2 == 0;
}

int iterate(mg_ctx* c, const double* f, double* x, hipStream_t s) {
  if (c->st) {
    if (c->o.precision == MG_FP32_IR)
      HIPCHK(c, mgk::stokes_ir_step(c->st, x, s, c->d_norm, c->o.inner_cycles));
    else
      HIPCHK(c, mgk::stokes_cycle(c->st, f, x, fine_r(c), true, s));
    return residual_norm(c, f, x, fine_r(c), 0, s);
  }
  LevelBuf& b = L_(c, c->level);
  if (ir_fused(c)) {
    const int st = ir_step_solve(c, x, s);
    return st != MG_OK ? st : residual_norm_f32(c, f, x, s);
  }
  if (sweep_norm(c)) {
    // the last post-smoothing sweep leaves r = f - A x (maintained by the
    // smoother) in b.r and sums its squared norm: no separate residual pass
    int nb = 0;
    SweepNorm sn;
    sn.part = c->d_part;
    sn.mode = norm_mode(c);
    sn.nb = &nb;
    int st = cycle_body<double>(c, c->level, f, x, b.r, true, s, sn);
    if (st != MG_OK) return st;
    HIPCHK(c, mgk::launch_sum(c->d_part, nb, c->d_norm, s));
    return MG_OK;
  }
  int st = c->o.precision == MG_FP32_IR ? ir_step(c, x, s) : cycle_body<double>(c, c->level, f, x, b.r, true, s);
  if (st != MG_OK) return st;
  return residual_norm(c, f, x, b.r, 0, s);
}

void drop_graph(mg_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  c->gexec = nullptr;
  c->g_f = nullptr;
  c->g_x = nullptr;
}

// records body(stream) on the context's capture stream (no execution) and
// instantiates the graph into *out
template <class Body>
int capture_graph(mg_ctx* c, Body&& body, hipGraphExec_t* out) {
  *out = nullptr;
  if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  c->capturing = true;
  int st = body(c->cap_stream);
  c->capturing = false;
  hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
  if (st != MG_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(c, MG_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    *out = nullptr;
    return fail(c, e == hipErrorOutOfMemory ? MG_ENOMEM : MG_EHIP,
                std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  return MG_OK;
}

// graph of iterate() for (f, x) and the current options / timing state
int ensure_graph(mg_ctx* c, const double* f, double* x) {
  if (c->gexec && c->g_f == f && c->g_x == x) return MG_OK;
  drop_graph(c);
  int st = capture_graph(c, [&](hipStream_t cs) { return iterate(c, f, x, cs); }, &c->gexec);
  if (st != MG_OK) return st;
  c->g_f = f;
  c->g_x = x;
  return MG_OK;
}

int check_level(const mg_ctx* c, int l, bool allow_coarsest) {
  if (l > c->level || l < c->k0) return 0;
  if (!allow_coarsest && l == c->k0) return 0;
  return 1;
}

}  // namespace

namespace {
// Stokes contexts: the CSR solver object plus the norm workspace of the context
int setup_stokes(mg_ctx* c, mg_ctx** out) {
  const char* g = std::getenv("MGKKT_NO_GRAPH");
  c->graphs = !(g && g[0] == '1');
  c->tail_allowed = false;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return MG_EHIP;
  }
  if (scratch_init(c->device) != hipSuccess) {
    delete c;
    return MG_EHIP;
  }
  int st = mgk::stokes_create(c->level, c->k0, c->alpha, c->o, &c->st, &c->err);
  if (st != MG_OK) {
    destroy_impl(c);
    return st;
  }
  c->npart = mgk::stokes_partials(c->st);
  if (hipMalloc(&c->d_part, c->npart * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->d_norm, 4 * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void**)&c->h_norm, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    destroy_impl(c);
    return MG_ENOMEM;
  }
  *out = c;
  return MG_OK;
}
}  // namespace

// ====================================================================== C ABI

extern "C" {

mg_opts mg_default_opts(int problem) {
  mg_opts o;
  o.smoother = MG_LSGS;
  o.nu1 = 2;
  o.nu2 = 2;
  o.gamma = 1;
  o.tau = -1.0;  // resolved at setup: 0.4 (Poisson NE, patch smoother) or 0.35 (Stokes NE)
  o.coarse_level = 1;
  o.precision = MG_FP64;
  o.max_cycles = 200;
  o.inner_cycles = 1;
  o.norm = MG_NORM_LINV;
  return o;
}

const char* mg_strerror(int status) {
  if (status > 0 || status < MG_ESTALL) return "unknown status";
  return kStatusText[-status];
}

const char* mg_last_error(const mg_ctx* ctx) {
  if (!ctx) return "no context";
  return ctx->err.c_str();
}

size_t mg_vec_len(const mg_ctx* ctx) {
  if (!ctx) return 0;
  return ctx->st ? mgk::stokes_len(ctx->st, ctx->level) : ctx->lv.back().len;
}

size_t mg_level_len(const mg_ctx* ctx, int level) {
  if (!ctx || level < ctx->k0 || level > ctx->level) return 0;
  if (ctx->st) return mgk::stokes_len(ctx->st, level);
  return ctx->lv[level - ctx->k0].len;
}

static int impl_mg_get_opts(const mg_ctx* ctx, mg_opts* out) {
  if (!ctx || !out) return MG_EINVAL;
  *out = ctx->o;
  return MG_OK;
}

static int setup_body(mg_ctx* c, int level, double alpha, int problem, const mg_opts* opts, mg_ctx** out);

static int impl_mg_setup(int level, double alpha, int problem, const mg_opts* opts, mg_ctx** out) {
  if (!out) return MG_EINVAL;
  *out = nullptr;
  if (problem != MG_POISSON && problem != MG_STOKES) return MG_EINVAL;
  if (!(alpha > 0.0) || !std::isfinite(alpha)) return MG_EINVAL;
  if (level < 2 || level > kMaxLevel) return MG_EINVAL;
  if (!valid_opts(opts, level)) return MG_EINVAL;
  if (unsupported_pair(problem, opts ? *opts : mg_default_opts(problem))) return MG_EUNSUPPORTED;
  if (problem == MG_STOKES && level > kMaxStokesLevel) return MG_EUNSUPPORTED;
  mg_ctx* c = new (std::nothrow) mg_ctx();
  if (!c) return MG_ENOMEM;
  try {
    return setup_body(c, level, alpha, problem, opts, out);
  } catch (...) {
    // every path that releases c returns at once, so c is still alive here
    destroy_impl(c);
    throw;
  }
}

static int setup_body(mg_ctx* c, int level, double alpha, int problem, const mg_opts* opts, mg_ctx** out) {
  c->problem = problem;
  c->level = level;
  c->alpha = alpha;
  c->o = opts ? *opts : mg_default_opts(problem);
  if (c->o.tau <= 0.0) c->o.tau = default_tau(problem, c->o.smoother);
  c->k0 = c->o.coarse_level;
  if (problem == MG_STOKES) return setup_stokes(c, out);
  {
    // MGKKT_PHASE_KERNELS=1 selects one launch per colour phase (comparison and testing)
    const char* e = std::getenv("MGKKT_PHASE_KERNELS");
    c->fused = !(e && e[0] == '1');
    // MGKKT_NO_SWEEP2=1 runs one sweep per launch on every level
    const char* e2 = std::getenv("MGKKT_NO_SWEEP2");
    c->sweep2 = !(e2 && e2[0] == '1');
    // MGKKT_NO_FUSED_TRANSFERS=1 launches the restriction and the
    // prolongation with the residual as kernels of their own
    const char* e3 = std::getenv("MGKKT_NO_FUSED_TRANSFERS");
    c->xfer_allowed = !(e3 && e3[0] == '1');
    // MGKKT_NO_TAIL=1 runs the coarse levels with the per-level kernels
    const char* t = std::getenv("MGKKT_NO_TAIL");
    c->tail_allowed = !(t && t[0] == '1');
    // MGKKT_NO_MAP=1 runs the tail's sub-cycle on every level instead of the coarse map
    const char* m = std::getenv("MGKKT_NO_MAP");
    c->map_allowed = !(m && m[0] == '1');
    // MGKKT_NO_DENSE_MAP=1 launches the tail instead of the dense map of its top level
    const char* dm = std::getenv("MGKKT_NO_DENSE_MAP");
    c->dmap_allowed = !(dm && dm[0] == '1') && !t_batch_instance;
    // MGKKT_NO_SWEEP_NORM=1 recomputes f - A x for the norm after every iterate
    const char* q = std::getenv("MGKKT_NO_SWEEP_NORM");
    c->sweep_norm_allowed = !(q && q[0] == '1');
    // MGKKT_NO_GRAPH=1 makes mg_solve launch every kernel eagerly
    const char* g = std::getenv("MGKKT_NO_GRAPH");
    c->graphs = !(g && g[0] == '1');
  }
  int st = MG_OK;
  auto bail = [&](int s) {
    destroy_impl(c);
    return s;
  };
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return MG_EHIP;
  }
  if (scratch_init(c->device) != hipSuccess) {
    delete c;
    return MG_EHIP;
  }
  c->lv.resize(level - c->k0 + 1);
  size_t max_blocks = 1;
  for (int l = c->k0; l <= level; l++) {
    LevelBuf& b = L_(c, l);
    b.level = l;
    // level 1 can only be the coarsest level, which is solved by the dense LU:
    // its stencil tables are never read, those of level 2 stand in
    LevelTables t = make_tables(l < 2 ? 2 : l, alpha, c->o.tau);
    b.lev = t.lev;
    const int n = 1 << l;
    b.lev.n = n;
    b.lev.ld = n + 1;
    b.lev.V = (n + 1) * (n + 1);
    b.len = 2 * (size_t)b.lev.V;
    if (hipMalloc(&b.d_tab, sizeof(Tab)) != hipSuccess) return bail(MG_ENOMEM);
    if (hipMemcpy(b.d_tab, &t.tab, sizeof(Tab), hipMemcpyHostToDevice) != hipSuccess) return bail(MG_EHIP);
    b.lev.tab = b.d_tab;
    const size_t bytes = b.len * sizeof(double);
    if (l < level) {
      if (hipMalloc(&b.x, bytes) != hipSuccess || hipMalloc(&b.f, bytes) != hipSuccess) return bail(MG_ENOMEM);
    }
    if (l > c->k0) {
      if (hipMalloc(&b.r, bytes) != hipSuccess || hipMalloc(&b.r2, bytes) != hipSuccess ||
          hipMalloc(&b.p, bytes) != hipSuccess)
        return bail(MG_ENOMEM);
    }
    const size_t nb = (size_t)((n + 1 + 63) / 64) * (size_t)((n + 1 + 3) / 4);
    if (nb > max_blocks) max_blocks = nb;
  }
  // coarsest level: FP64 LU with partial pivoting of A_{k0}
  {
    std::vector<double> A = dense_kkt(c->k0, alpha);
    std::vector<int> piv;
    const int N = 2 * ((1 << c->k0) + 1) * ((1 << c->k0) + 1);
    if (!lu_factor(N, A, piv)) return bail(fail(c, MG_EINVAL, "singular coarsest matrix"));
    c->ncoarse = N;
    // d_piv holds the row interchanges (N entries) followed by the permutation
    // they compose to: entry i of the permuted right-hand side is b[perm[i]]
    piv.resize(2 * N);
    for (int i = 0; i < N; i++) piv[N + i] = i;
    for (int k = 0; k < N; k++) std::swap(piv[N + k], piv[N + piv[k]]);
    if (hipMalloc(&c->d_lu, A.size() * sizeof(double)) != hipSuccess) return bail(MG_ENOMEM);
    if (hipMalloc(&c->d_piv, piv.size() * sizeof(int)) != hipSuccess) return bail(MG_ENOMEM);
    if (hipMemcpy(c->d_lu, A.data(), A.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_piv, piv.data(), piv.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
      return bail(MG_EHIP);
  }
  if (max_blocks < 1024) max_blocks = 1024;
  c->npart = max_blocks;
  if (hipMalloc(&c->d_part, max_blocks * sizeof(double)) != hipSuccess) return bail(MG_ENOMEM);
  if (hipMalloc(&c->d_norm, 4 * sizeof(double)) != hipSuccess) return bail(MG_ENOMEM);
  if (hipHostMalloc((void**)&c->h_norm, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return bail(MG_ENOMEM);
  if (c->o.precision == MG_FP32_IR && (st = alloc_fp32(c)) != MG_OK) return bail(st);
  if ((st = setup_tail(c)) != MG_OK) return bail(st);
  *out = c;
  return MG_OK;
}

void mg_destroy(mg_ctx* ctx) { destroy_impl(ctx); }

static int impl_mg_set_opts(mg_ctx* ctx, const mg_opts* opts) {
  if (!ctx || !opts) return MG_EINVAL;
  if (!valid_opts(opts, ctx->level)) return MG_EINVAL;
  if (opts->coarse_level != ctx->k0) return fail(ctx, MG_EINVAL, "coarse_level is fixed at setup");
  if (unsupported_pair(ctx->problem, *opts))
    return fail(ctx, MG_EUNSUPPORTED, "mg_set_opts: smoother not provided for this problem");
  mg_opts o = *opts;
  if (o.tau <= 0.0) o.tau = default_tau(ctx->problem, o.smoother);
  if (ctx->st) {
    if (o.smoother != ctx->o.smoother || o.precision != ctx->o.precision)
      return fail(ctx, MG_EUNSUPPORTED, "Stokes: smoother and precision are fixed at setup");
    ctx->o = o;
    mgk::stokes_set(ctx->st, o);
    drop_graph(ctx);
    ctx->opts_gen++;
    return MG_OK;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return MG_EHIP;
  if (o.precision == MG_FP32_IR) {
    int st = alloc_fp32(ctx);
    if (st != MG_OK) return st;
  }
  ctx->o = o;
  for (auto& b : ctx->lv) b.lev.tau = o.tau;
  drop_graph(ctx);
  ctx->opts_gen++;
  return setup_tail(ctx);
}

static int impl_mg_rhs(mg_ctx* ctx, const double* yd, double* f, void* stream) {
  if (!ctx || !yd || !f) return MG_EINVAL;
  if (ctx->st) {
    HIPCHK(ctx, mgk::stokes_rhs(ctx->st, yd, f, (hipStream_t)stream));
    return MG_OK;
  }
  HIPCHK(ctx, mgk::launch_rhs<double>(L_(ctx, ctx->level).lev, yd, f, (hipStream_t)stream));
  return MG_OK;
}

static int impl_mg_control(mg_ctx* ctx, const double* x, double* u, void* stream) {
  if (!ctx || !x || !u) return MG_EINVAL;
  if (ctx->problem != MG_POISSON) return fail(ctx, MG_EUNSUPPORTED, "mg_control: Poisson control only");
  HIPCHK(ctx, mgk::launch_control(L_(ctx, ctx->level).lev, x, u, (hipStream_t)stream));
  return MG_OK;
}

static int impl_mg_adjoint_grad(mg_ctx* ctx, const double* x, const double* xadj, double* grad_yd, double* grad_alpha,
                    void* stream) {
  if (!ctx || !x || !xadj || !grad_yd || !grad_alpha) return MG_EINVAL;
  if (ctx->problem != MG_POISSON) return fail(ctx, MG_EUNSUPPORTED, "mg_adjoint_grad: Poisson control only");
  hipStream_t s = (hipStream_t)stream;
  const LevelBuf& b = L_(ctx, ctx->level);
  int nb = 0;
  HIPCHK(ctx, mgk::launch_adjoint_grad(b.lev, x, xadj, grad_yd, ctx->d_part, &nb, s));
  HIPCHK(ctx, mgk::launch_sum(ctx->d_part, nb, grad_alpha, s, -1.0 / (ctx->alpha * ctx->alpha)));
  return MG_OK;
}

static int impl_mg_apply(mg_ctx* ctx, int level, const double* x, double* y, void* stream) {
  if (!ctx || !x || !y || !check_level(ctx, level, false)) return MG_EINVAL;
  if (ctx->st) {
    HIPCHK(ctx, mgk::stokes_apply(ctx->st, level, x, y, (hipStream_t)stream));
    return MG_OK;
  }
  HIPCHK(ctx, mgk::launch_apply<double>(L_(ctx, level).lev, x, y, (hipStream_t)stream));
  return MG_OK;
}

static int impl_mg_residual(mg_ctx* ctx, int level, const double* f, const double* x, double* r, double* norm_out,
                void* stream) {
  if (!ctx || !f || !x || !r || !check_level(ctx, level, false)) return MG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int nb = 0;
  if (ctx->st) {
    HIPCHK(ctx, mgk::stokes_residual(ctx->st, level, f, x, r, norm_out ? ctx->d_part : nullptr, 1, &nb, s));
    if (!norm_out) return MG_OK;
  } else {
    LevelBuf& b = L_(ctx, level);
    if (!norm_out) {
      HIPCHK(ctx, mgk::launch_residual<double>(b.lev, f, x, r, nullptr, 0, nullptr, s));
      return MG_OK;
    }
    HIPCHK(ctx, mgk::launch_residual<double>(b.lev, f, x, r, ctx->d_part, 1, &nb, s));
  }
  HIPCHK(ctx, mgk::launch_sum(ctx->d_part, nb, ctx->d_norm + 2, s));
  HIPCHK(ctx, hipMemcpyAsync(ctx->h_norm + 2, ctx->d_norm + 2, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  *norm_out = std::sqrt(ctx->h_norm[2]);
  return MG_OK;
}

// mg_residual's arithmetic with the norm partials in the static scratch and
// the norm left on the device: no allocation and no synchronisation
static int impl_mg_residual_nalloc(mg_ctx* ctx, int level, const double* f, const double* x, double* r,
                                   double* norm_dev, void* stream) {
  if (!ctx || !f || !x || !r || !norm_dev || !check_level(ctx, level, false)) return MG_EINVAL;
  const int nb = ctx->st ? mgk::stokes_residual_parts(ctx->st, level) : mgk::residual_blocks(1 << level);
  if (nb < 1 || nb > kScratchWords) {
    ctx->err = "mg_residual_nalloc: level " + std::to_string(level) + " needs " + std::to_string(nb) +
               " partial sums, the static scratch holds " + std::to_string(kScratchWords);
    return MG_EUNSUPPORTED;
  }
  double* part = scratch_ptr(ctx->device);
  if (!part) {
    ctx->err = "mg_residual_nalloc: no scratch address for device " + std::to_string(ctx->device);
    return MG_EHIP;
  }
  hipStream_t s = (hipStream_t)stream;
  int wrote = 0;
  if (ctx->st)
    HIPCHK(ctx, mgk::stokes_residual(ctx->st, level, f, x, r, part, 1, &wrote, s));
  else
    HIPCHK(ctx, mgk::launch_residual<double>(L_(ctx, level).lev, f, x, r, part, 1, &wrote, s));
  if (wrote != nb) {
    ctx->err = "mg_residual_nalloc: partial count mismatch";
    return MG_EHIP;
  }
  HIPCHK(ctx, mgk::launch_sum_sqrt(part, nb, norm_dev, s));
  return MG_OK;
}

static int impl_mg_smooth(mg_ctx* ctx, int level, double* x, double* r, int steps, void* stream) {
  if (!ctx || !x || !r || steps < 0 || !check_level(ctx, level, false)) return MG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (ctx->st) {
    HIPCHK(ctx, mgk::stokes_smooth(ctx->st, level, x, r, steps, s));
    return MG_OK;
  }
  LevelBuf& b = L_(ctx, level);
  double* cur = r;
  int st = smooth_steps<double>(ctx, level, x, cur, b.r2, b.p, steps, s);
  if (st != MG_OK) return st;
  if (cur != r) HIPCHK(ctx, hipMemcpyAsync(r, cur, b.len * sizeof(double), hipMemcpyDeviceToDevice, s));
  return MG_OK;
}

static int impl_mg_restrict(mg_ctx* ctx, int level, const double* r, double* fc, void* stream) {
  if (!ctx || !r || !fc || !check_level(ctx, level, false)) return MG_EINVAL;
  if (ctx->st) {
    HIPCHK(ctx, mgk::stokes_restrict(ctx->st, level, r, fc, (hipStream_t)stream));
    return MG_OK;
  }
  HIPCHK(ctx, mgk::launch_restrict<double>(L_(ctx, level).lev, L_(ctx, level - 1).lev, r, fc, nullptr, nullptr,
                                           (hipStream_t)stream));
  return MG_OK;
}

static int impl_mg_prolong_add(mg_ctx* ctx, int level, const double* xc, double* x, void* stream) {
  if (!ctx || !xc || !x || !check_level(ctx, level, false)) return MG_EINVAL;
  if (ctx->st) {
    HIPCHK(ctx, mgk::stokes_prolong_add(ctx->st, level, xc, x, (hipStream_t)stream));
    return MG_OK;
  }
  HIPCHK(ctx, mgk::launch_prolong_add<double>(L_(ctx, level).lev, L_(ctx, level - 1).lev, xc, x,
                                              (hipStream_t)stream));
  return MG_OK;
}

static int impl_mg_coarse_solve(mg_ctx* ctx, const double* f, double* x, void* stream) {
  if (!ctx || !f || !x) return MG_EINVAL;
  if (ctx->st) {
    HIPCHK(ctx, mgk::stokes_coarse_solve(ctx->st, f, x, (hipStream_t)stream));
    return MG_OK;
  }
  return coarse_solve_T<double>(ctx, f, x, (hipStream_t)stream);
}

static int impl_mg_cycle(mg_ctx* ctx, const double* f, double* x, void* stream) {
  if (!ctx || !f || !x) return MG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (ctx->st) {
    if (ctx->o.precision == MG_FP32_IR) {
      int st = residual_norm(ctx, f, x, fine_r(ctx), 0, s);
      if (st != MG_OK) return st;
      HIPCHK(ctx, mgk::stokes_ir_step(ctx->st, x, s, ctx->d_norm, ctx->o.inner_cycles));
      return MG_OK;
    }
    HIPCHK(ctx, mgk::stokes_cycle(ctx->st, f, x, fine_r(ctx), false, s));
    return MG_OK;
  }
  LevelBuf& b = L_(ctx, ctx->level);
  if (ctx->o.precision == MG_FP32_IR) {
    int st = residual_norm(ctx, f, x, b.r, 0, s);
    if (st != MG_OK) return st;
    return ir_step(ctx, x, s);
  }
  return cycle_body<double>(ctx, ctx->level, f, x, b.r, false, s);
}

static int impl_mg_capture_cycle(mg_ctx* ctx, const double* f, double* x, void* stream, mg_graph** out) {
  if (out) *out = nullptr;
  if (!ctx || !f || !x || !out) return MG_EINVAL;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  hipGraphExec_t exec = nullptr;
  int st = capture_graph(ctx, [&](hipStream_t cs) { return mg_cycle(ctx, f, x, cs); }, &exec);
  if (st != MG_OK) return st;
  hipError_t e = hipGraphUpload(exec, (hipStream_t)stream);
  if (e != hipSuccess) {
    (void)hipGraphExecDestroy(exec);
    return fail(ctx, MG_EHIP, std::string("hipGraphUpload: ") + hipGetErrorString(e));
  }
  *out = new mg_graph{exec, ctx, ctx->opts_gen};
  return MG_OK;
}

static int impl_mg_graph_launch(mg_graph* graph, void* stream) {
  if (!graph) return MG_EINVAL;
  mg_ctx* c = graph->ctx;
  if (graph->gen != c->opts_gen) return fail(c, MG_EINVAL, "mg_graph_launch: options changed since capture");
  HIPCHK(c, hipGraphLaunch(graph->exec, (hipStream_t)stream));
  return MG_OK;
}

void mg_graph_destroy(mg_graph* graph) {
  if (!graph) return;
  (void)hipGraphExecDestroy(graph->exec);
  delete graph;
}

static int impl_mg_solve(mg_ctx* ctx, const double* f, double* x, double tol, int* cycles_out, double* relres_out,
             void* stream) {
  if (!ctx || !f || !x || !(tol > 0.0) || !std::isfinite(tol)) return MG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int nb = 0;
  if (ctx->st)
    HIPCHK(ctx, mgk::stokes_vnorm(ctx->st, f, ctx->d_part, norm_mode(ctx), &nb, s));
  else
    HIPCHK(ctx, mgk::launch_vnorm(L_(ctx, ctx->level).lev, f, ctx->d_part, norm_mode(ctx), &nb, s));
  HIPCHK(ctx, mgk::launch_sum(ctx->d_part, nb, ctx->d_norm + 1, s));
  Monitor mon;
  int st = MG_OK;
  st = ir_fused(ctx) ? residual_norm_f32(ctx, f, x, s) : residual_norm(ctx, f, x, fine_r(ctx), 0, s);
  if (st != MG_OK) return st;
  for (int it = 0;; it++) {
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_norm, ctx->d_norm, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    const char* why = "";
    const int verdict = mon.check(ctx->h_norm[0], ctx->h_norm[1], tol, it, ctx->o.max_cycles, &why);
    if (cycles_out) *cycles_out = it;
    if (relres_out) *relres_out = mon.rel;
    if (verdict == MG_OK && it > 0 && sweep_norm(ctx)) {
      // the norm came from the residual the smoother maintains: confirm with
      // the recomputed residual f - A x (which then replaces it)
      if ((st = residual_norm(ctx, f, x, fine_r(ctx), 0, s)) != MG_OK) return st;
      HIPCHK(ctx, hipMemcpyAsync(ctx->h_norm, ctx->d_norm, sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(ctx, hipStreamSynchronize(s));
      const double rel = std::sqrt(ctx->h_norm[0]) / mon.nf;
      if (relres_out) *relres_out = rel;
      if (rel <= tol) return MG_OK;
      if (!std::isfinite(rel)) return fail(ctx, MG_ENAN, "non-finite residual norm");
    } else if (verdict == MG_OK) {
      return MG_OK;
    }
    if (verdict != kContinue && verdict != MG_OK) return fail(ctx, verdict, why);
    if (ctx->graphs && !ctx->timing) {
      if ((st = ensure_graph(ctx, f, x)) != MG_OK) return st;
      HIPCHK(ctx, hipGraphLaunch(ctx->gexec, s));
    } else if ((st = iterate(ctx, f, x, s)) != MG_OK) {
      return st;
    }
  }
}

static int impl_mg_timing_enable(mg_ctx* ctx, int enable) {
  if (!ctx) return MG_EINVAL;
  drop_graph(ctx);
  if (ctx->ev_used) (void)hipEventSynchronize(ctx->ev[ctx->ev_used - 1]);
  ctx->ev_used = 0;
  ctx->t_ms = 0.0;
  ctx->t_n = 0;
  ctx->timing = enable != 0;
  return MG_OK;
}

static int impl_mg_timing_read(mg_ctx* ctx, double* total_ms, long* launches) {
  if (!ctx || !total_ms || !launches) return MG_EINVAL;
  if (ctx->ev_used) {
    HIPCHK(ctx, hipEventSynchronize(ctx->ev[ctx->ev_used - 1]));
    for (size_t k = 0; k + 1 < ctx->ev_used; k += 2) {
      float ms = 0.f;
      HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev[k], ctx->ev[k + 1]));
      ctx->t_ms += ms;
    }
    ctx->ev_used = 0;
  }
  *total_ms = ctx->t_ms;
  *launches = ctx->t_n;
  return MG_OK;
}

}  // extern "C"

// ====================================================================== batch
//
// Independent instances (their own level, alpha and data) solved together.
// Every instance keeps its own context (workspace, tables, coarse LU, tail
// schedule); a batched V-cycle runs the levels from the highest finest level
// down to the tail level and back, and each step is one launch covering every
// instance whose finest level reaches that level (they share its geometry).
// The coarse-level tail runs one workgroup per instance.  One batched iterate
// is captured as a HIP graph; between replays the host reads all residual
// norms with one copy, applies the stopping rule per instance, and switches
// finished instances off through a device flag that every kernel checks.

struct mg_batch {
  int count = 0, k0 = 1, T = 0, Lmax = 0, device = 0;
  mg_opts o{};
  std::vector<mg_ctx*> inst;
  std::vector<int> level;
  int* d_active = nullptr;
  int* h_active = nullptr;
  double* d_norms = nullptr;  // gathered (||r||^2, ||f||^2) per instance
  double* h_norms = nullptr;
  double** d_normptr = nullptr;
  struct Group {
    int L = 0;
    int shape = 0;  // tile shape of the batched sweep on this level (picked at setup)
    std::vector<int> members;
    mgk::BInst<double>* d64 = nullptr;
    mgk::BInst<float>* d32 = nullptr;
  };
  std::vector<Group> groups;  // levels T+1 .. Lmax
  struct Fine {
    int F = 0;
    std::vector<int> members;
    mgk::BFine* d = nullptr;
  };
  std::vector<Fine> fine;  // one per distinct finest level
  void* d_tail64 = nullptr;
  void* d_tail32 = nullptr;
  size_t tail_lds = 0;
  std::vector<const double*> uf;
  std::vector<double*> ux;
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool graphs = true;
  std::string err;
};

namespace {

int bfail(mg_batch* b, int status, const std::string& msg) {
  if (b) b->err = msg;
  return status;
}

#define BCHK(b, expr)                                                                                      \
  do {                                                                                                     \
    hipError_t e_ = (expr);                                                                                \
    if (e_ != hipSuccess)                                                                                  \
      return bfail((b), e_ == hipErrorOutOfMemory ? MG_ENOMEM : MG_EHIP,                                   \
                   std::string(#expr) + ": " + hipGetErrorString(e_));                                     \
  } while (0)

void batch_free(mg_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (auto& g : b->groups) {
    (void)hipFree(g.d64);
    (void)hipFree(g.d32);
  }
  for (auto& f : b->fine) (void)hipFree(f.d);
  (void)hipFree(b->d_tail64);
  (void)hipFree(b->d_tail32);
  (void)hipFree(b->d_active);
  (void)hipFree(b->d_norms);
  (void)hipFree(b->d_normptr);
  if (b->h_active) (void)hipHostFree(b->h_active);
  if (b->h_norms) (void)hipHostFree(b->h_norms);
  for (auto c : b->inst) destroy_impl(c);
  delete b;
}

mg_batch::Group& group_of(mg_batch* b, int L) { return b->groups[L - b->T - 1]; }

// per-level descriptors of instance i at level L (FP64: the caller's f and x
// on the instance's finest level)
template <typename T>
mgk::BInst<T> make_binst(mg_batch* b, int i, int L, const double* uf, double* ux) {
  mg_ctx* c = b->inst[i];
  LevelBuf& lb = L_(c, L);
  LevelBuf& lc = L_(c, L - 1);
  Work<T> w = work(lb, (T*)nullptr), wc = work(lc, (T*)nullptr);
  mgk::BInst<T> a{};
  a.L = lb.lev;
  a.Lc = lc.lev;
  a.x = w.x;
  a.f = w.f;
  if constexpr (std::is_same<T, double>::value) {
    if (L == c->level) {
      a.x = ux;
      a.f = const_cast<double*>(uf);
    }
  }
  a.r = w.r;
  a.r2 = w.r2;
  a.p = w.p;
  a.xc = wc.x;
  a.fc = wc.f;
  a.rc = wc.r;
  a.active = b->d_active + i;
  return a;
}

// descriptors that hold the caller's pointers (FP64 levels, finest levels)
int batch_bind(mg_batch* b, const double* const* f, double* const* x, hipStream_t s) {
  bool same = !b->uf.empty();
  for (int i = 0; same && i < b->count; i++) same = b->uf[i] == f[i] && b->ux[i] == x[i];
  if (same) return MG_OK;
  BCHK(b, hipStreamSynchronize(s));
  b->uf.assign(f, f + b->count);
  b->ux.assign(x, x + b->count);
  for (auto& g : b->groups) {
    std::vector<mgk::BInst<double>> h;
    for (int i : g.members) h.push_back(make_binst<double>(b, i, g.L, f[i], x[i]));
    BCHK(b, hipMemcpy(g.d64, h.data(), h.size() * sizeof(h[0]), hipMemcpyHostToDevice));
  }
  for (auto& fg : b->fine) {
    std::vector<mgk::BFine> h;
    for (int i : fg.members) {
      mg_ctx* c = b->inst[i];
      LevelBuf& lb = L_(c, c->level);
      mgk::BFine a{};
      a.L = lb.lev;
      a.f = f[i];
      a.x = x[i];
      a.r = lb.r;
      a.f32 = lb.f32;
      a.x32 = lb.x32;
      a.r32 = lb.r32;
      a.part = c->d_part;
      a.norm = c->d_norm;
      a.active = b->d_active + i;
      h.push_back(a);
    }
    BCHK(b, hipMemcpy(fg.d, h.data(), h.size() * sizeof(h[0]), hipMemcpyHostToDevice));
  }
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
  return MG_OK;
}

template <typename T>
const mgk::BInst<T>* gdev(const mg_batch::Group& g);
template <>
const mgk::BInst<double>* gdev<double>(const mg_batch::Group& g) {
  return g.d64;
}
template <>
const mgk::BInst<float>* gdev<float>(const mg_batch::Group& g) {
  return g.d32;
}

template <typename T>
int batch_smooth(mg_batch* b, const mg_batch::Group& g, int steps, int& sel, hipStream_t s) {
  const int n = 1 << g.L, cnt = (int)g.members.size();
  const mgk::BInst<T>* d = gdev<T>(g);
  for (int it = 0; it < steps; it++) {
    switch (b->o.smoother) {
      case MG_NE:
        BCHK(b, mgk::launch_b_ne<T>(d, cnt, n, sel, s));
        break;
      case MG_LSGS:
        BCHK(b, mgk::launch_b_lsgs_sweep<T>(d, cnt, n, 0, sel, s, g.shape));
        sel ^= 1;
        break;
      case MG_SLSGS:
        BCHK(b, mgk::launch_b_lsgs_sweep<T>(d, cnt, n, 0, sel, s, g.shape));
        BCHK(b, mgk::launch_b_lsgs_sweep<T>(d, cnt, n, 1, sel ^ 1, s, g.shape));
        break;
      case MG_CGS:
        for (int col = 0; col < 7; col++) BCHK(b, mgk::launch_b_cgs_phase<T>(d, cnt, n, col, sel, s));
        break;
    }
  }
  return MG_OK;
}

// one batched V-cycle; on entry the finest-level residual of every instance
// is current in its r buffer
template <typename T>
int batch_cycle(mg_batch* b, hipStream_t s) {
  std::vector<int> sel(b->Lmax + 1, 0);
  int st;
  for (int L = b->Lmax; L > b->T; L--) {
    const mg_batch::Group& g = group_of(b, L);
    int sl = 0;
    if ((st = batch_smooth<T>(b, g, b->o.nu1, sl, s)) != MG_OK) return st;
    BCHK(b, mgk::launch_b_restrict<T>(gdev<T>(g), (int)g.members.size(), 1 << (L - 1), sl, L - 1 > b->T ? 1 : 0, s));
    sel[L] = sl;
  }
  BCHK(b, mgk::launch_b_tail<T>(std::is_same<T, double>::value ? b->d_tail64 : b->d_tail32, b->count, b->tail_lds, s));
  for (int L = b->T + 1; L <= b->Lmax; L++) {
    const mg_batch::Group& g = group_of(b, L);
    const int cnt = (int)g.members.size();
    int sl = sel[L];
    BCHK(b, mgk::launch_b_prolong_add<T>(gdev<T>(g), cnt, 1 << L, s));
    BCHK(b, mgk::launch_b_residual<T>(gdev<T>(g), cnt, 1 << L, sl, s));
    if ((st = batch_smooth<T>(b, g, b->o.nu2, sl, s)) != MG_OK) return st;
  }
  return MG_OK;
}

// finest-level residuals and their squared norms into norm[0] of every instance
int batch_residual_norms(mg_batch* b, hipStream_t s) {
  const int mode = b->o.norm == MG_NORM_LINV ? 2 : 1;
  for (auto& fg : b->fine) {
    const int cnt = (int)fg.members.size();
    BCHK(b, mgk::launch_b_residual_norm(fg.d, cnt, 1 << fg.F, mode, s));
    BCHK(b, mgk::launch_b_sum(fg.d, cnt, mgk::residual_blocks(1 << fg.F), 0, s));
  }
  return MG_OK;
}

// one iterate for every active instance, then the gathered norms
int batch_iterate(mg_batch* b, hipStream_t s) {
  int st;
  if (b->o.precision == MG_FP32_IR) {
    for (auto& fg : b->fine) {
      const size_t len = 2 * (size_t)((1 << fg.F) + 1) * ((1 << fg.F) + 1);
      BCHK(b, mgk::launch_b_to_f32_scaled(fg.d, (int)fg.members.size(), len, s));
      BCHK(b, mgk::launch_b_zero_x32(fg.d, (int)fg.members.size(), len, s));
    }
    if ((st = batch_cycle<float>(b, s)) != MG_OK) return st;
    for (auto& fg : b->fine) {
      const size_t len = 2 * (size_t)((1 << fg.F) + 1) * ((1 << fg.F) + 1);
      BCHK(b, mgk::launch_b_axpy_f32(fg.d, (int)fg.members.size(), len, s));
    }
  } else if ((st = batch_cycle<double>(b, s)) != MG_OK) {
    return st;
  }
  if ((st = batch_residual_norms(b, s)) != MG_OK) return st;
  BCHK(b, mgk::launch_b_gather_norms(b->d_normptr, b->count, b->d_norms, s));
  return MG_OK;
}

int batch_graph(mg_batch* b) {
  if (b->gexec) return MG_OK;
  if (!b->cap) BCHK(b, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  BCHK(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  int st = batch_iterate(b, b->cap);
  hipError_t e = hipStreamEndCapture(b->cap, &g);
  if (st != MG_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return bfail(b, MG_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->gexec = nullptr;
    return bfail(b, MG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  return MG_OK;
}

// Autotuner of the batched sweep's tile shape: per level, every candidate
// of launch_b_lsgs_sweep is timed on the batch's own level buffers (x, r and
// r2 of every instance; FP64 cycles use the level scratch p as x, since the
// caller's iterate is bound only at solve time), after zeroing them, and the
// fastest is kept.  One warm-up launch, then the median of 3 timed launches.
template <typename T>
int batch_autotune(mg_batch* b, hipStream_t s) {
  for (auto& g : b->groups) {
    const int n = 1 << g.L, cnt = (int)g.members.size();
    std::vector<mgk::BInst<T>> h;
    for (int i : g.members) {
      mgk::BInst<T> a = make_binst<T>(b, i, g.L, nullptr, nullptr);
      if constexpr (std::is_same<T, double>::value) a.x = a.p;
      const size_t len = L_(b->inst[i], g.L).len;
      BCHK(b, hipMemsetAsync(a.x, 0, len * sizeof(T), s));
      BCHK(b, hipMemsetAsync(a.r, 0, len * sizeof(T), s));
      BCHK(b, hipMemsetAsync(a.r2, 0, len * sizeof(T), s));
      h.push_back(a);
    }
    mgk::BInst<T>* d = nullptr;
    if (hipMalloc(&d, h.size() * sizeof(h[0])) != hipSuccess) return bfail(b, MG_ENOMEM, "autotune: allocation failed");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto done = [&](int st) {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      (void)hipFree(d);
      return st;
    };
    if (hipMemcpyAsync(d, h.data(), h.size() * sizeof(h[0]), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
      return done(bfail(b, MG_EHIP, "autotune: HIP setup failed"));
    float best = 0.0f;
    int best_shape = 0;
    for (int shape = 0; shape < mgk::b_sweep_shapes(); shape++) {
      if (mgk::launch_b_lsgs_sweep<T>(d, cnt, n, 0, 0, s, shape) != hipSuccess)
        return done(bfail(b, MG_EHIP, "autotune: sweep launch failed"));
      float t[3];
      for (int rep = 0; rep < 3; rep++) {
        if (hipEventRecord(e0, s) != hipSuccess ||
            mgk::launch_b_lsgs_sweep<T>(d, cnt, n, 0, rep & 1, s, shape) != hipSuccess ||
            hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t[rep], e0, e1) != hipSuccess)
          return done(bfail(b, MG_EHIP, "autotune: timing failed"));
      }
      std::sort(t, t + 3);
      if (shape == 0 || t[1] < best) {
        best = t[1];
        best_shape = shape;
      }
    }
    g.shape = best_shape;
    done(MG_OK);
  }
  return MG_OK;
}

}  // namespace

extern "C" {

static int batch_setup_body(mg_batch* b, int count, const int* levels, const double* alphas, int problem,
                            const mg_opts& o, mg_batch** out);

static int impl_mg_batch_setup(int count, const int* levels, const double* alphas, int problem, const mg_opts* opts,
                               mg_batch** out) {
  if (!out) return MG_EINVAL;
  *out = nullptr;
  if (count < 1 || count > kMaxBatch || !levels || !alphas) return MG_EINVAL;
  if (problem != MG_POISSON && problem != MG_STOKES) return MG_EINVAL;
  mg_opts o = mg_default_opts(problem);
  if (opts) o = *opts;
  if (!valid_opts(&o, -1)) return MG_EINVAL;
  for (int i = 0; i < count; i++) {
    if (levels[i] < kBatchMinLevel || levels[i] > kMaxLevel) return MG_EINVAL;
    if (!(alphas[i] > 0.0) || !std::isfinite(alphas[i])) return MG_EINVAL;
  }
  if (problem != MG_POISSON || o.gamma != 1 || o.inner_cycles != 1 || o.coarse_level > 2) return MG_EUNSUPPORTED;
  mg_batch* b = new mg_batch;
  try {
    return batch_setup_body(b, count, levels, alphas, problem, o, out);
  } catch (...) {
    batch_free(b);
    throw;
  }
}

static int batch_setup_body(mg_batch* b, int count, const int* levels, const double* alphas, int problem,
                            const mg_opts& o, mg_batch** out) {
  b->count = count;
  b->o = o;
  b->k0 = o.coarse_level;
  (void)hipGetDevice(&b->device);
  b->graphs = std::getenv("MGKKT_NO_GRAPH") == nullptr;
  auto bail = [&](int st) {
    batch_free(b);
    return st;
  };
  for (int i = 0; i < count; i++) {
    mg_ctx* c = nullptr;
    t_batch_instance = true;
    int st = mg_setup(levels[i], alphas[i], problem, &o, &c);
    t_batch_instance = false;
    if (st != MG_OK) return bail(st);
    b->inst.push_back(c);
    b->level.push_back(levels[i]);
    b->Lmax = std::max(b->Lmax, levels[i]);
    if (c->tail_T == 0) return bail(MG_EUNSUPPORTED);  // the coarse-level tail is required
    if (i == 0) b->T = c->tail_T;
    if (c->tail_T != b->T) return bail(MG_EUNSUPPORTED);
  }
  if (hipMalloc(&b->d_active, count * sizeof(int)) != hipSuccess ||
      hipMalloc(&b->d_norms, 2 * count * sizeof(double)) != hipSuccess ||
      hipMalloc(&b->d_normptr, count * sizeof(double*)) != hipSuccess ||
      hipHostMalloc((void**)&b->h_active, count * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&b->h_norms, 2 * count * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return bail(MG_ENOMEM);
  {
    std::vector<double*> np;
    for (auto c : b->inst) np.push_back(c->d_norm);
    if (hipMemcpy(b->d_normptr, np.data(), count * sizeof(double*), hipMemcpyHostToDevice) != hipSuccess)
      return bail(MG_EHIP);
  }
  // level groups; FP32 descriptors are fixed (library buffers only)
  for (int L = b->T + 1; L <= b->Lmax; L++) {
    mg_batch::Group g;
    g.L = L;
    for (int i = 0; i < count; i++)
      if (levels[i] >= L) g.members.push_back(i);
    if (hipMalloc(&g.d64, g.members.size() * sizeof(mgk::BInst<double>)) != hipSuccess) return bail(MG_ENOMEM);
    if (o.precision == MG_FP32_IR) {
      std::vector<mgk::BInst<float>> h;
      for (int i : g.members) h.push_back(make_binst<float>(b, i, L, nullptr, nullptr));
      if (hipMalloc(&g.d32, h.size() * sizeof(h[0])) != hipSuccess) return bail(MG_ENOMEM);
      if (hipMemcpy(g.d32, h.data(), h.size() * sizeof(h[0]), hipMemcpyHostToDevice) != hipSuccess)
        return bail(MG_EHIP);
    }
    b->groups.push_back(g);
  }
  for (int F = b->T + 1; F <= b->Lmax; F++) {
    mg_batch::Fine fg;
    fg.F = F;
    for (int i = 0; i < count; i++)
      if (levels[i] == F) fg.members.push_back(i);
    if (fg.members.empty()) continue;
    if (hipMalloc(&fg.d, fg.members.size() * sizeof(mgk::BFine)) != hipSuccess) return bail(MG_ENOMEM);
    b->fine.push_back(fg);
  }
  // tail schedules: level-T buffers of every instance (x_T starts at zero)
  {
    const size_t sz64 = mgk::tail_args_bytes<double>(), sz32 = mgk::tail_args_bytes<float>();
    std::vector<unsigned char> h64(sz64 * count), h32(sz32 * count);
    for (int i = 0; i < count; i++) {
      mg_ctx* c = b->inst[i];
      LevelBuf& lt = L_(c, b->T);
      mgk::make_tail_args<double>(c->tail, lt.f, lt.x, 1, b->d_active + i, h64.data() + i * sz64);
      if (o.precision == MG_FP32_IR)
        mgk::make_tail_args<float>(c->tail, lt.f32, lt.x32, 1, b->d_active + i, h32.data() + i * sz32);
    }
    if (hipMalloc(&b->d_tail64, h64.size()) != hipSuccess) return bail(MG_ENOMEM);
    if (hipMemcpy(b->d_tail64, h64.data(), h64.size(), hipMemcpyHostToDevice) != hipSuccess) return bail(MG_EHIP);
    if (o.precision == MG_FP32_IR) {
      if (hipMalloc(&b->d_tail32, h32.size()) != hipSuccess) return bail(MG_ENOMEM);
      if (hipMemcpy(b->d_tail32, h32.data(), h32.size(), hipMemcpyHostToDevice) != hipSuccess) return bail(MG_EHIP);
    }
    b->tail_lds = std::max(mgk::tail_lds_bytes<double>(b->k0, b->T),
                           o.precision == MG_FP32_IR ? mgk::tail_lds_bytes<float>(b->k0, b->T) : size_t(0));
  }
  // tile shapes of the batched LSGS sweeps (MGKKT_NO_AUTOTUNE=1: the default shape)
  if (o.smoother == MG_LSGS || o.smoother == MG_SLSGS) {
    const char* nt = std::getenv("MGKKT_NO_AUTOTUNE");
    if (!(nt && nt[0] == '1')) {
      for (int i = 0; i < count; i++) b->h_active[i] = 1;
      if (hipMemcpy(b->d_active, b->h_active, count * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        return bail(MG_EHIP);
      const int st = o.precision == MG_FP32_IR ? batch_autotune<float>(b, nullptr) : batch_autotune<double>(b, nullptr);
      if (st != MG_OK) return bail(st);
      if (hipDeviceSynchronize() != hipSuccess) return bail(MG_EHIP);
    }
  }
  *out = b;
  return MG_OK;
}

void mg_batch_destroy(mg_batch* b) { batch_free(b); }

int mg_batch_sweep_tile(const mg_batch* b, int level) {
  if (!b) return 0;
  for (const auto& g : b->groups)
    if (g.L == level) return mgk::b_sweep_tile(b->o.precision == MG_FP32_IR ? 1 : 0, g.shape);
  return 0;
}

int mg_batch_count(const mg_batch* b) { return b ? b->count : 0; }

size_t mg_batch_vec_len(const mg_batch* b, int i) {
  return (b && i >= 0 && i < b->count) ? mg_vec_len(b->inst[i]) : 0;
}

const char* mg_batch_last_error(const mg_batch* b) { return b ? b->err.c_str() : "no batch"; }

static int impl_mg_batch_rhs(mg_batch* b, const double* const* yd, double* const* f, void* stream) {
  if (!b || !yd || !f) return MG_EINVAL;
  for (int i = 0; i < b->count; i++)
    if (!yd[i] || !f[i]) return MG_EINVAL;
  for (int i = 0; i < b->count; i++) {
    const int st = mg_rhs(b->inst[i], yd[i], f[i], stream);
    if (st != MG_OK) return bfail(b, st, b->inst[i]->err);
  }
  return MG_OK;
}

static int impl_mg_batch_solve(mg_batch* b, const double* const* f, double* const* x, double tol, int* cycles_out,
                   double* relres_out, int* status_out, void* stream) {
  if (!b || !f || !x || !(tol > 0.0) || !std::isfinite(tol)) return MG_EINVAL;
  for (int i = 0; i < b->count; i++)
    if (!f[i] || !x[i]) return MG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int st;
  if ((st = batch_bind(b, f, x, s)) != MG_OK) return st;
  const int n = b->count, mode = b->o.norm == MG_NORM_LINV ? 2 : 1;
  // ||f|| and the initial residual of every instance
  for (int i = 0; i < n; i++) b->h_active[i] = 1;
  BCHK(b, hipMemcpyAsync(b->d_active, b->h_active, n * sizeof(int), hipMemcpyHostToDevice, s));
  for (auto& fg : b->fine) {
    const int cnt = (int)fg.members.size();
    BCHK(b, mgk::launch_b_vnorm(fg.d, cnt, 1 << fg.F, mode, s));
    BCHK(b, mgk::launch_b_sum(fg.d, cnt, mgk::residual_blocks(1 << fg.F), 1, s));
  }
  if ((st = batch_residual_norms(b, s)) != MG_OK) return st;
  BCHK(b, mgk::launch_b_gather_norms(b->d_normptr, n, b->d_norms, s));
  std::vector<Monitor> mon(n);
  std::vector<int> verdict(n, kContinue), cyc(n, 0);
  std::vector<double> rel(n, 0.0);
  std::string why0;
  for (int it = 0;; it++) {
    BCHK(b, hipMemcpyAsync(b->h_norms, b->d_norms, 2 * n * sizeof(double), hipMemcpyDeviceToHost, s));
    BCHK(b, hipStreamSynchronize(s));
    int live = 0;
    for (int i = 0; i < n; i++) {
      if (verdict[i] != kContinue) continue;
      const char* why = "";
      cyc[i] = it;
      verdict[i] = mon[i].check(b->h_norms[2 * i], b->h_norms[2 * i + 1], tol, it, b->o.max_cycles, &why);
      rel[i] = mon[i].rel;
      if (verdict[i] != kContinue && verdict[i] != MG_OK && why0.empty())
        why0 = "instance " + std::to_string(i) + ": " + why;
      b->h_active[i] = verdict[i] == kContinue ? 1 : 0;
      live += b->h_active[i];
    }
    if (!live) break;
    BCHK(b, hipMemcpyAsync(b->d_active, b->h_active, n * sizeof(int), hipMemcpyHostToDevice, s));
    if (b->graphs) {
      if ((st = batch_graph(b)) != MG_OK) return st;
      BCHK(b, hipGraphLaunch(b->gexec, s));
    } else if ((st = batch_iterate(b, s)) != MG_OK) {
      return st;
    }
  }
  int result = MG_OK;
  for (int i = 0; i < n; i++) {
    if (cycles_out) cycles_out[i] = cyc[i];
    if (relres_out) relres_out[i] = rel[i];
    if (status_out) status_out[i] = verdict[i];
    if (verdict[i] != MG_OK && result == MG_OK) result = verdict[i];
  }
  if (result != MG_OK) b->err = why0;
  return result;
}

}  // extern "C"

// ============================================================ exception guard
//
// Every int-returning entry point runs its body through guarded(): a host
// exception (std::bad_alloc from a std::vector of the setup or of the solve
// loop's bookkeeping, std::length_error from an oversized assembly) becomes a
// status code instead of crossing the C ABI.
namespace {
template <class F>
int guarded(std::string* err, F&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    try {
      if (err) *err = "host memory allocation failed";
    } catch (...) {
    }
    return MG_ENOMEM;
  } catch (const std::exception& e) {
    try {
      if (err) *err = std::string("host exception: ") + e.what();
    } catch (...) {
    }
    return MG_EUNSUPPORTED;
  } catch (...) {
    return MG_EHIP;
  }
}
std::string* err_of(mg_ctx* c) { return c ? &c->err : nullptr; }
std::string* err_of(const mg_ctx*) { return nullptr; }
std::string* err_of(mg_batch* b) { return b ? &b->err : nullptr; }
std::string* err_of(mg_graph* g) { return g ? &g->ctx->err : nullptr; }
}  // namespace

extern "C" {

int mg_get_opts(const mg_ctx* ctx, mg_opts* out) {
  return guarded(err_of(ctx), [&] { return impl_mg_get_opts(ctx, out); });
}

int mg_setup(int level, double alpha, int problem, const mg_opts* opts, mg_ctx** out) {
  return guarded(nullptr, [&] { return impl_mg_setup(level, alpha, problem, opts, out); });
}

int mg_set_opts(mg_ctx* ctx, const mg_opts* opts) {
  return guarded(err_of(ctx), [&] { return impl_mg_set_opts(ctx, opts); });
}

int mg_rhs(mg_ctx* ctx, const double* yd, double* f, void* stream) {
  return guarded(err_of(ctx), [&] { return impl_mg_rhs(ctx, yd, f, stream); });
}

int mg_control(mg_ctx* ctx, const double* x, double* u, void* stream) {
  return guarded(err_of(ctx), [&] { return impl_mg_control(ctx, x, u, stream); });
}

int mg_adjoint_grad(mg_ctx* ctx, const double* x, const double* xadj, double* grad_yd, double* grad_alpha, void* stream) {
  return guarded(err_of(ctx), [&] { return impl_mg_adjoint_grad(ctx, x, xadj, grad_yd, grad_alpha, stream); });
}

int mg_apply(mg_ctx* ctx, int level, const double* x, double* y, void* stream) {
  return guarded(err_of(ctx), [&] { return impl_mg_apply(ctx, level, x, y, stream); });
}

int mg_residual(mg_ctx* ctx, int level, const double* f, const double* x, double* r, double* norm_out, void* stream) {
  return guarded(err_of(ctx), [&] { return impl_mg_residual(ctx, level, f, x, r, norm_out, stream); });
}

int mg_residual_nalloc(mg_ctx* ctx, int level, const double* f, const double* x, double* r, double* norm_dev,
                       void* stream) {
  return guarded(err_of(ctx), [&] { return impl_mg_residual_nalloc(ctx, level, f, x, r, norm_dev, stream); });
}

int mg_smooth(mg_ctx* ctx, int level, double* x, double* r, int steps, void* stream) {
  return guarded(err_of(ctx), [&] { return impl_mg_smooth(ctx, level, x, r, steps, stream); });
}

int mg_restrict(mg_ctx* ctx, int level, const double* r, double* fc, void* stream) {
  return guarded(err_of(ctx), [&] { return impl_mg_restrict(ctx, level, r, fc, stream); });
}

int mg_prolong_add(mg_ctx* ctx, int level, const double* xc, double* x, void* stream) {
  return guarded(err_of(ctx), [&] { return impl_mg_prolong_add(ctx, level, xc, x, stream); });
}

int mg_coarse_solve(mg_ctx* ctx, const double* f, double* x, void* stream) {
  return guarded(err_of(ctx), [&] { return impl_mg_coarse_solve(ctx, f, x, stream); });
}

int mg_cycle(mg_ctx* ctx, const double* f, double* x, void* stream) {
  return guarded(err_of(ctx), [&] { return impl_mg_cycle(ctx, f, x, stream); });
}

int mg_capture_cycle(mg_ctx* ctx, const double* f, double* x, void* stream, mg_graph** out) {
  return guarded(err_of(ctx), [&] { return impl_mg_capture_cycle(ctx, f, x, stream, out); });
}

int mg_graph_launch(mg_graph* graph, void* stream) {
  return guarded(err_of(graph), [&] { return impl_mg_graph_launch(graph, stream); });
}

int mg_solve(mg_ctx* ctx, const double* f, double* x, double tol, int* cycles_out, double* relres_out, void* stream) {
  return guarded(err_of(ctx), [&] { return impl_mg_solve(ctx, f, x, tol, cycles_out, relres_out, stream); });
}

int mg_timing_enable(mg_ctx* ctx, int enable) {
  return guarded(err_of(ctx), [&] { return impl_mg_timing_enable(ctx, enable); });
}

int mg_timing_read(mg_ctx* ctx, double* total_ms, long* launches) {
  return guarded(err_of(ctx), [&] { return impl_mg_timing_read(ctx, total_ms, launches); });
}

int mg_batch_setup(int count, const int* levels, const double* alphas, int problem, const mg_opts* opts, mg_batch** out) {
  return guarded(nullptr, [&] { return impl_mg_batch_setup(count, levels, alphas, problem, opts, out); });
}

int mg_batch_rhs(mg_batch* b, const double* const* yd, double* const* f, void* stream) {
  return guarded(err_of(b), [&] { return impl_mg_batch_rhs(b, yd, f, stream); });
}

int mg_batch_solve(mg_batch* b, const double* const* f, double* const* x, double tol, int* cycles_out, double* relres_out, int* status_out, void* stream) {
  return guarded(err_of(b), [&] { return impl_mg_batch_solve(b, f, x, tol, cycles_out, relres_out, status_out, stream); });
}

}  // extern "C"
