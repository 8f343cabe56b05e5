// Internal declarations shared by the HIP kernels and the host orchestration
// of libmgkkt (not part of the public C ABI, see include/mgkkt.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>

#include "../../include/mgkkt.h"

namespace mgk {

// Neighbour offsets of the 7-point P1 stencil on the mesh whose squares are
// split along the (i,j)-(i+1,j+1) diagonal: the vertex itself, E, W, N, S,
// NE and SW.  Opposite directions are d and d^1 for d >= 1 (1/2, 3/4, 5/6).
constexpr int kNDir = 7;
constexpr int kDI[kNDir] = {0, 1, -1, 0, 0, 1, -1};
constexpr int kDJ[kNDir] = {0, 0, 0, 1, -1, 1, -1};

// Boundary tables of one level (device memory).  Vertex classes:
//   3x3 classes  c3(i)*3 + c3(j), c3 = 0 (index 0), 1 (inside), 2 (index n);
//   5x5 classes  c5(i)*5 + c5(j), c5 = 0, 1, 2 (inside), 3 (n-1), 4 (n).
// Coefficients towards neighbours outside the square are zero.
// Per 5x5 class, the block C5[c] holds everything one smoother update needs:
// M_{v,v+d} (d = 0..6), K_{v,v+d}, 1/W_{v+d} (0 for a neighbour outside the
// square), 1/N_yy, 1/N_ll, one pad entry.
constexpr int kC5 = 3 * kNDir + 3;
struct Tab {
  double M[9][kNDir];  // M_{v, v+d}
  double K[9][kNDir];  // K_{v, v+d}, K = Laplacian stiffness + M
  double Winv[9];      // 1 / W_v with W = diag(M + sqrt(alpha) K)
  double Nyi[25];      // 1 / (N_k)_{y_v y_v}
  double Nli[25];      // 1 / (N_k)_{l_v l_v}
  double C5[25][kC5];
};

// Scalars of one level, passed by value to every kernel.
struct Lev {
  int n;    // cells per side (2^level)
  int ld;   // vertices per row, n + 1
  int V;    // vertices, (n+1)^2; field offset of lambda
  double alpha, ainv, tau;
  double Mc, Mo;      // interior M: centre, each of the six neighbours
  double Kc, Ka, Kd;  // interior K: centre, E/W/N/S, NE/SW
  double Winv;        // interior 1 / W
  double Nyi, Nli;    // 1/N for vertices at distance >= 2 from the boundary
  const Tab* tab;     // device pointer
};

// ---- coarse-level tail (tail.hip): one workgroup runs the sub-cycle on
// levels k0..T from a host-built op list
constexpr int kTailMaxLevels = 6;  // highest tail level supported
constexpr int kTailThreads = 256;  // a few waves: the tail is a chain of small barrier-separated steps
enum { kTailSmooth = 1, kTailResidual = 2, kTailRestrict = 3, kTailCoarse = 4, kTailProlongResidual = 5, kTailApplyMap = 6 };
// Level of the precomputed coarse map: from x = 0 the sub-cycle on this level
// (and everything below it) is a fixed linear map of the level's residual,
// kept as a dense matrix (2 (2^3 + 1)^2 = 162 unknowns)
constexpr int kTailMapLevel = 3;
// dense coarse map of the tail's top level kDenseMapLevel: the whole
// sub-cycle on that level and below (a linear map of the level's right-hand
// side) as one N x N matrix, N = 2 (2^5 + 1)^2
constexpr int kDenseMapLevel = 5;
constexpr int kDenseMapMaxN = 2 * ((1 << kDenseMapLevel) + 1) * ((1 << kDenseMapLevel) + 1);
enum { MG_TAIL_NE = 0, MG_TAIL_LSGS = 1, MG_TAIL_SLSGS = 2, MG_TAIL_CGS = 3 };
struct TailLaunch {
  int k0, T, nops, smoother, ncoarse;
  double tau;
  const int4* ops;  // device op list (x = op, y = level, z = count)
  const double* lu;
  const int* piv;
  // coarse map of level kTailMapLevel: column-major N x N (entry (r, c) at
  // c * N + r), FP64 and FP32 copies; nullptr: not used
  const double* map64;
  const float* map32;
  int nmap;
  Lev lev[kTailMaxLevels + 1];
  size_t max_lds;
};

__host__ __device__ inline int cls3(int i, int n) { return i == 0 ? 0 : (i == n ? 2 : 1); }
__host__ __device__ inline int cls5(int i, int n) {
  return i <= 1 ? i : (i >= n - 1 ? 4 - (n - i) : 2);
}

// ---- batched launches: many independent instances of the same level in one
// launch; the instance is blockIdx.z (vertex-grid kernels) or blockIdx.y (tile
// sweep, one-dimensional kernels), its arguments come from a device array,
// and an instance whose flag is 0 is skipped (its blocks exit at once).
template <typename T>
struct BInst {
  Lev L, Lc;              // the level and the next coarser one
  T *x, *f, *r, *r2, *p;  // level buffers (r2: ping-pong partner of r)
  T *xc, *fc, *rc;        // coarser-level buffers
  const int* active;
};
// the finest level of an instance: the FP64 outer iteration
struct BFine {
  Lev L;
  const double* f;
  double *x, *r;
  float *f32, *x32, *r32;  // FP32 cycle buffers of the finest level (refinement)
  double *part, *norm;     // per-block partial sums; norm[0] = ||r||^2, norm[1] = ||f||^2
  const int* active;
};

// ---- kernel launchers (kernels.hip); all enqueue on stream s ----------------
// r = f - A x; with part != nullptr also per-block partial sums of ||r||^2,
// Euclidean (norm_mode 1) or in the L^{-1} norm (norm_mode 2)
template <typename T>
hipError_t launch_residual(const Lev& L, const T* f, const T* x, T* r, double* part, int norm_mode, int* nblocks,
                           hipStream_t s);
hipError_t launch_vnorm(const Lev& L, const double* v, double* part, int norm_mode, int* nblocks, hipStream_t s);
template <typename T>
hipError_t launch_apply(const Lev& L, const T* x, T* y, hipStream_t s);
template <typename T>
hipError_t launch_rhs(const Lev& L, const double* yd, T* f, hipStream_t s);
template <typename T>
hipError_t launch_ne(const Lev& L, T* x, T* r, T* p, hipStream_t s);
// one NE step in one pass over LDS tiles: r read from rin, written to rout
// (distinct buffers), x updated per vertex
template <typename T>
hipError_t launch_ne_tile(const Lev& L, T* x, const T* rin, T* rout, hipStream_t s);
template <typename T>
hipError_t launch_lsgs_phase(const Lev& L, int colour, T* x, T* r, hipStream_t s);
// Grid transfers folded into a tile-sweep launch (section 2: the defect
// restriction after the pre-smoothing, the coarse-grid correction and the new
// residual before the post-smoothing).
//  - prolongation (xc set; the first post-smoothing launch): the launch forms
//    x + P xc and r = f - A (x + P xc) on each tile's region from xin, xc and
//    f instead of reading r_in, and sweeps from there; xin is read on whole
//    regions, so it must not alias x;
//  - restriction (fc set; the last pre-smoothing launch): the tiles keep one
//    more ring of final residuals and write f_c = P^T r of the residual the
//    launch leaves (x_c = 0 and r_c = f_c as well where xc0 / rc are given)
//    instead of r_out.
//  - xin_zero: the launch takes the iterate it reads as zero (a refinement
//    step's first FP32 cycle starts from x = 0) and reads nothing from xin.
template <typename T>
struct SweepIO {
  const T* xc = nullptr;
  const T* f = nullptr;
  T* fc = nullptr;
  T* xc0 = nullptr;
  T* rc = nullptr;
  Lev Lc{};  // the coarse level
  bool xin_zero = false;
};
// one full LSGS sweep (all 7 colours; reverse = colours 6..0) reading r_in
// and writing r_out (distinct buffers), x updated in place
template <typename T>
hipError_t launch_lsgs_sweep(const Lev& L, int reverse, T* x, const T* rin, T* rout, hipStream_t s);
// the same sweep reading the iterate from xin and writing it to x
template <typename T>
hipError_t launch_lsgs_sweep_from(const Lev& L, int reverse, const T* xin, T* x, const T* rin, T* rout, hipStream_t s,
                                  const SweepIO<T>* io = nullptr);
// an FP64 sweep that also stores per-tile partial sums of ||r_out||^2
// (norm_mode 1: Euclidean, 2: L^{-1}) in part; *nparts = number of tiles
// two LSGS sweeps in one launch on levels with n <= lsgs_sweep2_max_n()
// (bit s of revmask: sweep s in reverse colour order); r from rin, the
// residual after both sweeps to rout
template <typename T>
hipError_t launch_lsgs_sweep2(const Lev& L, int revmask, const T* xin, T* x, const T* rin, T* rout, hipStream_t s,
                              const SweepIO<T>* io = nullptr);
int lsgs_sweep2_max_n();
hipError_t launch_lsgs_sweep_norm(const Lev& L, int reverse, const double* xin, double* x, const double* rin,
                                  double* rout, double* part, int norm_mode, int* nparts, hipStream_t s,
                                  const SweepIO<double>* io = nullptr);
template <typename T>
hipError_t launch_cgs_phase(const Lev& L, int colour, T* x, T* r, hipStream_t s);
// fused sweeps of the collective point smoother (7 colours, one launch per
// sweep; two sweeps per launch on levels with n <= lsgs_sweep2_max_n()); r
// read from rin and written to rout, the iterate read from xin and written
// to x; the _norm form also stores per-tile partial sums of ||r_out||^2
template <typename T>
hipError_t launch_cgs_sweep_from(const Lev& L, const T* xin, T* x, const T* rin, T* rout, hipStream_t s,
                                 const SweepIO<T>* io = nullptr);
template <typename T>
hipError_t launch_cgs_sweep2(const Lev& L, const T* xin, T* x, const T* rin, T* rout, hipStream_t s,
                             const SweepIO<T>* io = nullptr);
hipError_t launch_cgs_sweep_norm(const Lev& L, const double* xin, double* x, const double* rin, double* rout,
                                 double* part, int norm_mode, int* nparts, hipStream_t s,
                                 const SweepIO<double>* io = nullptr);
template <typename T>
hipError_t launch_restrict(const Lev& Lf, const Lev& Lc, const T* r, T* fc, T* xc_zero, T* rc_copy, hipStream_t s);
template <typename T>
hipError_t launch_prolong_add(const Lev& Lf, const Lev& Lc, const T* xc, T* x, hipStream_t s);
// x_out = x_in + P x_c and r = f - A x_out in one pass (x_out != x_in)
template <typename T>
hipError_t launch_prolong_residual(const Lev& Lf, const Lev& Lc, const T* xc, const T* xin, const T* f, T* xout, T* r,
                                   hipStream_t s);
template <typename T>
hipError_t launch_coarse_solve(int N, const double* lu, const int* piv, const T* f, T* x, hipStream_t s);

// f_T in, x_T in/out (first: x_T starts at zero); see TailLaunch
template <typename T>
hipError_t launch_tail(const TailLaunch& tl, const T* fT, T* xT, int first, hipStream_t s);
template <typename T>
size_t tail_lds_bytes(int k0, int Tl);
hipError_t tail_allow_lds(size_t bytes);

// *out = scale * (sum of the n partials)
hipError_t launch_sum(const double* part, int n, double* out, hipStream_t s, double scale = 1.0);
// *out = sqrt(sum of the n partials)
hipError_t launch_sum_sqrt(const double* part, int n, double* out, hipStream_t s);
// x = B r (accumulate 0) or x += B r (accumulate 1), B row-major N x N (N even, <= kDenseMapMaxN)
template <typename T>
hipError_t launch_dense_map(const T* B, int N, const T* r, T* x, int accumulate, hipStream_t s);
// gyd = M xa^y; part = per-block partial sums of (xa^lambda)^T M lambda
hipError_t launch_adjoint_grad(const Lev& L, const double* x, const double* xa, double* gyd, double* part,
                               int* nblocks, hipStream_t s);
// u = lambda / alpha
hipError_t launch_control(const Lev& L, const double* x, double* u, hipStream_t s);
hipError_t launch_sumsq(const double* v, size_t n, double* part, int* nblocks, hipStream_t s);

// batched forms (count instances of level n; `sel` picks r (0) or r2 (1) as
// the current residual buffer)
template <typename T>
hipError_t launch_b_residual(const BInst<T>* d, int count, int n, int sel, hipStream_t s);
template <typename T>
hipError_t launch_b_ne(const BInst<T>* d, int count, int n, int sel, hipStream_t s);
template <typename T>
hipError_t launch_b_cgs_phase(const BInst<T>* d, int count, int n, int colour, int sel, hipStream_t s);
// one LSGS sweep reading the `sel` buffer and writing the other
template <typename T>
hipError_t launch_b_lsgs_sweep(const BInst<T>* d, int count, int n, int reverse, int sel, hipStream_t s, int shape = 0);
int b_sweep_shapes();                              // tile-shape candidates of launch_b_lsgs_sweep
int b_sweep_tile(int precision_fp32, int shape);   // their tile edges
// f_c = P^T r (the `sel` buffer); with zero_coarse also x_c = 0, r_c = f_c
template <typename T>
hipError_t launch_b_restrict(const BInst<T>* d, int count, int nc, int sel, int zero_coarse, hipStream_t s);
template <typename T>
hipError_t launch_b_prolong_add(const BInst<T>* d, int count, int nf, hipStream_t s);
// finest level: r = f - A x with norm partials (norm_mode 1 Euclidean, 2 L^-1),
// or partials of ||f|| (vnorm); sums into norm[slot]
hipError_t launch_b_residual_norm(const BFine* d, int count, int n, int norm_mode, hipStream_t s);
hipError_t launch_b_vnorm(const BFine* d, int count, int n, int norm_mode, hipStream_t s);
hipError_t launch_b_sum(const BFine* d, int count, int nparts, int slot, hipStream_t s);
hipError_t launch_b_to_f32_scaled(const BFine* d, int count, size_t len, hipStream_t s);
hipError_t launch_b_zero_x32(const BFine* d, int count, size_t len, hipStream_t s);
hipError_t launch_b_axpy_f32(const BFine* d, int count, size_t len, hipStream_t s);
// out[2b] = norms[b][0], out[2b+1] = norms[b][1] for b < count
hipError_t launch_b_gather_norms(const double* const* norms, int count, double* out, hipStream_t s);
int residual_blocks(int n);  // partial sums written by a level-n residual
// batched tail: one workgroup per instance; `args` is a device array built
// with make_tail_args
template <typename T>
size_t tail_args_bytes();
template <typename T>
void make_tail_args(const TailLaunch& tl, const T* fT, T* xT, int first, const int* active, void* out);
template <typename T>
hipError_t launch_b_tail(const void* args, int count, size_t lds_bytes, hipStream_t s);

// ---- Stokes control (stokes.hip): one CSR-based solver object per context
struct Stokes;
int stokes_create(int level, int k0, double alpha, const mg_opts& o, Stokes** out, std::string* err);
void stokes_destroy(Stokes* S);
size_t stokes_len(const Stokes* S, int level);
size_t stokes_partials(const Stokes* S);  // norm partial sums written on the finest level
void stokes_set(Stokes* S, const mg_opts& o);  // nu1, nu2, gamma, tau
hipError_t stokes_rhs(Stokes* S, const double* vd, double* f, hipStream_t s);
hipError_t stokes_apply(Stokes* S, int l, const double* x, double* y, hipStream_t s);
hipError_t stokes_residual(Stokes* S, int l, const double* f, const double* x, double* r, double* part,
                           int norm_mode, int* nparts, hipStream_t s);
int stokes_residual_parts(const Stokes* S, int l);  // norm partial sums a level-l residual writes
hipError_t stokes_vnorm(Stokes* S, const double* v, double* part, int norm_mode, int* nparts, hipStream_t s);
hipError_t stokes_smooth(Stokes* S, int l, double* x, double* r, int steps, hipStream_t s);
hipError_t stokes_restrict(Stokes* S, int l, const double* r, double* fc, hipStream_t s);
hipError_t stokes_prolong_add(Stokes* S, int l, const double* xc, double* x, hipStream_t s);
hipError_t stokes_coarse_solve(Stokes* S, const double* f, double* x, hipStream_t s);
hipError_t stokes_project(Stokes* S, int l, double* x, hipStream_t s);
hipError_t stokes_cycle(Stokes* S, const double* f, double* x, double* r, bool current, hipStream_t s);
double* stokes_fine_r(Stokes* S);
hipError_t stokes_ir_step(Stokes* S, double* x, hipStream_t s, const double* nrm2, int inner);

// FP32-preconditioned iterative refinement glue
// refinement scale s = sqrt(*nrm2) read on the device (1 if the norm is zero)
hipError_t launch_to_f32_scaled(const double* r, size_t n, const double* nrm2, float* out, float* out2, hipStream_t s);
// r = f - A x with norm partials (norm_mode 1 / 2), stored only as r / s in
// FP32 to out and out2 (s = sqrt(*nrm2), 1 if zero)
hipError_t launch_residual_f32(const Lev& L, const double* f, const double* x, const double* nrm2, float* out,
                               float* out2, double* part, int norm_mode, int* nblocks, hipStream_t s);
hipError_t launch_axpy_f32(const float* c, size_t n, const double* nrm2, double* x, hipStream_t s);
hipError_t launch_zero_f32(float* v, size_t n, hipStream_t s);

}  // namespace mgk
