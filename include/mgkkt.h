/*
 * mgkkt.h -- C ABI of the MI355X (gfx950) all-at-once multigrid solver for the
 * discretised Poisson-control KKT system of Takacs, "Efficient smoothers for
 * all-at-once multigrid methods for Poisson and Stokes control problems"
 * (arXiv 1502.03917), section 1 eq. mp2:
 *
 *      [ M_k          K_k     ] [ y_k      ]   [ M_k y_D ]
 *      [ K_k   -alpha^-1 M_k  ] [ lambda_k ] = [    0    ]
 *
 * on the unit square, P1 (Courant) elements on the uniform mesh with n = 2^k
 * cells per side, every square split along its (i,j)-(i+1,j+1) diagonal,
 * K_k = stiffness matrix of -Laplace(y) + y with natural boundary conditions;
 * and of the Stokes-control KKT system of section 1 eq. mp3,
 *
 *      [ M_k    0     K_k        D_k^T ] [ v_k      ]   [ M_k v_D ]
 *      [ 0      0     D_k        0     ] [ p_k      ] = [    0    ]
 *      [ K_k  D_k^T  -alpha^-1 M_k  0  ] [ lambda_k ]   [    0    ]
 *      [ D_k    0     0          0     ] [ mu_k     ]   [    0    ]
 *
 * with Taylor-Hood elements on the same mesh: P2 velocity and multiplier
 * lambda (zero on the boundary; M_k, K_k the vector P2 mass and Laplacian
 * stiffness matrices), P1 pressure p and multiplier mu, D_k the divergence
 * (D_k q-row = -int q div phi).  The constant p and mu span the kernel of
 * A_k: iterates are shifted to zero mean (weights int phi_q) after every
 * finest-level iterate.
 *
 * Conventions shared by every entry point:
 *  - Vectors are contiguous FP64 arrays in DEVICE memory of the context's GPU.
 *  - Poisson control: a level-l vector has 2 (2^l+1)^2 entries, field-major
 *    [ y | lambda ]; vertex (i,j) (x = i h, y = j h, h = 2^-l) has index
 *    j (2^l+1) + i within a field.
 *  - Stokes control: a level-l vector (n = 2^l, m = 2n - 1) has
 *    4 m^2 + 2 (n+1)^2 entries, field-major [ v1 | v2 | p | lambda1 | lambda2 | mu ]:
 *    v1, v2, lambda1, lambda2 have one entry per interior P2 node, the node at
 *    (a h/2, b h/2), 1 <= a, b <= m, at index (b-1) m + (a-1) within the field;
 *    p and mu have one entry per vertex (i,j), index j (n+1) + i.  Field
 *    offsets: v1 0, v2 m^2, p 2 m^2, lambda1 2 m^2 + (n+1)^2, lambda2
 *    3 m^2 + (n+1)^2, mu 4 m^2 + (n+1)^2.
 *  - Caller-owned buffers are never freed, retained or resized by the library.
 *    The context owns its level workspace (allocated in mg_setup).
 *  - `stream` is a hipStream_t (NULL = default stream).  Work is enqueued in
 *    stream order; only mg_solve and the norm outputs synchronise the stream.
 *  - One context must not be used from two host threads or two streams at the
 *    same time; distinct contexts are independent.
 *  - Every entry point returns an mg_status (0 = success).  Argument checks run
 *    before any HIP call, so invalid arguments never touch the GPU.
 *    No exception crosses the ABI and the library never aborts.
 */
#ifndef MGKKT_H
#define MGKKT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_ctx mg_ctx;

/* problems: section 1, Poisson control (eq. mp2) and Stokes control (eq. mp3) */
enum mg_problem { MG_POISSON = 0, MG_STOKES = 1 };

/* smoothers of section 2:
 *  MG_NE    normal-equation smoother x += tau L^-1 A^T L^-1 (f - A x) (Alg. 1)
 *  MG_LSGS  least-squares Gauss-Seidel x += trig(N)^-1 A^T L^-1 (f - A x),
 *           N = A^T L^-1 A (Alg. 2).  Poisson: unknowns visited in 7 colours
 *           c(i,j) = (i + 2 j) mod 7; a vertex's y and lambda are updated
 *           together from one residual snapshot (their N entry is zero).
 *           Stokes: per velocity component 25 colours (a mod 5) + 5 (b mod 5)
 *           of the interior P2 nodes (v_c and lambda_c of a node together),
 *           then 9 colours (i mod 3) + 3 (j mod 3) of the vertices (p and mu
 *           of a vertex together)
 *  MG_SLSGS symmetric LSGS: one LSGS sweep, then one in reversed order (eq. mcNhat)
 *  MG_CGS   Poisson only: collective point Gauss-Seidel, 2x2 solve per vertex, 7 colours
 *  MG_VANKA Stokes only: patch (Vanka-type) smoother, one patch per vertex (its
 *           p and mu, and v, lambda at the vertex and at the midpoints of its
 *           edges), damped with tau (default 0.4), 9 colours (i mod 3) + 3 (j mod 3) */
enum mg_smoother { MG_NE = 0, MG_LSGS = 1, MG_SLSGS = 2, MG_CGS = 3, MG_VANKA = 4 };

/* arithmetic of the cycles: FP64 throughout, or FP32 cycles used as the
 * preconditioner of FP64 iterative refinement (outer residual, update and the
 * coarsest-level LU stay FP64) */
enum mg_precision { MG_FP64 = 0, MG_FP32_IR = 1 };

typedef enum mg_status {
  MG_OK = 0,
  MG_EINVAL = -1,      /* invalid argument (checked before any HIP call)     */
  MG_EHIP = -2,        /* a HIP runtime call failed; see mg_last_error        */
  MG_ENOMEM = -3,      /* device or host allocation failed                    */
  MG_ENOTCONV = -4,    /* max_cycles reached; x holds the last iterate        */
  MG_ENAN = -5,        /* non-finite residual norm                            */
  MG_EDIVERGE = -6,    /* residual grew above 1e3 times its initial value     */
  MG_EUNSUPPORTED = -7, /* valid but not provided by this build               */
  MG_ESTALL = -8        /* residual stagnated: the best relative residual of the last
                           10 iterates is not half the best of the 10 before (the
                           rounding floor of the arithmetic); x = last iterate */
} mg_status;

/* norm of the relative residual ||f - A x|| / ||f|| tested by mg_solve:
 *  MG_NORM_L2    Euclidean norm of the full block residual
 *  MG_NORM_LINV  ||r||_{L^-1} = (r^T L_k^-1 r)^{1/2}, L_k = diag(Q_k) of section 2
 *                (the dual of the norm ||.||_{L_k} in which the paper measures
 *                convergence).  The Euclidean ratio has an FP64 floor near
 *                eps h^-2 because x itself is rounded while f = M y_D is O(h^2):
 *                about 3e-9 at h = 1/2048, above a 1e-10 target. */
enum mg_norm { MG_NORM_L2 = 0, MG_NORM_LINV = 1 };

typedef struct {
  int smoother;     /* mg_smoother; default MG_LSGS                                  */
  int nu1, nu2;     /* pre-/post-smoothing steps; default 2, 2 (section 3)           */
  int gamma;        /* recursive coarse iterates: 1 = V-cycle (default), 2 = W-cycle */
  double tau;       /* NE / patch-smoother damping; <= 0 (default -1) selects section 3's
                       0.4 (Poisson NE, Stokes patch smoother) or 0.35 (Stokes NE)      */
  int coarse_level; /* k0: level solved exactly by FP64 LU; 1..3, default 1           */
  int precision;    /* mg_precision; default MG_FP64                                */
  int max_cycles;   /* cap of mg_solve; default 200                                  */
  int inner_cycles; /* FP32 cycles per refinement step (MG_FP32_IR); default 1       */
  int norm;         /* mg_norm of the stopping test of mg_solve; default MG_NORM_LINV */
} mg_opts;

/* defaults for a problem (see the field comments) */
mg_opts mg_default_opts(int problem);

/* Build a solver context for level `level` (n = 2^level cells per side),
 * regularisation `alpha` (> 0, finite) and problem MG_POISSON (eq. mp2) or
 * MG_STOKES (eq. mp3), with the scaling L_k of section 2 (Poisson:
 * diag(Q_k) = blockdiag(W, W / alpha), W = diag(M + alpha^1/2 K); Stokes:
 * blockdiag(W^, P^, W^ / alpha, P^ / alpha), W^ = diag(M + alpha^1/2 K),
 * P^ = alpha diag(D W^-1 D^T)) and one exact FP64 LU solve on the coarsest
 * level of section 2's cycle.  opts may be NULL (defaults).
 * Requires coarse_level+1 <= level <= 12 (Poisson) or <= 10 (Stokes: its
 * host assembly uses 32-bit row pointers).  Computes the per-level stencil
 * tables, the FP64 LU factors of the coarsest matrix and allocates the level
 * hierarchy on the current HIP device; *out is NULL on every error.
 * Errors: MG_EINVAL (argument), MG_EUNSUPPORTED (Stokes above level 10, the
 * patch smoother for Poisson, the collective smoother or coarse_level > 2 for
 * Stokes), MG_ENOMEM (device or host allocation), MG_EHIP. */
int mg_setup(int level, double alpha, int problem, const mg_opts *opts, mg_ctx **out);

/* Release the context and its device memory (NULL is allowed). */
void mg_destroy(mg_ctx *ctx);

/* Number of unknowns on the finest level: 2 (2^level+1)^2 (Poisson) or
 * 4 (2^(level+1)-1)^2 + 2 (2^level+1)^2 (Stokes); 0 for NULL. */
size_t mg_vec_len(const mg_ctx *ctx);
/* Number of unknowns on level l (0 if l is outside [coarse_level, level]). */
size_t mg_level_len(const mg_ctx *ctx, int level);

/* Read / replace the options (the level, alpha and coarse_level are fixed at
 * setup; for Stokes also the smoother and the precision).  mg_set_opts
 * returns MG_EUNSUPPORTED for the problem / smoother pairs mg_setup rejects. */
int mg_get_opts(const mg_ctx *ctx, mg_opts *out);
int mg_set_opts(mg_ctx *ctx, const mg_opts *opts);

/* Right-hand side of the finest level (device buffers, caller-owned).
 * Poisson (eq. mp2): f = (M_k y_D; 0); yd holds the nodal values of the
 * desired state ((2^l+1)^2 entries), f has 2 (2^l+1)^2 entries.
 * Stokes (eq. mp3): f = (M_k v_D; 0; 0; 0); yd holds [ v_D1 | v_D2 ] at the
 * interior P2 nodes (2 m^2 entries, the node order of the vector layout
 * above), f has mg_vec_len entries. */
int mg_rhs(mg_ctx *ctx, const double *yd, double *f, void *stream);

/* Control u = alpha^-1 lambda recovered from a solution x = (y; lambda) of
 * eq. mp2 (section 1: the optimality condition alpha M u = M lambda).
 * x: device, 2V entries; u: device, V entries (caller-owned).
 * Poisson control only (MG_EUNSUPPORTED otherwise). */
int mg_control(mg_ctx *ctx, const double *x, double *u, void *stream);

/* Reverse-mode derivative of a loss of the solution of eq. mp2 with respect
 * to the data y_D and the regularisation parameter alpha.  A_k is symmetric
 * (eq. mp2), so the adjoint system A x_adj = dLoss/dx is solved with the same
 * context (mg_solve on the right-hand side dLoss/dx).  Given the solution x
 * and x_adj (device, 2V entries each):
 *   grad_yd[V]    = M_k x_adj^y                    (f = (M_k y_D; 0))
 *   *grad_alpha   = -alpha^-2 (x_adj^lambda)^T M_k lambda
 *                   (dA/dalpha = blockdiag(0, alpha^-2 M_k))
 * grad_yd and grad_alpha (one double) are device memory; the result is
 * stream-ordered (no synchronisation).  Poisson control only. */
int mg_adjoint_grad(mg_ctx *ctx, const double *x, const double *xadj, double *grad_yd, double *grad_alpha,
                    void *stream);

/* y = A_l x on level l (section 1: eq. mp2, or eq. mp3 for Stokes). */
int mg_apply(mg_ctx *ctx, int level, const double *x, double *y, void *stream);

/* r = f - A_l x on level l; if norm_out is not NULL the Euclidean norm of r
 * is written there (this synchronises the stream). */
int mg_residual(mg_ctx *ctx, int level, const double *f, const double *x, double *r, double *norm_out,
                void *stream);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops or harnesses that forbid allocation): mg_residual without any
 * allocation or host synchronisation.  r = f - A_l x on level l as in
 * mg_residual, and the Euclidean norm of r written to norm_dev (ONE double in
 * device memory, caller-owned), stream-ordered.  The per-block partial sums
 * of the norm live in a static device array of the library (32768 doubles,
 * 256 KiB per GPU, kept until the process ends) instead of the context's
 * workspace; its address on each device is taken by mg_setup.  Every call on
 * one GPU shares that array, so calls that may overlap on one GPU (two
 * streams, two host threads) race and must be ordered by the caller.
 * Returns MG_EINVAL for a NULL argument or a level outside
 * [coarse_level, level], MG_EUNSUPPORTED when the level needs more partial
 * sums than the array holds (Poisson level 12; every other Poisson and
 * Stokes level fits), MG_EHIP for a launch failure.  Allocates nothing. */
int mg_residual_nalloc(mg_ctx *ctx, int level, const double *f, const double *x, double *r, double *norm_dev,
                       void *stream);

/* `steps` smoothing steps of the context's smoother on level l, in place on
 * (x, r) where r = f - A_l x on entry and is kept current (Alg. 1 / Alg. 2). */
int mg_smooth(mg_ctx *ctx, int level, double *x, double *r, int steps, void *stream);

/* f_c = I_l^{l-1} r: restriction = transpose of the canonical embedding, scale 1
 * (section 2); r on level l, f_c on level l-1, every field (Stokes: P2
 * interpolation for v and lambda, P1 for p and mu). */
int mg_restrict(mg_ctx *ctx, int level, const double *r, double *fc, void *stream);

/* x += I_{l-1}^l x_c: canonical embedding (P1 interpolation; Stokes: P2 for v
 * and lambda, P1 for p and mu), section 2. */
int mg_prolong_add(mg_ctx *ctx, int level, const double *xc, double *x, void *stream);

/* x = A_{k0}^{-1} f on the coarsest level by FP64 LU with partial pivoting
 * (section 2; Stokes: LU of A_{k0} bordered by the two zero-mean constraints
 * on p and mu). */
int mg_coarse_solve(mg_ctx *ctx, const double *f, double *x, void *stream);

/* One multigrid iterate on the finest level, in place on x (section 2):
 * r = f - A x, nu1 smoothing steps, restriction of the defect, gamma
 * recursive iterates from zero on the coarse-grid problem (exact LU on k0),
 * prolongation and correction, r = f - A x, nu2 smoothing steps.  With
 * precision MG_FP32_IR the iterate is one refinement step: FP64 residual,
 * inner_cycles FP32 cycles from zero on it, FP64 update.  Stream-ordered, no
 * host synchronisation.  With the tile-sweep smoothers (MG_LSGS, MG_SLSGS,
 * MG_CGS) and nu1, nu2 >= 1 the restriction runs inside the last
 * pre-smoothing launch and the prolongation with the new residual inside the
 * first post-smoothing launch of each level (the same arithmetic; the
 * environment variable MGKKT_NO_FUSED_TRANSFERS=1 at mg_setup, or timing
 * enabled with mg_timing_enable, launches them as kernels of their own). */
int mg_cycle(mg_ctx *ctx, const double *f, double *x, void *stream);

/* ---- one iterate as a replayable HIP graph (section 2's cycle) ------------
 * mg_capture_cycle records exactly the launches of mg_cycle(ctx, f, x) with
 * the context's current options into an executable HIP graph and returns it
 * in *out (caller-owned; free it with mg_graph_destroy before mg_destroy of
 * its context).  Capture runs on a private stream of the context and does not
 * execute anything; the graph is uploaded on `stream`.  Each
 * mg_graph_launch(g, stream) then performs one iterate in place on the x
 * captured, reading the f captured: both device buffers must stay allocated
 * while g is used.  A replay is bit-identical to an eager mg_cycle.  The graph
 * uses the context's workspace, so replays, eager calls and solves on one
 * context must be ordered on one stream.  mg_set_opts invalidates graphs
 * captured before it: their launch then returns MG_EINVAL.  Errors: MG_EINVAL
 * (NULL argument), MG_EHIP / MG_ENOMEM from capture or instantiation (*out =
 * NULL). */
typedef struct mg_graph mg_graph;
int mg_capture_cycle(mg_ctx *ctx, const double *f, double *x, void *stream, mg_graph **out);
int mg_graph_launch(mg_graph *graph, void *stream);
void mg_graph_destroy(mg_graph *graph);

/* Iterate section 2's multigrid cycle (or, with MG_FP32_IR, FP64 refinement
 * steps around FP32 cycles) from the initial guess in x until
 * ||f - A x|| <= tol ||f|| in the context's norm (mg_opts.norm; section 3
 * stops on a reduction of the error in the L_k norm, whose dual on residuals
 * is MG_NORM_LINV).  cycles_out (may be NULL) receives the number
 * of iterates done, relres_out (may be NULL) the final relative residual.
 * Synchronises on one norm per iterate.  Returns MG_OK, MG_ENOTCONV (x = last
 * iterate), MG_ESTALL (x = last iterate), MG_ENAN, MG_EDIVERGE, or an argument /
 * HIP error.  tol must be > 0. */
int mg_solve(mg_ctx *ctx, const double *f, double *x, double tol, int *cycles_out, double *relres_out,
             void *stream);

/* Per-launch timing of the finest-level smoothing kernels with HIP events on
 * the launch stream: enable (1) / disable (0) and reset; read the total time in
 * milliseconds and the number of timed launches.  While timing is enabled the
 * cycles launch the grid transfers as kernels of their own, so that every
 * timed launch is a plain smoothing step. */
int mg_timing_enable(mg_ctx *ctx, int enable);
int mg_timing_read(mg_ctx *ctx, double *total_ms, long *launches);

/* Static message for a status code. */
const char *mg_strerror(int status);
/* Last error message recorded on the context ("" if none; static text for NULL). */
const char *mg_last_error(const mg_ctx *ctx);

/* ---- batches of independent instances -------------------------------------
 * count instances of eq. mp2, instance i on level levels[i] (its own
 * (2^levels[i]+1)^2 vertex grid) with alpha alphas[i], all with the same
 * options.  Each instance owns a context's workspace; the batched V-cycle
 * (section 2) runs every level step as one launch over all instances whose
 * finest level reaches it, the coarse levels k0..5 as one workgroup per
 * instance, and each batched iterate is replayed from one HIP graph.
 * Instances converge (and stop) independently.
 * Requirements: MG_POISSON; 1 <= count <= 1024; every level in [6, 12];
 * gamma = 1 (V-cycle); inner_cycles = 1; coarse_level <= 2 (otherwise
 * MG_EUNSUPPORTED).  The batch must not be used from two host threads or
 * streams at once. */
typedef struct mg_batch mg_batch;

int mg_batch_setup(int count, const int *levels, const double *alphas, int problem, const mg_opts *opts,
                   mg_batch **out);
void mg_batch_destroy(mg_batch *batch);
/* number of instances (0 for NULL) */
int mg_batch_count(const mg_batch *batch);
/* unknowns of instance i, 2 (2^levels[i]+1)^2 (0 if out of range) */
size_t mg_batch_vec_len(const mg_batch *batch, int i);
/* Tile edge of the batched LSGS sweep on `level` (vertices 2^level+1 per
 * side).  For an LSGS or sLSGS batch, mg_batch_setup times every candidate
 * tile shape of that level on the batch's own buffers and keeps the fastest
 * (an addition to the method: the tile shape changes no result beyond
 * rounding); MGKKT_NO_AUTOTUNE=1 keeps the default shape.  0 for NULL or a
 * level that no instance reaches above the coarse tail. */
int mg_batch_sweep_tile(const mg_batch *batch, int level);
/* f_i = (M y_D,i; 0) for every instance: yd and f are HOST arrays of count
 * DEVICE pointers (instance i: (2^l+1)^2 and 2 (2^l+1)^2 entries). */
int mg_batch_rhs(mg_batch *batch, const double *const *yd, double *const *f, void *stream);
/* Solve every instance from its initial guess x_i (in/out) until its
 * relative residual (norm of opts.norm) is <= tol, as mg_solve does for one
 * context.  f and x are HOST arrays of count DEVICE pointers.  Per-instance
 * results go to the optional host arrays cycles_out, relres_out and
 * status_out (count entries; status as mg_solve would return).  Returns
 * MG_OK if every instance succeeded, else the status of the first failing
 * instance (message in mg_batch_last_error).  Synchronises the stream once
 * per iterate. */
int mg_batch_solve(mg_batch *batch, const double *const *f, double *const *x, double tol, int *cycles_out,
                   double *relres_out, int *status_out, void *stream);
const char *mg_batch_last_error(const mg_batch *batch);

#ifdef __cplusplus
}
#endif
#endif /* MGKKT_H */
