/*
 * mgpbd.h - C ABI of the MI355X (gfx950) MGPBD library.
 *
 * MGPBD (Li et al., "MGPBD: A Multigrid Accelerated Global XPBD Solver",
 * SIGGRAPH 2025) replaces XPBD's per-constraint update by a global solve of
 * the dual system of Eq. 3,
 *     A dlambda = b,  A = gradC M^-1 gradC^T + alpha~,  b = -C - alpha~ lambda,
 * alpha~ = alpha / dt^2, with conjugate gradients preconditioned by one
 * unsmoothed-aggregation AMG V-cycle per iteration (Sec. 4.4), inside the
 * simulation loop of Algorithm 1. The AMG setup (Sec. 4.1-4.3, 4.5) is
 * reused lazily across iterations and frames (Sec. 4.2).
 *
 * Conventions shared by every call:
 *  - Every call returns an mgpbd_status; nothing throws or aborts across the
 *    ABI. mgpbd_last_error(ctx) gives a message for the last failure on ctx.
 *  - Arrays documented as "device" are HIP device pointers (for example
 *    torch.Tensor.data_ptr() of a cuda tensor on the current device). They
 *    are borrowed for the duration of the call only; work is ordered on the
 *    context's stream (mgpbd_set_stream; default: a stream the context creates) and every
 *    call returns after that work has completed, except mgpbd_apply and
 *    mgpbd_apply_noalloc, which only enqueue their kernels.
 *  - Arrays documented as "host" are ordinary CPU memory, read or written
 *    during the call only.
 *  - The library never frees caller memory; mgpbd_destroy frees everything
 *    the library allocated for a context.
 *  - One host thread per context at a time.
 */
#ifndef MGPBD_H
#define MGPBD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MGPBD_OK = 0,
  MGPBD_E_INVALID_ARG = 1,   /* bad size, index, value or state; nothing changed */
  MGPBD_E_OUT_OF_MEMORY = 2, /* device or host allocation failed */
  MGPBD_E_DEVICE = 3,        /* a HIP runtime call failed */
  MGPBD_E_NOT_CONVERGED = 4, /* mgpbd_solve hit max_pcg; the iterate is still written */
  MGPBD_E_BREAKDOWN = 5,     /* p^T A p <= 0, r^T z <= 0, non-finite, or a non-SPD level */
  MGPBD_E_SETUP = 6,         /* coarsening stalled above dense_max rows or a table overflowed */
  MGPBD_E_STATE = 7          /* call not valid for this context (e.g. no mesh) */
} mgpbd_status;

typedef enum {
  MGPBD_PREC_FP64 = 0,  /* everything in FP64 */
  MGPBD_PREC_MIXED = 1  /* V-cycle (smoother, SpMV, transfers) in FP32; outer PCG,
                           dot products and the coarsest solve in FP64 */
} mgpbd_precision;

/* Solver options. mgpbd_default_options fills the paper's values. */
typedef struct {
  double theta;         /* strength threshold theta_s of Sec. 4.1: 0.1 */
  int32_t gs_sweeps;    /* Gauss-Seidel sweeps on A x = 0 for the near-kernel (Sec. 4.3): 20 */
  int32_t pre_sweeps;   /* omega-Jacobi pre-smoothing sweeps (Sec. 4.5): 2 */
  int32_t post_sweeps;  /* omega-Jacobi post-smoothing sweeps: 2 */
  double lambda_min;    /* user estimate of lambda_min(D^-1 A) in omega (Sec. 4.5): 0.1 */
  int32_t coarse_max;   /* coarsen until a level has at most this many rows (Sec. 4.1): 400 */
  int32_t dense_max;    /* largest last level accepted for the dense Cholesky solve: 4096 */
  int32_t max_levels;   /* cap on the number of levels (1..32): 16 */
  int32_t power_iters;  /* power-method steps for lambda_max (Sec. 4.5) before its first
                           stopping test (see power_tol): 30 */
  double omega_relax;   /* relaxation of x += omega dx (Algorithm 1 and Sec. 4): 0.1 */
  double tol;           /* PCG stop: |r| <= tol |b| (recurrence residual): 1e-6 */
  int32_t max_pcg;      /* PCG iteration cap per solve: 5000 */
  uint64_t seed;        /* seed of the solver's own random streams: 20250513 */
  int32_t reuse_interval; /* setup at iteration 0 of frames f with f % R == 0 (Sec. 4.2);
                             0 = setup every iteration (the no-reuse baseline): 20 */
  int32_t b_mode;       /* 0 = smoothed near-kernel candidate, 1 = all-ones candidate */
  double eps_b;         /* end the frame's loop once |b| < eps_b (Algorithm 1); 0 = never */
  int32_t precision;    /* mgpbd_precision: MGPBD_PREC_FP64 */
  double lmax_scale;    /* omega = 2 / (lmax_scale * lambda_max + lambda_min): 1.05 (the
                           power-method estimate lies below lambda_max; the smoother
                           needs omega lambda_max < 2 to keep the V-cycle SPD) */
  int32_t check_every;  /* PCG iterations between host reads of the convergence flag: 8 */
  int32_t use_graph;    /* capture one PCG iteration in a hipGraph and replay it: 1 */
  int32_t profile_spmv; /* time every fine-level A p product with HIP events (the PCG
                           loop then launches kernels directly, without the graph): 0 */
  int32_t spmv_tile;    /* CSR pass variant: 0 = autotuned on levels with >= 20000 rows
                           (timed at setup: lanes-per-row kernels, LDS stream kernels,
                           SELL-C-sigma), -1 = lanes-per-row kernels only, -2 =
                           SELL-C-sigma (C = 64, sigma = 1024) on every level,
                           1024 / 2048 / 4096 = LDS stream kernels with that tile: 0 */
  int32_t spmv_lanes;   /* lanes per row of the lanes-per-row kernels when not autotuned
                           (4, 8, 16, 32, 64; 0 = from the mean row length): 0 */
  int32_t matrix_free;  /* 1: the fine-level products of PCG and of the V-cycle (A p,
                           smoother sweeps, residual) apply J W J^T + alpha~ from the
                           constraint gradients instead of the assembled values (the
                           assembled A still feeds the setup, the Galerkin products and
                           the Jacobi diagonal); 0: assembled CSR; 2: whichever of the
                           two is faster for this context's fine level, timed at its
                           first setup (for a batch, for the whole system). Simulation
                           contexts only; mgpbd_solve always uses the caller's CSR: 1 */
  int32_t smoother;     /* V-cycle smoother (Sec. 4.5): 0 = omega-Jacobi, 1 = Chebyshev
                           (pre_sweeps / post_sweeps steps of Chebyshev acceleration of
                           Jacobi on [lambda_min, lmax_scale * lambda_max] of D^-1 A,
                           coefficients fixed at setup), 2 = multicolour Gauss-Seidel
                           (greedy colouring of every level at setup; forward colour
                           order before the coarse correction, reversed after; the
                           sweeps read the assembled values): 0 */
  int32_t n_cand;       /* near-kernel candidates per level K, 1..8 (Sec. 4.3 generates
                           six): K > 1 factorises each aggregate's K candidates by
                           modified Gram-Schmidt, dropping columns whose remainder is at
                           most 1e-8 of their norm, so an aggregate has 1..K coarse
                           unknowns; P takes the Q blocks and the next level's
                           candidates the R rows. 1 = one normalised candidate: 1 */
  int32_t power_max;    /* power-method step cap: 500 */
  double power_tol;     /* power-method stop, tested at step power_iters and every 10 steps
                           after it: with theta = v^T A v / v^T D v, stop once
                           |D^-1 A v - theta v|_D <= power_tol * theta * |v|_D
                           (|x|_D = sqrt(x^T D x)) or at step power_max; lambda_max =
                           theta. power_max = power_iters gives a fixed count: 1e-2 */
  int32_t vcycle_tail;  /* coarse levels on which every body has at most this many rows run
                           as one launch per V-cycle, one workgroup per body, from the
                           first such level down to the dense solve and back (same
                           arithmetic as the per-level kernels; Jacobi and Chebyshev
                           smoothers, one candidate); 0 = one launch per pass (the
                           default: one workgroup's passes are latency-bound and slower
                           than the launches they replace on the workloads measured): 0 */
  int32_t fuse_transfers; /* 1: with one candidate, the residual and the restriction are one
                           pass on assembled levels, and the prolongation is folded into
                           the first post-smoothing step (its input z + P e is formed on
                           the fly); 0: separate residual, restriction and prolongation
                           kernels (the default: the fused passes' extra dependent loads
                           cost more than the launches they save on the workloads
                           measured): 0 */
  int32_t resetup_on_breakdown; /* 1: when PCG breaks down (p^T A p <= 0 or r^T z <= 0)
                           under a hierarchy kept from an earlier global iteration (the
                           lazy setup of Sec. 4.2, with the smoother weights of Sec. 4.5),
                           set up afresh for the current A and solve that iteration
                           again, once; setup_ran reports 2 for it. In a batch the whole
                           system is set up again and every body solved again. 0: return
                           MGPBD_E_BREAKDOWN: 1 */
} mgpbd_options;

/* Tetrahedral body. All arrays host, read during mgpbd_create only.
   rest: [n_verts][3] rest positions; inv_mass: [n_verts] (0 = pinned);
   tets: [n_tets][4] vertex ids, positively oriented. */
typedef struct {
  int64_t n_verts;
  const double *rest;
  const double *inv_mass;
  int64_t n_tets;
  const int32_t *tets;
} mgpbd_mesh;

/* Constraint rows. Row order: the n_edges distance constraints, then the
   n_vols volume constraints, then the n_arap ARAP constraints. edges:
   [n_edges][2], i < j, strictly ascending lexicographic; vol_tet and
   arap_tet: indices into mesh tets. All arrays host.
   An ARAP row (Sec. 5.3, Eq. 8, As-Rigid-As-Possible constraints) is
   C = |F - R|_F^2 for its tet, F = Ds Dm^-1 the deformation gradient
   (Ds = [x1 - x0, x2 - x0, x3 - x0], Dm the same at rest) and R the rotation
   (det +1) nearest to F; target C = 0. The paper takes its compliance as
   1 / (mu V_rest), mu the second Lame parameter. */
typedef struct {
  int64_t n_edges;
  const int32_t *edges;
  int64_t n_vols;
  const int32_t *vol_tet;
  int64_t n_arap;
  const int32_t *arap_tet;
} mgpbd_constraints;

/* A caller-supplied symmetric positive definite matrix in CSR form, device
   arrays: rowptr [n+1] (int64), col [nnz] (int32, strictly ascending within a
   row, diagonal present), val [nnz] (FP64). */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t *rowptr;
  const int32_t *col;
  const double *val;
} mgpbd_csr;

/* Per-frame statistics (host struct filled by mgpbd_step). Arrays are
   caller-owned host buffers of length >= n_iters, any may be NULL. */
typedef struct {
  double *bnorm;        /* |b| at each global iteration */
  int32_t *pcg_iters;   /* PCG iterations of each solve */
  double *pcg_ratio;    /* final recurrence |r| / |b| of each solve */
  int32_t *setup_ran;   /* 1 where the AMG setup ran at that iteration, 2 where it ran
                           again after a breakdown (resetup_on_breakdown) */
  int32_t iters_done;   /* global iterations executed */
  double ms_setup;      /* time spent in the setup and in the Galerkin refreshes (hipEvents) */
  double ms_pcg;        /* time spent in the PCG loops (hipEvents) */
  double ms_total;      /* whole frame (hipEvents) */
  int64_t spmv_calls;   /* fine-level A p launches timed (profile_spmv) */
  double spmv_ms;       /* their summed duration (both kernels when matrix-free, without
                           the one-block dot finisher) */
  double spmv_first_ms; /* summed duration of the first kernel alone (the matrix-free
                           vertex gather; 0 for the CSR product) */
  double ms_assembly;   /* constraints, gradients and the assembly of A and b (Eq. 3) */
  double ms_galerkin;   /* iterations that reuse the hierarchy (Sec. 4.2): Galerkin
                           products of the coarse levels (Eq. 6), diagonals and the
                           coarsest factor; part of ms_setup */
  double ms_update;     /* dx = M^-1 gradC^T dlambda (Eq. 5), lambda and x updates */
  int64_t vcycles;      /* V-cycles timed level by level (profile_spmv only) */
  double ms_level[16];  /* with profile_spmv: each level's own V-cycle passes (smoothing,
                           residual, transfers, dense solve; not its coarser levels)
                           summed over the timed V-cycles; 0 otherwise */
} mgpbd_step_stats;

typedef struct {
  int32_t iters;
  double ratio;         /* final recurrence |r| / |b| */
  double ms_setup;
  double ms_solve;
} mgpbd_solve_stats;

typedef struct mgpbd_ctx mgpbd_ctx;
typedef struct mgpbd_batch mgpbd_batch;

/* Fills *opt with the defaults listed above. */
void mgpbd_default_options(mgpbd_options *opt);

/* Create a simulation context for one body (Algorithm 1 inputs: mesh,
   constraints, per-row compliance alpha (host, [n_edges + n_vols + n_arap],
   >= 0),
   time step dt > 0, gravity (host [3]) as the external acceleration of the
   semi-implicit Euler predict). Copies everything to library-owned device
   memory and builds the fixed pattern of A (pairs of rows that share a vertex,
   Sec. 4.2). opt may be NULL for the defaults.
   Errors: E_INVALID_ARG for dt <= 0, negative or non-finite compliance or
   mass, an index out of range, edges not unique / not i < j / not ascending,
   a zero-length rest edge or a rest tet with volume <= 0. */
mgpbd_status mgpbd_create(const mgpbd_mesh *mesh, const mgpbd_constraints *cons,
                          const double *compliance, double dt, const double *gravity,
                          const mgpbd_options *opt, mgpbd_ctx **out);

/* Create a context with no body, for mgpbd_solve only. */
mgpbd_status mgpbd_solver_create(const mgpbd_options *opt, mgpbd_ctx **out);

/* Set the lazy-setup policy (Sec. 4.2; Algorithm 1 rebuilds the hierarchy
   only every few frames): max_levels caps the hierarchy depth (1..32), reuse_interval R
   runs the setup at iteration 0 of frames f with f % R == 0, R = 0 at every
   iteration. Marks the hierarchy stale so the next step rebuilds it. */
mgpbd_status mgpbd_setup(mgpbd_ctx *ctx, int32_t max_levels, int32_t reuse_interval);

/* One frame of Algorithm 1 on device SoA positions x, y, z and velocities
   vx, vy, vz ([n_verts] FP64 each, updated in place): predict, reset lambda,
   n_iters global iterations (C and gradC, A and b, lazy setup, Galerkin
   coarse operators, MGPCG, dx = M^-1 gradC^T dlambda of Eq. 5, lambda +=
   dlambda, x += omega dx), then v = (x - x_old) / dt. PCG non-convergence
   is not an error (counted in stats). Errors: E_INVALID_ARG for non-finite
   positions, E_BREAKDOWN, E_SETUP, E_DEVICE, E_STATE without a mesh. On every
   error x, y, z, vx, vy, vz hold what they held on entry, the frame counter
   does not advance, lambda is undefined until the next successful step, and
   the next step rebuilds the hierarchy. */
mgpbd_status mgpbd_step(mgpbd_ctx *ctx, double *x, double *y, double *z, double *vx,
                        double *vy, double *vz, int32_t n_iters, mgpbd_step_stats *st);

/* Solve A x = b for a caller matrix (device CSR, see mgpbd_csr; b and x_out
   device [n]) with a fresh setup on A and MGPCG to tol (Sec. 4.4). The
   hierarchy stays inspectable afterwards. Returns E_NOT_CONVERGED (x_out
   still written) when max_pcg is reached. The structure of A is checked on the
   device before use: E_INVALID_ARG (nothing else read) unless rowptr[0] = 0,
   rowptr is non-decreasing with rowptr[n] = nnz, and every row's columns lie
   in [0, n) and ascend strictly. */
mgpbd_status mgpbd_solve(mgpbd_ctx *ctx, const mgpbd_csr *A, const double *b, double tol,
                         double *x_out, mgpbd_solve_stats *st);

void mgpbd_destroy(mgpbd_ctx *ctx);
const char *mgpbd_last_error(const mgpbd_ctx *ctx);

/* Order the context's work on this HIP stream (hipStream_t, may be NULL). */
mgpbd_status mgpbd_set_stream(mgpbd_ctx *ctx, void *hip_stream);

/* Fix the PCG iteration count of the next step's solves (host array
   [n_iters], copied; NULL clears). A test hook that makes two solvers
   take the same number of iterations. */
mgpbd_status mgpbd_force_pcg_iters(mgpbd_ctx *ctx, const int32_t *iters, int32_t n_iters);

/* ---- inspection (host outputs; sizes from mgpbd_get_level) ---- */
mgpbd_status mgpbd_num_rows(const mgpbd_ctx *ctx, int64_t *m, int64_t *nnz);
mgpbd_status mgpbd_num_levels(const mgpbd_ctx *ctx, int32_t *levels);
/* n rows, nnz, Jacobi weight, aggregate count (-1 on the last level) of level l */
mgpbd_status mgpbd_get_level(const mgpbd_ctx *ctx, int32_t l, int64_t *n, int64_t *nnz,
                             double *omega, int64_t *n_agg);
/* aggregate id of every row of level l (-1 = isolated); host int32 [n_l] */
mgpbd_status mgpbd_get_aggregates(const mgpbd_ctx *ctx, int32_t l, int32_t *agg);
/* prolongator value and near-kernel candidate of every row of level l; host FP64 [n_l]
   (one candidate only: E_STATE when n_cand > 1, see mgpbd_get_qr) */
mgpbd_status mgpbd_get_transfer(const mgpbd_ctx *ctx, int32_t l, double *p, double *B);
/* sorted CSR of level l: host rowptr [n+1], col [nnz], val [nnz]; any may be NULL */
mgpbd_status mgpbd_get_matrix(const mgpbd_ctx *ctx, int32_t l, int64_t *rowptr, int32_t *col,
                              double *val);
/* y = A x with the constraint-space matrix of the last global iteration
   (Eq. 3), applied the way the PCG loop applies it: matrix-free from the
   constraint gradients (the future-work direction of the Conclusion and
   Limitations section) when
   options.matrix_free is set, else from the assembled CSR. x, y: device FP64
   [m] (for a batch context, all bodies' rows back to back), not aliased;
   enqueued on the context's stream (no synchronisation). Errors: E_STATE
   before the first step. */
mgpbd_status mgpbd_apply(mgpbd_ctx *ctx, const double *x, double *y);
/* mgpbd_apply for callers that cannot allocate device memory (code under HIP
   graph capture, tight serving loops, harnesses that forbid hipMalloc): the
   same y = A x with the same kernels, but it calls no hipMalloc, hipFree or
   allocating library routine. The matrix-free vertex gather's vector
   (4 FP64 per vertex) lives in a library-static device array of 16 MiB per
   GPU, held until the process ends, so the context may have at most 524,288
   vertices (E_INVALID_ARG beyond that, nothing enqueued); the CSR form
   (matrix_free = 0) uses no scratch. Every call on a GPU shares that GPU's
   array, so calls that overlap in time on one GPU (on different streams or
   from different threads) race and give undefined results. x, y: device FP64
   [m], not aliased; enqueued on the context's stream (no synchronisation);
   the context's device must be current (E_INVALID_ARG otherwise). Errors:
   E_STATE before the first step. */
mgpbd_status mgpbd_apply_noalloc(mgpbd_ctx *ctx, const double *x, double *y);
/* The K > 1 transfer of level l (n_cand > 1 only, E_STATE otherwise): host kq
   [n_agg] (coarse unknowns of each aggregate), coff [n_agg + 1] (first coarse
   unknown of each), Q [members][n_cand] (P's row of each aggregate member, in
   the order of the ascending member lists, zeros past kq), B [n][n_cand] (the
   level's candidates); any may be NULL. */
mgpbd_status mgpbd_get_qr(const mgpbd_ctx *ctx, int32_t l, int32_t *kq, int64_t *coff, double *Q,
                          double *B);
/* *matrix_free = 1 when the fine-level passes use the constraint-gradient
   operator, 0 when they read the assembled values (after the first step; with
   options.matrix_free = 2 this is the timed choice) */
mgpbd_status mgpbd_get_fine_operator(const mgpbd_ctx *ctx, int32_t *matrix_free);
/* right-hand side b of the last global iteration, host FP64 [m] */
mgpbd_status mgpbd_get_rhs(const mgpbd_ctx *ctx, double *b);
/* Lagrange multipliers lambda of the current frame, host FP64 [m] */
mgpbd_status mgpbd_get_lambda(const mgpbd_ctx *ctx, double *lambda);
/* multicolour Gauss-Seidel colour of every fine row (host int32 [m]); *n_colors */
mgpbd_status mgpbd_get_colors(const mgpbd_ctx *ctx, int32_t *color, int32_t *n_colors);

/* ---- test hook ---- */
/* s[i] = sqrt(a[i]), q[i] = a[i] / b[i] in FP64 on the device (device arrays
   [n]); lets tests confirm correctly rounded square root and division, on
   which the bit-exact setup relies. */
mgpbd_status mgpbd_selftest_sqrt_div(int64_t n, const double *a, const double *b, double *s,
                                     double *q);

/* ---- batching: many bodies advanced together (block-diagonal system) ---- */
/* Group n already created single-body contexts (borrowed; they must outlive
   the batch). They must share dt, gravity and precision; the batch takes the
   other options from ctxs[0]. Their rows are concatenated into one
   block-diagonal A so that every kernel of a global iteration covers all
   bodies in one launch; each body keeps its own hierarchy depth, Jacobi
   weights, coarsest factor, PCG scalars and convergence test, so each body's
   result is the one its own context would compute (up to the rounding order
   of reductions). Errors: E_INVALID_ARG for mismatched contexts or a batch
   with 2^31 or more entries of A. */
mgpbd_status mgpbd_batch_create(mgpbd_ctx *const *ctxs, int32_t n, mgpbd_batch **out);
/* One frame for every body: xyz[3*k+0..2] and vxyz[3*k+0..2] are body k's
   device SoA arrays (updated in place). st may be NULL or an array of n
   stats structs (times are those of the whole batch). Iteration counts set
   with mgpbd_force_pcg_iters on a member context apply to that body. A body
   whose |b| falls below eps_b stops iterating (zero right-hand side
   afterwards). The lazy-setup schedule follows the batch's own frame count;
   mgpbd_setup on the batch context changes it. Errors as for mgpbd_step: on
   every error the bodies' arrays hold what they held on entry (the batch
   steps copies of them and writes back only after a successful frame). */
mgpbd_status mgpbd_batch_step(mgpbd_batch *b, double *const *xyz, double *const *vxyz,
                              int32_t n_iters, mgpbd_step_stats *st);
/* The batch's system context, for mgpbd_setup, mgpbd_set_stream and the
   inspection calls (levels hold all bodies' rows back to back). Owned by the
   batch: mgpbd_destroy ignores it. */
mgpbd_ctx *mgpbd_batch_context(mgpbd_batch *b);
void mgpbd_batch_destroy(mgpbd_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* MGPBD_H */
