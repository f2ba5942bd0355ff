/*
 * bamg.h -- one Levenberg-Marquardt linear solve of bundle adjustment on an
 * AMD Instinct MI355X (gfx950), with the unsmoothed-aggregation multigrid
 * preconditioner of Konolige and Brown, "Multigrid for Bundle Adjustment".
 *
 * Conventions for every entry point:
 *   - Array pointers are DEVICE memory (hipMalloc / torch CUDA tensors) unless
 *     the comment says (host). Arrays are dense, row-major, FP64 unless noted.
 *   - The caller owns every input, output and workspace buffer; the library
 *     never frees caller memory. Device memory the library needs comes from
 *     two places:
 *       * the plan's persistent arrays (the integer structure of one
 *         visibility graph, built by ba_plan_create) come through the
 *         allocation callbacks given to ba_plan_create (hipMalloc/hipFree when
 *         they are NULL) and are released by ba_plan_destroy;
 *       * everything one LM step computes (Jacobian planes, normal blocks, the
 *         multigrid hierarchy's numeric data, PCG vectors) lives in a
 *         workspace of ba_workspace_bytes() bytes that the caller passes to the
 *         calls that start a step (ws, ws_bytes). A workspace too small for
 *         the options is BA_ERR_WORKSPACE. The prepared step stays in that
 *         workspace: the stage calls that use it (ba_step_solve,
 *         ba_schur_apply, ...) need it untouched since the call that prepared
 *         it. With ws == NULL the plan keeps a workspace of its own, allocated
 *         through its callbacks when first needed (and grown when options
 *         need more).
 *     Memory returned by the callbacks and workspaces must be aligned to 256
 *     bytes (BA_ERR_ARG otherwise).
 *   - `stream` is a hipStream_t passed as void*; all device work is enqueued on
 *     it (the multigrid setup also uses side streams of the plan, forked from
 *     and joined back into `stream` with events, so ordering on `stream` is
 *     kept). Calls that return step results block until those results are ready
 *     (the solver reads its convergence test back to the host); the operator
 *     applications (ba_schur_apply, ba_schur_offdiag_apply, ba_precond_apply)
 *     do not block.
 *   - A negative status means nothing was written to the outputs; a message is
 *     available from ba_last_error() on the calling thread. BA_NOT_CONVERGED
 *     means the outputs hold the last iterate and the statistics are valid.
 *   - A plan is not thread-safe; distinct plans are independent.
 *
 * Camera parameters (9 per camera, the 9-parameter camera the paper uses,
 * Sections 2.1 and 6; model as in the Bundle Adjustment in the Large data the
 * paper cites in Section 4):  [w0 w1 w2 | t0 t1 t2 | f | k1 k2],
 *   x_cam = R(w) X + t, p = -(x_cam.x, x_cam.y) / x_cam.z,
 *   pixel = f (1 + k1 |p|^2 + k2 |p|^4) p,  residual f_o = pixel - u_o.
 * Points: 3 world coordinates each. Observations: (camera, point, u in R^2).
 */
#ifndef BAMG_H
#define BAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ba_plan ba_plan;

typedef enum {
  BA_OK = 0,
  BA_NOT_CONVERGED = 1,   /* iteration limit reached: outputs = last iterate */
  BA_ERR_ARG = -1,        /* bad argument (null pointer, size, option value) */
  BA_ERR_INDEX = -2,      /* an observation index is out of range */
  BA_ERR_STRUCTURE = -3,  /* point with < 2 views, camera with no view, duplicate (camera, point) */
  BA_ERR_GEOMETRY = -4,   /* non-finite input, or a point at/behind an observing camera (x_cam.z >= 0) */
  BA_ERR_NOT_SPD = -5,    /* a 3x3 point block, a 9x9/16x16 smoother block or the coarse matrix
                             is not positive definite, or PCG broke down (p'Sp <= 0, r'z <= 0) */
  BA_ERR_WORKSPACE = -6,  /* the workspace is smaller than ba_workspace_bytes() for the options */
  BA_ERR_HIP = -7,        /* a HIP runtime call failed, or an allocation callback returned NULL */
  BA_ERR_LIMIT = -8       /* a documented size limit was exceeded */
} ba_status;

enum { BA_PC_BLOCK_JACOBI = 0, BA_PC_MULTIGRID = 1, BA_PC_CLUSTER_JACOBI = 2 };
enum { BA_FP64 = 0, BA_MIXED = 1 };
enum { BA_OP_AUTO = 0, BA_OP_IMPLICIT = 1, BA_OP_EXPLICIT = 2 };
enum { BA_STOP_RESIDUAL = 0, BA_STOP_NASH_SOFER = 1 };
enum { BA_LOSS_SQUARED = 0, BA_LOSS_HUBER = 1 };
enum { BA_PROLONG_TENTATIVE = 0, BA_PROLONG_SMOOTHED = 1 };

typedef struct {
  int32_t precond;          /* BA_PC_BLOCK_JACOBI (point block Jacobi, Section 2.2), BA_PC_MULTIGRID,
                               or BA_PC_CLUSTER_JACOBI: visibility-based block Jacobi (Section 2.2), the
                               inverse of S's block-diagonal part over clusters of cameras, the
                               clusters being the level-0 aggregates of Algorithm 2 (single cameras
                               when the hierarchy has one level); BA_FP64 only */
  int32_t precision;        /* BA_FP64, or BA_MIXED: FP32 Schur product and preconditioner inside
                               FP64 iterative refinement; C^-1, coarse solve and outer residual FP64 */
  double lambda;            /* D = lambda * diag(J^T J) (Marquardt damping), default 1e-4 */
  double rtol;              /* stop when ||b - S dc||_2 <= rtol ||b||_2, default 1e-6 */
  int32_t max_iter;         /* PCG iteration limit (per refinement step in BA_MIXED), default 2000 */
  int32_t max_refine;       /* BA_MIXED: refinement steps, default 10 */
  double inner_rtol;        /* BA_MIXED: relative tolerance of each FP32 inner solve, default 1e-3 */
  int32_t agg_cap;          /* aggregate size cap, default 20 (Section 3.2) */
  int32_t cheb_degree;      /* Chebyshev steps per pre/post smoothing, default 2 (Section 3.4) */
  int32_t lanczos_steps;    /* operator applications for lambda_max, default 5 (Section 3.4) */
  int32_t coarse_max_nodes; /* stop coarsening at this many nodes, default 128 */
  int32_t max_levels;       /* default 12 */
  double cheb_lo, cheb_hi;  /* Chebyshev interval as fractions of lambda_max: 0.3, 1.1 (Section 3.4) */
  double min_coarsen_ratio; /* stop when a level keeps more than this fraction of nodes, 0.9 */
  int32_t level0_op;        /* operator for level-0 smoothing and Lanczos (Section 3.6): BA_OP_AUTO
                               picks the cheaper of the implicit product and the explicit S by
                               bytes moved per application; PCG itself always uses the implicit form */
  int32_t freeze_damping_in_grad; /* backward: 1 = treat D as a constant, 0 = differentiate D(x) */
  int32_t check_every;      /* PCG: read the convergence flag back every N iterations, default 4 */
  int32_t deterministic;    /* 1: no floating-point atomics anywhere in the step, so that two runs on
                               the same inputs give bitwise equal results (the Schur product stores
                               per-(tile, camera) sums and adds them in tile order; the explicit
                               level-0 S sums each camera pair's shared points in one wave);
                               slightly slower. Default 0 */
  int32_t stop_rule;        /* PCG stop rule. BA_STOP_RESIDUAL (default): the rtol test above.
                               BA_STOP_NASH_SOFER: also stop once i (Q_i - Q_{i-1}) / Q_i <= forcing,
                               Q_i = 1/2 dc_i^T S dc_i - dc_i^T b at PCG iteration i (the forcing rule
                               of Section 2.1 with a constant forcing sequence, Section 5). FP64 only:
                               BA_MIXED with BA_STOP_NASH_SOFER is BA_ERR_ARG. The backward pass
                               always uses the rtol test. */
  int32_t prolongator;      /* BA_PROLONG_TENTATIVE (default): the unsmoothed prolongator of Section
                               3.3, one QR block per node. BA_PROLONG_SMOOTHED: smoothed aggregation,
                               the alternative Section 3.5 and the scaling experiment of Section 5.2
                               set against it: P_s = (I - w D^-1 S) P with D the block diagonal of
                               the level's operator S and w = smooth_omega / lambda_max(D^-1 S)
                               (the smoother's Lanczos estimate); the coarse operators are
                               P_s^T S P_s, with wider block rows (fill-in). A plan-time choice:
                               ba_plan_create builds the coarse block patterns for it, and a
                               multigrid step whose option differs from the plan's is BA_ERR_ARG.
                               With BA_PC_MULTIGRID it needs BA_FP64. */
  double forcing;           /* tau of BA_STOP_NASH_SOFER, >= 0, default 0.1 */
  int32_t loss;             /* BA_LOSS_SQUARED (default), or BA_LOSS_HUBER: the robust loss of Section
                               5.4 on s_o = |f_o|^2, rho(s) = s for s <= a^2 and 2 a sqrt(s) - a^2
                               above (a = loss_scale; the paper's loss is a = 1). The step then solves
                               the reweighted system: each observation's residual and Jacobian rows
                               are multiplied by sqrt(rho'(s_o)) (iteratively reweighted least
                               squares, rho's own curvature left out). Not supported by
                               ba_lm_step_backward (BA_ERR_ARG). */
  int32_t graph;            /* 1: every PCG iteration is replayed from a HIP graph (the iteration's
                               ~30 launches recorded once per plan, workspace and options, then
                               reused across steps); 0 (default): launched kernel by kernel. Same
                               results either way; on MI355X the replay saves no time, because the
                               GPU, not the host's launch rate, bounds the iteration. */
  double loss_scale;        /* a of BA_LOSS_HUBER, > 0, default 1 (pixels) */
  double smooth_omega;      /* w * lambda_max of BA_PROLONG_SMOOTHED, in (0, 2), default 4/3 */
} ba_opts;

typedef struct {            /* (host) */
  int32_t iters;            /* PCG iterations (summed over refinement steps) */
  int32_t refine_steps;     /* BA_MIXED: outer refinement steps */
  int32_t levels;           /* multigrid levels (1 = direct solve on level 0) */
  int32_t nodes[16];        /* nodes per level */
  double rel_res;           /* final ||b - S dc|| / ||b|| (recursive residual; FP64 outer in MIXED) */
  double t_jacobian_ms;     /* residual + Jacobian + normal blocks */
  double t_setup_ms;        /* preconditioner numeric setup */
  double t_solve_ms;        /* PCG (and refinement) + back-substitution */
  int32_t fallback_fp64;    /* BA_MIXED: 1 if an FP32 inner solve broke down (FP32 rounding of S
                               exceeded its smallest eigenvalues) and the solve was finished by
                               FP64 PCG on the FP64 residual */
  int32_t reserved_stats;
  int32_t agg_min[16];      /* aggregate sizes of every level that has aggregates (Section 3.2 reports */
  int32_t agg_max[16];      /* 3 to 8, mean a little over 3, on its street scenes): smallest, largest */
  double agg_mean[16];      /* and mean number of nodes per aggregate; 0 on the coarsest level */
} ba_stats;

/* Allocation callbacks of a plan: alloc returns `bytes` bytes of device memory
 * aligned to 256 bytes (or NULL on failure), release frees what alloc
 * returned; ctx is passed through. */
typedef void* (*ba_alloc_fn)(size_t bytes, void* ctx);
typedef void (*ba_free_fn)(void* ptr, void* ctx);

/* What a workspace has to hold beyond one LM step (ba_workspace_bytes). */
enum { BA_USE_STEP = 0, BA_USE_BACKWARD = 1, BA_USE_LM = 2 };

/* Defaults listed above. (host) o. */
ba_status ba_opts_default(ba_opts* o);

/* Build the integer structure reused by every LM step on the same visibility:
 * observation order, point tiles, the covisibility counts W = V V^T
 * (Section 3.2), greedy aggregation (Algorithm 2) on every level and the
 * block patterns of the coarse operators (for o->prolongator; the other
 * fields of o are read at each step). Depends only on which camera sees
 * which point, never on parameter values.
 *   obs_cam, obs_pt: [n_obs] int32 device arrays, any order.
 *   Errors: BA_ERR_INDEX, BA_ERR_STRUCTURE, BA_ERR_LIMIT (n_obs >= 2^31, a
 *   point seen by more than 65535 cameras), BA_ERR_HIP.
 *   *out (host) receives the plan. */
ba_status ba_plan_create(int32_t n_cam, int32_t n_pt, int64_t n_obs, const int32_t* obs_cam,
                         const int32_t* obs_pt, const ba_opts* o, ba_alloc_fn alloc, ba_free_fn release,
                         void* ctx, void* stream, ba_plan** out);

void ba_plan_destroy(ba_plan* p);

/* Device bytes held by the plan (host): its persistent arrays, plus its own
 * workspace if it allocated one. */
size_t ba_plan_bytes(const ba_plan* p);

/* Bytes of the workspace a step with options o needs on this plan (host):
 * the step itself (Jacobian planes, normal blocks, PCG vectors), plus the
 * FP32 copies of BA_MIXED, the hierarchy of BA_PC_MULTIGRID, the cluster
 * blocks of BA_PC_CLUSTER_JACOBI, the weights of a robust loss and the partial
 * sums of deterministic mode, as o selects. `uses` adds BA_USE_BACKWARD (the
 * adjoint's per-observation terms, for ba_lm_step_backward) and/or BA_USE_LM
 * (candidate parameters and scalars, for ba_cost and ba_lm_solve). Returns 0
 * (and sets ba_last_error) on a bad argument. */
size_t ba_workspace_bytes(const ba_plan* p, const ba_opts* o, int32_t uses);

/* One LM step (Section 2.1): solve (J^T J + D) delta = -J^T f for
 * delta = [delta_cam; delta_pt] by PCG on the Schur complement
 * S = A - F^T E C^-1 E^T F applied implicitly (Section 3.6), preconditioned by
 * block Jacobi or the multigrid V-cycle (Algorithm 1), then back-substitution
 * delta_pt = -C^-1 (g_p + E^T F delta_cam).
 *   cams [n_cam][9], pts [n_pt][3], uv [n_obs][2] (observation order as given
 *   to ba_plan_create); D: optional explicit damping diagonal [9 n_cam + 3 n_pt]
 *   (camera entries first), NULL for D = lambda diag(J^T J). ws: workspace of
 *   ws_bytes >= ba_workspace_bytes(p, o, BA_USE_STEP) bytes, or NULL.
 *   Outputs delta_cam [n_cam][9], delta_pt [n_pt][3]; st (host) may be NULL. */
ba_status ba_lm_step(ba_plan* p, const ba_opts* o, const double* cams, const double* pts,
                     const double* uv, const double* D, void* ws, size_t ws_bytes, double* delta_cam,
                     double* delta_pt, ba_stats* st, void* stream);

/* Gradient of a scalar loss L(delta) of one LM step with respect to the step's
 * inputs, given gd_cam = dL/d delta_cam [n_cam][9] and gd_pt = dL/d delta_pt
 * [n_pt][3]. With mu = H^-1 [gd_cam; gd_pt] (H = J^T J + D, solved with the same
 * Schur system and preconditioner as the forward step, residual and Jacobian
 * recomputed):  dL/du_o = J_o mu_o and
 * dL/dx = -J^T J mu - sum_o sum_r Hess(pi_{o,r}) w_{o,r} (the second-order terms
 * of the reprojection; with D = lambda diag(J^T J) and freeze_damping_in_grad = 0
 * the damping's own dependence on x is included). D: the explicit damping
 * diagonal the forward step was taken with (as in ba_lm_step; a constant, so it
 * contributes no term of its own), or NULL for D = lambda diag(J^T J).
 * delta_cam/delta_pt are the forward outputs. ws: workspace of
 * ba_workspace_bytes(p, o, BA_USE_BACKWARD) bytes, or NULL.
 * Outputs g_cams [n_cam][9], g_pts [n_pt][3], g_uv [n_obs][2]. */
ba_status ba_lm_step_backward(ba_plan* p, const ba_opts* o, const double* cams,
                              const double* pts, const double* uv, const double* D,
                              const double* delta_cam, const double* delta_pt, const double* gd_cam,
                              const double* gd_pt, void* ws, size_t ws_bytes, double* g_cams,
                              double* g_pts, double* g_uv, ba_stats* st, void* stream);

/* ------------------------------------------------------------------------
 * Stage-level entry points. ba_lm_step = ba_step_prepare + ba_step_solve.
 * They expose each stage of the step so that it can be checked on its own.
 * ---------------------------------------------------------------------- */

/* Residual and Jacobian blocks per observation (Section 2.1):
 * f [n_obs][2], F [n_obs][2][9] = d pi/d camera, E [n_obs][2][3] = d pi/d point,
 * in the caller's observation order, without any robust weighting. Any output
 * may be NULL. ws as for ba_lm_step (BA_USE_STEP with default options suffices).
 * The workspace's per-observation buffers are reused, so a step
 * prepared earlier must be prepared again before ba_step_solve,
 * ba_schur_apply, ba_schur_offdiag_apply or ba_precond_apply (they return
 * BA_ERR_ARG until then). */
ba_status ba_eval_jacobian(ba_plan* p, const double* cams, const double* pts, const double* uv,
                           void* ws, size_t ws_bytes, double* f, double* F, double* E, void* stream);

/* Evaluate J, the damped normal blocks (Section 2.1), C^-1, the reduced
 * right-hand side b = -g_c + W C^-1 g_p, the block-Jacobi blocks and, for
 * BA_PC_MULTIGRID, the numeric multigrid setup (near-nullspace QR,
 * Galerkin operators, smoothers, coarse factorization), keeping them in the
 * workspace (ws as for ba_lm_step) for ba_step_solve / ba_schur_apply /
 * ba_precond_apply. */
ba_status ba_step_prepare(ba_plan* p, const ba_opts* o, const double* cams, const double* pts,
                          const double* uv, const double* D, void* ws, size_t ws_bytes, ba_stats* st,
                          void* stream);

/* PCG on S dc = b and back-substitution using the prepared step. */
ba_status ba_step_solve(ba_plan* p, const ba_opts* o, double* delta_cam, double* delta_pt,
                        ba_stats* st, void* stream);

/* y = S x with the implicit product A x - F^T (E (C^-1 (E^T (F x))))
 * (Section 3.6) of the prepared step. precision BA_FP64 or BA_MIXED (FP32
 * operands and accumulation; x, y are still FP64 at this boundary).
 * x, y: [n_cam][9]. Enqueued on `stream`; returns without waiting. */
ba_status ba_schur_apply(ba_plan* p, int32_t precision, const double* x, double* y,
                         void* stream);

/* y <- y - W C^-1 W^T x with W = F^T E: the point-elimination term of the
 * Schur complement S = A - W C^-1 W^T (Section 2.1) alone, as one kernel
 * launch (the implicit product of Section 3.6 without its A x part; in
 * FP64 it recomputes F and E from the prepared cameras and points rather
 * than reading them, with the same arithmetic as the stored blocks).
 * x [n_cam][9] is read, y [n_cam][9] is read and updated. precision as for
 * ba_schur_apply. Enqueued on `stream`; returns without waiting. */
ba_status ba_schur_offdiag_apply(ba_plan* p, int32_t precision, const double* x, double* y,
                                 void* stream);

/* z = M r: one preconditioner application of the prepared step (block Jacobi,
 * or one V-cycle of Algorithm 1 from a zero initial guess). [n_cam][9].
 * Enqueued on `stream`; returns without waiting. */
ba_status ba_precond_apply(ba_plan* p, const ba_opts* o, int32_t precision, const double* r,
                           double* z, void* stream);

/* Reduced right-hand side b [n_cam][9], point blocks C^-1 [n_pt][3][3] and
 * block-Jacobi blocks S_cc [n_cam][9][9] (before inversion) of the prepared
 * step. Any output may be NULL. */
ba_status ba_step_blocks(ba_plan* p, double* b, double* Cinv, double* Scc, void* stream);

/* ---- multigrid hierarchy inspection (after ba_plan_create; numeric parts
 * after ba_step_prepare with BA_PC_MULTIGRID). Sizes are (host) outputs. ---- */

/* Number of levels and nodes per level (nodes: (host) array of >= 16). */
ba_status ba_mg_levels(const ba_plan* p, int32_t* n_levels, int32_t* nodes);

/* Aggregate id of every node of `level` (Algorithm 2; ids in creation order):
 * agg [nodes(level)] int32 (device). Not defined on the coarsest level. */
ba_status ba_mg_aggregates(const ba_plan* p, int32_t level, int32_t* agg);

/* Covisibility counts W of `level` (Section 3.2; coarse levels
 * W_{l+1} = Ahat^T W_l Ahat) in CSR with sorted columns, diagonal included:
 * call with row_ptr == NULL to get *nnz (host); then row_ptr [nodes+1] int64,
 * col [nnz] int32, val [nnz] int64 (device). */
ba_status ba_mg_covisibility(const ba_plan* p, int32_t level, int64_t* nnz, int64_t* row_ptr,
                             int32_t* col, int64_t* val);

/* Numeric hierarchy of the prepared step, FP64:
 *   what = 0: operator of `level` as dense [n][n] (n = nodes*bs; level 0 gives
 *             the explicit S), only for n <= 16384;
 *   what = 1: tentative prolongator blocks P [nodes][bs][16] of `level`;
 *   what = 2: near-nullspace rows K [nodes][bs][16] of `level`;
 *   what = 3: inverse smoother blocks D^-1 [nodes][bs][bs] (not on the coarsest level);
 *   what = 4: lambda_max estimate of D^-1 S (1 value; not on the coarsest level);
 *   what = 5: coarsest level only: inverse of its operator, dense [n][n];
 *   what = 6: plans built for BA_PROLONG_SMOOTHED: the smoothed prolongator of
 *             `level` as dense [nodes*bs][nodes(level+1)*16], only for
 *             nodes*bs <= 16384. */
ba_status ba_mg_level_data(const ba_plan* p, int32_t level, int32_t what, double* out,
                           void* stream);

/* ------------------------------------------------------------------------
 * The Levenberg-Marquardt outer loop around the step (Section 2.1), with the
 * solver settings of Section 5: a trust region whose radius starts at 1e4
 * (damping D = diag(J^T J) / radius) and, with ba_opts.stop_rule =
 * BA_STOP_NASH_SOFER, a constant forcing sequence for the inner PCG. The paper
 * leaves the radius update to its nonlinear solver; this loop takes the update
 * of Madsen, Nielsen and Tingleff (2004), Section 3.2, in radius form.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t max_iters;              /* LM iterations, default 100 (Section 5) */
  int32_t reserved0;
  double radius0;                 /* initial trust-region radius, default 1e4 (Section 5) */
  double min_relative_decrease;   /* accept a step when rho exceeds this, default 1e-3 */
  double function_tol;            /* stop after an accepted step that lowers the cost by at most
                                     function_tol times the previous cost, default 1e-6 */
  double parameter_tol;           /* stop (before evaluating the candidate) when
                                     |delta| <= parameter_tol (|x| + parameter_tol), default 1e-8 */
  double min_radius;              /* stop when a rejection takes the radius below this, default 1e-32 */
  double max_radius;              /* cap of the radius, default 1e16 */
  double reserved[2];
} ba_lm_opts;

enum { BA_TERM_MAX_ITERS = 0, BA_TERM_FUNCTION = 1, BA_TERM_PARAMETER = 2, BA_TERM_RADIUS = 3 };

typedef struct {                  /* (host) one LM iteration */
  double cost;                    /* 1/2 sum_o |f_o|^2 at the start of the iteration */
  double cost_candidate;          /* at x + delta; +inf if the candidate puts a point at or behind an
                                     observing camera, or its cost is not finite */
  double model_decrease;          /* 1/2 |f|^2 - 1/2 |f + J delta|^2 */
  double rho;                     /* (cost - cost_candidate) / model_decrease; -inf if the candidate is
                                     invalid or model_decrease <= 0 */
  double radius;                  /* trust-region radius of this step (lambda = 1 / radius) */
  double step_norm;               /* |delta| over all camera and point parameters */
  int32_t accepted;
  int32_t pcg_iters;              /* PCG iterations of this step's linear solve */
  double t_ms;                    /* time of the iteration */
} ba_lm_iter;

typedef struct {                  /* (host) */
  int32_t iters;                  /* iterations recorded in the history */
  int32_t accepted;               /* accepted steps */
  int32_t termination;            /* BA_TERM_* */
  int32_t pcg_iters;              /* summed over all iterations */
  double cost0, cost;             /* initial and final cost */
  double t_ms;                    /* total time */
} ba_lm_summary;

/* Defaults listed above. (host) lo. */
ba_status ba_lm_opts_default(ba_lm_opts* lo);

/* Cost 1/2 sum_o rho(|pi_o - u_o|^2) at (cams, pts), rho the loss of o (NULL:
 * the squared loss, rho(s) = s), and the number of observations whose point is
 * at or behind the camera (x_cam.z >= 0) or whose residual is not finite
 * (those are left out of the sum). ws: ba_workspace_bytes(p, o, BA_USE_LM)
 * bytes, or NULL; it is bound as a step's workspace, so a prepared step in a
 * different workspace is no longer available afterwards. cost, n_invalid
 * (host); n_invalid may be NULL. Blocks until the values are ready. */
ba_status ba_cost(ba_plan* p, const ba_opts* o, const double* cams, const double* pts, const double* uv,
                  void* ws, size_t ws_bytes, double* cost, int64_t* n_invalid, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ba_cost
 * without a workspace. Its kernels' scratch (camera records, reduction
 * partials and counters) is a static device array of about 6.3 MB that each
 * GPU the library runs on holds until the process ends, which takes plans of
 * at most 32768 cameras (BA_ERR_LIMIT beyond). Every call on one GPU shares
 * that array, so calls that overlap on one GPU (other streams or threads)
 * race. Allocates nothing; otherwise as ba_cost. Blocks. */
ba_status ba_cost_noalloc(ba_plan* p, const ba_opts* o, const double* cams, const double* pts,
                          const double* uv, double* cost, int64_t* n_invalid, void* stream);

/* Levenberg-Marquardt from (cams, pts), updated in place [n_cam][9], [n_pt][3].
 * Each iteration solves one step (as ba_lm_step, with lambda = 1 / radius; the
 * lambda of o is ignored and D = lambda diag(J^T J)), evaluates the model
 * decrease and the candidate's cost, accepts or rejects the candidate and
 * updates the radius. Updates are additive on every parameter. An inner solve
 * that reaches max_iter is used as it stands; a step whose damped system is
 * not numerically positive definite (BA_ERR_NOT_SPD from the step) is a failed
 * step, recorded with an infinite candidate cost and handled as a rejection. o: the linear solver's options;
 * lo: the loop's. ws: ba_workspace_bytes(p, o, BA_USE_LM) bytes, or NULL.
 * history (host) holds lo->max_iters entries or is NULL;
 * summary (host) may be NULL. Returns BA_OK whatever the termination rule.
 * Errors: BA_ERR_GEOMETRY if the initial parameters put a point at or behind
 * an observing camera or are not finite; the errors of ba_lm_step. After an
 * error cams and pts hold the last accepted parameters. Afterwards the plan
 * holds the step prepared at the last iteration's parameters. Blocks. */
ba_status ba_lm_solve(ba_plan* p, const ba_opts* o, const ba_lm_opts* lo, double* cams, double* pts,
                      const double* uv, void* ws, size_t ws_bytes, ba_lm_iter* history,
                      ba_lm_summary* summary, void* stream);

const char* ba_status_str(ba_status e);
const char* ba_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BAMG_H */
