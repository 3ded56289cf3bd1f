/*
 * dnls.h -- C ABI of the batched differentiable nonlinear least-squares
 * (DNLS) inner step on MI355X (gfx950).
 *
 * The calls follow the problem statement of "Theseus: A Library for
 * Differentiable Nonlinear Optimization" (arXiv 2207.09442):
 *   - variables theta_j on Lie groups (SE(2), SE(3)) or R^3 (Section 2, Eq. nls);
 *   - cost functions c_i with scalar cost weights w_i = exp(l_i), residual
 *     r_i = w_i c_i (Eq. nls; Section 3 core API: Variable, CostFunction,
 *     CostWeight, Objective);
 *   - an optimizer: K Gauss-Newton or Levenberg-Marquardt steps
 *     (H + lambda I) delta = g, theta <- theta (-) delta by right retraction
 *     (Section 2 "Solving NLS"), with fixed or adaptive damping or Powell's
 *     dogleg (Section 3 optimizers), optionally Welsch-robust edges;
 *   - an implicit backward through the final iterate (Section 4.3,
 *     Proposition 1), with the factorisation kept from the forward pass
 *     (Section 4.2 "Backward for custom linear solvers"), and the other
 *     backward modes of Section 4.3: direct loss minimisation, unrolled and
 *     truncated differentiation, and Proposition 1 with the exact Hessian.
 *
 * Conventions
 *   SE(3) element storage: 12 doubles, the 3x4 matrix [R | t] row-major.
 *   SE(2) element storage: 4 doubles (x, y, cos theta, sin theta).
 *   Tangent order: [translation; rotation] -- (rho, phi) in R^6 for SE(3),
 *   (rho_x, rho_y, theta) for SE(2).  Perturbations act on the right:
 *   X <- X Exp(xi) (Appendix D, Eq. grad1).
 *   Relative-pose cost of edge (i, j) with measurement Z:
 *     c = Log(Z^-1 X_i^-1 X_j); prior on pose p with target P: c = Log(P^-1 X_p);
 *   pinhole reprojection of world point q by world-to-camera pose T:
 *     c = (fx x/z + cx, fy y/z + cy) - uv with (x, y, z) = R q + t.
 *   All indices are global over the batch and int32; graph b owns the
 *   half-open ranges [off[b], off[b+1]) of every per-graph table.
 *
 * Ownership: the caller owns every device buffer (inputs, outputs,
 * workspaces and the factor cache); the library never frees caller memory.
 * A plan owns only small immutable index tables that it copies to the
 * device at creation and frees in dnls_plan_destroy.  Plans are immutable
 * after creation, so concurrent calls on different streams with distinct
 * workspaces and outputs are allowed -- except for plans made with
 * DNLS_FLAG_GRAPH or DNLS_FLAG_PAIR, which keep launch state (a captured
 * graph, event counters): their calls must not overlap.
 *
 * Errors: argument and HIP runtime errors are returned as dnls_status and
 * described by dnls_last_error() (thread-local).  Numerical failures never
 * abort: they are reported per graph in the status output
 * (DNLS_GRAPH_NOT_PD, DNLS_GRAPH_NONFINITE); a failed graph keeps its last
 * iterate, repeats its last objective value and receives zero gradients
 * (DNLS_GRAPH_TIMEOUT, of the shared-factorisation schedules, leaves the
 * iterate undefined).
 * Kernel launches are asynchronous on the given stream; an asynchronous
 * device fault surfaces at the next synchronising call.
 */
#ifndef DNLS_H
#define DNLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dnls_plan_s* dnls_plan;

typedef enum {
  DNLS_OK = 0,
  DNLS_ERR_INVALID_ARG = 1,
  DNLS_ERR_UNSUPPORTED = 2,
  DNLS_ERR_HIP = 3,
  DNLS_ERR_WORKSPACE = 4,
  DNLS_ERR_NO_FACTOR = 5
} dnls_status;

/* per-graph numerical status written by dnls_solve */
enum { DNLS_GRAPH_OK = 0, DNLS_GRAPH_NOT_PD = 1, DNLS_GRAPH_NONFINITE = 2,
       /* DNLS_FLAG_PAIR: a workgroup of the graph's pair waited for its
        * partner beyond the poll limit (the cooperative launch makes the
        * pair co-resident, so this indicates a fault) */
       DNLS_GRAPH_TIMEOUT = 3 };

typedef enum { DNLS_SE2 = 2, DNLS_SE3 = 3 } dnls_group;

/* Linear solver of the normal equations (Section 4.2):
 *   DENSE  per-graph dense Cholesky of the pose system;
 *   SCHUR  bundle adjustment: points eliminated by the Schur complement,
 *          dense Cholesky of the camera system;
 *   SPARSE per-graph block-sparse supernodal Cholesky of the pose system. */
typedef enum { DNLS_SOLVER_DENSE = 0, DNLS_SOLVER_SCHUR = 1, DNLS_SOLVER_SPARSE = 2 } dnls_solver;

/* FP64: everything in float64.
 * MIXED: inside the K steps, residuals, Jacobians and the J^T J assembly are
 *   float32 with float32 accumulation; damping, factorisation, solves and
 *   retraction stay float64.  With refine > 0 the right-hand side and
 *   `refine` matrix-free float64 residual corrections per step are added (the
 *   factor of the float32-assembled matrix serves as preconditioner).  The
 *   final linearisation, whose factor the implicit backward reuses, is
 *   assembled in float64 in both precisions. */
typedef enum { DNLS_PREC_FP64 = 0, DNLS_PREC_MIXED = 1 } dnls_precision;

/* Problem structure (host pointers, read during dnls_plan_create only). */
typedef struct {
  int32_t batch;              /* B >= 1 graphs */
  int32_t group;              /* dnls_group of the pose variables */
  const int32_t* pose_off;    /* [B+1] pose ranges */
  const int32_t* edge_off;    /* [B+1] relative-pose cost ranges */
  const int32_t* edge_ij;     /* [2*E] (i, j) per edge, both in the edge's graph, i != j */
  const int32_t* prior_off;   /* [B+1] prior cost ranges */
  const int32_t* prior_var;   /* [P] pose of each prior */
  /* bundle adjustment (solver SCHUR), else NULL / 0 */
  const int32_t* point_off;   /* [B+1] R^3 point ranges */
  const int32_t* obs_off;     /* [B+1] observation ranges */
  const int32_t* obs_cam;     /* [O] camera (pose) index */
  const int32_t* obs_pt;      /* [O] point index */
  double fx, fy, cx, cy;      /* pinhole intrinsics */
  double huber_delta;         /* Huber threshold on ||w c|| (> 0), SCHUR only */
} dnls_problem;

/* Schedule of the SPARSE solver's factorisation and triangular solves.
 * WORKGROUP: both with one workgroup per graph (vector in LDS, no launches
 * between tile steps); SWEEPS: one launch per tile column / row with one
 * workgroup per tile, for both; HYBRID: per-column factorisation launches,
 * workgroup solves; PERSISTENT: the whole solve (every step of every graph,
 * linearisation to retraction, and the final linearisation) in one launch
 * of at most one workgroup per resident slot, which take the graphs from a
 * device-memory queue, largest first (Section 4.1 "Batching and
 * vectorization": graphs of uneven size batched in one launch); not with
 * DNLS_FLAG_ADAPTIVE_LM or DNLS_FLAG_DOGLEG, and the plan's solves must not
 * overlap (the queue is the plan's).  AUTO: for graphs of at most 6144
 * (padded) unknowns and 16 tile columns PERSISTENT with a fixed-damping
 * optimizer, else WORKGROUP; for graphs of at most 6144 unknowns beyond 16
 * tile columns BLOCK with float64 and fixed damping, else HYBRID; SWEEPS
 * beyond 6144 unknowns.  WORKGROUP, HYBRID and PERSISTENT
 * on a plan whose graphs exceed 6144 unknowns, and PERSISTENT with adaptive
 * damping or the dogleg, are DNLS_ERR_UNSUPPORTED.
 * BLOCK: the factor in d x d pose blocks (the block-sparse structure of the
 * Gauss-Newton matrix itself, no 48-wide tiles), factored left-looking by
 * levels of the elimination tree (every column of a level at once) with
 * the triangular solves by the same levels, one workgroup per graph, and
 * the whole solve in one persistent launch as PERSISTENT; same limits as
 * PERSISTENT (at most 6144 unknowns per graph, fixed damping). */
typedef enum {
  DNLS_SPSOLVE_AUTO = 0,
  DNLS_SPSOLVE_WORKGROUP = 1,
  DNLS_SPSOLVE_SWEEPS = 2,
  DNLS_SPSOLVE_HYBRID = 3,
  DNLS_SPSOLVE_PERSISTENT = 4,
  DNLS_SPSOLVE_BLOCK = 5
} dnls_sparse_solve;

/* dnls_options.flags */
enum {
  /* SPARSE and SCHUR: record the launch sequence of dnls_solve into a HIP
   * graph on the first call and replay it while the argument pointers stay
   * the same (every pointer of dnls_solve_args, edge_logc and huber_delta
   * included; recaptured when one changes).  The plan then holds mutable
   * state: calls with this flag must not overlap on one plan.  DENSE is a
   * single launch and ignores the flag. */
  DNLS_FLAG_GRAPH = 1,
  /* Every solver: Levenberg-Marquardt with adaptive damping (Sections 2 and 3),
   * starting from options.lambda: after each step the float64 objective is
   * evaluated at the retracted trial point; the step is kept iff it is
   * strictly smaller than the objective at theta_t, and then lambda is
   * divided by 10, otherwise theta_t is restored and lambda is multiplied by
   * 10; lambda stays in [1e-7, 1e7], per graph.  objective[b][t] is the
   * objective at theta_t, so a rejected step repeats it.  SCHUR: the same
   * rule on cameras and points together (lambda on both diagonal blocks). */
  DNLS_FLAG_ADAPTIVE_LM = 2,
  /* Every solver: Powell's dogleg (Section 3 optimizers) with a per-graph trust
   * radius starting at options.trust_radius (> 0): the Gauss-Newton step of
   * H + lambda I if its norm is within the radius, else the gradient cut at
   * the boundary if the Cauchy point alpha g (alpha = g^T g / g^T H g) lies
   * outside, else the point of the segment from alpha g to the Gauss-Newton
   * step at distance radius.  The step is kept iff the float64 objective
   * strictly decreases; with rho = actual / predicted decrease
   * (g^T delta - 1/2 delta^T (H + lambda I) delta) the radius becomes
   * ||delta|| / 4 if rho < 1/4 (or is not a number) and min(2 radius, 1e4)
   * if rho > 3/4 for a step on the boundary.  Excludes
   * DNLS_FLAG_ADAPTIVE_LM.  SCHUR: over cameras and points together (the
   * Gauss-Newton point from the Schur solve, the model's products matrix-free
   * from float64 records).  The mixed path linearises in float64 as well for
   * g and the model (SCHUR: every step in float64). */
  DNLS_FLAG_DOGLEG = 4,
  /* DENSE and SPARSE, fixed damping (not with DNLS_FLAG_ADAPTIVE_LM or
   * DNLS_FLAG_DOGLEG): dnls_solve also stores the iterates theta_0 ..
   * theta_{K-1} in the factor cache (factor_bytes grows by K V 12|4
   * doubles) for the unrolled backward (DNLS_BACKWARD_UNROLL). */
  DNLS_FLAG_KEEP_ITERATES = 8,
  /* DENSE, plain least squares with fixed or adaptive damping: when the
   * device can hold two workgroups per graph at once, dnls_solve runs each
   * graph on a pair of co-resident workgroups (cooperative launch) that
   * share every factorisation, for batches too small to fill the device;
   * otherwise (or with DNLS_FLAG_DOGLEG or Welsch edges) the one-workgroup
   * kernel runs.  SCHUR (without DNLS_FLAG_GRAPH): six co-resident
   * workgroups per problem share the camera-system factorisation when they
   * fit.  Results equal the one-workgroup path's up to rounding.  The plan
   * holds event counters: calls with this flag must not overlap on one
   * plan.  A wait between the workgroups gives up after a poll limit
   * (about a second; the environment variable DNLS_PAIR_SPIN, read at plan
   * creation, sets another count): the graph then gets DNLS_GRAPH_TIMEOUT
   * and undefined poses, and every workgroup exits. */
  DNLS_FLAG_PAIR = 16
};

typedef struct {
  int32_t solver;             /* dnls_solver */
  int32_t precision;          /* dnls_precision */
  int32_t iterations;         /* K >= 0 optimizer steps */
  int32_t refine;             /* 0..4 float64 correction sweeps (MIXED only) */
  double lambda;              /* Levenberg-Marquardt damping >= 0; 0 = Gauss-Newton */
  int32_t sparse_solve;       /* dnls_sparse_solve (SPARSE only) */
  int32_t flags;              /* DNLS_FLAG_* */
  double trust_radius;        /* DNLS_FLAG_DOGLEG: initial trust radius (> 0) */
  int32_t refine_last;        /* MIXED: run the refinement sweeps in the last
                                 refine_last steps only (negative: the first
                                 -refine_last steps; 0 = every step, the
                                 default); the other steps use the float32
                                 step.  Faster, but the float32 steps move
                                 the trajectory (~1e-6 relative after 10 LM
                                 steps of the 64-pose walks, gradients
                                 ~1e-5).  In -iterations..iterations. */
} dnls_options;

/* Arguments of dnls_solve (device pointers unless stated). */
typedef struct {
  double* poses;              /* [V][12|4] in: theta_0, out: theta_K (in place) */
  double* points;             /* [Vp][3] in/out (SCHUR), else NULL */
  const double* edge_meas;    /* [E][12|4] measurements Z */
  const double* edge_logw;    /* [E] log cost weights */
  const double* edge_tau;     /* [E][dof] or NULL: Z <- Z Exp(tau) */
  const double* prior_meas;   /* [P][12|4] prior targets */
  const double* prior_logw;   /* [P] */
  const double* obs_uv;       /* [O][2] measured pixels (SCHUR) */
  const double* obs_w;        /* [O] observation weights (SCHUR) */
  double* objective;          /* [B][K+1] out: S(theta_t) for t = 0..K */
  int32_t* status;            /* [B] out: DNLS_GRAPH_* */
  void* factor;               /* factor cache, factor_bytes, written for dnls_backward */
  void* workspace;            /* solve_ws bytes */
  const double* edge_logc;    /* [E] Welsch log-radii of the edges, or NULL: with
                                 c = exp(logc) an edge contributes
                                 1/2 rho(s) = 1/2 c^2 (1 - exp(-s / c^2)),
                                 s = ||w c_e||^2, and enters the normal
                                 equations reweighted by rho'(s) (first
                                 order).  Pose-graph solvers only. */
  const double* huber_delta;  /* [B] per-problem Huber radius (> 0), or NULL for
                                 the plan's huber_delta (SCHUR only; the
                                 robust kernel's radius as a solve input,
                                 so that it can be learned) */
} dnls_solve_args;

/* Arguments of dnls_backward: everything must be the state left by the
 * dnls_solve call that filled `factor` (same plan, same parameters). */
typedef struct {
  const double* poses;        /* [V][12|4] theta_K */
  const double* points;       /* [Vp][3] (SCHUR) else NULL */
  const double* edge_meas;
  const double* edge_logw;
  const double* edge_tau;     /* may be NULL (tau = 0) */
  const double* prior_meas;
  const double* prior_logw;
  const double* obs_uv;
  const double* obs_w;
  const int32_t* status;      /* [B] from dnls_solve */
  const void* factor;         /* from dnls_solve */
  const double* seed_pose;    /* [V][dof] v = dL/dtheta_K in tangent coordinates */
  const double* seed_point;   /* [Vp][3] or NULL (SCHUR) */
  double* grad_edge_logw;     /* [E] out or NULL */
  double* grad_edge_tau;      /* [E][dof] out or NULL (gradient at tau) */
  double* grad_prior_logw;    /* [P] out or NULL */
  double* grad_obs_w;         /* [O] out or NULL (SCHUR) */
  double* adjoint;            /* [V][dof] out or NULL: u = H*^-1 v (pose part);
                                 left untouched by DNLS_BACKWARD_DLM */
  void* workspace;            /* backward_ws bytes */
  int32_t mode;               /* dnls_backward_mode (0 = implicit) */
  double dlm_eps;             /* DNLS_BACKWARD_DLM: epsilon > 0 */
  int32_t sweeps;             /* DNLS_BACKWARD_EXACT: refinement sweeps in [0, 64] */
  int32_t steps;              /* DNLS_BACKWARD_UNROLL: last steps differentiated, in [1, K] */
  const double* edge_logc;    /* [E] Welsch log-radii as in dnls_solve, or NULL;
                                 not with DNLS_BACKWARD_EXACT / UNROLL
                                 (DNLS_ERR_UNSUPPORTED) */
  double* grad_edge_logc;     /* [E] out or NULL: gradient at the log-radii */
  const double* huber_delta;  /* [B] the per-problem radii given to dnls_solve,
                                 or NULL (SCHUR) */
  double* grad_obs_delta;     /* [O] out or NULL (SCHUR, implicit and DLM):
                                 gradient with respect to each observation's
                                 Huber radius, all equal to the problem's
                                 radius, so their sum over a problem is the
                                 gradient of its radius; zero inside the
                                 quadratic branch (s <= delta^2) */
  double* grad_huber_delta;   /* [B] out or NULL (SCHUR, implicit and DLM):
                                 gradient with respect to each problem's
                                 Huber radius, the sum of its observations'
                                 per-radius gradients, reduced on the device
                                 in a fixed order (needs no grad_obs_delta) */
} dnls_backward_args;

/* dnls_backward_args.mode */
typedef enum {
  /* Proposition 1: u = H*^-1 v with the cached factor (DENSE, FP64 plans:
   * plus one float64 refinement step u += H*^-1 (v - H* u) with H* applied
   * matrix-free; MIXED plans, held to 1e-5 of float64, skip it). */
  DNLS_BACKWARD_IMPLICIT = 0,
  /* Direct loss minimisation (Section 4.3, Appendix G), every solver: one
   * Gauss-Newton step from theta_K on S(theta) + ||eps theta - v/2||^2,
   * (H* + 2 eps^2 I) delta = -g* + eps v, theta_direct = theta_K Exp(delta),
   * then dL/dphi = (dS/dphi(theta_K) - dS/dphi(theta_direct)) / eps for the
   * log-weights and the tangent perturbations tau, with S the objective of
   * Section 2 (costs weighted by exp(2 log w)).  A first-order estimate of
   * the implicit gradient that approaches it linearly as eps -> 0; eps <= 0
   * or non-finite is DNLS_ERR_INVALID_ARG.  DENSE leaves the factor
   * untouched (the new system is factored in the workspace); SPARSE and
   * SCHUR factor it in the factor cache and then re-factor H* there (same
   * kernels and inputs as the solve's final linearisation), so the cache
   * holds the solve's factor again when the call has run.  SCHUR: cameras
   * and points take the step together (2 eps^2 on both diagonal blocks, the
   * point seed as v's point part, zero if NULL), gradients for the
   * observation weights (dS/dw = rho'(s) w |c|^2), the prior log-weights
   * and the observations' Huber radii (dS/ddelta = sqrt(s) - delta outside
   * the quadratic branch).
   * Graphs whose status is not OK get zero gradients. */
  DNLS_BACKWARD_DLM = 1,
  /* Proposition 1 with the exact Hessian of S in place of the Gauss-Newton
   * one (DENSE and SPARSE): Hx = the Hessian of S(theta_K Exp(delta)) at
   * delta = 0, i.e. J^T J plus the second-order terms of the costs
   * (differentiated by dual numbers) and of the retraction.  u = Hx^-1 v is
   * reached by `sweeps` steps of iterative refinement preconditioned by the
   * cached factor, u <- u + H*^-1 (v - Hx u) from u = H*^-1 v (sweeps = 0
   * is the Gauss-Newton result); it converges when the spectral radius of
   * I - H*^-1 Hx is below 1, i.e. for residuals small against the
   * curvature, and each sweep multiplies the error by about that radius.
   * Then the same per-cost VJP.  The adjoint output receives u. */
  DNLS_BACKWARD_EXACT = 2,
  /* Unrolled differentiation (Section 4.3; truncated when steps < K),
   * DENSE and SPARSE plans with DNLS_FLAG_KEEP_ITERATES: reverse sweep through the
   * last `steps` optimizer steps theta_{t+1} = theta_t Exp(-delta_t),
   * delta_t = (H_t + lambda I)^-1 g_t, recomputed in float64 at the kept
   * iterates (the mixed path's float32 assembly is not differentiated), for
   * the seed v = dL/dtheta_K; the parameter gradients sum over those steps
   * and the adjoint output receives dL/dtheta_{K-steps}.  A graph whose
   * solve failed, or whose float64 step matrix is not positive definite,
   * gets zero gradients.  The factor of H* is not read; SPARSE factors the
   * step matrices in the factor cache and then re-factors H* there (same
   * kernels and inputs as the solve's final linearisation). */
  DNLS_BACKWARD_UNROLL = 3
} dnls_backward_mode;

/* Validate the structure and build the plan: per-graph offsets, cost
 * incidence lists, the dense / Schur / supernodal block maps (symbolic
 * analysis, done once per structure).  This is the paper's Objective built
 * from Variables, CostFunctions and CostWeights (Section 3, core API) plus
 * the optimizer's settings (Section 2 "Solving NLS"; Section 3 optimizers);
 * the symbolic work is done once and reused by every numeric call, as the
 * paper's sparse solvers split symbolic and numeric factorisation
 * (Section 4.2; Appendix F).  `problem` and `options` are host pointers
 * read during the call only; *out receives a plan the caller releases with
 * dnls_plan_destroy.  Returns DNLS_ERR_INVALID_ARG on inconsistent offsets
 * or indices, DNLS_ERR_UNSUPPORTED on a combination the library does not
 * implement, DNLS_ERR_HIP if the index tables cannot be copied to the
 * device; *out is left NULL on error. */
dnls_status dnls_plan_create(dnls_plan* out, const dnls_problem* problem,
                             const dnls_options* options);

/* Byte sizes of the caller-owned buffers of a plan (host outputs, any may
 * be NULL): solve_ws, the workspace of dnls_solve; factor_bytes, the factor
 * cache that dnls_solve fills and dnls_backward reads (the factorisation of
 * the final linearisation that the backward reuses, Section 4.2 "Backward
 * for custom linear solvers"); backward_ws, the workspace of dnls_backward.
 * The library allocates none of them: like the paper's sparse solver
 * library, it owns no numeric memory (Appendix F).  Every buffer must be
 * 256-byte aligned.  DNLS_ERR_INVALID_ARG for a NULL plan. */
dnls_status dnls_plan_workspace(dnls_plan plan, size_t* solve_ws, size_t* factor_bytes,
                                size_t* backward_ws);

/* Work of one numeric factorisation of the whole batch, from the symbolic
 * analysis (host values, either pointer may be NULL).  algorithmic: the
 * block Cholesky of each graph's d x d block pattern with its fill in the
 * plan's elimination order (DENSE: (6N)^3/3 per graph, SCHUR: the camera
 * system), i.e. the flops the method needs (Section 4.2); executed: what the
 * kernels run, padded panels and whole tiles included. */
dnls_status dnls_plan_flops(dnls_plan plan, double* algorithmic, double* executed);

/* The schedule a plan resolved at creation (host values, either pointer may
 * be NULL): dense_pair = 1 if dnls_solve shares each factorisation among
 * co-resident workgroups (DNLS_FLAG_PAIR requested and they fit: a pair per
 * graph for DENSE, six per problem for SCHUR), else 0;
 * sparse_solve = the dnls_sparse_solve that AUTO resolved to (SPARSE), else
 * DNLS_SPSOLVE_AUTO. */
dnls_status dnls_plan_schedule(dnls_plan plan, int32_t* dense_pair, int32_t* sparse_solve);

/* Run K optimizer steps and the final linearisation on `stream` (a
 * hipStream_t, NULL = default stream): per step, cost evaluation, the
 * weighted normal equations, damping, factorisation, the step and the
 * retraction (Section 2 "Solving NLS", Eq. nls; Section 3 optimizers), then
 * the undamped linearisation at theta_K whose factor goes to args->factor
 * for the backward (Section 4.2).  Enqueues kernels only: the caller's
 * buffers must stay valid until the stream reaches them.  Returns
 * DNLS_ERR_INVALID_ARG for a missing required pointer,
 * DNLS_ERR_WORKSPACE for a misaligned factor or workspace,
 * DNLS_ERR_UNSUPPORTED for an input the plan's solver does not take,
 * DNLS_ERR_HIP if a launch fails; numerical failures go to args->status. */
dnls_status dnls_solve(dnls_plan plan, const dnls_solve_args* args, void* stream);

/* dnls_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, with the solve workspace taken from a
 * 256 MiB array inside the library instead of args->workspace, which must
 * be NULL.  Each device the library runs on holds its own copy of that
 * array until the process ends; its address is looked up once per device,
 * on the first call there, with that device current (the current device
 * must be the plan's and the stream's).  The call allocates nothing itself
 * and asks for no HIP graph.  Every call on a device shares that device's
 * array and nothing in it needs to start at zero (the solve writes before
 * it reads), so calls that overlap on one device (other streams, other
 * threads) race and must be serialised by the caller; the other buffers
 * (poses, factor cache, outputs) are the caller's as for dnls_solve, and
 * dnls_backward afterwards takes its own workspace as usual.  Returns
 * DNLS_ERR_INVALID_ARG if args->workspace is not NULL, DNLS_ERR_WORKSPACE
 * if the plan's solve_ws exceeds 256 MiB, DNLS_ERR_UNSUPPORTED for a plan
 * made with DNLS_FLAG_GRAPH, DNLS_ERR_HIP if the array's address cannot be
 * obtained; otherwise as dnls_solve. */
dnls_status dnls_solve_noalloc(dnls_plan plan, const dnls_solve_args* args, void* stream);

/* Implicit backward (Section 4.3, Proposition 1 and its proof in Appendix
 * H): u = H*^-1 v with the cached factor of the undamped Gauss-Newton
 * Hessian at theta_K (Section 4.2 "Backward for custom linear solvers"),
 * then dL/dphi = -d/dphi [u^T g(theta_K; phi)] for the log-weights, the
 * measurement tangent perturbations and the observation weights; or the
 * other modes of dnls_backward_mode.  Enqueues kernels only; outputs that
 * are NULL are skipped.  Returns DNLS_ERR_INVALID_ARG for a missing
 * required pointer or a bad mode parameter, DNLS_ERR_UNSUPPORTED for a mode
 * the plan's solver does not have, DNLS_ERR_HIP if a launch fails.  Graphs
 * whose status is not OK get zero gradients. */
dnls_status dnls_backward(dnls_plan plan, const dnls_backward_args* args, void* stream);

/* Projection operator of Appendix D: tangent gradient
 * v_k = <G, d/ds X Exp(s e_k)|_{s=0}> of a Euclidean gradient G given on the
 * element storage.  poses, grad: [n][12|4]; out: [n][dof] (device). */
dnls_status dnls_project_grad(int32_t group, int64_t n, const double* poses,
                              const double* grad, double* out, void* stream);

/* Free the plan's device tables and launch state (the caller's buffers
 * are not touched).  It waits for the plan's own work on the device to
 * finish first, so it may be called right after dnls_solve or
 * dnls_backward were enqueued.  NULL is accepted.  The paper's layer is a
 * Python object; this is its explicit end of life for C callers. */
dnls_status dnls_plan_destroy(dnls_plan plan);

/* Message of the last error on this thread ("" if none). */
const char* dnls_last_error(void);

/* Library version string. */
const char* dnls_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DNLS_H */
