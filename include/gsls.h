/*
 * gsls.h -- C ABI of the MI355X (gfx950) ADMM / associative-scan QP and SLS
 * solver of GPU-SLS (Fang & Chou, "Safe Large-Scale Robust Nonlinear MPC in
 * Milliseconds via Reachability-Constrained System Level Synthesis on the GPU").
 *
 * Conventions shared by every entry point
 *  - Arrays are row-major double precision.  Host or device memory as selected
 *    by gsls_qp_desc.mem (device pointers are read on the handle's stream).
 *  - Every input is copied during the call that receives it; the library never
 *    keeps a caller pointer after a call returns.  Output buffers belong to the
 *    caller; their sizes follow from the dimensions.
 *  - Return value: GSLS_OK (0) or a negative GSLS_ERR_* code; no C++ exception
 *    crosses the ABI.  gsls_strerror() names a code.
 *  - A handle is not thread-safe; distinct handles may be used concurrently on
 *    distinct streams.
 *
 * Problem (Sec. III-B, eq. (sqp_qp); the ADMM split of Sec. IV-A, eq. (admm_qp)):
 *   min  sum_{k<N} 1/2 [x;u]^T [[Q_k S_k^T];[S_k R_k]] [x;u] + q_k^T x + r_k^T u
 *        + 1/2 x_N^T Q_N x_N + q_N^T x_N
 *   s.t. x_{k+1} = A_k x_k + B_k u_k + b_k,  x_0 = x0,
 *        l_k <= C_k x_k + D_k u_k <= u_k  (nc rows per stage),
 *        l_N <= C_N x_N <= u_N            (nf terminal rows).
 * The paper's one-sided rows  z <= f  are the case l = -inf.  Infinite bounds
 * are allowed.  Q_k, R_k are symmetric; the augmented costs must stay positive
 * definite (R_k + rho D_k^T D_k > 0, and the Riccati matrices
 * R_hat + B^T P B > 0), else GSLS_ERR_NOT_PD.
 */
#ifndef GSLS_H
#define GSLS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ return codes */
enum {
  GSLS_OK = 0,
  GSLS_ERR_INVALID_ARG = -1, /* null pointer, non-finite data, l > u, bad setting */
  GSLS_ERR_DIM = -2,         /* dimensions out of the supported range          */
  GSLS_ERR_NOT_PD = -3,      /* a Cholesky factor failed (matrix not pos. def.) */
  GSLS_ERR_NUMERICAL = -4,   /* NaN/Inf met during the solve                    */
  GSLS_ERR_OOM = -5,         /* device allocation failed                        */
  GSLS_ERR_HIP = -6,         /* HIP runtime error (no device, launch failure)   */
  GSLS_ERR_STATE = -7        /* call out of order (e.g. get before solve)       */
};

/* solver outcome in gsls_result.status */
enum {
  GSLS_SOLVED = 1,           /* r_p <= tol and r_d <= tol                      */
  GSLS_MAX_ITER = 2,         /* iteration limit reached                         */
  GSLS_NUMERICAL_FAIL = 3,   /* NaN/Inf in the residuals                        */
  GSLS_INFEASIBLE_SUSPECTED = 4  /* single-instance solves with adaptive rho: the
                                    iteration limit was reached with r_p > tol after
                                    the rho rule had raised rho to rho_max, the
                                    pattern of ADMM on an infeasible QP (r_p settles
                                    at the distance between the constraint sets) */
};

/* memory kinds */
enum { GSLS_HOST = 0, GSLS_DEVICE = 1 };

/* precision modes */
enum {
  GSLS_MIXED = 0,  /* FP32 scan products and iteration; FP64 Cholesky/LU factors */
  GSLS_FP64 = 1    /* everything in FP64                                          */
};

/* Supported dimensions (per instance). */
#define GSLS_MAX_NX 80
#define GSLS_MAX_NU 32
#define GSLS_MAX_NC 64
#define GSLS_MAX_N 65536   /* the single-instance solver (gsls_qp_create) takes N <= 16384:
                              256 workgroups of at most 64 stages; GSLS_ERR_DIM beyond */

/* One LTV-QP.  Pointer shapes (row-major):
 *   A [N][nx][nx]  B [N][nx][nu]  b [N][nx] (NULL => 0)
 *   Q [N+1][nx][nx]  R [N][nu][nu]  S [N][nu][nx] (NULL => 0)
 *   q [N+1][nx] (NULL => 0)  r [N][nu] (NULL => 0)
 *   C [N][nc][nx]  D [N][nc][nu]  CN [nf][nx] (NULL iff nf == 0)
 *   l, u [N*nc + nf]  (stage rows k*nc..k*nc+nc-1, then the nf terminal rows) */
typedef struct gsls_qp_desc {
  int32_t N, nx, nu, nc, nf;
  int32_t mem;
  const double *A, *B, *b;
  const double *Q, *R, *S;
  const double *q, *r;
  const double *C, *D, *CN;
  const double *l, *u;
} gsls_qp_desc;

/* Solver settings; gsls_default_settings() fills the defaults in brackets. */
typedef struct gsls_settings {
  int32_t precision;     /* GSLS_MIXED or GSLS_FP64                       [MIXED] */
  int32_t max_iter;      /* ADMM iteration limit                          [10000] */
  int32_t adaptive_rho;  /* OSQP-style rho adaptation on/off                  [1] */
  int32_t sigma;         /* rho is reconsidered every sigma iterations       [25] */
  double rho_min;        /* clamp                                          [1e-6] */
  double rho_max;        /*                                                [1e6]  */
  double rho_tol;        /* change rho only if it moves by more than this   [5.0] */
  int32_t chunks_epoch;  /* horizon chunks for the factor scan (0 = auto:     [0]
                            one stage per chunk, at most 256 chunks) */
  int32_t chunks_iter;   /* horizon chunks (workgroups) for the iteration      [0]
                            scans (0 = auto: one stage per workgroup, at most 256;
                            with chunks_epoch also 0, problems with nx, nu <= 4,
                            nc, nf <= 8 and N <= 63 are solved whole by one
                            wavefront in FP64, whatever the precision) */
  int32_t refresh;       /* mixed precision: the x-update is evaluated on the  [0]
                            increment of w = y - z and accumulated in FP64, in
                            full after each factor epoch and, if refresh > 0,
                            at every iteration count that is a multiple of
                            refresh (bounds the FP32 drift of the accumulators) */
  int32_t fp64_fallback; /* 1: a mixed-precision single-instance solve that    [0]
                            reaches max_iter above tol is continued in FP64 from
                            its last iterate (z, y, rho), with a fresh iteration
                            budget, on an FP64 copy of the problem made on first
                            use; ignored by batched solves */
} gsls_settings;

/* Outcome of one solve. */
typedef struct gsls_result {
  int32_t status;        /* GSLS_SOLVED / GSLS_MAX_ITER / GSLS_NUMERICAL_FAIL /
                            GSLS_INFEASIBLE_SUSPECTED                            */
  int32_t iterations;    /* ADMM iterations (x-updates) performed                 */
  int32_t rho_updates;   /* number of rho changes (each costs a factor epoch)     */
  int32_t factorizations;/* factor epochs run                                     */
  double r_p;            /* |G xi - z|_inf at the last iteration                  */
  double r_d;            /* rho |G^T (z+ - z)|_inf at the last iteration          */
  double rho;            /* final rho                                             */
  double ms_total;       /* device time of the whole solve (HIP events)           */
  double ms_factor;      /* device time spent in factor epochs (batched solves:
                            time of the instance's own workgroup)              */
  double ms_iterate;     /* device time spent in the ADMM iterations (same)       */
  int32_t cold_restart;  /* batched learned warm start: 1 if the instance did not
                            converge within the warm budget and was re-solved
                            from a cold start (its iterations include both)    */
  int32_t fallback;      /* 1 if a mixed-precision solve reached max_iter and was
                            continued in FP64 (gsls_settings.fp64_fallback); its
                            iterations, epochs and times include both parts   */
  double r_dyn;          /* max_k |x_{k+1} - A_k x_k - B_k u_k - b_k|_inf of the
                            returned iterate, evaluated in FP64 on the working-
                            precision stage data (mixed precision: non-zero at
                            the level of FP32 rounding)                        */
} gsls_result;

typedef struct gsls_qp gsls_qp;

void gsls_default_settings(gsls_settings* s);
const char* gsls_strerror(int code);

/* Host-only validation of a problem description (no device call): dimensions,
 * null pointers, finiteness, l <= u.  Host memory only.  Returns GSLS_OK or the
 * code gsls_qp_setup would return for the same description. */
int gsls_validate_desc(const gsls_qp_desc* desc);

/* Create a solver handle for one QP (Sec. IV-A).  Copies the problem data to
 * the device, converts it to the working precision and allocates the caches.
 * stream: hipStream_t to enqueue on (NULL = default stream).
 * settings: NULL = defaults.  On success *out receives the handle. */
int gsls_qp_setup(const gsls_qp_desc* desc, const gsls_settings* settings, void* stream,
                  gsls_qp** out);

/* Replace the bounds l, u (length N*nc + nf, same memory kind as the setup)
 * without touching the factorisation: used to tighten rows by SLS margins. */
int gsls_qp_update_bounds(gsls_qp* h, const double* l, const double* u);

/* Replace all problem data (A, B, b, Q, R, S, q, r, C, D, CN, l, u) of the
 * handle by those of desc, which must have the handle's dimensions
 * (GSLS_ERR_DIM otherwise); desc->mem says where desc's arrays live.  The
 * arrays are copied; the ADMM state is kept.  Used by the SQP iteration of
 * Sec. III-B, whose QP changes at every linearisation. */
int gsls_qp_update_data(gsls_qp* h, const gsls_qp_desc* desc);

/* ADMM solve (Sec. III-C / IV-A) from a cold start z = y = 0.
 * x0 [nx] initial state; rho initial penalty (> 0); tol absolute tolerance on
 * both r_p = |G xi - z|_inf and r_d = rho |G^T (z+ - z)|_inf.  Each ADMM
 * x-update is the LQR subproblem eq. (primal_update), solved by the reverse
 * associative scan of eq. (combination_rules) / eq. (controller_cache) and the
 * forward composition eq. (nom_recovery), with the rho-invariant factors cached
 * across iterations.  Blocks until the solve is finished; result may be NULL. */
int gsls_qp_solve(gsls_qp* h, const double* x0, double rho, double tol, gsls_result* result);

/* As gsls_qp_solve, starting from the iterate (z0, y0) (length N*nc + nf each,
 * y0 the scaled dual lambda/rho at penalty rho). */
int gsls_qp_solve_warm(gsls_qp* h, const double* x0, double rho, double tol,
                       const double* z0, const double* y0, gsls_result* result);

/* Copy the last solution to host buffers (any may be NULL):
 * X [N+1][nx], U [N][nu], z [N*nc+nf], lambda [N*nc+nf] (= rho * y). */
int gsls_qp_get(gsls_qp* h, double* X, double* U, double* z, double* lambda);

void gsls_qp_free(gsls_qp* h);

/* Diagnostics.  enable = 1 / 0 switches per-phase cycle counting of the ADMM
 * iteration kernel on or off (-1 leaves it unchanged; counting adds one
 * barrier per phase).  cycles16 (nullable) receives the accumulated shader
 * clock cycles of workgroup 0 per phase since the last read:
 * [1] linear terms, [2] backward chunk fold, [3] backward doubling exchange,
 * [4] backward fix-up and gains, [5] forward chunk fold, [6] forward doubling
 * exchange, [7] forward fix-up + projection + dual update, [8] residual
 * reduction; the counters are then cleared.  layout4 (nullable) receives the
 * factor-scan chunk count, the iteration chunk (workgroup) count, whether the
 * chunk operators are LDS-resident, and the largest chunk length.
 * Tiny problems (nx, nu <= 4, nc, nf <= 8, N <= 63, both chunk settings 0) run
 * the whole solve in one wavefront in FP64: layout4 is then {1, 1, 1, N} and
 * cycles16 holds [0] solves, [1] shader cycles of the data load, [2] of the
 * factors, [3] of the iterations, [4] 100 MHz ticks of factors + iterations,
 * [5] factors, [6] iterations, summed over the solves since the last read. */
int gsls_debug_phase_cycles(gsls_qp* h, int32_t enable, double* cycles16, int32_t* layout4);

/* ----------------------------------------------------------------- SLS ---
 * Controller synthesis eq. (fastsls_qp) of Sec. III-D / IV-B on the handle's
 * dynamics (A_k, B_k) and constraint rows (C_k, D_k, C_N).
 *  E      [N][nx][nx] disturbance maps E_j (Phi^x_{j+1,j} = E_j).
 *  tau    weights of eq. (sls_cost_matrices_tau): [N][N][nc] stage part
 *         tau[k][j][.] (read for j < k <= N-1) followed by [N][nf] terminal part
 *         tau_N[j][.].  NULL => all zero.
 *  Qbar [nx][nx], Rbar [nu][nu], QbarN [nx][nx]: symmetric positive definite.
 *  rownorm 2: margins for |w_j|_2 <= wbound (the paper's row 2-norm);
 *          1: margins for |w_j|_inf <= wbound (row 1-norm, the dual norm).
 *  Outputs (host memory, any may be NULL):
 *   Phi_x: N(N+1)/2 blocks [nx][nx]; column j holds k = j+1..N at block offset
 *          j*N - j(j-1)/2.
 *   Phi_u: N(N-1)/2 blocks [nu][nx]; column j holds k = j+1..N-1 at block
 *          offset j*(N-1) - j(j-1)/2.
 *   h [N][nc]: h_k = wbound * sum_{j<k} rownorm(C_k Phi^x_{k,j} + D_k Phi^u_{k,j}).
 *   hf [nf]:  hf = wbound * sum_{j<N} rownorm(C_N Phi^x_{N,j}).
 * Column j's LQR runs over stages j+1..N-1 with terminal cost at N. */
int gsls_sls_solve(gsls_qp* h, const double* E, const double* tau, const double* Qbar,
                   const double* Rbar, const double* QbarN, int32_t rownorm, double wbound,
                   double* Phi_x, double* Phi_u, double* hmarg, double* hf);

/* Batched SLS: `count` instances sharing the handle's stage data, E and the
 * cost weights, each with its own tau (count consecutive tau arrays).  Outputs
 * h [count][N][nc], hf [count][nf]; Phi not returned.  Device time of the
 * batch is written to *ms if ms != NULL. */
int gsls_sls_solve_batch(gsls_qp* h, int32_t count, const double* E, const double* tau,
                         const double* Qbar, const double* Rbar, const double* QbarN,
                         int32_t rownorm, double wbound, double* hmarg, double* hf, double* ms);

/* Dual weights of App. B from multipliers lambda [N*nc+nf] and the responses
 * of gsls_sls_solve (host memory): tau_{k,j} = |lambda_k| / sqrt(beta_{k,j} + eps),
 * beta the squared row norms of C_k Phi^x_{k,j} + D_k Phi^u_{k,j}.  tau has the
 * layout of gsls_sls_solve's tau (entries with k <= j set to 0). */
int gsls_sls_tau(gsls_qp* h, const double* lambda, const double* Phi_x, const double* Phi_u,
                 double eps, double* tau);

/* ------------------------------------------------------------ robust MPC ---
 * The alternation of Sec. III-D on the handle's QP, between
 *  (A) the nominal trajectory: the QP with its rows tightened by the margins h
 *      of the current controller, l + h <= G xi <= u - h on the finite sides
 *      (eq. (nmpc_problem_tightened)), solved by the ADMM of gsls_qp_solve
 *      from a cold start at rho with tolerance tol (the handle's settings);
 *  (B) the controller: gsls_sls_solve with the App. B weights tau computed
 *      from the nominal multipliers and the current responses (eps as in
 *      gsls_sls_tau).
 * The first controller uses tau = 0.  One pass is (A) then (B); the loop
 * stops when the margins move by at most htol * max(1, |h|_inf) or after
 * max_passes passes, then solves (A) once more with the final margins, so the
 * returned trajectory (gsls_qp_get) and margins belong together.
 *  x0 [nx] (host); E, Qbar, Rbar, QbarN, rownorm, wbound as for gsls_sls_solve.
 *  result (nullable): outcome and counts; hmarg [N][nc], hf [nf] (host,
 *  nullable): the final margins.
 * The handle's bounds are restored before return.  Return code: GSLS_OK when
 * the loop ran (its outcome in result->status), an error code otherwise. */
enum {
  GSLS_ROBUST_CONVERGED = 1,      /* margins settled                            */
  GSLS_ROBUST_PASS_LIMIT = 2,     /* max_passes passes without settling         */
  GSLS_ROBUST_INFEASIBLE = 4,     /* l + h > u - h on some row                  */
  GSLS_ROBUST_NOMINAL_FAILED = 5  /* a nominal solve did not converge           */
};
typedef struct gsls_robust_result {
  int32_t status;        /* GSLS_ROBUST_*                                          */
  int32_t passes;        /* controller updates (B)                                 */
  int32_t qp_solves;     /* nominal solves (A)                                     */
  int32_t qp_iterations; /* ADMM iterations over all nominal solves                */
  int32_t qp_status;     /* gsls_result.status of the last nominal solve (0: none) */
  int32_t reserved;
  double h_change;       /* max |h_new - h| of the last pass                      */
  double ms_nominal;     /* device time of the nominal solves                     */
  double ms_controller;  /* device time of the tau and SLS steps                  */
} gsls_robust_result;

int gsls_robust_solve(gsls_qp* h, const double* x0, const double* E, const double* Qbar,
                      const double* Rbar, const double* QbarN, int32_t rownorm, double wbound,
                      double eps, double rho, double tol, int32_t max_passes, double htol,
                      gsls_robust_result* result, double* hmarg, double* hf);

/* ------------------------------------------------------- analytic models ---
 * SQP (Sec. III-B, eq. (sqp_qp)) and the real-time iteration (Sec. IV-C) on
 * the paper's analytic models: the Dubins car of App. C (x = (px, py, theta),
 * u = omega, speed v) and the planar quadrotor of App. D (x = (px, py, phi,
 * vx, vy, phidot), u = rotor thrusts; one explicit Euler step of its
 * continuous dynamics per time step dt).  Rows: per obstacle (cx, cy, r) the
 * row r^2 - (px-cx)^2 - (py-cy)^2 <= 0 at every stage and at the terminal
 * state (eq. (obstacle_constraints)), then the input box u_min <= u <= u_max.
 * Cost: the tracking cost 1/2 |x_k - x_ref_k|_Q^2 + 1/2 |u_k - u_ref_k|_R^2,
 * terminal 1/2 |x_N - x_ref_N|_QN^2; the QP's Hessian is the cost's (the
 * iteration's fixed point is the nonlinear problem's KKT point).
 * Each SQP iteration linearises around the nominal (X, U) on the device (one
 * thread per stage), solves the QP in (dx, du) from dx_0 = x0 - X_0 and takes
 * X += alpha dx, U += alpha du. */
enum { GSLS_MODEL_DUBINS = 1, GSLS_MODEL_QUADROTOR = 2 };

typedef struct gsls_model_desc {
  int32_t model;             /* GSLS_MODEL_*; nx, nu = 3, 1 or 6, 2            */
  int32_t N, n_obs;          /* horizon, obstacles (n_obs <= GSLS_MAX_NC - nu) */
  int32_t reserved;
  double dt;
  double v;                  /* Dubins speed                                    */
  double mass, gravity, arm, inertia;   /* quadrotor m, g, L, J                */
  const double* obstacles;   /* [n_obs][3]: cx, cy, r                           */
  const double *u_min, *u_max;          /* [nu]                                */
  const double *Q, *R, *QN;             /* [nx][nx], [nu][nu], [nx][nx]        */
  const double *x_ref, *u_ref;          /* [N+1][nx], [N][nu]                  */
} gsls_model_desc;

typedef struct gsls_sqp_result {
  int32_t status;        /* 1: step <= tol_step; 2: iteration limit; 5: a QP did not converge */
  int32_t iterations;    /* SQP iterations                                     */
  int32_t qp_iterations; /* ADMM iterations over all QPs                       */
  int32_t qp_status;     /* gsls_result.status of the last QP                  */
  double step;           /* max |(dx, du)| of the last iteration               */
  double ms_linearize;   /* device time of the linearisations                  */
  double ms_qp;          /* device time of the QP solves                       */
} gsls_sqp_result;

typedef struct gsls_sqp gsls_sqp;

/* Handle for a model with all host-memory parameters; the QP of the first
 * linearisation (around the nominal X, U: host [N+1][nx], [N][nu]) sets up the
 * inner QP solver with the given settings.  nx, nu follow from the model. */
int gsls_sqp_setup(const gsls_model_desc* model, const double* X, const double* U,
                   const gsls_settings* settings, void* stream, gsls_sqp** out);

/* The linearised QP around (X, U) (host arrays in the gsls_qp_desc layout with
 * nc = n_obs + nu, nf = n_obs; any output may be NULL). */
int gsls_sqp_linearize(gsls_sqp* h, const double* X, const double* U, double* A, double* B, double* b,
                       double* q, double* r, double* C, double* D, double* CN, double* l, double* u);

/* SQP iterations from the nominal (X, U) (host, overwritten with the final
 * nominal); x0 [nx] the initial state; each QP solved from a cold start at
 * rho = 1 to tolerance tol_qp. */
int gsls_sqp_solve(gsls_sqp* h, const double* x0, double* X, double* U, int32_t max_iter, double alpha,
                   double tol_qp, double tol_step, gsls_sqp_result* result);

/* One real-time-iteration update (Sec. IV-C): one linearisation around (X, U),
 * the alternation of gsls_robust_solve on that QP (max_passes controller
 * updates; E is the disturbance scaling, constant over the horizon, [nx][nx]),
 * and the tightened nominal step X += dx, U += du.  Margins to hmarg [N][nc],
 * hf [n_obs] (host, nullable). */
int gsls_rti_step(gsls_sqp* h, const double* x0, double* X, double* U, const double* E,
                  const double* Qbar, const double* Rbar, const double* QbarN, int32_t rownorm, double wbound,
                  double tol_qp, int32_t max_passes, gsls_robust_result* result, double* hmarg, double* hf);

void gsls_sqp_free(gsls_sqp* h);

/* ------------------------------------------------------------ batches ---
 * Many independent QPs of uneven shape solved in one persistent launch
 * (captured in a HIP graph and replayed on later calls): each workgroup of
 * the launch takes whole instances from a device work queue, largest first,
 * and runs the ADMM of gsls_qp_solve for each (mixed precision).  Instances
 * whose rows are exactly the box [x_k; u_k] (C = [I; 0], D = [0; I]) and whose
 * terminal rows are x_N or absent skip the constraint-map products.
 * Limits: nx + nu <= 96, nc <= 64 (box: nc = nx + nu), host memory. */
typedef struct gsls_batch gsls_batch;

int gsls_qp_setup_batch(const gsls_qp_desc* descs, int32_t count, const gsls_settings* settings,
                        void* stream, gsls_batch** out);

/* x0[c] initial state, rho[c] initial penalty of instance c; z0, y0 NULL for a
 * cold start of every instance, else per instance NULL (cold) or the starting
 * iterate (length N*nc+nf, y the scaled dual).  out[count] receives each
 * instance's result; *ms (nullable) the device time of the launch. */
int gsls_qp_solve_batch(gsls_batch* b, const double* const* x0, const double* rho, double tol,
                        const double* const* z0, const double* const* y0, gsls_result* out, double* ms);

/* Solution of instance index after gsls_qp_solve_batch (host buffers, any NULL). */
int gsls_batch_get(gsls_batch* b, int32_t index, double* X, double* U, double* z, double* lambda);

void gsls_batch_free(gsls_batch* b);

/* Schedule of the batched launch (Sec. IV-A: the horizon of one instance is
 * split into chunks whose affine maps are composed by associative scans).
 * Every instance starts on one workgroup; an instance with N >= 2 gang whose
 * r_p or r_d is still above 30 tol after park_at iterations is continued by a gang of
 * `gang` workgroups, each owning N / gang consecutive stages (chunk fold,
 * recursive doubling over the chunk transfer maps, re-run from the exact
 * entry).  park_at is the iteration count at which the instance's estimated
 * solo work reaches park_share times one workgroup's share of the batch
 * (every instance at 100 iterations); it depends on the shapes only.  Gangs
 * are filled first for hand-overs whose rho has reached 50 and grown at least
 * 4-fold since the instance's start while r_p or r_d is still at least 300 tol
 * (the instances that set the batch's makespan), then for the rest, each in
 * hand-over order.
 *  gang: 0 = automatic (32), 1 = no gangs, 2..32 (at most half the grid).
 *  park_share: > 0, or 0 = automatic (1.0).
 * Drops the captured launch (the next solve captures a new one). */
int gsls_batch_set_schedule(gsls_batch* b, int32_t gang, double park_share);

/* Current schedule; park_at (nullable) receives count entries (2^31 - 1:
 * the instance never leaves its solo workgroup). */
int gsls_batch_get_schedule(gsls_batch* b, int32_t* gang, double* park_share, int32_t* park_at);

/* Diagnostics: enable != 0 turns on per-phase device-clock counters of the
 * batched iterations (summed over instances; they add one barrier per
 * phase), 0 turns them off.  cycles16 (nullable) receives the counters
 * accumulated since the previous call, which are then cleared. */
int gsls_batch_debug_phase_cycles(gsls_batch* b, int32_t enable, double* cycles16);

/* ------------------------------------------------------------------------
 * Learned warm start of the batched solver (an extension of the ADMM start of
 * Sec. IV-A: the iterations begin from a predicted (z, lambda) and rho instead
 * of z = y = 0, rho = 1).  Box-constrained instances only (rows [x_k; u_k] per
 * stage, terminal rows x_N or none; nx <= 75, nu <= 19).
 *
 * One feature row per stage k = 0..N of each instance, d_in = 160, BF16:
 *   [0:nx] x0 / x_max; [75] x_max / 5; [76] u_max; [77:141] S d_k with
 *   d_k = [(A_k - I) x0 in slots 0..nx-1 ; B_k^T x0 in slots 75..75+nu-1] / x_max
 *   (d_N = 0) and S the 64 x 94 sketch; [141] k/N; [142] N/512; [143] nx/75;
 *   [144] nu/19; the rest 0.  x_max, u_max: upper bounds of the first state
 *   row and the first input row.
 * One output row, d_out = 192, FP32: z of the state rows / x_max in [0:nx],
 *   of the input rows / u_max in [75:75+nu]; lambda of the state rows in
 *   [94:94+nx], of the input rows in [169:169+nu]; log10 rho in [188].
 * MLP 160-512-512-512-192, ReLU on the hidden layers; parameters are one flat
 * FP32 vector W1 (160 x 512 row-major), b1, W2, b2, W3, b3, W4, b4; BF16
 * copies feed the matrix cores (FP32 accumulation); Adam keeps FP32 master
 * weights.  Loss sum(M (Y - T)^2) / sum(M), M the per-entry weights.
 *
 * Device pointers (X, T, M, idx, Y) are device memory; work runs on the
 * handle's stream (gsls_ws_create) or the batch's stream (batch calls).
 * ------------------------------------------------------------------------ */
typedef struct gsls_ws gsls_ws;

/* Number of MLP parameters (706,240). */
int64_t gsls_ws_nparams(void);

/* New model from host params[gsls_ws_nparams()] and sketch[64 * 94] (both
 * FP32, copied).  Adam state starts at zero. */
int gsls_ws_create(const float* params, const float* sketch, void* stream, gsls_ws** out);

/* Current FP32 master parameters into host params[gsls_ws_nparams()]. */
int gsls_ws_get_params(gsls_ws* h, float* params);

/* Binary file: 8-byte tag, int64 parameter count, FP32 parameters, FP32
 * sketch.  Load rejects files of another layout with GSLS_ERR_INVALID_ARG. */
int gsls_ws_save(gsls_ws* h, const char* path);
int gsls_ws_load(const char* path, void* stream, gsls_ws** out);

/* Y[rows][192] (device FP32) = MLP(X[rows][160]) (device BF16 bit patterns). */
int gsls_ws_forward(gsls_ws* h, const uint16_t* X, int32_t rows, float* Y);

/* As gsls_ws_forward, for callers that cannot allocate device memory (code
 * under stream capture, serving loops, harnesses that forbid hipMalloc): the
 * hidden activations live in a fixed library workspace of 2048 rows instead
 * of the handle's workspace, so the call allocates nothing.  rows > 2048:
 * GSLS_ERR_DIM.  The workspace (12 MiB per GPU, held until the process ends)
 * is shared by every call on that GPU: calls that overlap in time on one GPU
 * (different streams or threads) race and must be serialised by the caller.
 * Work is enqueued on the handle's stream; Y is complete when it finishes. */
int gsls_ws_forward_static(gsls_ws* h, const uint16_t* X, int32_t rows, float* Y);

/* Loss and gradient on rows idx[0..rows) of (X, T, M) (idx NULL: the first
 * rows rows): T, M device FP32 [*][192].  grad: host FP32 [nparams] or NULL;
 * loss: host or NULL.  No update. */
int gsls_ws_loss_grad(gsls_ws* h, const uint16_t* X, const float* T, const float* M, const int32_t* idx,
                      int32_t rows, float* grad, float* loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * gradient of those rows.  loss (host, nullable) synchronises to report it. */
int gsls_ws_train_step(gsls_ws* h, const uint16_t* X, const float* T, const float* M, const int32_t* idx,
                       int32_t rows, float lr, float* loss);

/* Number of feature rows of a batch: sum over instances of N + 1; instance c
 * owns a contiguous block of rows in batch order, stage k at offset k. */
int32_t gsls_ws_batch_rows(gsls_batch* b);

/* Feature rows of a batch for initial states x0 (host, NULL: the last ones
 * uploaded) into device X[rows][160]. */
int gsls_ws_features(gsls_ws* h, gsls_batch* b, const double* const* x0, uint16_t* X);

/* Target rows and loss weights (device FP32 [rows][192]) from the batch's
 * last solution: z, lambda = rho y (weight 1) and log10 of each instance's
 * final rho (weight 25); other entries weight 0. */
int gsls_ws_targets(gsls_batch* b, float* T, float* M);

/* Learned warm start + batched solve: features, MLP, start (rho0 =
 * 10^(mean of the rho column over the instance's rows) clamped to the
 * settings' [rho_min, rho_max]; z0 = prediction projected onto [l, u];
 * y0 = predicted lambda / rho0), then the persistent solve.  parts selects
 * the predicted parts of the start (GSLS_WS_RHO | GSLS_WS_Z | GSLS_WS_Y, at
 * least one); the others keep the cold start (rho0 = 1, z0 = 0, y0 = 0).  An
 * instance not converged after warm_budget iterations (0: no limit) restarts
 * cold (z = y = 0, rho = 1) and reports cold_restart = 1.  *ms: device time
 * of prediction and solve; *ms_predict (nullable): of the prediction alone. */
enum { GSLS_WS_RHO = 1, GSLS_WS_Z = 2, GSLS_WS_Y = 4, GSLS_WS_ALL = 7 };
int gsls_qp_solve_batch_ws(gsls_batch* b, gsls_ws* h, const double* const* x0, double tol, int32_t warm_budget,
                           int32_t parts, gsls_result* out, double* ms, double* ms_predict);

void gsls_ws_free(gsls_ws* h);

#ifdef __cplusplus
}
#endif
#endif /* GSLS_H */
