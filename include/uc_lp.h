/*
 * uc_lp.h -- C ABI of libuclp: restarted PDHG for unit-commitment LP
 * relaxations on one AMD Instinct MI355X (gfx950).
 *
 * The problem is the continuous relaxation that both legs of the paper's
 * concurrent GPU-CPU solver hand to their LP method (Sec. II-C: PDHG on the
 * GPU and barrier on CPU threads work on the same LP relaxation of the unit
 * commitment MILP; Sec. III-C: in the GPU pipeline PDHG takes the place of
 * the barrier solve):
 *
 *     min c'x   s.t.  a_i'x  = b_i   (sense 'E')
 *                     a_i'x >= b_i   (sense 'G')
 *                     a_i'x <= b_i   (sense 'L', negated internally)
 *                     lb <= x <= ub  (+-INFINITY allowed)
 *
 * The solve/poll/terminate surface (create, asynchronous solve, non-blocking
 * status, cancel) is what the concurrent driver of Algorithm 1 needs: start a
 * solve, poll it on a fixed interval, and terminate the slower leg.  The
 * default limits follow the PDHG parameter paragraph of Sec. II-D
 * (iteration limit 100,000, convergence tolerance 1e-4, absolute feasibility
 * tolerance 1e-5).
 *
 * Conventions for every function below
 *   - All pointers are HOST pointers unless stated otherwise.  Arrays passed
 *     in are deep-copied before the call returns; the caller keeps ownership.
 *   - Functions return UC_LP_OK (0) or a negative uc_lp_err code.  They never
 *     abort or throw across the ABI.  A thread-local message describing the
 *     last failure is available from uc_lp_last_error().
 *   - Index arrays are int32, CSR with row_ptr[0] = 0, row_ptr[m] = nnz,
 *     column indices in [0, n), no duplicate (row, column) pairs.
 *   - Dual values y follow the Lagrangian c'x - y'(Ax - b): y_i >= 0 on 'G'
 *     rows, y_i <= 0 on 'L' rows, free on 'E' rows.
 */
#ifndef UC_LP_H
#define UC_LP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct uc_lp uc_lp;          /* one LP instance                         */
typedef struct uc_engine uc_engine;  /* one GPU, an HBM budget and a slot table */

enum uc_lp_err {
  UC_LP_OK = 0,
  UC_LP_EINVAL = -1,   /* malformed input (see uc_lp_create)                   */
  UC_LP_ENOMEM = -2,   /* host or device allocation failed                      */
  UC_LP_EBUDGET = -3,  /* instance larger than the whole engine HBM budget      */
  UC_LP_EHIP = -4,     /* a HIP runtime call failed                             */
  UC_LP_ESTATE = -5,   /* call not valid in the handle's current state          */
  UC_LP_ENOTSUP = -6,  /* option value not supported                            */
  UC_LP_ETIMEOUT = -7  /* uc_lp_wait timed out (the solve keeps running)        */
};

/* Arithmetic of the iterates. */
enum uc_lp_precision {
  UC_LP_FP64 = 0,              /* FP64 matrix values and iterates                  */
  UC_LP_FP32_MIXED = 1,        /* FP32 values/iterates; FP64 KKT, restart, gap     */
  UC_LP_FP32_MIXED_POLISH = 2, /* FP32 until eps_rel, then FP64 until eps_polish   */
  UC_LP_FP32_REFINE = 3        /* FP32 until eps_rel, then rounds of iterative
                                  refinement with FP32 inner solves until the
                                  FP64-evaluated relative KKT error of the
                                  refined point is <= eps_polish (see
                                  eps_refine)                                      */
};

/* Solve status. */
enum uc_lp_status_code {
  UC_LP_IDLE = 0,        /* created, no solve requested                */
  UC_LP_QUEUED = 1,      /* waiting for an engine slot / HBM budget    */
  UC_LP_RUNNING = 2,
  UC_LP_OPTIMAL = 3,     /* stopping tolerance reached                 */
  UC_LP_ITER_LIMIT = 4,
  UC_LP_TIME_LIMIT = 5,
  UC_LP_CANCELLED = 6,   /* uc_lp_cancel was called                    */
  UC_LP_NUMERICAL = 7,   /* a non-finite KKT quantity appeared         */
  UC_LP_INFEASIBLE = 8,  /* detected by the minimal presolve           */
  UC_LP_FAILED = 9       /* device error during the solve              */
};

/* SpMV kernel family used by the PDHG half-steps. */
enum uc_lp_spmv_algo {
  UC_LP_SPMV_ROWSPLIT = 0,  /* row blocks of bounded nnz, LDS-staged products */
  UC_LP_SPMV_MERGEPATH = 1  /* equal shares of rows+nnz per workgroup         */
};

typedef struct {
  int32_t precision;     /* uc_lp_precision, default UC_LP_FP32_MIXED_POLISH   */
  int32_t kkt_every;     /* iterations between KKT/restart checks, default 64  */
  int32_t ruiz_iters;    /* Ruiz equilibration passes, default 10              */
  int32_t power_iters;   /* power-iteration steps for ||A||_2, default 64      */
  int64_t iter_limit;    /* total iteration limit, default 100000              */
  double eps_rel;        /* relative KKT stopping tolerance, default 1e-4      */
  double eps_abs_feas;   /* optional extra stopping requirement: inf-norm of
                            the unscaled row violation <= this; default 0 (off).
                            The paper's PDHG runs set 1e-5 (Sec. II-D).        */
  double eps_polish;     /* relative KKT target of the FP64 polish, 1e-8       */
  double time_limit_s;   /* wall-clock limit of one solve, default 3600        */
  double step_scale;     /* eta = step_scale / (upper bound on ||A_hat||_2),
                            default 0.99                                      */
  int32_t spmv_algo;     /* uc_lp_spmv_algo; the PDHG half-steps support
                            UC_LP_SPMV_ROWSPLIT only (ENOTSUP otherwise)       */
  int32_t verbose;       /* 0 = silent, 1 = one line per check on stderr       */
  int32_t timing;        /* 1 = time the middle primal and dual launch of each
                            check interval with dispatch-attached HIP events   */
  int32_t restart_to_current; /* 0: restart at the PDHG output T(z) (default);
                            1: restart at the current Halpern iterate z         */
  /* adaptive restart on the fixed-point residual r = ||z - T(z)||_P, checked
     every kkt_every iterations (Applegate et al. 2021; Lu & Yang 2024) */
  double restart_sufficient;  /* restart if r <= this * r(restart start), 0.2 */
  double restart_necessary;   /* ... or r <= this * r(start) and r grew, 0.9  */
  double restart_artificial;  /* ... or inner iterations >= this * total, 0.36 */
  double pw_smoothing;   /* primal weight: log w <- s log(dy/dx) + (1-s) log w
                            at each restart, default 0.8; 0 keeps w fixed.
                            (The published PDLP values are 0.8 necessary and
                            0.5 smoothing; 0.9 / 0.8 took fewer iterations to
                            1e-4 on every synthetic UC family measured.)      */
  double halpern_gamma;  /* reflection of the Halpern step in [0, 1]:
                            z <- w((1+g) T(z) - g z) + (1-w) z_restart;
                            1 = reflected Halpern (default), 0 = plain         */
  double pw_max_change;  /* bound on one primal-weight update: the new weight
                            stays within [w / this, w * this]; default 4,
                            0 = unbounded                                     */
  int32_t fp32_stall_checks; /* FP32 phase: continue in FP64 when the relative
                            KKT error has not fallen below 0.9 of its best
                            value for this many checks and that best is within
                            10x of the target; default 24, 0 = never.
                            (Near its rounding floor the FP32 iteration can
                            take restarts on residual noise whose primal-weight
                            updates then stall it; both guards bound that.)  */
  int32_t reserved;      /* must be 0                                         */
  double pw_integral;    /* integral gain of the primal-weight update: log w
                            also moves by -this * (sum of past errors
                            log w - log(dy/dx)); default 0                    */
  double pw_balance;     /* at a restart log w also moves by this * log(rel.
                            primal residual / rel. dual residual), raising the
                            dual step while the primal residual lags;
                            default 0.5, 0 = off                              */
  double pw_balance_polish; /* the gain used instead, in both phases, by
                            UC_LP_FP32_MIXED_POLISH; default 0 (toward 1e-8
                            the term did not pay: the 64-LP serving stream took
                            8.21M iterations without it, 8.91M with 0.5)      */
  double eps_gap_rel;    /* UC_LP_FP64 and UC_LP_FP32_MIXED: OPTIMAL also needs
                            the relative duality gap |pobj - dobj| /
                            (1 + |pobj| + |dobj|), accumulated in FP64, to be
                            <= this; the solve continues past the eps_rel
                            milestone (t_to_eps_s) until the gap closes.  In
                            the FP32 phase a gap that stops improving
                            (fp32_stall_checks checks without a 10% gain)
                            continues in FP64.  A closed gap does not bound
                            the objective error while the primal residual is
                            still at the eps_rel level (on the 6,049-bus
                            benchmark LP a gap of 8.7e-8 left the objective
                            3e-6 away from the optimum at a primal residual of
                            2e-5); UC_LP_FP32_MIXED_POLISH with a smaller
                            eps_polish does.  Default 0 = off.  Ignored by
                            UC_LP_FP32_MIXED_POLISH.                          */
  /* UC_LP_FP32_REFINE: iterative refinement for LP (Gleixner, Steffy & Wolter,
     INFORMS J. Computing 28(3), 2016) with this library's FP32 PDHG as the
     inner solver.  After the FP32 solve reaches eps_rel, its point (x*, y*)
     is kept in FP64; each round forms, on the device, the correction
     problem of the same matrix whose data are the FP64 residuals of
     (x*, y*) scaled up by D_P = 1/||primal violation||, D_D = 1/||dual
     residual|| (each at most refine_growth times the previous round's):
       c~ = D_D (c - A'y*), b~ = D_P (b - A x*), l~ = D_P (l - x*),
       u~ = D_P (u - x*), inequality duals y~ >= -D_D y*,
     solves it in FP32 from (0, 0), and adds the correction
     (x~/D_P, y~/D_D) to (x*, y*), projected onto the bounds and y_G >= 0.
     A correction solve measures its KKT error on the scale of the point it
     corrects (residuals divided by D_P, D_D, duality gap by D_P D_D, each
     relative as in the main solve) and stops once that estimate of the
     refined point's error has fallen to eps_refine times its value at the
     round start, or to eps_polish, or when it stalls (fp32_stall_checks).
     The solve is OPTIMAL once the relative KKT error of (x*, y*) on the
     original problem, evaluated in FP64, is <= eps_polish; ITER_LIMIT at
     iter_limit iterations over all rounds or after refine_max_rounds
     rounds.  A run that ends short of eps_polish returns the best refined
     point of its round boundaries (a round can end worse than it began).  Refinement runs in the scaled space of the solve, and the
     primal weight carries over, times the change of D_D / D_P.           */
  double eps_refine;     /* error reduction asked of each round, 1e-2         */
  double refine_growth;  /* bound on the growth of D_P and D_D per round, 1e4 */
  int32_t refine_max_rounds; /* default 200 (a round is a restart of the inner
                            solve: the iteration limit is the real bound)    */
  int32_t reserved2;     /* must be 0                                         */
  double pw_balance_refine; /* the residual-balance gain (as pw_balance) used
                            inside the correction problems, in [0, 1],
                            default 0.5                                       */
  double refine_diverge; /* a correction problem whose relative KKT error
                            rises above this times the best of its round
                            ends the round at once (0: never; else > 1),
                            default 0                                         */
} uc_lp_opts;

typedef struct {
  int32_t status;          /* uc_lp_status_code                               */
  int32_t precision_now;   /* arithmetic of the current / final phase         */
  int64_t iters;           /* PDHG iterations, all phases                     */
  int64_t iters_fp64;      /* of which in FP64 (polish or FP64 mode)          */
  int64_t restarts;
  double t_total_s;        /* solve start -> finish (or now)                  */
  double t_setup_s;        /* transpose, scaling, power iteration             */
  double t_to_eps_s;       /* solve start -> first check with rel_kkt<=eps_rel
                              (and the absolute feasibility tolerance); -1 if
                              not reached                                      */
  double t_queue_s;        /* solve request -> admission into a slot          */
  double pobj, dobj;       /* unscaled, original problem                      */
  double rel_primal, rel_dual, rel_gap, rel_kkt;
  double abs_primal_inf;   /* inf-norm of unscaled row violations             */
  double pobj_at_eps;      /* primal objective at the eps_rel milestone       */
  double rel_kkt_at_eps;
  int64_t iters_at_eps;    /* iterations at the eps_rel milestone             */
  double norm_a_est;       /* power-iteration estimate ||B v||^(1/2) of
                              ||A_hat||_2 (from below; see norm_a_bound)       */
  double omega;            /* current primal weight                           */
  double primal_kernel_us; /* mean duration of timed primal half-step kernels
                              (the FP32 ones when the solve had an FP32 phase) */
  double dual_kernel_us;   /* mean duration of timed dual half-step kernels    */
  int64_t timed_launches;  /* number of launches in each mean above           */
  int32_t m_presolved, n_presolved;  /* sizes after the minimal presolve      */
  int64_t nnz_presolved;
  int64_t device_bytes;    /* device memory held by this instance             */
  double primal_bytes;     /* algorithmic bytes of one primal half-step launch
                              in the current precision: matrix values and
                              indices, row pointers, one read of y, and the
                              per-column streams the kernel reads or writes
                              (c, l, u skipped where a row block holds one
                              known value)                                     */
  double dual_bytes;       /* the same for one dual half-step launch           */
  double rel_gap_at_eps;   /* relative duality gap at the eps_rel milestone    */
  double fp_residual;      /* fixed-point residual ||z - T(z)||_P of the last
                              check, in the scaled space, with P the metric of
                              the PDHG step [[I/tau, A_hat'], [A_hat, I/sigma]]
                              (the quantity the adaptive restarts compare)     */
  double norm_a_bound;     /* upper bound on ||A_hat||_2 that sets the step:
                              1, the bound the Pock-Chambolle scaling (alpha
                              = 1) guarantees; norm_a_est shows its tightness */
  double eta;              /* step: tau = eta / omega, sigma = eta * omega,
                              eta = step_scale / norm_a_bound                 */
  int32_t refine_rounds;   /* UC_LP_FP32_REFINE: correction problems solved
                              (or being solved); the KKT fields above then
                              describe the refined point (x*, y*) at the last
                              round boundary                                   */
  int32_t reserved_i;
  double rel_kkt_inner;    /* UC_LP_FP32_REFINE: relative KKT error of the
                              running correction problem at the last check    */
} uc_lp_info;

/* Fill *opts with the defaults listed in uc_lp_opts. */
void uc_lp_opts_default(uc_lp_opts* opts);

/* ---- engine: one device, one HBM budget, up to max_slots resident solves --
 * Instances created against an engine are uploaded when they are admitted
 * into a slot (FIFO order, when a slot is free and the budget allows) and are
 * iterated together by batched kernels that cover every resident instance.
 * device: HIP device ordinal.  hbm_budget_bytes: 0 = 90% of free memory.
 * max_slots: 1..1024.  Returns EINVAL, EHIP or ENOMEM on failure. */
int uc_engine_create(int device, size_t hbm_budget_bytes, int32_t max_slots,
                     uc_engine** out);
/* Cancels every running or queued solve, waits for the worker, frees all.
 * NULL is a no-op.  Instances of the engine must be destroyed first. */
void uc_engine_destroy(uc_engine* eng);

/* Create one LP instance.
 * eng == NULL: a private engine on device 0 is created; the instance is
 *   validated, presolved and uploaded before the call returns.
 * eng != NULL: validated and presolved now; uploaded at admission.
 * Arrays: row_ptr[m+1], col_idx[nnz], val[nnz], c[n], b[m], sense[m]
 *   ('E', 'G' or 'L'), lb[n], ub[n].
 * EINVAL: m or n < 1, nnz < 0, row_ptr not monotone or row_ptr[0] != 0 or
 *   row_ptr[m] != nnz, column index outside [0, n) or repeated within a row,
 *   NaN or infinite matrix value, cost or right-hand side, lb > ub,
 *   lb = +inf or ub = -inf, unknown sense code.
 * EBUDGET: the instance needs more device memory than the engine budget.
 * ENOTSUP: every column is fixed, or no row keeps an entry in a free column
 *   (nothing is left for PDHG).
 * The minimal presolve removes fixed columns (lb == ub) and empty rows; an
 * empty row that cannot be satisfied makes the instance INFEASIBLE (reported
 * by uc_lp_status after uc_lp_solve, not as an error here). */
int uc_lp_create(uc_engine* eng, int32_t m, int32_t n, int64_t nnz,
                 const int32_t* row_ptr, const int32_t* col_idx, const double* val,
                 const double* c, const double* b, const char* sense,
                 const double* lb, const double* ub, const uc_lp_opts* opts,
                 uc_lp** out);

/* uc_lp_create with the problem in DEVICE memory of the engine's device
 * (device 0 when eng == NULL), e.g. the storage of torch tensors: the same
 * arrays, types and validation as uc_lp_create.  The arrays are read on
 * hip_stream (NULL: the null stream), so after the work the caller enqueued
 * there, and deep-copied (through the host: the minimal presolve and the
 * row-block partition are host work) before the call returns; the caller
 * keeps ownership and may reuse them at once.  EINVAL also when a pointer
 * is not device memory of that device; EHIP when a copy fails.  The
 * caller's current device is restored on return.  A process that also uses
 * PyTorch must initialise torch's GPU before it loads this library: torch
 * ships its own HIP runtime under the same soname, and the process can hold
 * only one of the two. */
int uc_lp_create_device(uc_engine* eng, int32_t m, int32_t n, int64_t nnz,
                        const int32_t* row_ptr, const int32_t* col_idx, const double* val,
                        const double* c, const double* b, const char* sense,
                        const double* lb, const double* ub, const uc_lp_opts* opts,
                        void* hip_stream, uc_lp** out);

/* Replace c, b, lb, ub (any may be NULL = keep) of an instance that is not
 * running; the matrix is unchanged.  Same validation as uc_lp_create. */
int uc_lp_update_data(uc_lp* lp, const double* c, const double* b,
                      const double* lb, const double* ub);

/* Start an asynchronous solve.  x0[n], y0[m] (original space) warm-start the
 * iterates; NULL = start from the projection of 0 and y = 0.  ESTATE if a
 * solve of this handle is queued or running. */
int uc_lp_solve(uc_lp* lp, const double* x0, const double* y0);

/* Non-blocking snapshot of the solve state.  Safe to call from any thread
 * while the solve runs. */
int uc_lp_status(const uc_lp* lp, uc_lp_info* out);

/* Block until the solve is no longer QUEUED/RUNNING or timeout_s elapses
 * (timeout_s < 0: no limit).  ETIMEOUT on timeout. */
int uc_lp_wait(uc_lp* lp, double timeout_s);

/* Request termination of a queued or running solve (the step of Algorithm 1
 * that stops the slower leg).  Takes effect at the next check
 * (at most kkt_every iterations later); the status becomes CANCELLED.
 * OK if nothing is running. */
int uc_lp_cancel(uc_lp* lp);

/* Copy the final iterate, unscaled and in the original row/column order:
 * x[n], y[m] (either may be NULL).  ESTATE unless the status is terminal
 * (OPTIMAL, ITER_LIMIT, TIME_LIMIT, CANCELLED or NUMERICAL). */
int uc_lp_get_solution(const uc_lp* lp, double* x, double* y);

/* uc_lp_get_solution into DEVICE buffers x[n], y[m] (double; either may be
 * NULL) of the instance's device, enqueued on hip_stream (NULL: the null
 * stream): the values are there when the stream reaches the copies.  The
 * copies read the handle's host copy of the solution, so the handle is
 * neither destroyed nor solved again until the stream has passed them.  The
 * caller owns the buffers.  ESTATE as uc_lp_get_solution; EINVAL for
 * pointers that are not device memory of that device. */
int uc_lp_get_solution_device(const uc_lp* lp, double* x, double* y, void* hip_stream);

/* Cancel if running, wait, release device memory.  NULL is a no-op. */
void uc_lp_destroy(uc_lp* lp);

/* Thread-local description of the last failure ("" if none). */
const char* uc_lp_last_error(void);

/* ---- scenario batches sharing one matrix --------------------------------
 * Solve n_scen LPs that share the matrix of `base` (created with eng ==
 * NULL) and differ in c, b, lb, ub: arrays c[n_scen*n], b[n_scen*m],
 * lb[n_scen*n], ub[n_scen*n], scenario-major.  One read of the matrix per
 * half-step serves every scenario.  x0[n], y0[m] (may be NULL) warm-start all
 * scenarios from one point.  Blocks until all scenarios stop.  Solutions are
 * written to x[n_scen*n], y[n_scen*m] and per-scenario results to
 * info[n_scen].  n_scen in 1..16.  ENOTSUP for other counts.
 * Device memory: the call allocates the scenarios' interleaved vectors for
 * its duration (info[].device_bytes; ENOMEM if that fails).  Once at most
 * half the scenarios are still unfinished it moves them to a smaller set of
 * arrays holding only their lanes, allocated and released inside the call;
 * without memory for that set it keeps the full layout.  Host threads: one
 * per scenario for validation and presolve, up to 16 for unpacking the
 * results.  uc_lp_cancel(base) from another thread stops the batch. */
int uc_lp_solve_scenarios(uc_lp* base, int32_t n_scen, const double* c,
                          const double* b, const double* lb, const double* ub,
                          const double* x0, const double* y0, double* x,
                          double* y, uc_lp_info* info);

/* ---- step-level entry points (the same kernels the solve runs) -----------
 * These expose single steps of the method so that each can be compared
 * element by element with an independent implementation.  They act on the
 * instance's internal problem: fixed columns and empty rows removed, 'L'
 * rows negated, 'E' rows first.  They require a handle created with
 * eng == NULL that is not running, and they run the instance's setup
 * (transpose, scaling, power iteration) if it has not run yet. */

/* Internal sizes and maps: row_map[m_int] gives the original row of each
 * internal row (negative = negated 'L' row, encoded -(row+1)), col_map[n_int]
 * the original column of each internal column.  Any pointer may be NULL. */
int uc_lp_internal_dims(uc_lp* lp, int32_t* m_int, int32_t* n_int, int64_t* nnz_int,
                        int32_t* m_eq, int32_t* row_map, int32_t* col_map);

/* The transpose built on the device: t_row_ptr[n_int+1],
 * t_col[nnz_int], t_val[nnz_int] of the UNSCALED internal matrix, with the
 * entries of each transposed row in increasing original row order. */
int uc_lp_get_transpose(uc_lp* lp, int32_t* t_row_ptr, int32_t* t_col, double* t_val);

/* Diagonal scaling A_hat = D_r A D_c of the internal problem: d_row[m_int],
 * d_col[n_int]; and the power-iteration estimate of ||A_hat||_2. */
int uc_lp_get_scaling(uc_lp* lp, double* d_row, double* d_col, double* norm_est);

/* One PDHG step on the scaled internal problem, in the given precision
 * (UC_LP_FP64 or UC_LP_FP32_MIXED): from (x, y), anchor (x0, y0), inner
 * iteration index k and steps tau, sigma, computes
 *   x_hat = proj_[l,u](x - tau (c - A'y)),
 *   y_hat = proj_Y(y + sigma (b - A (2 x_hat - x))),
 *   x_next = w ((1+g) x_hat - g x) + (1 - w) x0,  y_next likewise,
 *   w = (k+1)/(k+2), g = the handle's halpern_gamma (1 by default).
 * All vectors are FP64 host arrays of internal length (x*: n_int, y*: m_int);
 * FP32 mode rounds the inputs to FP32 and widens the outputs. */
int uc_lp_debug_step(uc_lp* lp, int32_t precision, const double* x, const double* y,
                     const double* x0, const double* y0, int64_t k, double tau,
                     double sigma, double* x_hat, double* y_hat, double* x_next,
                     double* y_next);

/* `iters` consecutive PDHG iterations on the scaled internal problem, run
 * by the same launches as one check interval of a solve: iterations
 * 0 .. iters-2 are the solve's non-check half-steps (the Halpern step taken
 * inside the kernels; with halpern_gamma = 1 the primal iterate is rebuilt
 * from x_bar and the anchor instead of stored), iteration iters-1 is a
 * check: x_hat, y_hat = T(z) are stored, the FP64 KKT kernels run on them,
 * and the finish kernel takes the last Halpern step (no restart).
 * Starting point z = (x, y) at inner index k with anchor (x0, y0).
 * Outputs: x_hat, y_hat = T(z) of the last iteration, x_next, y_next the
 * iterate after all `iters` steps, *fp_residual = ||z - T(z)||_P of the last
 * iteration from the check kernels' FP64 scalars (P as in
 * uc_lp_info.fp_residual, with the given tau, sigma).
 * block_threads: workgroup size of the half-steps, 0 = the solve's own
 * choice for this launch size, 256 or 512 to force one (the two give the
 * same bits).  iters in 1..4096.  precision UC_LP_FP64 or UC_LP_FP32_MIXED
 * (FP32 rounds the inputs and widens the outputs).  All vectors are FP64
 * host arrays of internal length; fp_residual may be NULL.
 * uc_lp_debug_step is this call with iters = 1. */
int uc_lp_debug_iterate(uc_lp* lp, int32_t precision, int32_t iters, int32_t block_threads,
                        const double* x, const double* y, const double* x0, const double* y0,
                        int64_t k, double tau, double sigma, double* x_hat, double* y_hat,
                        double* x_next, double* y_next, double* fp_residual);

/* KKT quantities of an ORIGINAL-space pair (x[n], y[m]), evaluated by the
 * solver's own FP64 check kernels.  Fills pobj, dobj, rel_* and
 * abs_primal_inf of *out (other fields zero). */
int uc_lp_eval_kkt(uc_lp* lp, const double* x, const double* y, uc_lp_info* out);

/* One round boundary of iterative refinement (UC_LP_FP32_REFINE), by the
 * kernels the solve runs, on the scaled internal problem (A_hat, c_hat =
 * D_c c, b_hat = D_r b, l_hat = l / D_c, u_hat = u / D_c):
 *   x* <- proj_[l_hat,u_hat](x* + x~ inv_dp),  y* <- y* + y~ inv_dd with
 *   inequality rows projected to >= 0 (first != 0: x* = y* = 0 before);
 *   r = b_hat - A_hat x*, d = c_hat - A_hat' y*, violation v (E rows r, G rows
 *   max(r, 0)), dual residual e = d - lambda(d) (lambda by the finiteness
 *   of the bounds);
 *   D_P = min(1/||v||_2, growth dp_prev) (growth dp_prev if ||v|| = 0), D_D
 *   likewise from ||e||_2 and dd_prev; omega = omega_prev (D_D/D_P) /
 *   (dd_prev/dp_prev);
 *   c~ = D_D d, b~ = D_P r, l~ = D_P (l_hat - x*), u~ = D_P (u_hat - x*),
 *   ylo = -D_D y* on inequality rows (-inf on equality rows).
 * Inputs (host): x_star[n_int], y_star[m_int] (FP64, ignored if first),
 * x_corr[n_int], y_corr[m_int] (FP32, the correction solve's output),
 * par[6] = {inv_dp, inv_dd, dp_prev, dd_prev, growth, omega_prev}.
 * Outputs (host, any may be NULL): x_new[n_int], y_new[m_int] (FP64);
 * data64[3 n_int + m_int] = c~, l~, u~, b~ (FP64); data32[3 n_int + 2 m_int]
 * = c~, l~, u~, b~, ylo as the FP32 inner solve receives them (c~, b~ to
 * nearest; l~ and ylo rounded up, u~ rounded down, so every FP32-feasible
 * correction maps back into the FP64 box and onto y >= 0);
 * scal[14] = {D_P, D_D, omega, ||v||^2, ||e||^2 (scaled space),
 *   unscaled sum of squared violations, b_hat'y*, inf-norm of unscaled
 *   violations, unscaled sum of squared dual residuals, sum of l lambda+ +
 *   u lambda-, c_hat'x*, ||b~||_2 and ||c~||_2 unscaled, relative KKT error
 *   of (x*, y*) on the original problem}.
 * Same handle requirements as the other step-level entry points. */
int uc_lp_debug_refine(uc_lp* lp, const double* x_star, const double* y_star, const float* x_corr,
                       const float* y_corr, int32_t first, const double* par, double* x_new,
                       double* y_new, double* data64, float* data32, double* scal);

/* Standalone SpMV y = A x on host arrays, through the same SpMV kernels:
 * precision UC_LP_FP64 (FP64 values, FP64 accumulation) or UC_LP_FP32_MIXED
 * (values and x rounded to FP32, FP32 accumulation); algo uc_lp_spmv_algo.
 * device: HIP ordinal.  Same CSR validation as uc_lp_create. */
int uc_spmv(int device, int32_t m, int32_t n, int64_t nnz, const int32_t* row_ptr,
            const int32_t* col_idx, const double* val, const double* x, double* y,
            int32_t precision, int32_t algo);

/* Time the SpMV kernels on device-resident data: `copies` independent copies
 * of the matrix (so the working set can exceed the last-level cache) are
 * multiplied round-robin `reps` times.  Writes the mean kernel time in
 * microseconds to *us_per_spmv. */
int uc_spmv_bench(int device, int32_t m, int32_t n, int64_t nnz, const int32_t* row_ptr,
                  const int32_t* col_idx, const double* val, int32_t precision,
                  int32_t algo, int32_t copies, int32_t reps, double* us_per_spmv);

/* Time the solve's own half-step kernels (the non-check launches of the
 * given precision, UC_LP_FP64 or UC_LP_FP32_MIXED) on `copies` device copies
 * of this instance (matrix, scaled data and iterates), launched round-robin
 * so that consecutive launches read different copies and, with enough
 * copies, the working set exceeds the last-level cache.  `reps` iterations
 * (one primal and one dual launch each, every launch timed by start/stop
 * events attached to its dispatch).  Writes the mean duration of one primal
 * and of one dual launch in microseconds, and their algorithmic bytes (the
 * model of uc_lp_info.primal_bytes / dual_bytes; either pointer may be NULL).
 * copies 1..64, reps 1..4096.  Needs a handle created with eng == NULL that
 * is not running; allocates the copies for the duration of the call (ENOMEM
 * if they do not fit).  The handle's iterates are reset as at a cold start
 * (a later uc_lp_solve starts from its own initial point anyway). */
int uc_lp_bench_half_steps(uc_lp* lp, int32_t precision, int32_t copies, int32_t reps,
                           double* primal_us, double* dual_us, double* primal_bytes,
                           double* dual_bytes);

/* Merge-path SpMV y = A x (the kernels of uc_spmv with UC_LP_SPMV_MERGEPATH)
 * on caller-owned DEVICE arrays, allocating nothing: for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).
 * row_ptr[m+1], col_idx[nnz] int32 and val[nnz], x[n], y[m] of the precision
 * (UC_LP_FP64: double, UC_LP_FP32_MIXED: float, FP32 accumulation) are device
 * (or managed) memory of `device`; the CSR must be valid (row_ptr[0] = 0,
 * non-decreasing, row_ptr[m] = nnz, column indices in [0, n)): it is on the
 * device and is not checked.  The kernels run on hip_stream (NULL: the null
 * stream) and the call returns once they are enqueued; y is complete when
 * the stream reaches them.  Same results, bit for bit, as uc_spmv on the
 * same values.
 * Scratch: a static 4 MiB array on each device (workgroup coordinates and
 * carries, 20 bytes per 1,792 rows + entries), held until the process ends;
 * m + nnz up to about 3.7e8.  Larger inputs: ENOTSUP, before any launch.  The
 * kernels overwrite every scratch entry they read, so nothing needs clearing,
 * but calls that overlap in time on one device (other streams, other host
 * threads) share the scratch and race: serialize them.
 * EINVAL: bad sizes, NULL or non-device pointers.  EHIP: launch failure.
 * The caller's current device is restored on return. */
int uc_spmv_merge_noalloc(int device, int32_t m, int32_t n, int64_t nnz, const int32_t* row_ptr,
                          const int32_t* col_idx, const void* val, const void* x, void* y,
                          int32_t precision, void* hip_stream);

/* Device stream-copy bandwidth in GB/s for `bytes` per buffer (calibration
 * of the roofline and of hardware traffic counters). */
int uc_copy_bench(int device, size_t bytes, int32_t reps, double* gbps);

#ifdef __cplusplus
}
#endif
#endif /* UC_LP_H */
