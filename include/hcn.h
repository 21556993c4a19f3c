/*
 * hcn.h -- C ABI of the MI355X complex double-double / quad-double Newton
 * corrector for polynomial homotopy continuation.
 *
 * The method is the path tracker of Verschelde & Yu, "Accelerating
 * Polynomial Homotopy Continuation on a Graphics Processing Unit with Double
 * Double and Quad Double Arithmetic": evaluation and differentiation of a
 * polynomial system by reverse-mode differentiation of every monomial
 * (Section 3.2, Table 1) and summation (Section 3.3), a linear solve by
 * modified Gram-Schmidt (Section 1; Fig. 2), Newton's method (equations (2)
 * and (3), Fig. 2) and predictor-corrector tracking of the homotopy of
 * equation (1) (Fig. 3, equation (4)).
 *
 * Numbers.  A real is P doubles, most significant limb first, the limbs
 * non-overlapping: P = 1 is double (D), P = 2 double-double (DD), P = 4
 * quad-double (QD), the three modes of Section 3.1.  A complex number is
 * [2][P]: the real limbs, then the imaginary limbs.  The batch, the serving
 * loop and the mixed-precision corrector take DD and QD.
 *
 * Memory.  Pointers named *_dev are device pointers (hipMalloc or a torch
 * CUDA tensor); everything else is host memory.  Device arrays are
 * contiguous float64 / int32 in the layouts stated per argument; B is a
 * batch of independent problems, the leading index.  All device work is
 * enqueued on `stream` (a hipStream_t; NULL = the null stream) and is
 * asynchronous unless stated otherwise.
 *
 * Errors.  Every call returns an int: HCN_OK, a negative error code or, for
 * outcome codes, a positive value.  Argument errors (HCN_EINVAL) are found
 * on the host before anything is enqueued; the message is available from
 * hcn_last_error() (thread-local).  Launch failures are HCN_EDEVICE.
 * Per-problem outcomes (singular matrix, NaN, divergence) are written to
 * device status arrays and never to the return value.
 */
#ifndef HCN_H
#define HCN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HCN_OK 0
#define HCN_EINVAL (-1)
#define HCN_ENOMEM (-2)
#define HCN_EDEVICE (-3)
#define HCN_ESINGULAR (-4)
#define HCN_NOT_CONVERGED 1
#define HCN_DIVERGED 2
#define HCN_MAX_STEPS 3
#define HCN_STEP_TOO_SMALL 4
#define HCN_NAN 5

#define HCN_DD 2
#define HCN_QD 4

/* Thread-local text of the last error on this thread ("" if none). */
const char *hcn_last_error(void);

/* ABI version (major * 100 + minor). */
int hcn_version(void);

/* ------------------------------------------------------------------------
 * Polynomial systems (Section 3.1: the fully expanded distributed
 * representation; Section 3.2: monomials sorted by their number of
 * variables, with position tables laid out for coalesced access).
 * --------------------------------------------------------------------- */

typedef struct hcn_sys_s *hcn_sys;

/* Copy a system to the device.  Host tables, caller-owned, copied:
 *   eq_ptr  [N+1]   equations as a CSR over monomials (eq_ptr[0] = 0),
 *   mon_ptr [nmon+1] monomials as a CSR over (variable, exponent) pairs,
 *   var, exp [npairs] variable index in 0..n-1, distinct within a
 *           monomial, exponent 1..255; a monomial with no pair is a
 *           constant term,
 *   coef    [nmon][2][P] complex coefficients.
 * Requires P in {1, 2, 4} and 1 <= n <= N <= 4096 (a monomial has at most n
 * pairs; those of more than 64 variables are evaluated by a loop form of
 * the reverse mode).
 * The handle owns its device tables; it is immutable and may be shared by
 * calls on any stream.  Synchronous (returns after the upload). */
/* hcn_sys_free gives up the caller's reference.  A batch that lists the
 * system (hcn_batch_add) and a serving request that names it
 * (hcn_server_submit) hold references of their own, so the device tables
 * are freed only when the last of them lets go. */
int hcn_sys_load(hcn_sys *out, int N, int n, int P, const int32_t *eq_ptr,
                 const int32_t *mon_ptr, const int32_t *var, const int32_t *exp,
                 const double *coef);

int hcn_sys_free(hcn_sys sys);

typedef struct {
    int N, n, P, nmon;
    int max_k;        /* most variables in one monomial */
    int nslots;       /* values plus partials written per evaluation */
    int nnz_jac;      /* structurally non-zero Jacobian entries */
    size_t device_bytes;
} hcn_sys_info_t;

int hcn_sys_info(hcn_sys sys, hcn_sys_info_t *info);

/* Total degree of each equation (host array of N). */
int hcn_sys_degrees(hcn_sys sys, int32_t *degrees);

/* ------------------------------------------------------------------------
 * Evaluation and differentiation (Sections 3.2-3.3): f(x) and the full
 * Jacobian by reverse-mode differentiation of every monomial (forward,
 * backward and cross products, Table 1) times its coefficient, then one
 * sum per output.
 * --------------------------------------------------------------------- */

/* Workspace bytes for hcn_eval_jac with B points. */
size_t hcn_eval_ws_bytes(hcn_sys sys, int B);

/* x_dev [B][n][2][P] -> f_dev [B][N][2][P] and J_dev [B][n][N][2][P]
 * (column-major: J[k][i] = df_i/dx_k).  J_dev may be NULL: then only the
 * values are formed (products without their gradients).  ws_dev: hcn_eval_ws_bytes()
 * bytes of device memory, or NULL to let the call allocate and free it on
 * the stream. */
int hcn_eval_jac(hcn_sys sys, int B, const double *x_dev, double *f_dev,
                 double *J_dev, void *ws_dev, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Linear solve by modified Gram-Schmidt (Section 1; Fig. 2,
 * GPU_Modified_Gram_Schmidt) on the augmented matrix [A | b] followed by
 * back substitution.
 * --------------------------------------------------------------------- */

size_t hcn_mgs_ws_bytes(int B, int N, int n, int P);

/* Solve A dx = b (least squares when N > n), B independent problems.
 *   A_dev  [B][n][N][2][P] column-major, overwritten by Q,
 *   b_dev  [B][N][2][P], overwritten by its component orthogonal to Q,
 *   dx_dev [B][n][2][P] solution,
 *   R_dev  [B][n+1][n][2][P] column-major R (column j holds r_kj, k <= j;
 *          column n holds Q^H b), or NULL,
 *   status_dev [B] int32: HCN_OK, HCN_ESINGULAR (some r_kk zero or not
 *          finite; dx is then undefined) or HCN_NAN.
 * Requires 1 <= n <= N <= 4096. */
int hcn_mgs_solve(int B, int N, int n, int P, double *A_dev, double *b_dev,
                  double *dx_dev, double *R_dev, int32_t *status_dev,
                  void *ws_dev, size_t ws_bytes, void *stream);

/* Select the MGS variant used by every solve (process-wide): 0 automatic
 * (5 for large single problems, else 1), 1 one workgroup per problem,
 * 2 right-looking across workgroups (one launch per column step, the
 * trailing matrix re-read every step), 4 tiled (Section 1: right-looking
 * over panels of T columns, each panel factored by one workgroup with its
 * columns in registers, then one launch applies the panel to every later
 * column, held in registers: 2 ceil(n/T) launches), 5 pipelined (one
 * cooperative launch: the columns stay in the LDS of persistent workgroups,
 * column j in workgroup j mod G; the owner of a column publishes q_k in
 * place as soon as it is projected and normalised, and every workgroup
 * applies the q_k in order to its own later columns, the next column
 * first).  1 and 4 differ from 2 only by the rounding of their
 * reductions; 5 gives the bits of 2.  4 falls back to 2 when N > 512 (DD,
 * FP64) or N > 256 (QD); 5 falls back to 2 when the columns of one
 * workgroup do not fit its LDS or the workgroups cannot all be resident.
 * A problem whose pipelined solve could not finish (a bounded wait ran
 * out) reports HCN_EDEVICE in its status.  EINVAL outside {0, 1, 2, 4, 5}. */
int hcn_set_mgs_variant(int variant);

/* Panel width T of variant 4 (process-wide), 1 <= T <= 16; default 16.
 * EINVAL outside that range. */
int hcn_set_mgs_panel(int T);

/* Bound on each wait of variant 5 (process-wide), in polls of the awaited
 * words (about a microsecond each); default 4194304 (seconds).  A wait that
 * runs out stops the problem, which then reports HCN_EDEVICE; a small
 * bound lets a test take that path with every kernel ending normally.
 * EINVAL for polls < 0. */
int hcn_set_mgs_wait_limit(long long polls);

/* How the monomial kernels form the common factor of R1 (process-wide;
 * default 1): 1 the same products in every lane of a wavefront (a product by
 * y^0 = 1 where a variable's exponent is 1, powers tabulated per point in
 * LDS, exponent scalings by mul_d, which is exact for exponents 1 and 2),
 * 0 branching on each exponent.  Both give bitwise the same results for
 * normalised inputs; the first avoids running both sides of the branches
 * across a wavefront whose lanes differ in exponents. */
int hcn_set_mon_uniform(int on);

/* Monomial form of the evaluation with gradients (process-wide; default 0):
 * 0 the reverse mode, one lane per monomial (Section 3.2, Table 1); 1 the
 * tree mode of Section 3.2: a group of G lanes (the power of two >= the
 * most variables in a monomial of the system, at least 4, at most 64) per
 * monomial forms the product of its factors' powers, the prefix and suffix
 * products of its variables by log2 G levels of shuffles, and every partial
 * as prefix x suffix; systems with monomials of more than 64 variables, and
 * value-only evaluations, keep the reverse mode.  The two forms round
 * differently (reductions of products in another order); both are within
 * the stated tolerance of the plain definition. */
int hcn_set_mon_tree(int on);

/* Point chunking (process-wide) of hcn_newton_step, hcn_newton,
 * hcn_newton_mixed and hcn_track_paths: each Newton iteration runs its
 * monomial and summation launches over chunks of points whose monomial
 * scratch takes about `bytes` (a multiple of 64 points, at least 64), so that
 * the scratch one launch writes is still in the last-level cache when the
 * next reads it; the solve covers the whole batch.  0 (the default) runs
 * every launch over the whole batch.  Results are bitwise the same for every
 * setting. */
int hcn_set_chunk_bytes(size_t bytes);

/* Kernel-variant table used by the one-workgroup MGS: lane-group width
 * (8, 16 or 32 lanes per column) and the storage of [A | b] during the
 * factorisation, mgs_lds: 0 global memory, 1 staged in LDS (when it fits in
 * 80 KB), 2 held in the registers of the lane groups that own the columns
 * (when N <= group * 4 and the columns fit), 3 in registers one panel of
 * columns at a time, left-looking (Section 1: each q column is read once per
 * later panel instead of the trailing matrix at every step; DD and FP64,
 * when N <= group * 16); the slot-table batch treats 2 as 0.
 * Problems of batches of at most 64 use 2 when it fits.  Per precision P
 * (1 = the FP64 solve of the mixed-precision step, 2, 4)
 * and row count N (bucketed to the next power of two >= 8).  Defaults: for
 * DD and FP64 with 32 < N <= 256 storage 3 (16 lanes up to N = 128 in DD and
 * N = 64 in FP64, 32 beyond), else 16 lanes and global memory.
 * Every choice gives bitwise the same results, and it depends
 * only on (P, N), so a problem's result does not depend on the batch it is
 * solved in.  save/load: text, one "P N group lds" line per entry.
 * hcn_autotune (batch section) fills the table by timing.  EINVAL for a
 * group other than 8/16/32 or mgs_lds outside 0..3. */
int hcn_tune_set(int P, int N, int mgs_group, int mgs_lds);
int hcn_tune_get(int P, int N, int *mgs_group, int *mgs_lds);
int hcn_tune_save(const char *path);
int hcn_tune_load(const char *path);

/* Autotuner: times hcn_newton_step of `sys` at the B points x_dev (device
 * [B][n][2][P], left unchanged) for every lane-group width and storage choice
 * (reps steps each after a warm-up pass, HIP events on `stream`), stores the
 * choice in the table for (P, N) and returns it with its time: the fastest,
 * or [A | b] staged in LDS when that is within 5 % of the fastest and fits
 * every row count of the bucket (it moves a tenth of the global-memory
 * form's HBM traffic).  Synchronous. */
int hcn_autotune(hcn_sys sys, int B, const double *x_dev, int reps, int *best_group,
                 int *best_lds, double *best_ms, void *stream);

/* ------------------------------------------------------------------------
 * Newton's method (equation (2); Fig. 2).  The system is either f alone
 * (gamma == NULL) or the homotopy of equation (1),
 *   h(x, t) = gamma (1-t)^k g(x) + t^k f(x),
 * with the total-degree start system g_i = x_i^{d_i} - 1 (d_i the degree
 * of f_i; requires N == n).  gamma: host [2][P].  t_dev: device [B]
 * doubles (ignored when gamma == NULL).  Norms are infinity norms over the
 * leading limbs of the real and imaginary parts, in double.
 * --------------------------------------------------------------------- */

size_t hcn_newton_ws_bytes(hcn_sys sys, int B);

/* One iteration without tests: evaluate, solve J dx = -h, x += dx.
 *   x_dev [B][n][2][P] updated in place,
 *   norms_dev [B][2] doubles: ||h(x)|| before the update and ||dx||,
 *   status_dev [B]: HCN_OK, HCN_ESINGULAR or HCN_NAN (x unchanged). */
int hcn_newton_step(hcn_sys sys, const double *gamma, int relax_k, int B,
                    const double *t_dev, double *x_dev, double *norms_dev,
                    int32_t *status_dev, void *ws_dev, size_t ws_bytes,
                    void *stream);

/* hcn_newton_step without allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses
 * that forbid hipMalloc).  The same launches as hcn_newton_step, with the
 * workspace in a fixed device array of HCN_STATIC_WS_BYTES that the
 * library's code object holds on every GPU it runs on until the process
 * ends.  Its address on a device is looked up once, on the first call on
 * that device.  The call allocates nothing, creates no events (profiling
 * is held off for it) and leaves nothing in the array that a later call
 * relies on: no part of it must start at zero.
 * Arguments as hcn_newton_step without ws_dev / ws_bytes; EINVAL (before any
 * launch) when hcn_newton_ws_bytes(sys, B) exceeds HCN_STATIC_WS_BYTES
 * (complex DD: about 107 points of the dense n = 32 system, 3 of the sparse
 * n = 512 one).  All calls on one GPU share its array: calls whose work can overlap
 * on the device (other host threads, or streams not ordered with each
 * other) race on it; calls on one stream are ordered and safe. */
#define HCN_STATIC_WS_BYTES (64u << 20)
int hcn_newton_step_static(hcn_sys sys, const double *gamma, int relax_k, int B,
                           const double *t_dev, double *x_dev, double *norms_dev,
                           int32_t *status_dev, void *stream);

typedef struct {
    int max_iter;       /* iterations (evaluations) at most */
    double tol_res;     /* success when ||h|| < tol_res */
    double tol_dx;      /* success when ||dx|| < tol_dx */
    double max_eq_val;  /* fail when ||h|| exceeds the previous one,
                           initially max_eq_val */
} hcn_newton_params;

/* Fig. 2 per problem, every decision taken on the device:
 *   status_dev [B]: HCN_OK (converged), HCN_DIVERGED, HCN_NOT_CONVERGED,
 *                   HCN_ESINGULAR or HCN_NAN,
 *   iters_dev  [B]: evaluations performed,
 *   norms_dev  [B][2]: last residual norm and last update norm. */
int hcn_newton(hcn_sys sys, const double *gamma, int relax_k, int B,
               const double *t_dev, double *x_dev, const hcn_newton_params *prm,
               double *norms_dev, int32_t *status_dev, int32_t *iters_dev,
               void *ws_dev, size_t ws_bytes, void *stream);

/* Mixed precision: Fig. 2 where each iteration evaluates the residual h(x)
 * in DD/QD (values only), takes its rounding to FP64 as right-hand side,
 * forms the Jacobian in FP64 at the leading limbs of x, solves by MGS in
 * FP64 and adds the FP64 correction to x in DD/QD; the iteration reaches
 * full DD/QD accuracy while kappa(J) 2^-53 < 1.  Arguments, tests and outputs
 * as hcn_newton; workspace from hcn_newton_mixed_ws_bytes. */
size_t hcn_newton_mixed_ws_bytes(hcn_sys sys, int B);
int hcn_newton_mixed(hcn_sys sys, const double *gamma, int relax_k, int B,
                     const double *t_dev, double *x_dev, const hcn_newton_params *prm,
                     double *norms_dev, int32_t *status_dev, int32_t *iters_dev,
                     void *ws_dev, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Path tracking (Fig. 3 with the step bounds of equation (4)), the step
 * size controlled on the device: trial t = min(1, t_acc + dt); prediction
 * by the polynomial through the last accepted points (Section 3.1: degree
 * predictor_order, or one less than the number of points accepted so far,
 * the start point included; Lagrange form, weights from the double
 * differences of the t values); Fig. 2 corrector; on success accept and, once more than two
 * successes are counted, double dt up to max_dt; on failure reset the count
 * and halve dt, failing below min_dt; fail after more than max_steps steps.
 * At t = 1 Newton's method refines with end_tol and end_iters.
 * --------------------------------------------------------------------- */

typedef struct {
    int max_iter;
    double tol_res, tol_dx, max_eq_val, max_dt, min_dt;
    int max_steps, end_iters;
    double end_tol;
    int predictor_order;  /* degree of the extrapolation, 0..4 (EINVAL otherwise):
                             0 constant, 1 secant, up to 4 (Section 4.2) */
} hcn_track_params;

typedef struct {
    int32_t status;       /* HCN_OK, HCN_MAX_STEPS, HCN_STEP_TOO_SMALL, HCN_NAN */
    int32_t steps;        /* predictor-corrector steps taken */
    int32_t newton_iters; /* evaluations while tracking */
    int32_t end_iters;    /* evaluations of the refinement at t = 1 */
    int32_t end_status;   /* Fig. 2 outcome of the refinement */
    int32_t accepted;     /* accepted steps */
    double t;             /* last accepted t */
    double res_norm, dx_norm;
} hcn_path_result;

size_t hcn_track_ws_bytes(hcn_sys sys, int B);

/* Track B paths of the homotopy from the start solutions x0_dev
 * [B][n][2][P] (solutions of g) to x_out_dev [B][n][2][P]; results_dev [B]
 * hcn_path_result in device memory.  The host only enqueues steps and
 * polls a device counter of unfinished paths: it blocks until every path
 * has finished. */
int hcn_track_paths(hcn_sys sys, const double *gamma, int relax_k, int B,
                    const double *x0_dev, const hcn_track_params *prm,
                    double *x_out_dev, hcn_path_result *results_dev,
                    void *ws_dev, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Batches: a slot table of up to `capacity` paths of any number of systems
 * of one precision, tracked together (Fig. 3 per path, the step size of
 * each path its own).  Every kernel launch covers every occupied slot; the
 * step is captured once into a HIP graph (on the caller's stream, or for
 * the legacy null stream on a stream of the batch's own joined to it by
 * events) and replayed; the work lists are rebuilt when slots are added or
 * released.  A path's arithmetic depends
 * only on its own system, start point, gamma and the tuning table, so its
 * result is bitwise the same alone and in any mix.  Sizing: every system
 * added must have N == n <= max_n and at most max_nslots evaluation slots
 * (hcn_sys_info); at most max_systems distinct systems per batch.
 * --------------------------------------------------------------------- */

typedef struct hcn_batch_s *hcn_batch;

/* flags: HCN_BATCH_MIXED runs every corrector iteration in mixed precision
 * (residual and update in DD/QD, Jacobian and MGS in FP64, as
 * hcn_newton_mixed). */
#define HCN_BATCH_MIXED 1

int hcn_batch_create(hcn_batch *out, int P, int capacity, int max_n, int max_nslots,
                     int max_systems, const hcn_track_params *prm, int relax_k, int flags);
int hcn_batch_destroy(hcn_batch b);
size_t hcn_batch_device_bytes(hcn_batch b);
const char *hcn_batch_last_error(void);

/* Occupy a free slot with a path of `sys` from x0_dev ([n][2][P], device;
 * read by work enqueued on `stream`, keep it alive until then) with gamma
 * (host [2][P]); the path starts at t = 0. */
int hcn_batch_add(hcn_batch b, int slot, hcn_sys sys, const double *gamma,
                  const double *x0_dev, void *stream);

/* Free a slot (its result is no longer available). */
int hcn_batch_release(hcn_batch b, int slot);

/* Slots whose system has at least min_n unknowns (0, the default: none)
 * solve with the tiled MGS (hcn_set_mgs_variant 4; panels of 16 columns,
 * 8 for DD/FP64 with N > 256 and QD with N > 64), launched across all such
 * slots, instead of one workgroup per slot: lower latency per step for
 * large systems.  Systems too large for the tiled kernels (N > 512, QD
 * N > 256) keep the one-workgroup solve.  The choice depends only on a
 * slot's own system, so its results stay the same alone and in any mix; it
 * changes the rounding of the reductions against the one-workgroup solve.
 * Takes effect at the next step.  EINVAL for a NULL batch or min_n < 0. */
int hcn_batch_set_split(hcn_batch b, int min_n);

/* How hcn_batch_step runs plain steps (default 0): 0 a captured graph of
 * the step's launches (monomials, sums and solve over all slots), replayed
 * once per step; 1 one persistent workgroup per slot that runs the requested
 * steps of its own path, stage after stage, without returning to the host,
 * and stops when its path is done: no launch or graph overhead per stage,
 * for small systems and few paths (Section 2: a single path is latency
 * bound).  Both give bitwise the same results.  The persistent form covers
 * the plain corrector with the one-workgroup solve; a batch in mixed
 * precision or with slots on the tiled solve (hcn_batch_set_split) keeps the
 * graph.  EINVAL for a NULL batch. */
int hcn_batch_set_persistent(hcn_batch b, int on);

/* Enqueue `steps` predictor-corrector steps of every unfinished path. */
int hcn_batch_step(hcn_batch b, int steps, void *stream);

/* Number of occupied, unfinished slots (>= 0) or an error; done_host (NULL
 * or [capacity]) receives 1 for finished slots.  Waits for the stream. */
int hcn_batch_poll(hcn_batch b, int32_t *done_host, void *stream);

/* Result of a finished slot: x_out_dev ([n][2][P], device, or NULL) and
 * *res_host (or NULL).  Waits for the stream when res_host is given. */
int hcn_batch_result(hcn_batch b, int slot, double *x_out_dev, hcn_path_result *res_host,
                     void *stream);

/* Work done so far per slot: counts_host [capacity][2] = residual
 * evaluations and linear solves since the slot's path started (0 for empty
 * slots).  Waits for the stream. */
int hcn_batch_counts(hcn_batch b, int32_t *counts_host, void *stream);

/* Step every occupied slot to the end, polling after every `chunk` steps. */
int hcn_batch_run(hcn_batch b, int chunk, void *stream);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of path-tracking requests of many systems
 * and two precisions.  One slot-table batch (a lane, on its own stream) per
 * precision and size class of the system (n <= 24, 25..63, >= 64); a lane's
 * slot count is its share of budget_bytes (qd_share for QD, split evenly
 * over the classes) divided by the device footprint of one slot sized for
 * the largest system of its class (N == n <= max_n, at most max_nslots
 * evaluation slots), so requests are admitted by device-memory footprint:
 * a request waits in its lane's FIFO queue until a slot is free.
 * hcn_server_pump visits every lane whose last round has finished on the
 * device (it never waits for a busy one): it harvests finished paths,
 * admits queued requests and launches the lane's next round of
 * steps_per_round steps.  Requests admitted while others run join the same
 * launches, and a result does not depend on the mix; systems with n >= 48
 * solve with the tiled MGS across workgroups (hcn_batch_set_split).
 * serial != 0 runs one path at a time, oldest request first (a baseline).
 * Times are seconds on the server's monotonic clock (hcn_server_now).  The
 * lanes progress independently only when their streams land on different
 * hardware queues: HIP's GPU_MAX_HW_QUEUES (default 4) should be at least
 * the number of lanes plus the caller's streams.
 * --------------------------------------------------------------------- */

typedef struct hcn_server_s *hcn_server;

int hcn_server_create(hcn_server *out, size_t budget_bytes, double qd_share, int max_n,
                      int max_nslots, const hcn_track_params *dd_prm,
                      const hcn_track_params *qd_prm, int steps_per_round, int serial);
int hcn_server_destroy(hcn_server s);
const char *hcn_server_last_error(void);
double hcn_server_now(hcn_server s);
int hcn_server_capacity(hcn_server s, int *dd_slots, int *qd_slots);

/* Queue a request; gamma host [2][P], x0 host [n][2][P] (copied). */
int hcn_server_submit(hcn_server s, int64_t id, hcn_sys sys, const double *gamma,
                      const double *x0, double t_arrival);

/* One scheduling pass (no wait on busy lanes); returns the number of paths
 * in flight, or a negative error code. */
int hcn_server_pump(hcn_server s);

/* Pop one completed request: returns 1 (and fills the outputs that are not
 * NULL; x_out host [n][2][P]) or 0 when none is waiting. */
int hcn_server_fetch(hcn_server s, int64_t *id, double *x_out, hcn_path_result *res,
                     double *t_arrival, double *t_admit, double *t_done);
int hcn_server_queued(hcn_server s, int *dd, int *qd);

/* ------------------------------------------------------------------------
 * Elementwise arithmetic (the DD/QD layer itself, Section 3.1), for
 * checking it bit for bit.  op codes: 0 add, 1 sub, 2 mul, 3 div, 4 sqrt
 * (a only), 5 mul by double (b_dev: [count] doubles); on complex numbers
 * [count][2][P]: 10 add, 11 sub, 12 mul, 13 conj(a) * b, 14 |a|^2 (out:
 * real [count][P]), 15 real scaling (b_dev: real [count][P]); error-free
 * transformations on doubles [count] -> [count][2]: 20 TwoSum, 21
 * FastTwoSum, 22 TwoProd.
 * --------------------------------------------------------------------- */
int hcn_elementwise(int op, int P, int count, const double *a_dev,
                    const double *b_dev, double *out_dev, void *stream);

/* ------------------------------------------------------------------------
 * Kernel timing (measurement support, not part of the method).  When
 * enabled, every kernel launch of the library is bracketed by two HIP
 * events recorded on its launch stream.  Kernel names: "eval_monomials",
 * "eval_sums", "mgs".  hcn_profile_query waits for the recorded events and
 * returns the summed event time of one kernel name and its launch count.
 * --------------------------------------------------------------------- */
int hcn_profile_enable(int on);
int hcn_profile_reset(void);
int hcn_profile_query(const char *kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* HCN_H */
