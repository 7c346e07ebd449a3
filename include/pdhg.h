/*
 * pdhg.h -- C-ABI of the MI355X (gfx950) PDHG linear-programming library.
 *
 * The library solves  min c'x  s.t.  Gx >= h,  Ax = b,  l <= x <= u
 * (the primal LP of Section 2.2 of arXiv 2508.16806) with restarted
 * Primal-Dual Hybrid Gradient (Algorithm 1 in the sign-consistent form of
 * Appendices C/D, with the Section 2.4 enhancements: Ruiz scaling, adaptive
 * restarts and primal-weight updates).  Every step of the iteration runs in
 * hand-written HIP kernels; this header is the whole public surface.
 *
 * Conventions shared by every call
 *  - All functions return an int status: PDHG_OK (0) or a negative PDHG_ERR_*
 *    code.  No C++ exception crosses the ABI.  pdhg_last_error() returns a
 *    thread-local human-readable message for the last failure in the thread.
 *  - A "stream" argument is a hipStream_t (0 = the null stream).  Work is
 *    stream-ordered; calls that return host data synchronise that stream.
 *  - Memory-space flags (PDHG_MEM_HOST / PDHG_MEM_DEVICE) tell whether a
 *    caller pointer is host memory or device memory of the current device.
 *  - A handle may be used by one stream (one thread) at a time.
 *  - Rows: row_type[i] is PDHG_ROW_GE for a row of G (">=") and PDHG_ROW_EQ
 *    for a row of A ("=").  Internally the rows are reordered so that all
 *    ">=" rows come first (the stacked K = [G; A], q = [h; b] of Section 2.2);
 *    every row-indexed vector crossing this ABI is in the CALLER's row order.
 *  - Infinite bounds are IEEE infinities (l_j = -INFINITY, u_j = +INFINITY).
 */
#ifndef PDHG_H
#define PDHG_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define PDHG_OK 0
#define PDHG_ERR_INVALID_ARG -1 /* NULL pointer, bad option value, bad index   */
#define PDHG_ERR_SHAPE -2       /* row_ptr not monotone, column out of range,  */
                                /* nnz mismatch, row_type count mismatch       */
#define PDHG_ERR_BOUNDS -3      /* l_j > u_j, l_j = +inf or u_j = -inf          */
#define PDHG_ERR_NONFINITE -4   /* NaN anywhere, or +-inf in K, c or rhs       */
#define PDHG_ERR_NOMEM -5       /* workspace smaller than pdhg_workspace_bytes */
#define PDHG_ERR_HIP -6         /* a HIP runtime call failed                   */
#define PDHG_ERR_STATE -7       /* call not valid in the handle's state        */

/* ---- solve status (pdhg_result.status) ----------------------------------- */
#define PDHG_OPTIMAL 0          /* relative KKT error <= eps (Section 2.3.2)   */
#define PDHG_ITERATION_LIMIT 1
#define PDHG_TIME_LIMIT 2
#define PDHG_NUMERICAL_ERROR 3  /* a reduction in the check became NaN/inf     */
#define PDHG_PRIMAL_INFEASIBLE 4 /* a dual ray certifies it (Section 2.4.5)     */
#define PDHG_DUAL_INFEASIBLE 5   /* a primal ray certifies it: the LP is         */
                                 /* unbounded if it is feasible                 */

/* ---- enumerations ---------------------------------------------------------- */
#define PDHG_MEM_HOST 0
#define PDHG_MEM_DEVICE 1
#define PDHG_PREC_F64 0  /* iterates, matrix and arithmetic in FP64            */
#define PDHG_PREC_F32 1  /* FP32 iterates and matrix, FP64 accumulation, FP64  */
                         /* KKT check, restart test and primal-weight update   */
#define PDHG_ROW_GE 0
#define PDHG_ROW_EQ 1
#define PDHG_SOL_RESULT 0  /* point returned by the last pdhg_solve            */
#define PDHG_SOL_CURRENT 1 /* current iterate z                                 */
#define PDHG_SOL_AVERAGE 2 /* running average of the current restart epoch     */

/* One LP in CSR form (Section 2.2).  All pointers live in the memory space
 * `mem`.  They are BORROWED: pdhg_setup copies and converts everything it
 * needs before it returns, after which the caller may free them.
 *   row_ptr  m+1 int64, monotone, row_ptr[0] = 0, row_ptr[m] = nnz
 *   col      nnz int32 in [0, n); duplicate entries in a row are summed
 *   val      nnz double, finite
 *   c        n double, finite               (cost)
 *   rhs      m double, finite               (h_i for ">=" rows, b_i for "=" rows)
 *   l, u     n double, l_j <= u_j, l_j < +inf, u_j > -inf
 *   row_type m uint8 (PDHG_ROW_GE / PDHG_ROW_EQ), or NULL: all rows are "="  */
typedef struct {
    int64_t n;
    int64_t m;
    int64_t nnz;
    const int64_t *row_ptr;
    const int32_t *col;
    const double *val;
    const double *c;
    const double *rhs;
    const double *l;
    const double *u;
    const uint8_t *row_type;
    int32_t mem;
} pdhg_lp;

/* Solver options.  pdhg_default_opts fills the paper's constants:
 * eps = 1e-4 (Section 2.3.2), step = 0.9 / ||K~||_2 (Sections 4.1-4.2),
 * restart constants 0.2 / 0.8 / 0.36 (Section 2.4.2), eps_zero = 1e-6
 * (Section 2.4.3), and the choices the paper leaves open: 10 Ruiz passes,
 * a KKT check every 64 iterations, power iteration to a 1e-6 relative change
 * or 1000 passes. */
typedef struct {
    int32_t precision;      /* PDHG_PREC_F32 (default) or PDHG_PREC_F64             */
    int32_t ruiz_iters;     /* Ruiz passes; 0 disables scaling                      */
    int32_t use_restarts;   /* adaptive restarts (Section 2.4.2)                     */
    int32_t use_pw_update;  /* primal-weight updates (Algorithm 4)                   */
    int32_t check_every;    /* iterations between KKT checks, 1..4096                */
    int32_t power_max_iters;
    int64_t max_iters;      /* iteration limit                                       */
    double eps;             /* relative KKT tolerance                                */
    double time_limit;      /* seconds of pdhg_solve; <= 0: none                     */
    double step_size;       /* eta; <= 0 picks step_frac / ||K~||_2                  */
    double step_frac;
    double primal_weight;   /* omega_0; <= 0 picks ||c~|| / ||q~|| (1 if either small)*/
    double power_tol;
    double beta_suff, beta_nec, beta_art;
    double eps_zero;
    int32_t unroll_capacity;   /* max steps pdhg_iterate may record (0: none)       */
    int32_t unroll_checkpoint; /* checkpoint spacing C for the adjoint replay       */
    int32_t use_graph;         /* capture iteration chunks in a hipGraph            */
    int32_t xcd_remap;         /* XCD-contiguous workgroup numbering                */
    /* Row-length bins (autotuner output).  Bin k takes rows of length
     * <= bin_len[k] (and above bin k-1's limit) and sweeps each with 2^k lanes
     * (k = 0..6) or a whole 256-lane workgroup (k = 7).  0 keeps the default
     * 4, 8, 16, 32, 64, 128, 512, inf. */
    int32_t bin_len_dual[8];   /* rows of K   (dual sweep)                        */
    int32_t bin_len_primal[8]; /* rows of K^T (primal sweep)                      */
    /* Rows handled by one lane group in bins 0..4 (1, 2 or 4; 0 means 1): the
     * group interleaves the loads of its rows.  Bins 5..7 take one row per
     * group (0 or 1); other values, and negative bin_len, are rejected. */
    int32_t bin_rows_dual[8];
    int32_t bin_rows_primal[8];
    int32_t max_grid;          /* workgroups per solve-time sweep launch (0: 8192);  */
                               /* a launch walks the row blocks of the instances   */
                               /* still running                                    */
    /* Adaptive step size (Section 2.4.4, Algorithm 5), 0 or 1.  Each attempt
     * takes the PDHG step with the instance's trial step eta from the current
     * iterate, forms etabar = ||(x'-x, y'-y)||_w^2 / |2 (y'-y)' K~ (x'-x)|
     * with ||(a, b)||_w^2 = w ||a||^2 + ||b||^2 / w (+inf when the product
     * is 0) and the next trial step eta' = min((1 - (k+1)^-0.3) etabar,
     * (1 + (k+1)^-0.6) eta), k = attempts of this solve including this one;
     * the candidate becomes the iterate when eta <= etabar.  The first
     * attempt of every pdhg_solve tries the fixed step above.  Averages are
     * weighted by the accepted steps (Section 2.4.2).  Iteration counts,
     * check_every and max_iters count attempts.  pdhg_iterate always takes
     * fixed steps. */
    int32_t adaptive_step;
    /* Infeasibility detection (Section 2.4.5, Algorithm 6), 0 or 1.  At every
     * check, on the difference of the last step in the original variables
     * (dx, dy, dlambda with lambda = proj_Lambda(c - K'y); with adaptive steps
     * only when the last attempt was accepted): the LP is reported
     * PDHG_DUAL_INFEASIBLE when c'dx < 0 and ||A dx||, -min(G dx) and the
     * largest violation of dx_j in the recession cone of [l_j, u_j] are all
     * <= infeas_tol * |c'dx|; else PDHG_PRIMAL_INFEASIBLE when
     * psi = q'dy + l'dlambda^+ + u'dlambda^- > 0 (-inf when an infinite bound
     * meets a nonzero multiplier) and ||K'dy + dlambda|| and -min(dy_ineq)
     * are <= infeas_tol * psi.  The returned point is the current iterate. */
    int32_t detect_infeas;
    double infeas_tol;         /* default 1e-4                                      */
    /* Largest point count of pdhg_fishnet (0, or a power of two in 2..64): the
     * workspace then holds that many interleaved candidate points. */
    int32_t fishnet_points;
    /* Admission of a batch's instances into pdhg_solve's running set (batch
     * > 1; 0: all run from the start).  Instances enter in order of
     * decreasing per-iteration sweep bytes 2 (e + 4) nnz + 8 (n + m + 2) +
     * e (9 n + 6 m), e = 4 (FP32) or 8 (FP64) (values, columns and row
     * pointers of K~ and K~^T, the swept and gathered vectors; ties by
     * index) while the running ones' bytes stay within this budget, and
     * always at least one runs; a finished instance frees its share at the
     * next check.  A waiting instance has had its starting-point check and
     * takes no step, so its iterates, iteration count and status are the
     * ones it reaches alone.  Sizing the budget below the 256 MB Infinity
     * Cache keeps the running matrices resident between iterations; the
     * default, 192e6, also keeps enough instances running to fill the GPU.
     * Waiting instances at a time limit end with PDHG_TIME_LIMIT and their
     * starting point. */
    int64_t batch_resident_bytes;
    /* Per-instance ring of check records kept by pdhg_solve (0: none): the
     * last trace_capacity records of the solve, read with pdhg_get_trace.
     * The solve loop never waits for them. */
    int32_t trace_capacity;
    /* Column slices of the dual sweep (the product K~ xbar of Algorithm 1),
     * 0 or 1: none (default).  With S in 2..16, every row of K~ with at least
     * 16 S entries is swept in S passes over the column ranges
     * [s n/S, (s+1) n/S) of its instance (FP64 partial sums per row; the last
     * pass adds them in pass order and updates y), so each pass gathers from
     * an n/S-entry slice of xbar that stays in one XCD's L2.  Such rows keep
     * their entries grouped by slice, are binned by their per-slice length,
     * and every product over them sums in that order.  Applies to pdhg_solve
     * (the adaptive step's dual sweep and the products K~ x of its checks
     * included) and to pdhg_iterate without recording; the recorded steps of
     * the adjoint, pdhg_kkt and fishnet sweep whole rows. */
    int32_t col_slices;
    /* The same for the primal sweep (the product K~^T y): rows of K~^T
     * (columns of the LP) with at least 16 S entries are swept in S passes
     * over the row ranges [s m/S, (s+1) m/S) of K~ of their instance, so each
     * pass gathers from an m/S-entry slice of y; 0 or 1: none (default).
     * The entries of every column are in row order, so slicing changes no
     * entry order, only where the FP64 sums are split.  Fixed steps only:
     * the adaptive step's primal sweep takes whole rows. */
    int32_t col_slices_t;
} pdhg_opts;

/* Relative KKT error terms (Section 2.3.2, conditions term1-term3) on the
 * ORIGINAL (unscaled) LP, FP64 throughout:
 *   pres = ||(Ax - b, [h - Gx]^+)||_2, dres = ||c - K'y - lambda||_2 with
 *   lambda = proj_Lambda(c - K'y), pobj = c'x, dobj = q'y + l'lambda^+ +
 *   u'lambda^- (a product with an infinite bound is skipped: lambda is 0
 *   there), gap = |dobj - pobj|, rel_gap = gap / (1 + |dobj| + |pobj|),
 *   rel_pres = pres / (1 + ||q||), rel_dres = dres / (1 + ||c||),
 *   rel_kkt = max(rel_gap, rel_pres, rel_dres).  rel_kkt <= eps iff all three
 *   termination conditions hold. */
typedef struct {
    double pres, dres, pobj, dobj, gap;
    double rel_pres, rel_dres, rel_gap, rel_kkt;
} pdhg_kkt_out;

typedef struct {
    int32_t status;      /* PDHG_OPTIMAL, ..._ITERATION_LIMIT, ..._TIME_LIMIT, ..._NUMERICAL_ERROR */
    int32_t from_avg;    /* returned point: 1 = epoch average, 0 = current iterate */
    int64_t iters;       /* PDHG iterations of this solve                           */
    int32_t restarts;
    int32_t power_iters;
    double knorm;        /* power-iteration estimate of ||K~||_2                    */
    double eta, omega0, omega, tau, sigma;
    pdhg_kkt_out kkt;    /* of the returned point (last check)                      */
    double seconds;      /* wall time of pdhg_solve                                 */
    int64_t accepted;    /* accepted steps (= iters without adaptive steps)         */
    double eta_next;     /* trial step of the next attempt (= eta without them)     */
} pdhg_result;

/* One check of pdhg_solve (Sections 2.3.2 and 2.4.2): written after the
 * restart / primal-weight / termination decision of that check, with the
 * inputs of that decision (KKT_omega values are on the scaled LP). */
typedef struct {
    int64_t iter;         /* iterations (attempts) of the solve at the check      */
    int32_t restarted;    /* a restart happened at this check                     */
    int32_t cand_avg;     /* the restart candidate is the epoch average           */
    double kkt_cand;      /* KKT_omega of the candidate (scaled LP, omega before) */
    double omega;         /* primal weight after the check                        */
    double rel_kkt_cur;   /* relative KKT error of the iterate (original LP)      */
    double rel_kkt_avg;   /* of the average (+inf without restarts)               */
    double eta_next;      /* step of the next attempt                             */
    int64_t accepted;     /* accepted steps so far                                */
    int64_t t_inner;      /* iterations of the restart epoch at the check         */
    double kkt0;          /* the epoch's reference KKT_omega(z_n^0) at the check  */
    double kkt_prev;      /* previous candidate's KKT_omega (+inf at epoch start) */
    double omega_before;  /* primal weight of the check's metrics                 */
    double delta_x;       /* on restart: ||x^ - x_n^0||, scaled (0 otherwise)     */
    double delta_y;       /* on restart: ||y^ - y_n^0||, scaled (0 otherwise)     */
    double kkt0_next;     /* the reference after the check (new on restart)       */
    double cand_pres;     /* candidate's primal residual, scaled LP               */
    double cand_dres;     /* candidate's dual residual, scaled LP                 */
    double cand_gap;      /* candidate's |dobj - pobj|, scaled LP                 */
} pdhg_trace_rec;

typedef struct {
    int64_t n, m, m_ineq, nnz;
    double knorm, eta, omega, tau, sigma;
    double setup_seconds;
    int32_t precision, batch;
    int64_t workspace_bytes;
    int32_t nseg_primal, nseg_dual; /* row-length bins in use                     */
    int64_t nblk_primal, nblk_dual; /* workgroups per primal / dual sweep         */
    /* phases of setup_seconds: validation and row binning, building the
     * device images of K~ and K~^T on the host, copying them to the device,
     * and the device work (Ruiz scaling, FP32 copies, power iteration) */
    double setup_plan_seconds, setup_host_seconds, setup_copy_seconds, setup_device_seconds;
    double setup_power_seconds;     /* the power iteration's part of the device work */
    int32_t power_iters_max;        /* most power iterations of any instance        */
    int32_t record_valid;           /* pdhg_backward has a tape for the current data */
    int64_t record_generation;      /* bumped by each recording pdhg_iterate and each
                                     * pdhg_set_data: a caller that keeps the value
                                     * from its recording call can tell whether the
                                     * tape is still the one it recorded           */
} pdhg_info;

/* Average device time per launch of each phase kernel (milliseconds). */
typedef struct {
    double ms_primal;   /* fused K~^T y sweep + primal update + averaging      */
    double ms_dual;     /* fused K~ xbar sweep + dual update + averaging       */
    double ms_check;    /* FP64 KKT partial sums of iterate and average        */
    double ms_control;  /* per-instance reduction + restart / stop decisions,
                         * timed on a check that restarts (omega update)      */
    double ms_restart;  /* restart copy of every running instance's candidate
                         * (0 when restarts are off)                          */
    int32_t reps;
    double ms_primal_ad; /* adaptive step: K~^T y sweep + candidate x' + sums   */
    double ms_dual_ad;   /* adaptive step: K~ x' sweep + candidate y' + sums    */
    double ms_step_ad;   /* adaptive step: per-instance accept / reject         */
} pdhg_kernel_times;

typedef struct pdhg_handle pdhg_handle;

/* Fills *o with the defaults listed above. */
void pdhg_default_opts(pdhg_opts *o);

/* Device bytes the workspace passed to pdhg_setup must hold for `batch` LPs
 * (lp points to an array of `batch` descriptors).  Reads the sparsity pattern
 * (copying it to the host if it lives on the device).  Returns 0 and sets the
 * last error when the input is invalid. */
size_t pdhg_workspace_bytes(const pdhg_lp *lp, int32_t batch, const pdhg_opts *o);

/* Validates and copies `batch` LPs into the caller-owned device workspace
 * `ws` (at least pdhg_workspace_bytes bytes, 256-byte aligned; it must outlive
 * the handle), reorders rows to [G; A], builds CSR(K) and CSR(K'), runs Ruiz
 * scaling (Algorithm 3) and the power iteration (Algorithm 2) on the GPU,
 * picks eta, omega_0, tau = eta/omega, sigma = eta*omega (Section 2.3.1) and
 * sets x0 = proj_X(0), y0 = 0.  On success *out is a new handle (free it
 * with pdhg_destroy).  Errors: PDHG_ERR_INVALID_ARG, _SHAPE, _BOUNDS,
 * _NONFINITE, _NOMEM, _HIP. */
int pdhg_setup(const pdhg_lp *lp, int32_t batch, const pdhg_opts *o, void *ws, size_t ws_bytes,
               hipStream_t stream, pdhg_handle **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call hipMalloc, harnesses that forbid
 * it): pdhg_setup with the workspace in a fixed device array that the library
 * holds on every GPU it runs on (PDHG_NOALLOC_MAX_BYTES bytes, kept until the
 * process ends).  The call allocates no device memory and no pinned host
 * memory (pdhg_setup maps a pinned array of done flags; here the flags sit in
 * the fixed array and pdhg_solve copies them out after each chunk, which ends
 * its overlap of chunks).  Same arguments, results and errors as pdhg_setup
 * without ws / ws_bytes; the device is the calling thread's current device and
 * `stream` (NULL: the null stream) must belong to it.  Errors besides
 * pdhg_setup's: PDHG_ERR_NOMEM when pdhg_workspace_bytes plus the done flags
 * exceed PDHG_NOALLOC_MAX_BYTES; PDHG_ERR_STATE while a handle from this call
 * is still live on the device (one at a time per device: the array keeps the
 * last handle's contents; pdhg_destroy frees it for the next call).  Calls
 * that overlap on one device (a second thread setting up while the first
 * handle runs) are refused, not raced. */
#define PDHG_NOALLOC_MAX_BYTES (64ull << 20)
int pdhg_setup_noalloc(const pdhg_lp *lp, int32_t batch, const pdhg_opts *o, hipStream_t stream,
                       pdhg_handle **out);

/* Changes the run-time options of a handle: use_restarts, use_pw_update,
 * check_every, max_iters, eps, time_limit, beta_*, eps_zero, use_graph.  The
 * other fields of *o (precision, scaling, step, power iteration, unroll
 * capacity, bins) are fixed at setup and ignored here. */
int pdhg_set_opts(pdhg_handle *h, const pdhg_opts *o);

/* Runs k fixed-step PDHG iterations (Algorithm 1, theta = 1) from the
 * handle's current iterate with the current tau and sigma: no averaging,
 * restarts or checks.  Asynchronous.  State persists across calls, so
 * pdhg_iterate(k1) then pdhg_iterate(k2) equals pdhg_iterate(k1 + k2).
 * record != 0 stores checkpoints for pdhg_backward (k <= unroll_capacity);
 * a recorded call replaces the previous record. */
int pdhg_iterate(pdhg_handle *h, int64_t k, int32_t record, hipStream_t stream);

/* Full restarted solve to opts.eps (Sections 2.3-2.4) from the handle's
 * current iterate.  Blocks until every instance has stopped; res points to
 * `batch` results.  Every instance of a batch follows exactly the iteration,
 * check and restart sequence it would follow alone. */
int pdhg_solve(pdhg_handle *h, pdhg_result *res, hipStream_t stream);

/* Writes instance `inst`'s point (which = PDHG_SOL_*) in the ORIGINAL
 * variables: x (n), y (m, caller row order) and lambda = proj_Lambda(c - K'y)
 * (n).  Any output pointer may be NULL.  Pointers are in memory space `mem`. */
int pdhg_get_solution(pdhg_handle *h, int32_t inst, int32_t which, double *x, double *y,
                      double *lambda, int32_t mem, hipStream_t stream);

/* Sets instance `inst`'s current iterate to (x, y) given in the original
 * variables (y in caller row order); x is projected onto [l, u] and the
 * inequality entries of y onto y >= 0.  The restart epoch starts here. */
int pdhg_set_state(pdhg_handle *h, int32_t inst, const double *x, const double *y, int32_t mem,
                   hipStream_t stream);

/* Replaces the cost, right-hand side and bounds of every instance (arrays
 * concatenated over the batch in the caller's layout; NULL keeps a vector).
 * The matrix, the Ruiz factors and the step parameters stay those of setup.
 * Host arrays are validated like pdhg_setup's; device arrays are trusted.
 * Once the arrays pass validation the recorded tape of pdhg_iterate is
 * dropped (pdhg_backward then fails with PDHG_ERR_STATE). */
int pdhg_set_data(pdhg_handle *h, const double *c, const double *rhs, const double *l, const double *u,
                  int32_t mem, hipStream_t stream);

/* Fishnet casting (Section 2.5, Algorithm 7): a multi-start warm start for a
 * handle of one LP (batch 1, opts.fishnet_points >= npoints at setup).
 * npoints = 2^p candidate points (2..64) start at (r / sqrt(n)) g_q with
 * r = ||K~||_2 (the handle's power-iteration estimate) and g_q the caller's
 * standard normal draws G (npoints x n, point-major, caller column order,
 * scaled variables), and y_q = K~ x_q.  Each round runs k fixed PDHG steps
 * (the handle's tau, sigma) on every live point, keeps the half with the
 * smallest duality gap |dobj - pobj| (ties by index, best first) and, in odd
 * rounds that start with more than two points, appends as many new points,
 * new point a = sum_s w_as (kept point s) with w_as = |g_as| / sum_s |g_as|
 * from the caller's draws wraw (consumed a row of (kept count) at a time;
 * equal weights for an all-zero row).  Rounds end when one point is left; it
 * becomes the current iterate and the start of a restart epoch, so the next
 * pdhg_solve starts from it.  The rounds and draw count for npoints come from
 * pdhg_fishnet_rounds.  gaps (rounds x npoints) and keep (rounds x npoints,
 * kept indices best first, -1 beyond) may be NULL.  G, wraw, gaps and keep
 * live in memory space `mem`.  All points run together: each sweep reads a
 * matrix entry once for every point.  Synchronous.  Errors: _INVALID_ARG,
 * _STATE (batch > 1 or no fishnet workspace), _NONFINITE (host draws). */
int pdhg_fishnet(pdhg_handle *h, int32_t npoints, int32_t k, const double *G, const double *wraw, int64_t nw,
                 int32_t mem, double *gaps, int32_t *keep, hipStream_t stream);

/* Rounds of Algorithm 7 for npoints points and the number of repopulation
 * draws pdhg_fishnet consumes (host only). */
int pdhg_fishnet_rounds(int32_t npoints, int32_t *rounds, int64_t *draws);

/* Relative KKT error of a caller point (x, y) on instance `inst`'s original
 * LP (y in caller row order).  FP64 throughout; synchronous. */
int pdhg_kkt(pdhg_handle *h, int32_t inst, const double *x, const double *y, int32_t mem,
             pdhg_kkt_out *out, hipStream_t stream);

/* Adjoint of the last recorded pdhg_iterate on the whole batch.  Given
 * gx = dL/dx_K and gy = dL/dy_K (original variables, concatenated over the
 * batch, y parts in caller row order), writes dL/dc, dL/drhs, dL/dl, dL/du,
 * dL/dx_0 and dL/dy_0 in the original variables (tau, sigma and the Ruiz
 * factors are constants).  Output pointers may be NULL.  The replay uses the
 * checkpoints stored every unroll_checkpoint steps.  PDHG_ERR_STATE when no
 * recording pdhg_iterate ran since setup or since the last pdhg_set_data
 * (the tape would replay against other data); pdhg_info.record_generation
 * tells a caller whether a later recording call replaced its tape. */
int pdhg_backward(pdhg_handle *h, const double *gx, const double *gy, double *gc, double *grhs,
                  double *gl, double *gu, double *gx0, double *gy0, int32_t mem,
                  hipStream_t stream);

/* Phase timers: average device time per launch of each phase kernel over
 * `reps` launches on `stream`, from HIP events.  The two sweeps run
 * alternately, primal then dual, with an event after each launch, as in the
 * iteration (each finds the caches as the other leaves them); likewise the
 * adaptive attempt's primal sweep, dual sweep and step decision.  The packet
 * that each separating event adds is measured (the same sequence timed with
 * events at its ends only) and taken out evenly; a kernel shorter than that
 * packet gets its proportional share of the unseparated total instead (so
 * every figure is positive).  The check,
 * control and restart kernels, which run once per check interval, are timed
 * back to back.  The sweeps advance the iterate (fixed steps); solver counters
 * are restored.  1 <= reps <= 10000 (one event per launch is created),
 * else PDHG_ERR_INVALID_ARG.  Synchronous. */
int pdhg_time_kernels(pdhg_handle *h, int32_t reps, pdhg_kernel_times *out, hipStream_t stream);

/* Autotuner of the launch layout for `batch` LPs (lp as for pdhg_setup): times
 * the primal and dual sweeps (pdhg_time_kernels, `reps` launches each) over
 *   bins:  bin_len = f * 2^k (k = 0..5), w, inf for f in {2, 4, 8, 16},
 *          w in {512, 2048} (w >= 64 f), best limits per operator;
 *   rows per lane group in bins 0..4: 1, 2 or 4, best per operator;
 *   launch shape: xcd_remap in {0, 1} x max_grid in {4096, 8192, 16384,
 *          65536}, best by primal + dual + check / check_every;
 *   column slices on that layout: none, then col_slices = col_slices_t
 *          = S in {2, 4, 8} with each bin candidate for the dual sweep;
 *          the fastest dual (S, bins) and the fastest primal S are kept
 *          where they beat the unsliced sweep by at least 2%;
 * every other option is taken from *base.  *best receives the chosen
 * options; out_json (may be NULL) a JSON record of every trial and the
 * choice.  Each trial sets the LP up in the caller's workspace `ws`, which
 * must hold the largest candidate: *ws_needed (may be NULL) receives that
 * size, and a NULL or smaller workspace fails with PDHG_ERR_NOMEM after
 * setting it.  Synchronous. */
int pdhg_autotune(const pdhg_lp *lp, int32_t batch, const pdhg_opts *base, void *ws, size_t ws_bytes,
                  size_t *ws_needed, int32_t reps, hipStream_t stream, pdhg_opts *best, const char *out_json);

/* Ruiz factors of instance `inst` (Algorithm 3): the scaled problem is
 * K~ = diag(rho) K diag(kappa), x = kappa x~, y = rho y~.  rho has m entries
 * (caller row order), kappa n entries; either pointer may be NULL. */
int pdhg_get_scaling(pdhg_handle *h, int32_t inst, double *rho, double *kappa, int32_t mem,
                     hipStream_t stream);

/* Check records of instance `inst` from the last pdhg_solve (needs
 * opts.trace_capacity > 0 at setup): *total receives the number of checks
 * the solve made (the first check after the starting point counts as 1),
 * out the last min(*total, trace_capacity, cap) of them, oldest first (host
 * memory).  Synchronous on `stream`. */
int pdhg_get_trace(pdhg_handle *h, int32_t inst, pdhg_trace_rec *out, int32_t cap, int64_t *total,
                   hipStream_t stream);

/* Sizes, step parameters and launch layout of the handle (instance 0's
 * parameters for a batch). */
int pdhg_get_info(const pdhg_handle *h, pdhg_info *info);

/* Releases the handle (not the caller's workspace). */
void pdhg_destroy(pdhg_handle *h);

/* Thread-local message for the last error ("" if none). */
const char *pdhg_last_error(void);

/* Thread-local status code (PDHG_ERR_*) of the last failure in the thread,
 * PDHG_OK if none: the code behind a pdhg_workspace_bytes that returned 0. */
int pdhg_last_error_code(void);

#ifdef __cplusplus
}
#endif

#endif /* PDHG_H */
