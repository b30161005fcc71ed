/*
 * lsefit.h -- C ABI of the MI355X (gfx950) moment-pass least-squares fit.
 *
 * The operation (Sec. II of Dasgupta, "An Analytical Evaluation of Matricizing
 * Least-Square-Errors Curve Fitting ..."): given n >= 2 pairs (x_i, y_i) and a
 * degree m, find a_0..a_m of f(x) = a_0 + a_1 x + ... + a_m x^m minimising
 * Pi = sum_i [y_i - f(x_i)]^2.  The zero-gradient conditions are the normal
 * equations sum_i x_i^j y_i = sum_k a_k sum_i x_i^(j+k), j = 0..m, i.e. AX = B
 * with the Hankel matrix A_jk = S_(j+k) of power sums S_p = sum_i x_i^p (so
 * A_00 = S_0 = n) and B_j = T_j = sum_i x_i^j y_i; the system is solved by
 * Gaussian elimination (end of Sec. II).
 *
 * The library computes the power sums of the shifted, scaled variable
 * t_i = (x_i - c)/s in one streaming pass over device memory, solves the
 * (m+1)x(m+1) system in float64 with partial pivoting, and maps the solution b
 * (t-basis) back to a (x-basis): a_k = sum_{j>=k} b_j C(j,k) (-c)^(j-k) s^-j.
 * The least-squares minimiser does not depend on (c, s); they only improve
 * conditioning.
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers owned by the caller (for example
 *    torch tensors), except the option structs, which are host memory read
 *    during the call only.  The library never frees or retains them past the
 *    call, except that a plan caches a captured graph that refers to the
 *    arrays of its last call (see fit_batched).
 *  - x and y share one dtype (LSEFIT_F32 or LSEFIT_F64); gradients have it too.
 *    Integer codes (dtype, status) travel as int32_t, so that any value a
 *    caller passes is well defined and an unknown one is reported as
 *    INVALID_ARG (or "unknown status") rather than read as an enumeration.
 *    Coefficients and power sums are always float64, lowest power first.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL is the default stream).
 *    No entry point synchronises the device except fit_plan_tune.
 *  - The return value reports argument and launch errors found on the host
 *    (INVALID_ARG, WORKSPACE, DEVICE, UNSUPPORTED); it never waits for the GPU.
 *    Numerical outcomes are written per fit to the device array `status`
 *    (OK, SINGULAR, NONFINITE, INVALID_ARG for a bad degree or segment); the
 *    coefficients of a fit whose status is not OK are NaN.
 *  - SINGULAR: fewer than m+1 points, or a pivot of magnitude at most 2^-40
 *    times the largest entry of A (in the t variable).  Fewer than m+1
 *    distinct x values always end there.  NONFINITE: a NaN or Inf reached the
 *    power sums or the solution.
 *  - Results are bitwise reproducible from run to run for the same inputs,
 *    options and schedule: every reduction has a fixed order and no floating
 *    point atomics are used.
 */
#ifndef LSEFIT_H
#define LSEFIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LSEFIT_MAX_DEGREE 8
#define LSEFIT_MAX_DEGREE_CHEBYSHEV 16

typedef enum {
    LSEFIT_OK = 0,
    LSEFIT_ERR_INVALID_ARG = 1,
    LSEFIT_ERR_SINGULAR = 2,
    LSEFIT_ERR_NONFINITE = 3,
    LSEFIT_ERR_WORKSPACE = 4,
    LSEFIT_ERR_DEVICE = 5,
    LSEFIT_ERR_UNSUPPORTED = 6
} lsefit_status;

typedef enum { LSEFIT_F32 = 0, LSEFIT_F64 = 1 } lsefit_dtype;

/* How the power sums are accumulated.
 *  LSEFIT_PREC_F64:  every point is promoted to float64; t, its powers and the
 *                    lane sums are float64.
 *  LSEFIT_PREC_F32C: float32 inputs only; t and its powers in float32, lane
 *                    sums as compensated (Kahan) float32 pairs folded once per
 *                    group of four points, promoted to float64 for the
 *                    cross-lane and cross-wave combine; followed by
 *                    `refine_steps` passes of iterative refinement in which the
 *                    residual r_i = y_i - sum_j b_j t_i^j and the sums
 *                    sum_i t_i^j r_i are float64, and A delta = R corrects b. */
typedef enum { LSEFIT_PREC_F64 = 0, LSEFIT_PREC_F32C = 1 } lsefit_precision;

/* Where (c, s) come from.
 *  LSEFIT_RANGE_GIVEN: c = center, s = scale for every fit (s > 0; a power
 *                      of two keeps t exact).
 *  LSEFIT_RANGE_AUTO:  monomial basis: from a sample of x (single fit: up to
 *                      256 evenly strided points, first and last included;
 *                      batched: the first 8 and the last 8 points of each
 *                      fit, all of a shorter one): s = 2^ceil(log2(half-range))
 *                      and c = the mid-range rounded to a multiple of s/8,
 *                      replaced by 0 when it is below 2^-6 times the
 *                      half-range; c is then rounded to float32.  The result
 *                      does not depend on this choice except through rounding.
 *                      Chebyshev basis: from the exact extent [lo, hi] of the
 *                      finite x of each fit (one extra pass over x):
 *                      c = hi/2 + lo/2, s = hi/2 - lo/2 (1 when zero), so
 *                      that t covers [-1, 1], where the T_k are orthogonal;
 *                      on a sub-interval their Gram matrix loses its
 *                      conditioning quickly with the degree. */
typedef enum { LSEFIT_RANGE_GIVEN = 0, LSEFIT_RANGE_AUTO = 1 } lsefit_range_mode;

/* How the (m+1)x(m+1) normal system A X = B is solved.
 *  LSEFIT_SOLVER_GEPP:     Gaussian elimination with partial pivoting (the
 *                          method of the end of Sec. II).
 *  LSEFIT_SOLVER_CHOLESKY: A = L L^T (A is symmetric positive definite for a
 *                          determined fit), one of the "methods other than
 *                          Gaussian elimination" Sec. V names.  SINGULAR when a
 *                          diagonal of the factorisation is at most 2^-40 max|A|. */
typedef enum { LSEFIT_SOLVER_GEPP = 0, LSEFIT_SOLVER_CHOLESKY = 1 } lsefit_solver;

/* The basis the normal equations are written in.
 *  LSEFIT_BASIS_MONOMIAL:  powers of t, the method of Sec. II (degree <= 8).
 *  LSEFIT_BASIS_CHEBYSHEV: Chebyshev polynomials T_k(t) (degree <= 16), for the
 *      higher orders Sec. V leaves open: the pass sums C_k = sum T_k(t_i) and
 *      D_j = sum y_i T_j(t_i) by the recurrence T_(k+1) = 2t T_k - T_(k-1), and
 *      the Gram matrix is G_jk = (C_(j+k) + C_|j-k|) / 2 (C_0 = n), which stays
 *      well conditioned where the power-sum matrix does not.  float64 sums only
 *      (LSEFIT_PREC_F64).  Results: single fits write c_0..c_m (Chebyshev
 *      coefficients in t) followed by a_0..a_m (x-basis); batched fits write
 *      c_0..c_m and, when coef_stride >= m + 3, the fit's center and scale.
 *      fit_moments writes [c, s, C_0..C_2m, D_0..D_m] (same length 3m+4) and
 *      fit_solve reads that layout.  fit_residuals evaluates the fitted
 *      series by Clenshaw's recurrence.  fit_backward takes grad_coef =
 *      dL/dc of the Chebyshev coefficients and needs the range given
 *      (LSEFIT_RANGE_GIVEN; with the automatic range the coefficients also
 *      move with the extreme x: UNSUPPORTED). */
typedef enum { LSEFIT_BASIS_MONOMIAL = 0, LSEFIT_BASIS_CHEBYSHEV = 1 } lsefit_basis;

/* What fit_batched writes per fit in the monomial basis.
 *  LSEFIT_OUTPUT_X:       a_0..a_m (x-basis) at coef[f * coef_stride], the
 *                         rest of the row untouched.
 *  LSEFIT_OUTPUT_X_AND_T: also the t-basis solution b_0..b_m from
 *                         coef[f * coef_stride + M + 1] on and the fit's c, s
 *                         at coef[f * coef_stride + 2M + 2] and + 2M + 3
 *                         (M = opt->degree, the largest degree of the call;
 *                         needs coef_stride >= 2M + 4).  For data far from 0
 *                         (x near 1000, say) the x-basis coefficients are
 *                         large and cancel when f(x) is evaluated in float64;
 *                         f(x) = sum_j b_j ((x - c)/s)^j does not.
 * Single-fit calls always write a and then b, and report (c, s) in their
 * moments; the Chebyshev basis writes its own coefficients (see above); both
 * ignore this field. */
typedef enum { LSEFIT_OUTPUT_X = 0, LSEFIT_OUTPUT_X_AND_T = 1 } lsefit_output_basis;

typedef struct lsefit_options {
    int32_t degree;        /* single fit: m in 1..LSEFIT_MAX_DEGREE (Chebyshev basis:
                              1..LSEFIT_MAX_DEGREE_CHEBYSHEV); batched: the
                              largest degree present (each degrees[f] must be <= it) */
    int32_t precision;     /* lsefit_precision */
    int32_t refine_steps;  /* LSEFIT_PREC_F32C: 0 or 1 refinement passes; ignored otherwise */
    int32_t range_mode;    /* lsefit_range_mode */
    double center;         /* c for LSEFIT_RANGE_GIVEN */
    double scale;          /* s for LSEFIT_RANGE_GIVEN, > 0 */
    int32_t solver;        /* lsefit_solver */
    int32_t basis;         /* lsefit_basis */
    int32_t output_basis;  /* lsefit_output_basis (fit_batched, monomial basis) */
} lsefit_options;

/* Launch schedule of the streaming kernels.  Any valid schedule gives the
 * same numbers up to the summation order it implies.
 *  waves:          total wavefronts of the persistent streaming grid; each owns
 *                  an equal share of the tiles (balanced by tile count)
 *  waves_per_block: 1, 2 or 4
 *  tile:           balancing granularity in points (>= 64); a tile never spans
 *                  two fits, a wave streams the consecutive tiles of one fit
 *                  as one segment
 *  unroll:         vector loads in flight per lane and array: 1, 2 or 4 */
typedef struct lsefit_schedule {
    int32_t waves;
    int32_t waves_per_block;
    int32_t tile;
    int32_t unroll;
} lsefit_schedule;

typedef struct lsefit_plan lsefit_plan;   /* opaque: schedule, workspace, captured graph */

/* Bytes of workspace needed by fit_moments/fit_solve (batch = 1, total_points = n)
 * or by fit_batched/fit_backward (batch fits) with `schedule` (NULL: the default
 * schedule).  The workspace holds per-wave partial sums, the tile table and one
 * record per fit (c, s, power sums, t-basis solution) that fit_backward reads.
 * Its contents on entry to a fitting call do not matter (every call writes what
 * it reads), so a caller need not clear it; fit_backward and fit_residuals read
 * what the preceding fit left there. */
size_t lsefit_workspace_bytes(int64_t batch, int32_t max_degree, const lsefit_schedule* schedule);
/* (max_degree up to LSEFIT_MAX_DEGREE_CHEBYSHEV for Chebyshev-basis calls) */

/* The schedule used when no plan is given (initially sized to this device's
 * compute units: 8 waves per unit, 4 per block, tiles of 2,048 points, 2
 * vectors in flight).  lsefit_set_default_schedule replaces it for the whole
 * process (NULL restores the initial one); it is not synchronised with calls
 * running on other host threads.  Workspace sizes depend on it.  While the
 * initial schedule is in force, the power-sum, refinement and residual passes
 * of a single fit (monomial basis) over fewer than 32 MiB of points run 4
 * waves per unit instead (4 vectors in flight for float64 points), which
 * needs no more workspace; a schedule set by the caller is used as given. */
lsefit_status lsefit_default_schedule(lsefit_schedule* out);
lsefit_status lsefit_set_default_schedule(const lsefit_schedule* schedule);

/* Power-sum pass of one fit (Sec. II: the sums that form A and B).
 *  x, y:     n points, dtype dt, any alignment (16-byte aligned is fastest)
 *  n:        >= degree + 1
 *  opt:      degree, precision, range
 *  ws:       >= lsefit_workspace_bytes(1, degree, NULL) bytes, device
 *  moments:  output, device float64 [3m+4] = c, s, S_0..S_2m, T_0..T_m of
 *            t = (x - c)/s (S_0 = n exactly)
 * Errors: INVALID_ARG (null pointer, n < m+1, bad degree/option), UNSUPPORTED
 * (F32C with float64 data), WORKSPACE (ws too small), DEVICE (launch failure). */
lsefit_status fit_moments(const void* x, const void* y, int64_t n, int32_t dt,
                          const lsefit_options* opt, void* ws, size_t ws_bytes,
                          double* moments, void* stream);

/* Assembly of A (Hankel, A_jk = S_(j+k)) and B (B_j = T_j), Gaussian
 * elimination with partial pivoting (end of Sec. II), optional refinement
 * (LSEFIT_PREC_F32C with refine_steps > 0: x, y, n, dt must then be the data
 * the moments came from), and the change back to the x-basis.
 *  moments:  device [3m+4] as written by fit_moments
 *  coef:     output, device float64 [2(m+1)]: a_0..a_m (x-basis), then
 *            b_0..b_m (t-basis)
 *  status:   output, device int32 [1]
 * x and y may be NULL when no refinement is requested. */
lsefit_status fit_solve(const double* moments, const lsefit_options* opt,
                        const void* x, const void* y, int64_t n, int32_t dt,
                        void* ws, size_t ws_bytes, double* coef, int32_t* status, void* stream);

/* fit_moments followed by fit_solve in one call, with fewer launches: the
 * kernel that sums the per-block partial sums also solves (two launches for
 * LSEFIT_PREC_F64; two more for the refinement pass of LSEFIT_PREC_F32C).
 *  coef:     output, device float64 [2(m+1)]: a_0..a_m (x-basis), b_0..b_m (t-basis)
 *  status:   output, device int32 [1]
 *  moments:  optional output (NULL to skip), device float64 [3m+4] as in fit_moments
 * Errors as fit_moments. */
lsefit_status fit_single(const void* x, const void* y, int64_t n, int32_t dt, const lsefit_options* opt,
                         void* ws, size_t ws_bytes, double* coef, int32_t* status, double* moments, void* stream);

/* fit_single for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and launches as fit_single, with the workspace in a static
 * device array of LSEFIT_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends.  The call itself allocates
 * nothing (no hipMalloc, hipFree or allocating library routine; its launches
 * are never timed by lsefit_timing_*, whose events are created on demand).
 *  x, y, n, dt, opt, coef, status, moments, stream: as fit_single
 * The array is shared by every call on one GPU and keeps the last call's
 * contents; nothing in it needs to start at zero (every call writes what it
 * reads).  Calls that overlap on one GPU -- on different streams, or from
 * different host threads -- race on it and give undefined results; serialise
 * them (one stream per GPU).  A fit_residuals call on this workspace is not
 * possible (the array is not exposed).
 * Errors as fit_single, plus WORKSPACE when the workspace of this call
 * (lsefit_workspace_bytes(1, opt->degree, NULL), which grows with the default
 * schedule's wave count) exceeds LSEFIT_NOALLOC_SCRATCH_BYTES, and DEVICE when
 * the array's address cannot be resolved on the current device. */
#define LSEFIT_NOALLOC_SCRATCH_BYTES (4u << 20)
lsefit_status fit_single_noalloc(const void* x, const void* y, int64_t n, int32_t dt,
                                 const lsefit_options* opt, double* coef, int32_t* status, double* moments,
                                 void* stream);

/* One fit through an orthogonal factorisation instead of the normal equations
 * (the QR route of Sec. III, which Sec. V's "methods other than Gaussian
 * elimination" points to): every lane of the streaming pass keeps a triangular
 * factor of the rows (1, t, .., t^m | y) it reads, updated with square-root-free
 * Givens rotations (Gentleman), and the factors are merged lane -> wave ->
 * block -> fit in a fixed order (a tall-skinny tree).  The error is governed by
 * cond(V), V_ik = t_i^k, not by cond(V)^2 as for the power sums; the pass costs
 * about (m+1)(m+2)/2 + 12(m+1) float64 operations per point instead of the
 * 5m+1 of the power sums.
 *  x, y, n, dt, ws: as fit_single (same workspace size)
 *  opt:      degree 1..LSEFIT_MAX_DEGREE, range (as fit_single); precision
 *            must be LSEFIT_PREC_F64 and basis monomial (else UNSUPPORTED);
 *            solver and refine_steps are ignored
 *  coef:     output, device float64 [2(m+1)]: a_0..a_m (x-basis), b_0..b_m (t-basis)
 *  status:   output, device int32 [1]; SINGULAR when fewer than m+1 points or
 *            some |R_ii| <= 2^-40 max_k |R_kk|
 *  info:     optional output (NULL to skip), device float64 [3]: c, s and the
 *            residual sum of squares sum_i (y_i - f(x_i))^2 (NaN unless OK)
 * fit_residuals may follow on the same workspace.  Errors as fit_moments. */
lsefit_status fit_qr(const void* x, const void* y, int64_t n, int32_t dt, const lsefit_options* opt,
                     void* ws, size_t ws_bytes, double* coef, int32_t* status, double* info, void* stream);

/* fit_qr for B independent fits over CSR segments (layout as fit_batched):
 * every wave factors its segment of each fit it streams, and one thread per
 * fit merges the fit's factors in wave order and solves.
 *  coef:     output, device float64 [B * coef_stride]: a_0..a_m of fit f
 *  status:   output, device int32 [B]
 *  sse:      optional output (NULL to skip), device float64 [B]: the residual
 *            sum of squares of each fit (NaN unless OK)
 *  ws:       >= lsefit_workspace_bytes(B, opt->degree, NULL) bytes (the
 *            default schedule; no plan)
 * opt, errors and limits as fit_qr; fit_residuals may follow on the same ws. */
lsefit_status fit_qr_batched(const void* x, const void* y, const int64_t* offsets, const int32_t* degrees,
                             int64_t batch, int32_t dt, const lsefit_options* opt, void* ws, size_t ws_bytes,
                             double* coef, int32_t coef_stride, int32_t* status, double* sse, void* stream);

/* B independent fits over CSR segments: fit f owns points offsets[f] ..
 * offsets[f+1]-1 of x and y (Sec. II applied to each segment).
 *  offsets:   device int64 [B+1], non-decreasing, offsets[0] = 0, every
 *             offset within x and y (which the library cannot check: x and
 *             y have no length argument); a fit whose end lies before its
 *             start gets status INVALID_ARG and no points
 *  degrees:   device int32 [B], each in 1..opt->degree
 *  coef:      output, device float64 [B * coef_stride]: a_0..a_m of fit f at
 *             f*coef_stride; coef_stride >= opt->degree + 1; entries past m
 *             untouched (LSEFIT_OUTPUT_X_AND_T: also b and (c, s), see
 *             lsefit_output_basis; coef_stride >= 2 opt->degree + 4)
 *  status:    output, device int32 [B]
 *  plan:      NULL -> the default schedule and the caller's workspace `ws`;
 *             otherwise the plan's tuned schedule and its own workspace (ws
 *             and ws_bytes ignored) and, in the graph form (see
 *             fit_plan_tune), after the first call with the same arguments,
 *             one replay of a captured HIP graph.
 * All fits run in one launch of the persistent streaming kernel (plus the
 * tile table before it -- one kernel for at most 32 blocks of 256 fits and a
 * power-of-two tile, else two -- and one solve kernel after it). */
lsefit_status fit_batched(const void* x, const void* y, const int64_t* offsets, const int32_t* degrees,
                          int64_t batch, int32_t dt, const lsefit_options* opt,
                          lsefit_plan* plan, void* ws, size_t ws_bytes,
                          double* coef, int32_t coef_stride, int32_t* status, void* stream);

/* Reverse-mode derivative of the batched fit.  Given grad_coef = dL/da
 * (device float64 [B * coef_stride]) for the coefficients that fit_batched
 * returned, writes dL/dx and dL/dy (device, dtype dt, one per point):
 *   lambda = A_t^-1 M^T dL/da  (M maps t-basis b to x-basis a; A_t symmetric)
 *   dL/dy_i = q(t_i),  dL/dx_i = (q'(t_i) r_i - q(t_i) f'(t_i)) / s
 * with q(t) = sum_j lambda_j t^j, f(t) = sum_j b_j t^j, r_i = y_i - f(t_i),
 * powers recomputed per point (nothing per point is stored by the forward).
 * Chebyshev basis (range given): lambda = G^-1 dL/dc with the forward's Gram
 * matrix, q = sum_j lambda_j T_j and f = sum_j c_j T_j (Clenshaw's recurrence
 * and its derivative).  Points of fits whose status is not OK get NaN.
 * `plan`/`ws` must be the ones the forward call used, unchanged since (the
 * per-fit records and the tile table are read from there); lambda is written
 * into that workspace.  The tile table carries the tile size it was built
 * with, so the default schedule may change between the two calls (the pass
 * cuts every fit where the forward did); `ws_bytes` must still cover the
 * workspace size of the schedule in force (else WORKSPACE).  The streaming
 * pass of the adjoint keeps no partial sums: it runs its own launch shape
 * (16 waves per compute unit, 2 per block, 1 vector in flight per lane), not
 * the plan's, unless the caller has set a default schedule, which it then
 * uses; the gradients are the same bits under any shape.  Monomial basis: up
 * to opt->degree 3 the streaming pass solves for each fit's lambda itself
 * (one launch); above, one thread per fit solves first (two launches), with
 * the same operations. */
lsefit_status fit_backward(const void* x, const void* y, const int64_t* offsets, const int32_t* degrees,
                           int64_t batch, int32_t dt, const lsefit_options* opt,
                           lsefit_plan* plan, void* ws, size_t ws_bytes,
                           const double* grad_coef, int32_t coef_stride,
                           void* grad_x, void* grad_y, void* stream);

/* Residuals of fitted polynomials: the fitted values and errors of Table V
 * (Sec. III), e_i = y_i - f(x_i), and the sum of squared errors Pi = sum e_i^2
 * of Sec. II, per fit.  Must follow a fit on the same workspace (or plan), with
 * the same x, y and options: the per-fit (c, s) and t-basis coefficients are
 * read from there, and e_i is formed in the t variable in float64 (Chebyshev
 * basis: f = sum_j c_j T_j(t) by Clenshaw's recurrence).
 *  offsets:    NULL -> one fit of n points (after fit_single or fit_solve;
 *              degrees and batch ignored); else the batch of fit_batched
 *  sse:        output, device float64 [batch] (or [1]); NaN for fits whose
 *              status is not OK
 *  residuals:  optional output (NULL to skip), device, dtype dt, one per point */
lsefit_status fit_residuals(const void* x, const void* y, const int64_t* offsets, const int32_t* degrees,
                            int64_t batch, int64_t n, int32_t dt, const lsefit_options* opt,
                            lsefit_plan* plan, void* ws, size_t ws_bytes, double* sse, void* residuals,
                            void* stream);

/* Plans for repeated batched calls of one shape.  fit_plan_create allocates
 * the plan's workspace (device memory, freed by fit_plan_destroy) for up to
 * `batch` fits of degree <= max_degree.  fit_plan_tune times candidate
 * schedules on the given data (it synchronises `stream`): every candidate
 * with `reps` calls, then the four fastest again with 3 * reps calls each,
 * keeping the fastest of those.  It then times that schedule as eager
 * launches and as replays of a captured graph on the same call and keeps the
 * faster form (eager when the graph cannot be captured or replayed), unless
 * fit_plan_set_graph chose one (enable 1: replay a captured graph, 0: launch
 * eagerly; a new plan replays graphs).  fit_plan_get_graph reports the form
 * in use.  fit_plan_set_schedule installs a known schedule (for example from
 * a cache).  A plan must be used from one stream at a time. */
lsefit_status fit_plan_create(lsefit_plan** plan, int64_t batch, int32_t max_degree, int32_t dt,
                              int32_t precision);
lsefit_status fit_plan_tune(lsefit_plan* plan, const void* x, const void* y, const int64_t* offsets,
                            const int32_t* degrees, int64_t batch, const lsefit_options* opt,
                            double* coef, int32_t coef_stride, int32_t* status, void* stream,
                            int32_t reps, double* best_ms_out);
/* Schedule cache of fit_plan_tune (for callers that tune the same shapes in
 * many processes).  With a path set, fit_plan_tune first looks the call's
 * shape up in that text file: the key is the device (architecture, compute
 * units), dtype, options, batch and the total points rounded down to a power
 * of two.  On a hit it installs the cached schedule and the cached form (when
 * the line records one and the caller did not set one), runs the fit once
 * with it (coef and status are written as by a tuning run), writes the cached
 * time to best_ms_out and times nothing; on a miss it tunes as usual and
 * appends the result as one line.  Appends within a process are serialised; a file
 * that cannot be read is treated as empty and one that cannot be written is
 * left alone (the tuned schedule is still installed).  path NULL or "" turns
 * the cache off.  The string is copied. */
lsefit_status fit_plan_set_tune_cache(lsefit_plan* plan, const char* path);
lsefit_status fit_plan_set_schedule(lsefit_plan* plan, const lsefit_schedule* schedule);
lsefit_status fit_plan_get_schedule(const lsefit_plan* plan, lsefit_schedule* out);
lsefit_status fit_plan_set_graph(lsefit_plan* plan, int32_t enable);
lsefit_status fit_plan_get_graph(const lsefit_plan* plan, int32_t* enabled);
void fit_plan_destroy(lsefit_plan* plan);

/* A short description of a status code: any lsefit_status value, and
 * "unknown status" for every other integer. */
const char* lsefit_status_string(int32_t status);

/* Read-bandwidth probe, for measurement only (no part of the fit): streams two
 * float32 arrays of n elements (n rounded down to a multiple of 4; both
 * 16-byte aligned) with the schedule's grid and 16-byte loads and writes one
 * float per block into out[out_count >= number of blocks].  pattern 0: each
 * wave reads one contiguous share (the layout of the power-sum pass);
 * pattern 1: the grid strides over 16-byte vectors; pattern 2: each block
 * reads one contiguous share and its waves take turns over its 16-byte
 * vectors (the waves of a block together walk one stream).  nontemporal: 1 uses
 * non-temporal loads.  Timed as kind 4 by lsefit_timing_read.  Serves to
 * measure the read bandwidth the device attains with each load pattern. */
lsefit_status lsefit_read_probe(const float* x, const float* y, int64_t n, const lsefit_schedule* schedule,
                                int32_t pattern, int32_t nontemporal, float* out, size_t out_count, void* stream);

/* Copy probe, for measurement only (no part of the fit): reads two float32
 * arrays x, y of n elements (n rounded down to a multiple of 4) and writes
 * them to ox, oy with 16-byte loads and stores -- 8 bytes read and 8 written
 * per point, the traffic of the adjoint pass of fit_backward.  All four
 * pointers 16-byte aligned; pattern and nontemporal as lsefit_read_probe
 * (nontemporal applies to the loads and the stores).  Timed as kind 4. */
lsefit_status lsefit_copy_probe(const float* x, const float* y, float* ox, float* oy, int64_t n,
                                const lsefit_schedule* schedule, int32_t pattern, int32_t nontemporal,
                                void* stream);

/* Kernel timing for profiling.  While enabled, the main kernel of every
 * streaming launch made by the calls above (outside graph capture; never by
 * fit_single_noalloc) carries a clock slot: the first thread of block 0 (the
 * first block to start) stores the device's constant-rate wall clock
 * (hipDeviceAttributeWallClockRate) when it starts, and every wave folds the
 * clock into one of 32 separate lines of the slot with an atomic maximum when
 * it leaves; a launch's duration is the span from that start to the latest
 * end, taken by the kernel itself.  No event or marker is enqueued, so timed
 * launches run back to back like untimed ones; the cost is one atomic per
 * wave, spread over 32 memory lines.  The first enable allocates a device
 * pool of 16,384 slots (2 KiB each, kept until the process ends); launches
 * past the pool are not timed.  lsefit_timing_reset waits for the device and
 * clears the totals and the pool; lsefit_timing_read waits for the device and
 * returns the summed duration of one kernel kind in milliseconds and the
 * number of timed launches since the last reset.
 *  kind: 0 = power-sum pass (k_moments, or the Chebyshev / QR streaming pass),
 *        1 = refinement pass, 2 = adjoint streaming pass (not its per-fit
 *        solve), 3 = per-fit combine and solve (the finish kernel of a single
 *        fit), 4 = read or copy probe, 5 = residual pass (not its per-fit
 *        fold), 6 = range pass (Chebyshev basis, automatic range; not its
 *        per-fit fold), 7 = tile table of a batch (its first launch: the
 *        whole table when the batch has at most 32 blocks of 256 fits and a
 *        power-of-two tile, else the per-block counts, not the block offsets).
 * Not synchronised with calls on other host threads. */
lsefit_status lsefit_timing_enable(int32_t enable);
lsefit_status lsefit_timing_reset(void);
lsefit_status lsefit_timing_read(int32_t kind, double* total_ms, int64_t* launches);

/* Device ordinal's compute-unit count as the library sees it (0 on error). */
int32_t lsefit_device_cus(void);

#ifdef __cplusplus
}
#endif

#endif /* LSEFIT_H */
