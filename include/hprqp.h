/*
 * hprqp.h -- C ABI of the MI355X (gfx950) HPR-QP library, libhprqp.so.
 *
 * HPR-QP (arXiv 2507.02470) solves the convex QP of Section 1, problem
 * "QP-primal-0":
 *
 *     min_x  1/2 <x, Q x> + <c, x>   s.t.  l <= A x <= u,   L <= x <= U,
 *
 * i.e. the composite problem "QP-primal" with phi = indicator of the box
 * C = [L, U] and K = [l, u].  The library runs the dual Halpern
 * Peaceman-Rachford iteration of Algorithm 4 on the restricted Wolfe dual
 * ("QP-dual"), with the restart rule of Section 3.2 and the sigma update of
 * Algorithm 5, in FP64, entirely in hand-written HIP kernels.
 *
 * Conventions shared by every entry point:
 *  - Every array pointer is a DEVICE pointer (memory of the GPU current at
 *    hprqp_create / hprqp_batch_create) unless its comment says "host".
 *    Input arrays are borrowed: the caller keeps them alive and unchanged
 *    for the lifetime of the handle.  Outputs are caller-allocated.
 *  - Indices are int32, values double.  CSR arrays: rowptr has rows+1
 *    entries starting at 0 and non-decreasing; columns lie in [0, cols).
 *    The columns of a row may come in any order and may repeat: every
 *    product adds a row's entries in an order fixed by the data (results
 *    are deterministic and differ from those of a sorted copy by rounding
 *    only).
 *  - Infinite bounds are IEEE +-INFINITY; l_i == u_i marks an equality row.
 *  - All GPU work is enqueued on the stream given at creation; entry points
 *    return after the results they report are complete.
 *  - Errors are returned as hprqp_status; a message for the calling thread
 *    is available from hprqp_last_error().  Non-convergence is not an
 *    error: it is reported in hprqp_info.term.
 */
#ifndef HPRQP_H
#define HPRQP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HPRQP_OK = 0,
  HPRQP_ERR_ARG = 1,          /* NULL handle/pointer, bad option value          */
  HPRQP_ERR_SHAPE = 2,        /* bad sizes, CSR not monotone, column out of range */
  HPRQP_ERR_BOUNDS = 3,       /* l > u, L > U, NaN in a bound, non-finite c      */
  HPRQP_ERR_HIP = 4,          /* a HIP runtime call failed                       */
  HPRQP_ERR_OOM = 5,          /* device allocation failed                        */
  HPRQP_ERR_UNSUPPORTED = 6   /* option or problem kind not supported here       */
} hprqp_status;

typedef enum {
  HPRQP_SOLVED = 0,           /* max(eta_p, eta_d, eta_gap) <= tol               */
  HPRQP_MAX_ITER = 1,
  HPRQP_TIME_LIMIT = 2,
  HPRQP_NUMERICAL = 3         /* NaN/Inf met at a check                          */
} hprqp_term;

typedef enum {
  HPRQP_Q_ZERO = 0,           /* Q = 0 (the LP case of Remark 2.1)               */
  HPRQP_Q_CSR = 1,            /* explicit symmetric CSR, both triangles stored   */
  HPRQP_Q_KRON = 2,           /* matrix-free Q = B (x) C [- I(x)S - T(x)I] (4.5)  */
  HPRQP_Q_LOWRANK = 3,        /* Q = diag(d) + F F^T                              */
  HPRQP_Q_GRAM = 4            /* matrix-free Q = Ahat^T Ahat, Ahat sparse (Lasso) */
} hprqp_qkind;

/* Problem data (Section 1, "QP-primal"): min 1/2<x,Qx> + <c,x> + phi(x)
 * s.t. l <= Ax <= u, with phi(x) = l1_weight ||x||_1 + delta_[L,U](x)
 * (l1_weight = 0: the CQP "QP-primal-0").  Q must be self-adjoint PSD. */
typedef struct {
  int32_t n, m;               /* variables, rows of A (m may be 0: Remark 2.1)  */
  int32_t qkind;              /* hprqp_qkind                                      */
  /* HPRQP_Q_CSR: n x n, full symmetric storage */
  const int32_t *q_rowptr, *q_col; const double *q_val; int64_t q_nnz;
  /* HPRQP_Q_KRON: Q vec(X) = vec(C X B^T), X kron_s x kron_p column-major,
   * n = kron_s * kron_p; B (kron_p x kron_p) and C (kron_s x kron_s) dense
   * column-major, each symmetric PSD */
  int32_t kron_p, kron_s; const double *kron_B, *kron_C;
  /* HPRQP_Q_LOWRANK: Q = diag(lr_d) + F F^T, F n x lr_rank row-major */
  int32_t lr_rank; const double *lr_d, *lr_F;
  const double *c, *L, *U;    /* n each: objective and box C = [L, U]          */
  const int32_t *a_rowptr, *a_col; const double *a_val; int64_t a_nnz;  /* A, m x n */
  const double *l, *u;        /* m each: K = [l, u]                              */
  double l1_weight;           /* >= 0: weight of ||x||_1 in phi (Lasso, Section 4.4) */
  /* HPRQP_Q_GRAM: Q = Ahat^T Ahat applied as two products; Ahat gram_p x n CSR */
  int32_t gram_p; const int32_t *gram_rowptr, *gram_col; const double *gram_val; int64_t gram_nnz;
  /* HPRQP_Q_KRON, optional (NULL: 0): Q = B (x) C - I (x) S - T (x) I, i.e.
   * Q vec(X) = vec(C X B^T - S X - X T^T), the QAP-relaxation operator of
   * Section 4.5 (C = Ahat, B = Bhat up to the factor 2 of 1/2<x,Qx>); S
   * kron_s x kron_s and T kron_p x kron_p, dense column-major.  Q must stay
   * PSD (the LP conditions on the eigenvalues of S, T of Section 4.5). */
  const double *kron_S, *kron_T;
} hprqp_problem;

typedef struct {
  double tol;                 /* stopping tolerance on max(eta_p, eta_d, eta_gap); 1e-8 */
  int64_t max_iter;           /* iteration cap                                           */
  double time_limit_s;        /* wall-clock cap checked at each check; <= 0: none; 3600  */
  int32_t check_every;        /* restart/termination test cadence; 100                   */
  double sigma0;              /* <= 0: sigma0 = ||b||/||c|| rule of Section 4.1           */
  double lambda_A, lambda_Q;  /* <= 0: power method (Section 4.1) at create               */
  const double *power_start_A;  /* device, m: power-method start on A A^T; NULL: all ones */
  const double *power_start_Q;  /* device, n: power-method start on Q;     NULL: all ones */
  double alpha1, alpha2, alpha3;  /* restart parameters of Section 3.2; 0.2, 0.8, 0.5     */
  int32_t enable_restart;     /* 1 */
  int32_t enable_sigma_update;/* 1 */
  int32_t use_graph;          /* 1: replay each check segment as a captured HIP graph    */
  int32_t spmv_autotune;      /* 1: time lanes-per-row choices for A, A^T, Q at create   */
  int32_t trace_iters;        /* record the first K iterations into trace_host           */
  double *trace_host;         /* host, K x (2m + 4n) doubles, rows [y, w, x, ybar, wbar, xbar];
                                 y, w, x is the state carried into the next iteration
                                 (in the scaled variables when preconditioned)            */
  int32_t log_cap;            /* capacity (rows) of check_log_host                       */
  double *check_log_host;     /* host, rows of 10 doubles: k, t, R~, eta_p, eta_d, eta_gap,
                                 sigma used, restarted (0/1), sigma next, restart count  */
  int32_t profile_kernels;    /* 1: time the four per-iteration products with HIP events on
                                 the solve stream (the plain iterations of every 4th check
                                 segment, launched without a graph), see hprqp_kernel_stats */
  int32_t precondition;       /* 1: diagonal preconditioning of Section 4.1 at create, for
                                 explicit Q (HPRQP_Q_CSR, HPRQP_Q_ZERO) with l1_weight = 0;
                                 ignored otherwise (the paper applies none to a matrix-free
                                 Q, and a scaled ||x||_1 needs per-variable weights): symmetric
                                 scaling of K = [[Q, A^T], [A, 0]] by ruiz_iters Ruiz passes
                                 (divide each scale by the square root of the inf-norm of
                                 its row) and one Pock-Chambolle pass with alpha = 1 (the
                                 1-norm).  The method runs on Q~ = DQD, A~ = EAD, c~ = Dc,
                                 [L,U]/D, E[l,u]; termination is tested on the given problem
                                 and inputs/outputs stay in the given variables.  0          */
  int32_t ruiz_iters;         /* Ruiz passes of the preconditioning; 10                  */
  int32_t spmv_lanes;         /* -1: SpMV kernel per matrix from its row lengths (and the
                                 autotuner); 0: the CSR-stream kernel; -2: the CSR-stream
                                 kernel gathering from an LDS copy of the input vector
                                 (matrices with at most 14336 columns, else 0); -3: the
                                 panel-ordered product (columns cut into 4 panels walked in
                                 the same order by a persistent grid; an extra copy of the
                                 matrix; rows of at most 4096 nonzeros, else the default);
                                 -4: the column-split product (a copy of the matrix in
                                 column panels, each workgroup gathering from its panel's
                                 slice of the vector in LDS, per-panel partial sums added
                                 in panel order; matrices with more than 14336 columns and
                                 on average at least 8 nonzeros per row in a 2048-column
                                 panel or 2 in a 16384-column one, else the default);
                                 1, 2, 4, ..., 256: that many lanes per row, for every
                                 matrix; -100 - g (g = 1, 2, 4, ..., 64): g lanes per row
                                 gathering from an LDS copy of the input vector (at most
                                 14336 columns, else g lanes from memory); -1             */
  int32_t method;             /* 0: HPR-QP (Algorithm 4 on the restricted Wolfe dual).
                                 1, 2: HPR applied to the primal reformulations of
                                 Appendix A, the baselines of Table 1: 1 = Algorithm 6 on
                                 "QP-primal-s" (A x = s; state x, y), 2 = Algorithm 7 on
                                 "QP-primal-sv" (A x = s, x = v; state x, v, y, t).  Same
                                 stopping test, check cadence and restart criteria; the
                                 merit R~ uses the metric of the reformulation, sigma is
                                 updated to the minimiser of the sigma-dependent part of
                                 ||ubar - u^{r,0}||_M^2 (smoothed as in Algorithm 5), and
                                 sigma0 = ||c||/||b|| (the reciprocal rule; an explicit
                                 sigma0 is used as given).  w0 starts v (method 2; unused
                                 by 1); t starts at 0.  Outputs: ybar, zbar (the x-step's
                                 multiplier), w = xbar (1) or vbar (2), xbar.  Trace rows
                                 hold [y, v, x, ybar, vbar, xbar] (method 1: x in the v
                                 places).  Per-solve option; 0                               */
  int32_t kron_kernel;        /* HPRQP_Q_KRON product kernel: -1 choose (the K-split kernel for
                                 factors up to 384, else the LDS-tiled one, timed against each
                                 other when spmv_autotune = 1); 0: K-split kernel (one 16 x 16
                                 tile per block, K over 8 waves); 1, 2, 4, 8: LDS-tiled kernel
                                 (64 x 64 tiles) with that many split-K groups (2 to 8 only
                                 while the tiles are fewer than 4 per compute unit); -1      */
  int32_t small_path;         /* method 0 with explicit (CSR) or zero Q: run each check segment
                                 as one workgroup (the four products as phases separated by
                                 barriers, same fused epilogues) instead of four launches per
                                 iteration.  -1: when n <= 4096 and m <= 4096; 0: never; 1:
                                 always (HPRQP_ERR_UNSUPPORTED for other Q kinds).  Segments
                                 timed by profile_kernels use the four-launch path; -1       */
  int32_t batch_threads;      /* batched solve: 0: threads per workgroup of each size class by
                                 default or by the autotuner (spmv_autotune = 1); 64, 128, 256
                                 or 512: that many for every class it can hold (n <= 4 x
                                 threads), the default for the others; 0                    */
} hprqp_options;

typedef struct {
  int32_t term;               /* hprqp_term                                        */
  int64_t iters;              /* iterations done                                   */
  int32_t restarts;
  int32_t n_log;              /* rows written to check_log_host                    */
  double sigma, sigma0, lambda_A, lambda_Q;
  double eta_p, eta_d, eta_gap; /* at the returned point                          */
  double pobj, dobj;
  double R_last;              /* merit R~ at the last check                        */
  double t_setup_s, t_solve_s;  /* seconds: create (incl. power method), solve    */
  double t_precond_s;         /* seconds of create spent on the preconditioning   */
  double qwx_gap;             /* ||Q(w - x)||_inf at the returned point (w the shadow
                                 w_Q of Proposition 2.4; 0 up to rounding at a
                                 solution, where w - x lies in ker Q): a diagnostic,
                                 not part of the stopping test (which uses Q x)      */
} hprqp_info;

typedef struct hprqp_handle hprqp_handle;
typedef struct hprqp_batch hprqp_batch;

/* Fills the defaults of Section 4.1 (tol 1e-8, alpha = 0.2/0.8/0.5,
 * check_every 100, time limit 3600 s, power method, sigma0 rule). */
void hprqp_default_options(hprqp_options *opt);

/* Validates the problem (bounds, CSR structure, finiteness), builds A^T as
 * an explicit CSR on the device (rows of A^T ordered by row of A, so every
 * product is deterministic), runs the power method when lambda_A/lambda_Q
 * are not given (Section 4.1), computes sigma0 and allocates the workspace
 * (about 34 n + 15 m doubles plus A^T, plus a reordered copy of each matrix
 * whose product runs on the panel-ordered or column-split layout, and the
 * latter's per-panel partial sums).  The problem arrays are borrowed.
 * Returns HPRQP_ERR_BOUNDS / HPRQP_ERR_SHAPE on invalid data. */
hprqp_status hprqp_create(const hprqp_problem *prob, const hprqp_options *opt,
                          hipStream_t stream, hprqp_handle **out);

/* Runs Algorithm 4 from (y0, w0, x0) (each may be NULL: origin, Section 4.1)
 * and writes the last bar iterate ubar = (ybar, zbar, wbar, xbar), the output
 * of Algorithm 4: y (m), z (n), w (n; the unprojected shadow w_Q of
 * Proposition 2.4), x (n).  With options.method = 1 or 2 it runs Algorithm 6
 * or 7 instead (see hprqp_options.method for the meaning of w0 and w).
 * info may be NULL. */
hprqp_status hprqp_solve(hprqp_handle *h, const double *y0, const double *w0, const double *x0,
                         double *y, double *z, double *w, double *x, hprqp_info *info);

/* The state of Algorithm 4 at the start of an outer epoch (Algorithm 5:
 * restart index r, the first inner iterate u^{r,0}, sigma_r, the total
 * iteration count k at that point, and the restart-test state of
 * Section 4.1: the merit at the first restart, which the sigma update and
 * the alpha3 tightening compare against, and the current alpha3).  All
 * other quantities of an epoch (anchors, A^T y, Q w, the merit at t = 0)
 * are recomputed from these exactly, so a solve resumed from this state
 * repeats the iterations that followed it bit for bit.  y (m), w, x (n)
 * are DEVICE arrays owned by the caller, in the handle's internal
 * variables (scaled when the handle is preconditioned), so the state is
 * meant for a handle made from the same problem with the same create
 * options. */
typedef struct {
  int64_t k;           /* iterations done before the epoch                         */
  int32_t restarts;    /* r                                                        */
  int32_t reserved;
  double sigma;        /* sigma_r                                                  */
  double R0ref;        /* merit at the first restart; negative before it           */
  double alpha3;       /* current alpha3 of eq:restart_3                           */
  double *y, *w, *x;   /* u^{r,0}: y (m), w, x (n)                                 */
} hprqp_state;

/* hprqp_solve (method 0 only; HPRQP_ERR_UNSUPPORTED otherwise) with
 * checkpoint and resume.  resume (may be NULL: the origin as start, k = 0)
 * starts the solve from a saved epoch start instead of a warm start; its
 * k must be below options.max_iter, which counts the iterations of both
 * solves together.  save (may be NULL) receives the state at the start of
 * the last epoch of this solve (its arrays must be given; they may be those
 * of resume, for a checkpoint kept in place, but not the output arrays).  A solve
 * stopped by max_iter or the time limit and resumed from its saved state
 * returns what one uninterrupted solve returns (the same iterates and
 * info, apart from the timings), since it redoes the partial epoch from
 * its start.  info->iters is the total k, restarts the total r; the check
 * log of the resumed solve holds the checks after the saved k. */
hprqp_status hprqp_solve_resume(hprqp_handle *h, const hprqp_state *resume, hprqp_state *save, double *y,
                                double *z, double *w, double *x, hprqp_info *info);

/* Replaces the per-solve options of a handle (tol, max_iter, time limit,
 * check_every, alpha's, restart/sigma switches, graph use, trace/log
 * buffers, kernel timing).  The setup-time choices made by hprqp_create
 * (lambda_A, lambda_Q, sigma0, power-method start, SpMV tuning) are kept. */
hprqp_status hprqp_set_options(hprqp_handle *h, const hprqp_options *opt);

/* Stopping quantities of Section 4.1 at the point (y, z, x), taken with Q x
 * as in the paper's eta_d and gap, in the given problem's variables (also
 * when the handle is preconditioned).  Writes eta_p, eta_d, eta_gap, pobj,
 * dobj and qwx_gap = ||Q(w - x)||_inf of *info_host (host struct; the other
 * fields are zeroed); w is the shadow iterate w_Q of Proposition 2.4 and may
 * be NULL (qwx_gap is then NaN).  y (m), z, w, x (n) are device arrays. */
hprqp_status hprqp_residuals(hprqp_handle *h, const double *y, const double *z, const double *w,
                             const double *x, hprqp_info *info_host);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc, code that must not grow the device heap):
 * the same quantities as hprqp_residuals -- eta_p, eta_d, eta_gap, pobj, dobj
 * and qwx_gap = ||Q(w - x)||_inf (w may be NULL: NaN) of the problem as given
 * -- without a handle and without allocating.  The problem is validated as
 * at hprqp_create (HPRQP_ERR_BOUNDS / HPRQP_ERR_SHAPE); A^T y is formed by
 * FP64 atomic additions (no stored transpose), so the last bits of eta_d and
 * the dual objective can differ between calls.  Workspace: a 32 MiB device
 * array of the library, one per GPU, held until the process ends; a problem
 * needing more than 8 (n [m > 0] + n [w given] + n [Kronecker Q] + (gram_p + n)
 * [Gram Q]) bytes beyond its 1.7 MiB of fixed parts is rejected with
 * HPRQP_ERR_UNSUPPORTED (n = 1e6 with m > 0 and w fits).  Calls on one GPU
 * share that array and are serialised within the process; calls from two
 * processes on one GPU use separate copies.  The work runs on `stream` and
 * the call returns after it (it synchronises the stream, so it cannot be
 * captured into a graph).  y (m), z, w, x (n) are device arrays; info_host is
 * a host struct whose other fields are zeroed. */
hprqp_status hprqp_residuals_noalloc(const hprqp_problem *prob, const double *y, const double *z,
                                     const double *w, const double *x, hprqp_info *info_host,
                                     hipStream_t stream);

/* Applies one operator of the handle: op 0: out = Q in (n -> n), op 1:
 * out = A in (n -> m), op 2: out = A^T in (m -> n, using the stored A^T). */
hprqp_status hprqp_apply(hprqp_handle *h, int32_t op, const double *in, double *out);

/* The power-method estimates of create (before the 1.01 safety factor),
 * and the number of products each took; any pointer may be NULL. */
hprqp_status hprqp_power_info(hprqp_handle *h, double *est_A, int32_t *it_A,
                              double *est_Q, int32_t *it_Q);

/* Scale factors of the preconditioning (precondition = 1 at create): D (n)
 * for the variables and E (m) for the rows of A, written to the device arrays
 * D and E (either may be NULL).  Without preconditioning both are all ones. */
hprqp_status hprqp_scaling(hprqp_handle *h, double *D, double *E);

/* Kernel timing of the last hprqp_solve made with profile_kernels = 1:
 * avg_ms_host[i] = mean duration (ms) and launches_host[i] = number of timed
 * launches of product i, i = 0: Q xhat (with its epilogue), 1: A v, 2: A^T ybar,
 * 3: Q A^T(ybar - y) with the Halpern epilogue (methods 1, 2: 0 = Q x or Q v,
 * 1 = A x, 2 = A^T(2 ybar - y), 3 unused).  Also reports the
 * kernel choice of A, A^T and Q (g_host[3], may be NULL): g > 0 lanes per row,
 * 0 the CSR-stream kernel, -1 its variant gathering from LDS, -3 the
 * panel-ordered product, -4 the column-split product, -100 - g the row-split
 * kernel with g lanes gathering from LDS. */
hprqp_status hprqp_kernel_stats(hprqp_handle *h, double *avg_ms_host, int64_t *launches_host, int32_t *g_host);

void hprqp_destroy(hprqp_handle *h);

/* ---------------------------------------------------------------------
 * Batched solve: many independent QPs (sizes may differ) solved by
 * persistent kernels, one workgroup per instance at a time, with the whole
 * of Algorithm 4 + 5 (restart, sigma update, termination) on the device.
 * The instances are cut into size classes, each run on a kernel of a block
 * size of its own (hprqp_batch_shapes); the kernels run at once, all but
 * one on streams of the library's, joined to `stream` before the solve
 * returns.  Supported: qkind HPRQP_Q_LOWRANK with lr_rank <= 16
 * and n <= 2048, m <= 64 per instance, at most n nonzeros in a row of A
 * (no preconditioning: Q is matrix-free).
 * --------------------------------------------------------------------- */

/* probs: host array of `count` problems whose arrays are device pointers;
 * instances may share arrays (e.g. one Q and A with per-instance c, l, u:
 * shared arrays are detected by address, so an A is transposed once and an F
 * padded once however many instances use it).  The library concatenates the
 * instances itself; the per-instance offsets of the vectors are those of
 * hprqp_solve_batch.  The options apply to every instance (power method per
 * instance when lambda_A/lambda_Q <= 0, from an all-ones start); time_limit_s
 * counts from the start of hprqp_solve_batch, and an instance still running
 * then stops at its next check with HPRQP_TIME_LIMIT (0: no limit).
 * Instances are scheduled largest first (hprqp_batch_set_priority sets
 * another order). */
hprqp_status hprqp_batch_create(int32_t count, const hprqp_problem *probs,
                                const hprqp_options *opt, hipStream_t stream, hprqp_batch **out);

/* Solves every instance.  Vectors are concatenated in instance order:
 * y0/y use offsets sum_{j<i} m_j, w0/x0/z/w/x use offsets sum_{j<i} n_j.
 * y0, w0, x0 may each be NULL (origin for every instance).  infos_host:
 * host array of `count` hprqp_info (may be NULL); qwx_gap of each is taken
 * at the instance's returned point after the solve kernels. */
hprqp_status hprqp_solve_batch(hprqp_batch *b, const double *y0, const double *w0, const double *x0,
                               double *y, double *z, double *w, double *x, hprqp_info *infos_host);

/* Shapes of the batched solver: the instances are cut into 4 size classes
 * (n <= 256, 512, 1024, 2048) and each class runs on a persistent kernel of
 * 64, 128, 256 or 512 threads per workgroup (a thread holds up to 4 entries,
 * so a class needs 4 x threads >= its largest n).  By default 256 threads up
 * to n = 1024 and 512 above; with spmv_autotune = 1 at hprqp_batch_create,
 * every fitting block size is timed on a sample of the class (100 iterations
 * per instance, up to 8 instances per compute unit) and the fastest is kept
 * unless the default is within 5% of it.  Host outputs (each may be NULL):
 * class_count_host[4] instances per class, class_threads_host[4] the chosen
 * threads per workgroup, class_us_host[4 * 4] the measured kernel time per
 * instance-iteration in microseconds of class c with 64 << j threads at
 * [4 c + j] (0 where not timed). */
hprqp_status hprqp_batch_shapes(hprqp_batch *b, int32_t *class_count_host, int32_t *class_threads_host,
                                double *class_us_host);

/* Elapsed time of the last hprqp_solve_batch kernels (HIP events on `stream`
 * around them), seconds. */
/* A plain streaming copy dst[i] = src[i], i < n (device arrays of doubles
 * that do not overlap), with 16-byte loads and stores when both are 16-byte
 * aligned.  Not part of the solver: the benchmark runs it to scale the HBM
 * byte counters by what they read for a known number of bytes, and to
 * measure the HBM rate plain streaming reaches.  ms_host (may be NULL)
 * receives its duration from HIP events on `stream` (and the call then
 * waits for the copy).  HPRQP_ERR_ARG for n < 0 or a NULL array. */
hprqp_status hprqp_stream_copy(const double *src, double *dst, int64_t n, hipStream_t stream, double *ms_host);

/* Queue order of the next hprqp_solve_batch calls.  A persistent kernel
 * takes its instances from a queue; the batch ends when the last instance
 * ends, so a long solve taken late sets the time of the whole batch.  With
 * priority (device array of `count` floats, a predicted length of each
 * solve, e.g. the score of hprqp_mlp_warm_start) each kernel takes its
 * instances highest priority first (ties, and non-finite priorities last, in
 * the default order); NULL restores the default (largest n first).  Results
 * do not depend on the order, only the time does. */
hprqp_status hprqp_batch_set_priority(hprqp_batch *b, const float *priority);

double hprqp_batch_last_kernel_s(hprqp_batch *b);

void hprqp_batch_destroy(hprqp_batch *b);

/* Message describing the last error of the calling thread ("" if none). */
const char *hprqp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HPRQP_H */
