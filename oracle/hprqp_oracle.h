/*
 * hprqp_oracle.h -- plain single-threaded FP64 CPU oracle for HPR-QP.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * What it computes (arXiv 2507.02470, "HPR-QP"):
 *   - the CCQP of Section 1 (problem "QP-primal"): min 1/2<x,Qx> + <c,x> + phi(x)
 *     s.t. l <= Ax <= u, with phi(x) = lambda ||x||_1 + delta_[L,U](x) (lambda = 0:
 *     the CQP "QP-primal-0"; m = 0, Q = Ahat^T Ahat: the Lasso of Section 4.4);
 *   - Algorithm 4 (HPR-QP, Section 3) with the closed-form subproblem updates
 *     of Section 3.1 ("update-z", "update-x", "update-w", "update-y"), the
 *     restart criteria of Section 3.2 ("eq:restart_1".."eq:restart_3") and
 *     Algorithm 5 (SigmaUpdate, Section 3.3);
 *   - the merit R~ = ||u - ubar||_M with M the metric of Section 2.3
 *     ("eq:metric-M");
 *   - the stopping quantities eta_p, eta_d, eta_gap of Section 4.1;
 *   - HPR applied to the primal reformulations "QP-primal-s" and
 *     "QP-primal-sv" (Algorithms 6 and 7 of Appendix A), the baselines of
 *     Table 1, with the restart rule carried over from HPR-QP.
 * Every product A x, A^T y, Q x is recomputed directly from the data each
 * time it is needed (no cached linear combinations).
 */
#ifndef HPRQP_ORACLE_H
#define HPRQP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_Q_ZERO = 0, ORC_Q_CSR = 1, ORC_Q_KRON = 2, ORC_Q_LOWRANK = 3, ORC_Q_GRAM = 4 };
enum { ORC_SOLVED = 0, ORC_MAX_ITER = 1, ORC_TIME_LIMIT = 2, ORC_NUMERICAL = 3 };

typedef struct {
  int n, m;
  int qkind;
  const int *q_rowptr, *q_col; const double *q_val;      /* CSR, full symmetric   */
  int kron_p, kron_s; const double *kron_B, *kron_C;     /* Q = B (x) C, col-major */
  int lr_rank; const double *lr_d, *lr_F;                /* Q = diag(d) + F F^T, F row-major n x r */
  const double *c, *L, *U;                               /* box C = [L, U]        */
  const int *a_rowptr, *a_col; const double *a_val;      /* A, m x n CSR          */
  const double *l, *u;                                   /* K = [l, u]            */
  double l1_weight;       /* lambda >= 0: phi(x) = lambda ||x||_1 + delta_[L,U](x)   */
  int gram_p; const int *gram_rowptr, *gram_col; const double *gram_val;
                          /* Q = Ahat^T Ahat, Ahat p x n CSR (matrix-free Q)          */
  const double *kron_S, *kron_T;  /* Kronecker Q only, may be NULL: Q = B (x) C
                          - I (x) S - T (x) I (the QAP relaxation of Section 4.5),
                          S s x s, T p x p, column-major                             */
} orc_problem;

typedef struct {
  double tol;             /* stop when max(eta_p, eta_d, eta_gap) <= tol            */
  int64_t max_iter;
  int check_every;        /* restart/termination test cadence                        */
  double time_limit_s;    /* <= 0: none                                               */
  double sigma0;          /* <= 0: ||b||/||c|| rule                                   */
  double lambda_A, lambda_Q;  /* <= 0: power method from the given start vectors      */
  const double *power_start_A;  /* m-vector (start of the power method on A A^T)     */
  const double *power_start_Q;  /* n-vector (start of the power method on Q)         */
  double alpha1, alpha2, alpha3;
  int enable_restart, enable_sigma_update;
  int trace_iters;        /* record the first K iterations into `trace`               */
  double *trace;          /* K x (2m + 4n): [y, w, x (carried state), ybar, wbar, xbar] */
  int log_cap;            /* capacity (rows) of check_log                             */
  double *check_log;      /* rows of 10: k, t, R, eta_p, eta_d, eta_gap, sigma_used,
                             restarted, sigma_next, r                                 */
  int precondition;       /* explicit Q (CSR or zero) and phi a box indicator only:
                             solve the diagonally scaled problem, stop on the
                             residuals of the given one                               */
  int ruiz_iters;         /* Ruiz passes of the scaling (Section 4.1: 10)             */
  int method;             /* 0: HPR-QP (Algorithm 4); 1, 2: HPR on the primal
                             reformulation "QP-primal-s" (Algorithm 6) or
                             "QP-primal-sv" (Algorithm 7) of Appendix A             */
} orc_options;

typedef struct {
  int term; int64_t iters; int restarts; int n_log;
  double sigma, sigma0, lambda_A, lambda_Q;
  double eta_p, eta_d, eta_gap, pobj, dobj;
  double R_last, t_solve_s;
} orc_info;

/* Linear operators (definitions written out). */
void orc_apply_Q(const orc_problem *P, const double *x, double *out);
void orc_apply_A(const orc_problem *P, const double *x, double *out);
void orc_apply_AT(const orc_problem *P, const double *y, double *out);

/* Power method: Rayleigh-quotient estimate of lambda_1(A A^T) (which=0) or
 * lambda_1(Q) (which=1) from `start`, stopping at relative change <= tol or
 * after maxit products.  Returns the raw estimate; *iters gets the count.   */
double orc_power(const orc_problem *P, int which, const double *start, int maxit,
                 double tol, int *iters);

/* sigma0 rule of Section 4.1 (parameter setting). */
double orc_sigma0(const orc_problem *P);

/* theta_1, theta_2, theta_3 and the cross term <A^T dy - Q dw, dx> for a
 * difference (dy, dw, dx); out[4].                                          */
void orc_thetas(const orc_problem *P, double lamA, double lamQ,
                const double *dy, const double *dw, const double *dx, double *out);
/* ||(dy, dw, dz, dx)||_M^2 for the metric M of Algorithm 3 (z-block is 0).  */
double orc_mnorm2(const orc_problem *P, double sigma, double lamA, double lamQ,
                  const double *dy, const double *dw, const double *dx);
/* Algorithm 5 without the smoothing: argmin of f(sigma) by golden section. */
double orc_sigma_argmin(double th1, double th2, double th3, double lamQ);
/* Restart test of Section 3.2 at a check ("eq:restart_1".."eq:restart_3"):
 * bit 1, 2, 4 set for the criterion that holds (0: no restart).  R: merit of
 * the iteration just completed; Rr0: merit of the epoch's first iteration;
 * Rprev: merit at the epoch's previous check, negative if there is none;
 * t, k: iterations done in the epoch and in total.                          */
int orc_restart_test(double R, double Rr0, double Rprev, int64_t t, int64_t k,
                     double alpha1, double alpha2, double alpha3);
/* alpha_3 after a restart with ratio R~_{r,tau_r-1}/R~_{0,tau_0-1} (Section
 * 4.1): 0.2 when ratio <= 0.1, else unchanged.                             */
double orc_alpha3_next(double alpha3, double ratio);

/* Diagonal preconditioning (Section 4.1, "Preconditioning"): scale factors
 * D (n, variables) and E (m, rows of A) of the symmetric scaling of
 * K = [[Q, A^T], [A, 0]]: `ruiz_iters` Ruiz passes (each scale divided by the
 * square root of the inf-norm of its row of the currently scaled K), then,
 * if pock_chambolle, one Pock-Chambolle pass with alpha = 1 (divided by the
 * square root of the 1-norm of the row).  Explicit Q (CSR or zero) only.
 * The scaled problem is  Q~ = D Q D, A~ = E A D, c~ = D c, [L, U]~ = [L, U]/D,
 * [l, u]~ = E [l, u];  its solution maps back as x = D x~, w = D w~,
 * z = z~ / D, y = E y~.                                                      */
void orc_scaling(const orc_problem *P, int ruiz_iters, int pock_chambolle, double *D, double *E);

/* Prox of sigma phi for phi(x) = lambda ||x||_1 + delta_[L,U](x), entry j:
 * the soft threshold of r at sigma lambda, clamped to [L_j, U_j].           */
double orc_prox(const orc_problem *P, int j, double sigma, double r);

/* eta_p, eta_d, eta_gap, pobj, dobj at (y, z, x); out[5]. */
void orc_residuals(const orc_problem *P, const double *y, const double *z,
                   const double *x, double *out);

/* One pass of Steps 1-3 of Algorithm 6 (variant 1) or 7 (variant 2) from the
 * state (x, v, y, t) (v, t, vb, tb: variant 2 only, else unused).  Writes
 * sbar, ybar (m), vbar, tbar, xbar and zbar (n), zbar the multiplier of the
 * x-step (-zbar in the subdifferential of phi at xbar).                    */
void orc_primal_step(const orc_problem *P, int variant, double sigma, double lamA, double lamQ,
                     const double *x, const double *v, const double *y, const double *t,
                     double *sb, double *yb, double *vb, double *tb, double *xb, double *zb);
/* ||(dx, dv, dy, dt)||_M^2 for the metric of Algorithm 6/7 (dv, dt: variant 2). */
double orc_primal_mnorm2(const orc_problem *P, int variant, double sigma, double lamA, double lamQ,
                         const double *dx, const double *dv, const double *dy, const double *dt);

/* Algorithm 4 (method 0), or Algorithm 6/7 (method 1/2: w0 is the start of
 * v for method 2 and unused for method 1; the output w is xbar for method 1
 * and vbar for method 2).  y0/w0/x0 may be NULL (origin).  Outputs ubar =
 * (y, z, w, x). */
int orc_solve(const orc_problem *P, const orc_options *opt,
              const double *y0, const double *w0, const double *x0,
              double *y, double *z, double *w, double *x, orc_info *info);

#ifdef __cplusplus
}
#endif
#endif
