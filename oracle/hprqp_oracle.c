/*
 * hprqp_oracle.c -- plain single-threaded FP64 CPU oracle for HPR-QP
 * (arXiv 2507.02470).  TEST INFRASTRUCTURE ONLY: see hprqp_oracle.h.
 *
 * Written for checkability by eye, not for speed: scalar loops, products
 * recomputed from the data every time, no blocking, fusion or caching.
 * Build without -ffast-math (IEEE binary64, round to nearest even).
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes of the repository as well):
 *  - Halpern weight 1/(t+2) with the inner counter t of the current epoch
 *    (Algorithm 4 prints the global counter; Algorithm 3 and the restart
 *    rationale of Section 3.2 use the per-epoch count).
 *  - Restart/termination are tested every `check_every` iterations and at
 *    max_iter; termination is tested before restart.
 *  - The restart criteria use the R~ of the iteration just completed; the
 *    epoch reference R~_{r,0} is the R~ of the epoch's first iteration;
 *    criterion 2 compares with the previous check of the same epoch and is
 *    skipped at an epoch's first check.
 *  - The smoothing reference R~_{0,tau_0-1} is the R~ that triggered the
 *    first restart; alpha_3 drops to 0.2 for good once the ratio used for
 *    beta is <= 0.1 at a restart.
 *  - theta_3 is clamped at 0 (only theta_1, theta_2 are clamped at 1e-12 in
 *    Algorithm 5); the golden-section search runs on log(sigma) over the
 *    bracket where f' changes sign, to a relative width of 1e-12.
 *  - The Halpern step is applied to (y, w, x) only: z^{r,t} is never read by
 *    the updates of Algorithm 4 (zbar is recomputed from (y, w, x)).
 *  - A term of the dual objective whose bound is infinite counts 0 when its
 *    multiplier is exactly 0.
 *  - HPR on the primal reformulations (Appendix A, method 1 and 2): the
 *    paper says only that they use restart and sigma strategies similar to
 *    HPR-QP's.  Here: the same restart criteria on R~ = ||u - ubar||_M with
 *    the metric M of the reformulation (derived from the steps, see
 *    orc_primal_mnorm2); sigma <- minimiser of the sigma-dependent part of
 *    ||ubar - u^{r,0}||_M^2, smoothed as in Algorithm 5; sigma0 = ||c||/||b||;
 *    the multiplier t of x = v starts at 0; s is read by no step and is not
 *    carried.
 */
#include "hprqp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* ------------------------------------------------------------------------ */
/* Small vector helpers                                                      */
/* ------------------------------------------------------------------------ */
static double *vnew(int k) { return (double *)calloc((size_t)(k > 0 ? k : 1), sizeof(double)); }
static double dot(const double *a, const double *b, int k) {
  double s = 0.0;
  for (int i = 0; i < k; ++i) s += a[i] * b[i];
  return s;
}
static double nrm2(const double *a, int k) { return sqrt(dot(a, a, k)); }
static double nrminf(const double *a, int k) {
  double s = 0.0;
  for (int i = 0; i < k; ++i) { double v = fabs(a[i]); if (v > s) s = v; }
  return s;
}
static double clamp(double v, double lo, double hi) {
  /* projection of one coordinate onto [lo, hi] (lo <= hi, either infinite) */
  if (v < lo) return lo;
  if (v > hi) return hi;
  return v;
}
static double now_s(void) {
  struct timespec ts; clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* ------------------------------------------------------------------------ */
/* Linear operators                                                          */
/* ------------------------------------------------------------------------ */
void orc_apply_Q(const orc_problem *P, const double *x, double *out) {
  const int n = P->n;
  if (P->qkind == ORC_Q_ZERO) {
    for (int i = 0; i < n; ++i) out[i] = 0.0;
  } else if (P->qkind == ORC_Q_CSR) {
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int k = P->q_rowptr[i]; k < P->q_rowptr[i + 1]; ++k) s += P->q_val[k] * x[P->q_col[k]];
      out[i] = s;
    }
  } else if (P->qkind == ORC_Q_KRON) {
    /* (B (x) C) vec(X) = vec(C X B^T), X s x p column-major (Section 4.5). */
    const int p = P->kron_p, s = P->kron_s;
    const double *B = P->kron_B, *C = P->kron_C;
    double *T = vnew(s * p);
    for (int b = 0; b < p; ++b)             /* T = C X */
      for (int i = 0; i < s; ++i) {
        double acc = 0.0;
        for (int a = 0; a < s; ++a) acc += C[i + (size_t)s * a] * x[a + (size_t)s * b];
        T[i + (size_t)s * b] = acc;
      }
    for (int j = 0; j < p; ++j)             /* out = T B^T */
      for (int i = 0; i < s; ++i) {
        double acc = 0.0;
        for (int b = 0; b < p; ++b) acc += T[i + (size_t)s * b] * B[j + (size_t)p * b];
        out[i + (size_t)s * j] = acc;
      }
    /* QAP relaxation (Section 4.5): Q = B (x) C - I (x) S - T (x) I, i.e.
     * out -= vec(S X) + vec(X T^T) */
    if (P->kron_S)
      for (int j = 0; j < p; ++j)
        for (int i = 0; i < s; ++i) {
          double acc = 0.0;
          for (int a = 0; a < s; ++a) acc += P->kron_S[i + (size_t)s * a] * x[a + (size_t)s * j];
          out[i + (size_t)s * j] -= acc;
        }
    if (P->kron_T)
      for (int j = 0; j < p; ++j)
        for (int i = 0; i < s; ++i) {
          double acc = 0.0;
          for (int b = 0; b < p; ++b) acc += x[i + (size_t)s * b] * P->kron_T[j + (size_t)p * b];
          out[i + (size_t)s * j] -= acc;
        }
    free(T);
  } else if (P->qkind == ORC_Q_GRAM) {
    /* Q x = Ahat^T (Ahat x) */
    const int p = P->gram_p;
    double *t = vnew(p);
    for (int i = 0; i < p; ++i) {
      double acc = 0.0;
      for (int k = P->gram_rowptr[i]; k < P->gram_rowptr[i + 1]; ++k) acc += P->gram_val[k] * x[P->gram_col[k]];
      t[i] = acc;
    }
    for (int j = 0; j < n; ++j) out[j] = 0.0;
    for (int i = 0; i < p; ++i)
      for (int k = P->gram_rowptr[i]; k < P->gram_rowptr[i + 1]; ++k) out[P->gram_col[k]] += P->gram_val[k] * t[i];
    free(t);
  } else { /* ORC_Q_LOWRANK: diag(d) x + F (F^T x) */
    const int r = P->lr_rank;
    double *t = vnew(r);
    for (int k = 0; k < r; ++k) {
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc += P->lr_F[(size_t)j * r + k] * x[j];
      t[k] = acc;
    }
    for (int i = 0; i < n; ++i) {
      double acc = P->lr_d[i] * x[i];
      for (int k = 0; k < r; ++k) acc += P->lr_F[(size_t)i * r + k] * t[k];
      out[i] = acc;
    }
    free(t);
  }
}

void orc_apply_A(const orc_problem *P, const double *x, double *out) {
  for (int i = 0; i < P->m; ++i) {
    double s = 0.0;
    for (int k = P->a_rowptr[i]; k < P->a_rowptr[i + 1]; ++k) s += P->a_val[k] * x[P->a_col[k]];
    out[i] = s;
  }
}

void orc_apply_AT(const orc_problem *P, const double *y, double *out) {
  for (int j = 0; j < P->n; ++j) out[j] = 0.0;
  for (int i = 0; i < P->m; ++i)
    for (int k = P->a_rowptr[i]; k < P->a_rowptr[i + 1]; ++k) out[P->a_col[k]] += P->a_val[k] * y[i];
}

/* ------------------------------------------------------------------------ */
/* Power method (Section 4.1, parameter setting)                            */
/* ------------------------------------------------------------------------ */
double orc_power(const orc_problem *P, int which, const double *start, int maxit,
                 double tol, int *iters) {
  const int k = (which == 0) ? P->m : P->n;
  if (k == 0) { if (iters) *iters = 0; return 0.0; }
  double *v = vnew(k), *w = vnew(k), *tmp = vnew(P->n);
  double nv = nrm2(start, k);
  for (int i = 0; i < k; ++i) v[i] = start[i] / nv;
  double lam = 0.0, lam_old = 0.0;
  int it = 0;
  for (it = 1; it <= maxit; ++it) {
    if (which == 0) { orc_apply_AT(P, v, tmp); orc_apply_A(P, tmp, w); }   /* A A^T v */
    else orc_apply_Q(P, v, w);
    lam = dot(v, w, k);                                                     /* Rayleigh quotient */
    double nw = nrm2(w, k);
    if (nw == 0.0) break;
    if (it > 1 && fabs(lam - lam_old) <= tol * fabs(lam)) break;
    lam_old = lam;
    for (int i = 0; i < k; ++i) v[i] = w[i] / nw;
  }
  if (iters) *iters = (it > maxit) ? maxit : it;
  free(v); free(w); free(tmp);
  return lam;
}

/* sigma0 = ||b|| / ||c||, b_i = max(|l_i|, |u_i|) with infinite entries read as 0. */
double orc_sigma0(const orc_problem *P) {
  double sb = 0.0;
  for (int i = 0; i < P->m; ++i) {
    double a = isinf(P->l[i]) ? 0.0 : fabs(P->l[i]);
    double b = isinf(P->u[i]) ? 0.0 : fabs(P->u[i]);
    double bi = a > b ? a : b;
    sb += bi * bi;
  }
  double nb = sqrt(sb), nc = nrm2(P->c, P->n);
  if (nb >= 1e-16 && nb <= 1e16 && nc >= 1e-16 && nc <= 1e16) return nb / nc;
  return 1.0;
}

/* ------------------------------------------------------------------------ */
/* Metric M (Section 2.3, "eq:metric-M") and the theta's ("eq:theta")       */
/* ------------------------------------------------------------------------ */
void orc_thetas(const orc_problem *P, double lamA, double lamQ,
                const double *dy, const double *dw, const double *dx, double *out) {
  const int n = P->n, m = P->m;
  double *Qdw = vnew(n), *ATdy = vnew(n), *QATdy = vnew(n);
  orc_apply_Q(P, dw, Qdw);
  orc_apply_AT(P, dy, ATdy);
  orc_apply_Q(P, ATdy, QATdy);
  /* theta_1 = lamA ||dy||^2 + lamQ ||dw||_Q^2 - 2 <Q dw, A^T dy> */
  out[0] = lamA * dot(dy, dy, m) + lamQ * dot(dw, Qdw, n) - 2.0 * dot(Qdw, ATdy, n);
  /* theta_2 = ||dx||^2 */
  out[1] = dot(dx, dx, n);
  /* theta_3 = ||A^T dy||_Q^2 */
  out[2] = dot(ATdy, QATdy, n);
  /* cross term of M: <A_Q (dy, dw), dx> = <A^T dy - Q dw, dx> */
  double cr = 0.0;
  for (int i = 0; i < n; ++i) cr += (ATdy[i] - Qdw[i]) * dx[i];
  out[3] = cr;
  free(Qdw); free(ATdy); free(QATdy);
}

/* With T_1 = S + S_sGS, S_y = lamA I - A A^*, S_w = Q(lamQ I - Q) and
 * S_sGS1 = sigma^2 A Q (sigma Q^2 + Q + sigma S_w)^{-1} Q A^* (which on the
 * range of Q equals sigma^2/(1+sigma lamQ) A Q A^*), the quadratic form of M
 * splits into the theta's:
 *   ||du||_M^2 = sigma th1 + th2/sigma + sigma^2 th3/(1+sigma lamQ) + 2 cross. */
double orc_mnorm2(const orc_problem *P, double sigma, double lamA, double lamQ,
                  const double *dy, const double *dw, const double *dx) {
  double th[4];
  orc_thetas(P, lamA, lamQ, dy, dw, dx, th);
  return sigma * th[0] + th[1] / sigma + sigma * sigma * th[2] / (1.0 + sigma * lamQ) + 2.0 * th[3];
}

/* Divided difference (f(a) - f(b)) / (a - b) of f(sigma) = th1 s + th2/s +
 * s^2 th3/(1 + lamQ s) ("eq:update-sigma-approx"), written without
 * cancellation:  th1 - th2/(a b) + th3 (a + b + lamQ a b)/((1+lamQ a)(1+lamQ b)). */
static double f_sigma_slope(double a, double b, double th1, double th2, double th3, double lamQ) {
  return th1 - th2 / (a * b) + th3 * (a + b + lamQ * a * b) / ((1.0 + lamQ * a) * (1.0 + lamQ * b));
}

/* argmin_{sigma > 0} f(sigma) by golden-section search (Algorithm 5, step 4).
 * f' = th1 + (th3/lamQ)(1 - (1+lamQ s)^-2) - th2/s^2, so the minimiser lies in
 * [sqrt(th2/(th1 + th3/lamQ)), sqrt(th2/th1)]; the search runs on log(sigma).
 * The comparison f(c) < f(d) (c < d) is taken as the sign of the divided
 * difference, which keeps it exact down to rounding instead of sqrt(eps). */
double orc_sigma_argmin(double th1, double th2, double th3, double lamQ) {
  double hi = sqrt(th2 / th1);
  if (th3 <= 0.0 || lamQ <= 0.0) return hi;
  double lo = sqrt(th2 / (th1 + th3 / lamQ));
  double a = log(lo), b = log(hi);
  const double g = 0.5 * (sqrt(5.0) - 1.0);
  for (int it = 0; it < 200 && (b - a) > log1p(1e-12); ++it) {
    double c = b - g * (b - a), d = a + g * (b - a);
    /* f(c) < f(d)  <=>  slope(c, d) > 0 since c < d */
    if (f_sigma_slope(exp(c), exp(d), th1, th2, th3, lamQ) > 0.0) b = d;
    else a = c;
  }
  return exp(0.5 * (a + b));
}

/* Restart test of Section 3.2, taken at a check.  R is the merit R~ of the
 * iteration just completed, Rr0 that of the epoch's first iteration (the
 * reference R~_{r,0}), Rprev that of the previous check of the same epoch
 * (negative: this is the epoch's first check, and the comparison of the second
 * criterion has nothing to compare with); t and k are the iterations done in
 * the epoch and in total.  Returns a bit mask of the criteria that hold:
 *   1  sufficient decay, "eq:restart_1":          R <= alpha1 Rr0
 *   2  insufficient local progress, "eq:restart_2": R <= alpha2 Rr0 and R > Rprev
 *   4  excessively long inner loop, "eq:restart_3": t >= alpha3 k
 * Any nonzero mask ends the epoch.                                         */
int orc_restart_test(double R, double Rr0, double Rprev, int64_t t, int64_t k,
                     double alpha1, double alpha2, double alpha3) {
  int mask = 0;
  if (R <= alpha1 * Rr0) mask |= 1;
  if (Rprev >= 0.0 && R <= alpha2 * Rr0 && R > Rprev) mask |= 2;
  if ((double)t >= alpha3 * (double)k) mask |= 4;
  return mask;
}

/* alpha_3 for the epochs after a restart (Section 4.1, parameter setting):
 * tightened to 0.2 once the ratio R~_{r,tau_r-1}/R~_{0,tau_0-1} of the
 * restart is at most 0.1, and kept there.                                  */
double orc_alpha3_next(double alpha3, double ratio) {
  return (ratio <= 0.1) ? 0.2 : alpha3;
}

/* ------------------------------------------------------------------------ */
/* Diagonal preconditioning (Section 4.1, "Preconditioning")               */
/* ------------------------------------------------------------------------ */
/* Row norms of the scaled K = diag(D, E) [[Q, A^T], [A, 0]] diag(D, E):
 * p = 0: inf-norm, p = 1: 1-norm.  For variable j the row holds row j of
 * D Q D and column j of E A D; for constraint i, row i of E A D.          */
static void scaled_row_norms(const orc_problem *P, const double *D, const double *E, int p,
                             double *nx, double *ny) {
  const int n = P->n, m = P->m;
  double *nq = vnew(n), *na = vnew(n);
  if (P->qkind == ORC_Q_CSR)
    for (int i = 0; i < n; ++i)
      for (int k = P->q_rowptr[i]; k < P->q_rowptr[i + 1]; ++k) {
        const double a = fabs(D[i] * P->q_val[k] * D[P->q_col[k]]);
        if (p == 0) { if (a > nq[i]) nq[i] = a; } else nq[i] += a;
      }
  for (int i = 0; i < m; ++i) {
    ny[i] = 0.0;
    for (int k = P->a_rowptr[i]; k < P->a_rowptr[i + 1]; ++k) {
      const int j = P->a_col[k];
      const double a = fabs(E[i] * P->a_val[k] * D[j]);
      if (p == 0) { if (a > ny[i]) ny[i] = a; if (a > na[j]) na[j] = a; }
      else { ny[i] += a; na[j] += a; }
    }
  }
  for (int j = 0; j < n; ++j) nx[j] = (p == 0) ? (nq[j] > na[j] ? nq[j] : na[j]) : nq[j] + na[j];
  free(nq); free(na);
}

static void divide_by_sqrt(double *f, const double *nrm, int k) {
  for (int i = 0; i < k; ++i)
    if (nrm[i] > 0.0) f[i] /= sqrt(nrm[i]);
}

void orc_scaling(const orc_problem *P, int ruiz_iters, int pock_chambolle, double *D, double *E) {
  const int n = P->n, m = P->m;
  double *nx = vnew(n), *ny = vnew(m);
  for (int j = 0; j < n; ++j) D[j] = 1.0;
  for (int i = 0; i < m; ++i) E[i] = 1.0;
  for (int it = 0; it < ruiz_iters; ++it) {          /* Ruiz equilibration */
    scaled_row_norms(P, D, E, 0, nx, ny);
    divide_by_sqrt(D, nx, n);
    divide_by_sqrt(E, ny, m);
  }
  if (pock_chambolle) {                              /* Pock-Chambolle, alpha = 1 */
    scaled_row_norms(P, D, E, 1, nx, ny);
    divide_by_sqrt(D, nx, n);
    divide_by_sqrt(E, ny, m);
  }
  free(nx); free(ny);
}

/* ------------------------------------------------------------------------ */
/* phi(x) = lambda ||x||_1 + delta_[L,U](x): prox and conjugate              */
/* ------------------------------------------------------------------------ */
double orc_prox(const orc_problem *P, int j, double sigma, double r) {
  const double t = sigma * P->l1_weight;
  double v = r;
  if (t > 0.0) v = (r > t) ? r - t : ((r < -t) ? r + t : 0.0);   /* soft threshold */
  return clamp(v, P->L[j], P->U[j]);
}

/* -phi_j^*(-z) for phi_j(x) = lambda |x| + delta_[L_j,U_j](x):
 * phi_j^*(s) = sup_{L <= x <= U} (s x - lambda |x|), attained at L, U or 0.
 * It is +inf (dual objective -inf) when L = -inf and z > lambda, or when
 * U = +inf and z < -lambda.  With lambda > 0 a multiplier that exceeds
 * lambda by rounding only (by at most 1e-12 max(1, lambda)) counts as
 * lambda.  Sets *inf and returns 0 in the infinite case.                  */
static double neg_conj_phi(const orc_problem *P, int j, double z, int *inf) {
  const double lam = P->l1_weight, L = P->L[j], U = P->U[j];
  const double slack = lam > 0.0 ? 1e-12 * (lam > 1.0 ? lam : 1.0) : 0.0;
  if ((isinf(L) && z > lam + slack) || (isinf(U) && z < -lam - slack)) { *inf = 1; return 0.0; }
  double best = -INFINITY;
  if (!isinf(L)) { double v = -z * L - lam * fabs(L); if (v > best) best = v; }
  if (!isinf(U)) { double v = -z * U - lam * fabs(U); if (v > best) best = v; }
  if (L <= 0.0 && 0.0 <= U && best < 0.0) best = 0.0;
  return -best;
}

/* ------------------------------------------------------------------------ */
/* Stopping quantities (Section 4.1, "Termination")                         */
/* ------------------------------------------------------------------------ */
void orc_residuals(const orc_problem *P, const double *y, const double *z,
                   const double *x, double *out) {
  const int n = P->n, m = P->m;
  double *Ax = vnew(m), *Qx = vnew(n), *ATy = vnew(n);
  orc_apply_A(P, x, Ax);
  orc_apply_Q(P, x, Qx);
  orc_apply_AT(P, y, ATy);
  /* primal: ||Ax - Pi_K(Ax)||_inf / (1 + max(||b||_inf, ||Ax||_inf)) */
  double rp = 0.0, nb = 0.0;
  for (int i = 0; i < m; ++i) {
    double d = fabs(Ax[i] - clamp(Ax[i], P->l[i], P->u[i]));
    if (d > rp) rp = d;
    double a = isinf(P->l[i]) ? 0.0 : fabs(P->l[i]);
    double b = isinf(P->u[i]) ? 0.0 : fabs(P->u[i]);
    if (a > nb) nb = a;
    if (b > nb) nb = b;
  }
  double nAx = nrminf(Ax, m);
  double eta_p = rp / (1.0 + (nb > nAx ? nb : nAx));
  /* dual: ||-Qx + A^T y + z - c||_inf / (1 + max(||c||, ||A^T y||, ||Qx||)) */
  double rd = 0.0;
  for (int j = 0; j < n; ++j) {
    double d = fabs(-Qx[j] + ATy[j] + z[j] - P->c[j]);
    if (d > rd) rd = d;
  }
  double den = nrminf(P->c, n);
  double t1 = nrminf(ATy, n), t2 = nrminf(Qx, n);
  if (t1 > den) den = t1;
  if (t2 > den) den = t2;
  double eta_d = rd / (1.0 + den);
  /* objectives: P = 1/2 x'Qx + c'x + phi(x);
   * D = -1/2 x'Qx - delta*_K(-y) - phi*(-z), where
   * -delta*_K(-y) = sum_i (l_i y_i^+ + u_i y_i^-). */
  double xQx = dot(x, Qx, n), cx = dot(P->c, x, n);
  double l1 = 0.0;
  for (int j = 0; j < n; ++j) l1 += fabs(x[j]);
  double pobj = 0.5 * xQx + cx + P->l1_weight * l1;          /* phi(x) on the box */
  double sup = 0.0; int dual_inf = 0;
  for (int i = 0; i < m; ++i) {
    if (y[i] > 0.0) { if (isinf(P->l[i])) dual_inf = 1; else sup += P->l[i] * y[i]; }
    else if (y[i] < 0.0) { if (isinf(P->u[i])) dual_inf = 1; else sup += P->u[i] * y[i]; }
  }
  for (int j = 0; j < n; ++j) sup += neg_conj_phi(P, j, z[j], &dual_inf);   /* -phi^*(-z) */
  double dobj = dual_inf ? -INFINITY : (-0.5 * xQx + sup);
  double eta_gap;
  if (dual_inf) eta_gap = INFINITY;
  else {
    double ap = fabs(pobj), ad = fabs(dobj);
    eta_gap = fabs(pobj - dobj) / (1.0 + (ap > ad ? ap : ad));
  }
  out[0] = eta_p; out[1] = eta_d; out[2] = eta_gap; out[3] = pobj; out[4] = dobj;
  free(Ax); free(Qx); free(ATy);
}

/* ------------------------------------------------------------------------ */
/* Algorithm 4 (HPR-QP) with Algorithm 5 (SigmaUpdate)                      */
/* ------------------------------------------------------------------------ */
/* P: the problem iterated on; P0, D, E (when D != NULL): the given problem
 * whose residuals at the unscaled point (E ybar, zbar / D, D xbar) decide
 * termination (P is then the scaled problem of orc_scaling).              */
static int solve_core(const orc_problem *P, const orc_problem *P0, const double *D, const double *E,
                      const orc_options *opt, const double *y0, const double *w0, const double *x0,
                      double *y_out, double *z_out, double *w_out, double *x_out, orc_info *info) {
  const int n = P->n, m = P->m;
  const double t_start = now_s();
  memset(info, 0, sizeof(*info));

  /* ---- parameters (Section 4.1) ---- */
  double lamA = opt->lambda_A, lamQ = opt->lambda_Q;
  if (lamA <= 0.0) {
    lamA = (m > 0) ? 1.01 * orc_power(P, 0, opt->power_start_A, 5000, 1e-6, NULL) : 0.0;
  }
  if (lamQ <= 0.0) {
    lamQ = (P->qkind == ORC_Q_ZERO) ? 0.0 : 1.01 * orc_power(P, 1, opt->power_start_Q, 5000, 1e-6, NULL);
  }
  double sigma = (opt->sigma0 > 0.0) ? opt->sigma0 : orc_sigma0(P);
  info->lambda_A = lamA; info->lambda_Q = lamQ; info->sigma0 = sigma;
  const int T = opt->check_every > 0 ? opt->check_every : 1;

  /* ---- state u = (y, w, x), anchor u^{r,0}, bars ---- */
  double *y = vnew(m), *w = vnew(n), *x = vnew(n);
  double *ya = vnew(m), *wa = vnew(n), *xa = vnew(n);
  double *yb = vnew(m), *wb = vnew(n), *xb = vnew(n), *zb = vnew(n);
  double *ATy = vnew(n), *Qw = vnew(n), *rz = vnew(n), *xh = vnew(n), *wh = vnew(n);
  double *Qwh = vnew(n), *vv = vnew(n), *ry = vnew(m), *dyv = vnew(m), *ATd = vnew(n);
  double *dy = vnew(m), *dw = vnew(n), *dx = vnew(n);
  if (y0) memcpy(y, y0, sizeof(double) * m);
  if (w0) memcpy(w, w0, sizeof(double) * n);
  if (x0) memcpy(x, x0, sizeof(double) * n);

  int64_t k = 0;
  int r = 0, term = -1;
  double alpha3 = opt->alpha3;
  double R0ref = -1.0;       /* R~_{0, tau_0 - 1} */
  double R = 0.0;
  const int rowlen = 2 * m + 4 * n;

  while (term < 0) {
    /* ---- new outer iteration r: anchor u^{r,0} ---- */
    memcpy(ya, y, sizeof(double) * m); memcpy(wa, w, sizeof(double) * n); memcpy(xa, x, sizeof(double) * n);
    int64_t t = 0;
    double Rr0 = -1.0, Rprev = -1.0;
    int restarted = 0;
    while (!restarted && term < 0) {
      const double sQ = sigma * lamQ;
      /* z-step and x-step ("update-z", "update-x"):
       *   r_z = x + sigma(-Q w + A^T y - c),  xbar = Pi_C(r_z),  zbar = (xbar - r_z)/sigma */
      orc_apply_AT(P, y, ATy);
      orc_apply_Q(P, w, Qw);
      for (int j = 0; j < n; ++j) {
        rz[j] = x[j] + sigma * (-Qw[j] + ATy[j] - P->c[j]);
        xb[j] = orc_prox(P, j, sigma, rz[j]);
        zb[j] = (xb[j] - rz[j]) / sigma;
        xh[j] = 2.0 * xb[j] - x[j];                                   /* xhat */
      }
      /* first w-step ("update-w"): w_{1/2} = (sigma lamQ w + xhat)/(1 + sigma lamQ) */
      for (int j = 0; j < n; ++j) wh[j] = (sQ * w[j] + xh[j]) / (1.0 + sQ);
      /* y-step ("update-y"): r_y = A(xhat + sigma(Q w - Q w_{1/2})) - sigma lamA y,
       *   ybar = (Pi_K(r_y) - r_y) / (sigma lamA) */
      orc_apply_Q(P, wh, Qwh);
      for (int j = 0; j < n; ++j) vv[j] = xh[j] + sigma * (Qw[j] - Qwh[j]);
      orc_apply_A(P, vv, ry);
      for (int i = 0; i < m; ++i) {
        ry[i] -= sigma * lamA * y[i];
        yb[i] = (clamp(ry[i], P->l[i], P->u[i]) - ry[i]) / (sigma * lamA);
      }
      /* second w-step ("update-w"): wbar = w_{1/2} + sigma/(1+sigma lamQ) A^T(ybar - y) */
      for (int i = 0; i < m; ++i) dyv[i] = yb[i] - y[i];
      orc_apply_AT(P, dyv, ATd);
      for (int j = 0; j < n; ++j) wb[j] = wh[j] + sigma / (1.0 + sQ) * ATd[j];

      /* merit R~ = ||u - ubar||_M of this iteration (needed at the epoch's
       * first iteration and at every check) */
      const int is_check = ((k + 1) % T == 0) || (k + 1 >= opt->max_iter);
      if (t == 0 || is_check) {
        for (int i = 0; i < m; ++i) dy[i] = y[i] - yb[i];
        for (int j = 0; j < n; ++j) { dw[j] = w[j] - wb[j]; dx[j] = x[j] - xb[j]; }
        double m2 = orc_mnorm2(P, sigma, lamA, lamQ, dy, dw, dx);
        R = sqrt(m2 > 0.0 ? m2 : 0.0);
      }

      /* Halpern step: u^{r,t+1} = 1/(t+2) u^{r,0} + (t+1)/(t+2) (2 ubar - u) */
      const double rho = 1.0 / (double)(t + 2);
      for (int i = 0; i < m; ++i) y[i] = rho * ya[i] + (1.0 - rho) * (2.0 * yb[i] - y[i]);
      for (int j = 0; j < n; ++j) {
        w[j] = rho * wa[j] + (1.0 - rho) * (2.0 * wb[j] - w[j]);
        x[j] = rho * xa[j] + (1.0 - rho) * (2.0 * xb[j] - x[j]);
      }
      t += 1; k += 1;
      if (t == 1) Rr0 = R;

      double sigma_used = sigma;
      if (is_check) {
        double res[5];
        if (D) {
          for (int i = 0; i < m; ++i) dy[i] = E[i] * yb[i];
          for (int j = 0; j < n; ++j) { dw[j] = zb[j] / D[j]; dx[j] = D[j] * xb[j]; }
          orc_residuals(P0, dy, dw, dx, res);
        } else {
          orc_residuals(P, yb, zb, xb, res);
        }
        info->eta_p = res[0]; info->eta_d = res[1]; info->eta_gap = res[2];
        info->pobj = res[3]; info->dobj = res[4];
        double kkt = res[0];
        if (res[1] > kkt) kkt = res[1];
        if (res[2] > kkt) kkt = res[2];
        int do_restart = 0;
        if (!(kkt == kkt) || !(R == R)) term = ORC_NUMERICAL;        /* NaN guard */
        else if (kkt <= opt->tol) term = ORC_SOLVED;
        else if (k >= opt->max_iter) term = ORC_MAX_ITER;
        else if (opt->time_limit_s > 0.0 && now_s() - t_start >= opt->time_limit_s) term = ORC_TIME_LIMIT;
        else if (opt->enable_restart)
          do_restart = orc_restart_test(R, Rr0, Rprev, t, k, opt->alpha1, opt->alpha2, alpha3) != 0;
        Rprev = R;
        if (term < 0 && do_restart) {
          if (R0ref < 0.0) R0ref = R;
          double ratio = R / R0ref;
          if (opt->enable_sigma_update) {
            /* Algorithm 5 with dy = ybar - y^{r,0}, dw = wbar - w^{r,0}, dx = xbar - x^{r,0} */
            double th[4];
            for (int i = 0; i < m; ++i) dy[i] = yb[i] - ya[i];
            for (int j = 0; j < n; ++j) { dw[j] = wb[j] - wa[j]; dx[j] = xb[j] - xa[j]; }
            orc_thetas(P, lamA, lamQ, dy, dw, dx, th);
            double th1 = th[0] > 1e-12 ? th[0] : 1e-12;
            double th2 = th[1] > 1e-12 ? th[1] : 1e-12;
            double th3 = th[2] > 0.0 ? th[2] : 0.0;
            double snew = orc_sigma_argmin(th1, th2, th3, lamQ);
            double beta = exp(-ratio);
            sigma = exp(beta * log(snew) + (1.0 - beta) * log(sigma));
          }
          alpha3 = orc_alpha3_next(alpha3, ratio);
          /* u^{r+1,0} = ubar^{r,tau_r} */
          memcpy(y, yb, sizeof(double) * m); memcpy(w, wb, sizeof(double) * n); memcpy(x, xb, sizeof(double) * n);
          r += 1;
          restarted = 1;
        }
        if (opt->check_log && info->n_log < opt->log_cap) {
          double *row = opt->check_log + 10 * (size_t)info->n_log;
          row[0] = (double)k; row[1] = (double)t; row[2] = R; row[3] = res[0]; row[4] = res[1];
          row[5] = res[2]; row[6] = sigma_used; row[7] = (double)restarted; row[8] = sigma; row[9] = (double)r;
          info->n_log += 1;
        }
      }
      if (opt->trace && k <= opt->trace_iters) {
        double *row = opt->trace + (size_t)(k - 1) * rowlen;
        memcpy(row, y, sizeof(double) * m); row += m;
        memcpy(row, w, sizeof(double) * n); row += n;
        memcpy(row, x, sizeof(double) * n); row += n;
        memcpy(row, yb, sizeof(double) * m); row += m;
        memcpy(row, wb, sizeof(double) * n); row += n;
        memcpy(row, xb, sizeof(double) * n);
      }
    }
  }

  /* output ubar of the last iteration (Algorithm 4, "Output") */
  memcpy(y_out, yb, sizeof(double) * m);
  memcpy(z_out, zb, sizeof(double) * n);
  memcpy(w_out, wb, sizeof(double) * n);
  memcpy(x_out, xb, sizeof(double) * n);
  info->term = term; info->iters = k; info->restarts = r; info->sigma = sigma; info->R_last = R;
  info->t_solve_s = now_s() - t_start;

  free(y); free(w); free(x); free(ya); free(wa); free(xa); free(yb); free(wb); free(xb); free(zb);
  free(ATy); free(Qw); free(rz); free(xh); free(wh); free(Qwh); free(vv); free(ry); free(dyv); free(ATd);
  free(dy); free(dw); free(dx);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* HPR on the primal reformulations (Appendix A): the two baselines of       */
/* Table 1.  Variant 1 splits Ax = s ("QP-primal-s", Algorithm 6), variant 2  */
/* also x = v ("QP-primal-sv", Algorithm 7).                                 */
/* ------------------------------------------------------------------------ */
/* One pass of Steps 1-3 from the state (x, v, y, t) (v, t: variant 2 only;
 * s is read by no step, so it is not part of the state):
 *   Step 1/2:  sbar = Pi_K(r), r = Ax - y/sigma (the minimiser of L_sigma
 *              over s), ybar = y + sigma (sbar - Ax) = sigma (sbar - r);
 *   variant 2: vbar = (sigma x - t + lamQ v - Q v)/(lamQ + sigma)  (the v-part
 *              of Step 1 with the proximal term S_v = lamQ I - Q),
 *              tbar = t + sigma (vbar - x);
 *   Step 3, variant 1 (S_x = lamQ I - Q + sigma(lamA I - A^T A)): the quadratic
 *              part of the subproblem becomes tau/2 ||x||^2, tau = lamQ + sigma lamA,
 *              so xbar = prox_{phi/tau}(x - (Q x + c - A^T(2 ybar - y))/tau);
 *   Step 3, variant 2 (S_x = sigma(lamA I - A^T A)): kappa = sigma (1 + lamA),
 *              xbar = prox_{phi/kappa}((sigma lamA x + sigma vbar + tbar
 *                                        + A^T(2 ybar - y) - c)/kappa).
 * zbar = tau (xbar - r) (kappa for variant 2), r the prox argument: the
 * multiplier with -zbar in the subdifferential of phi at xbar.            */
void orc_primal_step(const orc_problem *P, int variant, double sigma, double lamA, double lamQ,
                     const double *x, const double *v, const double *y, const double *t,
                     double *sb, double *yb, double *vb, double *tb, double *xb, double *zb) {
  const int n = P->n, m = P->m;
  double *Ax = vnew(m), *e = vnew(m), *g = vnew(n), *Qin = vnew(n);
  orc_apply_A(P, x, Ax);
  for (int i = 0; i < m; ++i) {
    /* ybar = y + sigma (sbar - Ax) written as sigma (sbar - r), r = Ax - y/sigma
     * (the same number up to rounding): ybar is exactly 0 where the
     * projection is inactive, so its sign always matches the active bound */
    const double r = Ax[i] - y[i] / sigma;
    sb[i] = clamp(r, P->l[i], P->u[i]);
    yb[i] = sigma * (sb[i] - r);
    e[i] = 2.0 * yb[i] - y[i];
  }
  orc_apply_AT(P, e, g);
  if (variant == 1) {
    const double tau = lamQ + sigma * lamA;
    orc_apply_Q(P, x, Qin);
    for (int j = 0; j < n; ++j) {
      double r = x[j] - (Qin[j] + P->c[j] - g[j]) / tau;
      xb[j] = orc_prox(P, j, 1.0 / tau, r);
      zb[j] = tau * (xb[j] - r);
    }
  } else {
    const double kap = sigma * (1.0 + lamA);
    orc_apply_Q(P, v, Qin);
    for (int j = 0; j < n; ++j) {
      vb[j] = (sigma * x[j] - t[j] + lamQ * v[j] - Qin[j]) / (lamQ + sigma);
      tb[j] = t[j] + sigma * (vb[j] - x[j]);
      double r = (sigma * lamA * x[j] + sigma * vb[j] + tb[j] + g[j] - P->c[j]) / kap;
      xb[j] = orc_prox(P, j, 1.0 / kap, r);
      zb[j] = kap * (xb[j] - r);
    }
  }
  free(Ax); free(e); free(g); free(Qin);
}

/* ||du||_M^2 for the metric of the preconditioned proximal-point form of
 * Algorithms 6 and 7 (0 in T(ubar) + M(ubar - u), T the KKT operator of the
 * reformulation; the s-block of M is 0):
 *   variant 1: <dx, (tau I - Q) dx> - 2 <A dx, dy> + ||dy||^2 / sigma;
 *   variant 2: kappa ||dx||^2 - 2 <A dx, dy> - 2 <dx, dt> + (||dy||^2 + ||dt||^2)/sigma
 *              + <dv, (lamQ I - Q) dv>.                                    */
double orc_primal_mnorm2(const orc_problem *P, int variant, double sigma, double lamA, double lamQ,
                         const double *dx, const double *dv, const double *dy, const double *dt) {
  const int n = P->n, m = P->m;
  double *Adx = vnew(m), *Qd = vnew(n);
  orc_apply_A(P, dx, Adx);
  double r = -2.0 * dot(Adx, dy, m) + dot(dy, dy, m) / sigma;
  if (variant == 1) {
    orc_apply_Q(P, dx, Qd);
    r += (lamQ + sigma * lamA) * dot(dx, dx, n) - dot(dx, Qd, n);
  } else {
    orc_apply_Q(P, dv, Qd);
    r += sigma * (1.0 + lamA) * dot(dx, dx, n) - 2.0 * dot(dx, dt, n) + dot(dt, dt, n) / sigma
         + lamQ * dot(dv, dv, n) - dot(dv, Qd, n);
  }
  free(Adx); free(Qd);
  return r;
}

/* Algorithms 6/7 with the restart and sigma strategy carried over from
 * HPR-QP (readings listed in the header comment of this file):
 *   merit R~ = ||u - ubar||_M (metric above), restart criteria of Section 3.2;
 *   sigma update: the minimiser of the sigma-dependent part of
 *   ||ubar - u^{r,0}||_M^2, i.e. sqrt(th2/th1) with th1 = lamA ||Dx||^2
 *   (variant 2: (1 + lamA) ||Dx||^2) and th2 = ||Dy||^2 (+ ||Dt||^2), both
 *   clamped at 1e-12, then the smoothing of Algorithm 5 with beta = exp(-ratio);
 *   sigma0 = ||c|| / ||b|| (the reciprocal of the HPR-QP rule: here sigma
 *   multiplies the primal residual);  state (x, v, y, t) from (x0, w0, y0, 0).
 * Output: ubar with w = xbar (variant 1) or vbar (variant 2).              */
static int solve_primal(const orc_problem *P, const orc_problem *P0, const double *D, const double *E,
                        const orc_options *opt, const double *y0, const double *w0, const double *x0,
                        double *y_out, double *z_out, double *w_out, double *x_out, orc_info *info) {
  const int n = P->n, m = P->m, var = opt->method;
  const double t_start = now_s();
  memset(info, 0, sizeof(*info));
  double lamA = opt->lambda_A, lamQ = opt->lambda_Q;
  if (lamA <= 0.0) lamA = (m > 0) ? 1.01 * orc_power(P, 0, opt->power_start_A, 5000, 1e-6, NULL) : 0.0;
  if (lamQ <= 0.0)
    lamQ = (P->qkind == ORC_Q_ZERO) ? 0.0 : 1.01 * orc_power(P, 1, opt->power_start_Q, 5000, 1e-6, NULL);
  double sigma = opt->sigma0;
  if (sigma <= 0.0) {
    double d = orc_sigma0(P);
    sigma = (d == 1.0) ? 1.0 : 1.0 / d;
  }
  info->lambda_A = lamA; info->lambda_Q = lamQ; info->sigma0 = sigma;
  const int T = opt->check_every > 0 ? opt->check_every : 1;

  double *x = vnew(n), *v = vnew(n), *y = vnew(m), *t = vnew(n);
  double *xa = vnew(n), *va = vnew(n), *ya = vnew(m), *ta = vnew(n);
  double *xb = vnew(n), *vb = vnew(n), *yb = vnew(m), *tb = vnew(n), *sb = vnew(m), *zb = vnew(n);
  double *dx = vnew(n), *dv = vnew(n), *dy = vnew(m), *dt = vnew(n);
  if (x0) memcpy(x, x0, sizeof(double) * n);
  if (w0 && var == 2) memcpy(v, w0, sizeof(double) * n);
  if (y0) memcpy(y, y0, sizeof(double) * m);

  int64_t k = 0;
  int r = 0, term = -1;
  double alpha3 = opt->alpha3, R0ref = -1.0, R = 0.0;
  const int rowlen = 2 * m + 4 * n;
  while (term < 0) {
    memcpy(xa, x, sizeof(double) * n); memcpy(va, v, sizeof(double) * n);
    memcpy(ya, y, sizeof(double) * m); memcpy(ta, t, sizeof(double) * n);
    int64_t it = 0;
    double Rr0 = -1.0, Rprev = -1.0;
    int restarted = 0;
    while (!restarted && term < 0) {
      orc_primal_step(P, var, sigma, lamA, lamQ, x, v, y, t, sb, yb, vb, tb, xb, zb);
      const int is_check = ((k + 1) % T == 0) || (k + 1 >= opt->max_iter);
      if (it == 0 || is_check) {
        for (int j = 0; j < n; ++j) { dx[j] = x[j] - xb[j]; dv[j] = v[j] - vb[j]; dt[j] = t[j] - tb[j]; }
        for (int i = 0; i < m; ++i) dy[i] = y[i] - yb[i];
        double m2 = orc_primal_mnorm2(P, var, sigma, lamA, lamQ, dx, dv, dy, dt);
        R = sqrt(m2 > 0.0 ? m2 : 0.0);
      }
      /* Steps 4-5: u <- 1/(t+2) u^{r,0} + (t+1)/(t+2) (2 ubar - u) */
      const double rho = 1.0 / (double)(it + 2);
      for (int j = 0; j < n; ++j) {
        x[j] = rho * xa[j] + (1.0 - rho) * (2.0 * xb[j] - x[j]);
        if (var == 2) {
          v[j] = rho * va[j] + (1.0 - rho) * (2.0 * vb[j] - v[j]);
          t[j] = rho * ta[j] + (1.0 - rho) * (2.0 * tb[j] - t[j]);
        }
      }
      for (int i = 0; i < m; ++i) y[i] = rho * ya[i] + (1.0 - rho) * (2.0 * yb[i] - y[i]);
      it += 1; k += 1;
      if (it == 1) Rr0 = R;
      double sigma_used = sigma;
      if (is_check) {
        double res[5];
        if (D) {
          for (int i = 0; i < m; ++i) dy[i] = E[i] * yb[i];
          for (int j = 0; j < n; ++j) { dv[j] = zb[j] / D[j]; dx[j] = D[j] * xb[j]; }
          orc_residuals(P0, dy, dv, dx, res);
        } else {
          orc_residuals(P, yb, zb, xb, res);
        }
        info->eta_p = res[0]; info->eta_d = res[1]; info->eta_gap = res[2];
        info->pobj = res[3]; info->dobj = res[4];
        double kkt = res[0];
        if (res[1] > kkt) kkt = res[1];
        if (res[2] > kkt) kkt = res[2];
        int do_restart = 0;
        if (!(kkt == kkt) || !(R == R)) term = ORC_NUMERICAL;
        else if (kkt <= opt->tol) term = ORC_SOLVED;
        else if (k >= opt->max_iter) term = ORC_MAX_ITER;
        else if (opt->time_limit_s > 0.0 && now_s() - t_start >= opt->time_limit_s) term = ORC_TIME_LIMIT;
        else if (opt->enable_restart)
          do_restart = orc_restart_test(R, Rr0, Rprev, it, k, opt->alpha1, opt->alpha2, alpha3) != 0;
        Rprev = R;
        if (term < 0 && do_restart) {
          if (R0ref < 0.0) R0ref = R;
          double ratio = R / R0ref;
          if (opt->enable_sigma_update && !(var == 1 && m == 0)) {
            double nx = 0.0, ny = 0.0, nt = 0.0;
            for (int j = 0; j < n; ++j) {
              nx += (xb[j] - xa[j]) * (xb[j] - xa[j]);
              if (var == 2) nt += (tb[j] - ta[j]) * (tb[j] - ta[j]);
            }
            for (int i = 0; i < m; ++i) ny += (yb[i] - ya[i]) * (yb[i] - ya[i]);
            double th1 = (var == 1 ? lamA : 1.0 + lamA) * nx, th2 = ny + nt;
            if (th1 < 1e-12) th1 = 1e-12;
            if (th2 < 1e-12) th2 = 1e-12;
            double snew = sqrt(th2 / th1);
            double beta = exp(-ratio);
            sigma = exp(beta * log(snew) + (1.0 - beta) * log(sigma));
          }
          alpha3 = orc_alpha3_next(alpha3, ratio);
          memcpy(x, xb, sizeof(double) * n); memcpy(y, yb, sizeof(double) * m);
          if (var == 2) { memcpy(v, vb, sizeof(double) * n); memcpy(t, tb, sizeof(double) * n); }
          r += 1;
          restarted = 1;
        }
        if (opt->check_log && info->n_log < opt->log_cap) {
          double *row = opt->check_log + 10 * (size_t)info->n_log;
          row[0] = (double)k; row[1] = (double)it; row[2] = R; row[3] = res[0]; row[4] = res[1];
          row[5] = res[2]; row[6] = sigma_used; row[7] = (double)restarted; row[8] = sigma; row[9] = (double)r;
          info->n_log += 1;
        }
      }
      if (opt->trace && k <= opt->trace_iters) {
        /* [y, v, x, ybar, vbar, xbar]; variant 1 has no v: x stands in its place */
        double *row = opt->trace + (size_t)(k - 1) * rowlen;
        memcpy(row, y, sizeof(double) * m); row += m;
        memcpy(row, var == 2 ? v : x, sizeof(double) * n); row += n;
        memcpy(row, x, sizeof(double) * n); row += n;
        memcpy(row, yb, sizeof(double) * m); row += m;
        memcpy(row, var == 2 ? vb : xb, sizeof(double) * n); row += n;
        memcpy(row, xb, sizeof(double) * n);
      }
    }
  }
  memcpy(y_out, yb, sizeof(double) * m);
  memcpy(z_out, zb, sizeof(double) * n);
  memcpy(w_out, var == 2 ? vb : xb, sizeof(double) * n);
  memcpy(x_out, xb, sizeof(double) * n);
  info->term = term; info->iters = k; info->restarts = r; info->sigma = sigma; info->R_last = R;
  info->t_solve_s = now_s() - t_start;
  free(x); free(v); free(y); free(t); free(xa); free(va); free(ya); free(ta);
  free(xb); free(vb); free(yb); free(tb); free(sb); free(zb); free(dx); free(dv); free(dy); free(dt);
  return 0;
}

static int solve_method(const orc_problem *P, const orc_problem *P0, const double *D, const double *E,
                        const orc_options *opt, const double *y0, const double *w0, const double *x0,
                        double *y_out, double *z_out, double *w_out, double *x_out, orc_info *info) {
  if (opt->method == 1 || opt->method == 2)
    return solve_primal(P, P0, D, E, opt, y0, w0, x0, y_out, z_out, w_out, x_out, info);
  return solve_core(P, P0, D, E, opt, y0, w0, x0, y_out, z_out, w_out, x_out, info);
}

int orc_solve(const orc_problem *P, const orc_options *opt,
              const double *y0, const double *w0, const double *x0,
              double *y_out, double *z_out, double *w_out, double *x_out, orc_info *info) {
  if (!opt->precondition || (P->qkind != ORC_Q_CSR && P->qkind != ORC_Q_ZERO) || P->l1_weight != 0.0)
    return solve_method(P, NULL, NULL, NULL, opt, y0, w0, x0, y_out, z_out, w_out, x_out, info);
  /* Section 4.1: solve the scaled problem, stop on the given one */
  const int n = P->n, m = P->m;
  const int nq = (P->qkind == ORC_Q_CSR) ? P->q_rowptr[n] : 0;
  const int na = (m > 0) ? P->a_rowptr[m] : 0;
  double *D = vnew(n), *E = vnew(m);
  orc_scaling(P, opt->ruiz_iters, 1, D, E);
  double *qv = vnew(nq), *av = vnew(na), *c = vnew(n), *L = vnew(n), *U = vnew(n), *l = vnew(m), *u = vnew(m);
  for (int i = 0; i < n && P->qkind == ORC_Q_CSR; ++i)
    for (int k = P->q_rowptr[i]; k < P->q_rowptr[i + 1]; ++k) qv[k] = D[i] * P->q_val[k] * D[P->q_col[k]];
  for (int i = 0; i < m; ++i)
    for (int k = P->a_rowptr[i]; k < P->a_rowptr[i + 1]; ++k) av[k] = E[i] * P->a_val[k] * D[P->a_col[k]];
  for (int j = 0; j < n; ++j) { c[j] = D[j] * P->c[j]; L[j] = P->L[j] / D[j]; U[j] = P->U[j] / D[j]; }
  for (int i = 0; i < m; ++i) { l[i] = E[i] * P->l[i]; u[i] = E[i] * P->u[i]; }
  orc_problem S = *P;
  S.q_val = qv; S.a_val = av; S.c = c; S.L = L; S.U = U; S.l = l; S.u = u;
  /* a warm start given in the original variables enters scaled */
  double *ys = NULL, *ws = NULL, *xs = NULL;
  if (y0) { ys = vnew(m); for (int i = 0; i < m; ++i) ys[i] = y0[i] / E[i]; }
  if (w0) { ws = vnew(n); for (int j = 0; j < n; ++j) ws[j] = w0[j] / D[j]; }
  if (x0) { xs = vnew(n); for (int j = 0; j < n; ++j) xs[j] = x0[j] / D[j]; }
  int rc = solve_method(&S, P, D, E, opt, ys, ws, xs, y_out, z_out, w_out, x_out, info);
  for (int i = 0; i < m; ++i) y_out[i] *= E[i];
  for (int j = 0; j < n; ++j) { z_out[j] /= D[j]; w_out[j] *= D[j]; x_out[j] *= D[j]; }
  free(D); free(E); free(qv); free(av); free(c); free(L); free(U); free(l); free(u);
  free(ys); free(ws); free(xs);
  return rc;
}
