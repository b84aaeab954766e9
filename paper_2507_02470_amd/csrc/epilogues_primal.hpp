// epilogues_primal.hpp -- per-row epilogues of HPR applied to the primal
// reformulations of arXiv 2507.02470, Appendix A: Algorithm 6 on
// "QP-primal-s" (split A x = s) and Algorithm 7 on "QP-primal-sv" (also
// x = v).  These are the baselines HPR-QP is compared with in Table 1.
//
// Closed forms of the steps (from the augmented Lagrangian and the stated
// proximal terms; S_x makes the x-subproblem's quadratic part isotropic):
//   s/y-step (both):  r = A x - y/sigma,  sbar = Pi_K(r),  ybar = sigma (sbar - r)
//                     (= y + sigma (sbar - A x), exactly 0 where Pi_K is inactive)
//   x-step, Alg. 6:   tau = lamQ + sigma lamA,
//                     xbar = prox_{phi/tau}(x - (Q x + c - A^T(2 ybar - y))/tau)
//   v-step, Alg. 7:   vbar = (sigma x - t + lamQ v - Q v)/(lamQ + sigma),
//                     tbar = t + sigma (vbar - x)
//   x-step, Alg. 7:   kappa = sigma (1 + lamA),
//                     xbar = prox_{phi/kappa}((sigma lamA x + sigma vbar + tbar
//                                             + A^T(2 ybar - y) - c)/kappa)
//   zbar = tau (xbar - r_x) (kappa for Alg. 7): the x-step's multiplier.
//   Halpern (Steps 4-5): u+ = rho u_a + (1 - rho)(2 ubar - u), rho = 1/(t+2).
// Each iteration is three products: Q x (Alg. 6) or Q v (Alg. 7), A x, and
// A^T (2 ybar - y); a vector gathered by a product is never written by that
// product's epilogue (v+ is written by the A^T epilogue of Alg. 7).
//
// Merit pieces (du = u - ubar), reduction index -> meaning:
//   0 |dx|^2, 1 <dx, Q dx> (Alg. 6) or |dv|^2 (Alg. 7), 2 <A dx, dy>, 3 |dy|^2,
//   4 |dt|^2, 5 <dx, dt>, 6 <dv, Q dv>;
// sigma-update pieces (D = ubar - u_a): |Dx|^2, |Dy|^2, |Dt|^2.
#pragma once
#include "common.hpp"

struct PrimalScalars {
  double sigma, rho, tau, kappa;
  __device__ void load(const DevParams* p, int j) {
    sigma = p->sigma;
    rho = 1.0 / (double)(p->t0 + j + 2);
    tau = p->lamQ + sigma * p->lamA;        // Algorithm 6
    kappa = sigma * (1.0 + p->lamA);        // Algorithm 7
  }
};

// A-product epilogue (q = (A x)_i): s/y-step and the Halpern step of y.
//   e = 2 ybar - y (gathered next by A^T);  acc[0] = |dy|^2, acc[1] = |Dy|^2.
struct EpiPY {
  const double *l, *u, *ya;
  double *y, *ybar, *e, *ax, *dy;
  int want_r, check, store_bar;
  double sigma, rho;
  static constexpr int NR = 2;
  static constexpr unsigned MAXMASK = 0u;
  __device__ void setup(const DevParams* p, int j) { PrimalScalars s; s.load(p, j); sigma = s.sigma; rho = s.rho; }
  __device__ __forceinline__ void operator()(int i, double q, double* acc) const {
    const double yi = ld_stream(y + i), yai = ld_stream(ya + i);
    const double r = q - yi / sigma;
    const double yb = sigma * (clampd(r, ld_stream(l + i), ld_stream(u + i)) - r);
    const double ei = 2.0 * yb - yi;
    e[i] = ei;
    st_stream(y + i, rho * yai + (1.0 - rho) * ei);
    if (store_bar) ybar[i] = yb;
    if (want_r) {
      ax[i] = q; dy[i] = yi - yb;
      acc[0] += (yi - yb) * (yi - yb);
    }
    if (check) acc[1] += (yb - yai) * (yb - yai);
  }
};

// Algorithm 6, A^T-product epilogue (q = (A^T e)_i; 0 without constraints):
// x-step from Q x (qx) and the Halpern step of x.
//   acc[0] = |dx|^2, acc[1] = |Dx|^2.
struct EpiP1X {
  const double *qx, *c, *L, *U, *xa;
  double *x, *XB, *ZB, *dx;
  int want_r, check, store_bar;
  double l1;
  double rho, tau;
  static constexpr int NR = 2;
  static constexpr unsigned MAXMASK = 0u;
  __device__ void setup(const DevParams* p, int j) { PrimalScalars s; s.load(p, j); rho = s.rho; tau = s.tau; }
  __device__ __forceinline__ void operator()(int i, double q, double* acc) const {
    const double xi = ld_stream(x + i), xai = ld_stream(xa + i);
    const double r = xi - (ld_stream(qx + i) + ld_stream(c + i) - q) / tau;
    const double xb = prox_phi(r, (1.0 / tau) * l1, ld_stream(L + i), ld_stream(U + i));
    st_stream(x + i, rho * xai + (1.0 - rho) * (2.0 * xb - xi));
    if (store_bar) XB[i] = xb;
    if (check) ZB[i] = tau * (xb - r);
    if (want_r) { dx[i] = xi - xb; acc[0] += (xi - xb) * (xi - xb); }
    if (check) acc[1] += (xb - xai) * (xb - xai);
  }
};

// Algorithm 7, Q-product epilogue (q = (Q v)_i): v/t-step, the Halpern step of
// t, and h = sigma vbar + tbar for the x-step.  v itself is gathered by this
// product, so its Halpern step waits for the A^T epilogue.
//   acc[0] = |dv|^2, acc[1] = |dt|^2, acc[2] = |Dt|^2.
struct EpiP2V {
  const double *v, *x, *ta;
  double *t, *vbar, *hv, *qv, *dv, *dt, *tbar;
  int want_r, check;
  double sigma, rho, lamQ;
  static constexpr int NR = 3;
  static constexpr unsigned MAXMASK = 0u;
  __device__ void setup(const DevParams* p, int j) {
    PrimalScalars s; s.load(p, j); sigma = s.sigma; rho = s.rho; lamQ = p->lamQ;
  }
  __device__ __forceinline__ void operator()(int i, double q, double* acc) const {
    const double vi = ld_stream(v + i), ti = ld_stream(t + i), xi = ld_stream(x + i), tai = ld_stream(ta + i);
    const double vb = (sigma * xi - ti + lamQ * vi - q) / (lamQ + sigma);
    const double tb = ti + sigma * (vb - xi);
    vbar[i] = vb;
    hv[i] = sigma * vb + tb;
    st_stream(t + i, rho * tai + (1.0 - rho) * (2.0 * tb - ti));
    if (want_r) {
      qv[i] = q; dv[i] = vi - vb; dt[i] = ti - tb;
      acc[0] += (vi - vb) * (vi - vb);
      acc[1] += (ti - tb) * (ti - tb);
    }
    if (check) { tbar[i] = tb; acc[2] += (tb - tai) * (tb - tai); }
  }
};

// Algorithm 7, A^T-product epilogue (q = (A^T e)_i; 0 without constraints):
// x-step and the Halpern steps of x and v.
//   acc[0] = |dx|^2, acc[1] = <dx, dt>, acc[2] = |Dx|^2.
struct EpiP2X {
  const double *hv, *c, *L, *U, *xa, *va, *vbar, *dt;
  double *x, *v, *XB, *ZB, *dx;
  int want_r, check, store_bar;
  double l1;
  double sigma, rho, kappa, lamA;
  static constexpr int NR = 3;
  static constexpr unsigned MAXMASK = 0u;
  __device__ void setup(const DevParams* p, int j) {
    PrimalScalars s; s.load(p, j); sigma = s.sigma; rho = s.rho; kappa = s.kappa; lamA = p->lamA;
  }
  __device__ __forceinline__ void operator()(int i, double q, double* acc) const {
    const double xi = ld_stream(x + i), xai = ld_stream(xa + i);
    const double r = (sigma * lamA * xi + ld_stream(hv + i) + q - ld_stream(c + i)) / kappa;
    const double xb = prox_phi(r, (1.0 / kappa) * l1, ld_stream(L + i), ld_stream(U + i));
    st_stream(x + i, rho * xai + (1.0 - rho) * (2.0 * xb - xi));
    st_stream(v + i, rho * ld_stream(va + i) + (1.0 - rho) * (2.0 * ld_stream(vbar + i) - ld_stream(v + i)));
    if (store_bar) XB[i] = xb;
    if (check) ZB[i] = kappa * (xb - r);
    if (want_r) {
      dx[i] = xi - xb;
      acc[0] += (xi - xb) * (xi - xb);
      acc[1] += (xi - xb) * dt[i];
    }
    if (check) acc[2] += (xb - xai) * (xb - xai);
  }
};

// Merit: q = (A xbar)_i;  acc[0] += (A x - A xbar)_i dy_i = (A dx)_i dy_i
struct EpiMeritA {
  const double *ax, *dy;
  static constexpr int NR = 1;
  static constexpr unsigned MAXMASK = 0u;
  __device__ void setup(const DevParams*, int) {}
  __device__ __forceinline__ void operator()(int i, double q, double* acc) const { acc[0] += (ax[i] - q) * dy[i]; }
};

// Merit: q = (Q ubar_blk)_i; acc[0] += d_i (Q u_blk - Q ubar_blk)_i = <d, Q d>
struct EpiMeritQ {
  const double *qold, *d;
  static constexpr int NR = 1;
  static constexpr unsigned MAXMASK = 0u;
  __device__ void setup(const DevParams*, int) {}
  __device__ __forceinline__ void operator()(int i, double q, double* acc) const { acc[0] += d[i] * (qold[i] - q); }
};
