// epilogues.hpp -- per-row epilogues fused into the Q / A / A^T products of
// one HPR-QP iteration (Algorithm 4 with the closed forms of Section 3.1).
//
// Names follow the paper: xh = xhat, wh = wbar_{Q}^{t+1/2}, yb/wb/xb/zb =
// ybar/wbar_Q/xbar/zbar, *_a = anchor u^{r,0}.  Linearity caches (GPU only):
// ATy = A^T y and Qw = Q w_Q are carried through the Halpern step instead of
// being recomputed (they are reset from exact products at every restart).
#pragma once
#include "common.hpp"

// out_i = q_i
struct EpiStore {
  double* out;
  static constexpr int NR = 0;
  static constexpr unsigned MAXMASK = 0u;
  __device__ void setup(const DevParams*, int) {}
  __device__ __forceinline__ void operator()(int i, double q, double*) const { out[i] = q; }
};

// Q-apply #1:  q1 = Q xhat;  v = xhat + sigma (Qw - Q w_half)
//   with Q w_half = (sigma lamQ Qw + q1)/(1 + sigma lamQ)  ("update-w", first line)
//   which simplifies to v = xhat + kappa (Qw - q1), kappa = sigma/(1+sigma lamQ).
// v is the argument of A in r_y ("update-y").
struct EpiQ1 {
  const double* xh; const double* Qw; double* v; double* q1;
  double kappa;
  static constexpr int NR = 0;
  // panel-ordered product: prefetched chunks, four row blocks per workgroup
  // (random QP, n = 1e6: 45.9 against 46.4 us; A v and A^T ybar lose with it)
  static constexpr bool PANEL_PREFETCH = true;
  static constexpr unsigned MAXMASK = 0u;
  __device__ void setup(const DevParams* p, int j) { IterScalars s; s.load(p, j); kappa = s.kappa; }
  __device__ __forceinline__ void operator()(int i, double q, double*) const {
    st_stream(q1 + i, q);                                   // read once, by Q-apply #2
    v[i] = xh[i] + kappa * (ld_stream(Qw + i) - q);          // v is gathered next: keep it cached
  }
};

// A-product:  r_y = A v - sigma lamA y;  ybar = (Pi_K(r_y) - r_y)/(sigma lamA)  ("update-y");
// Halpern:    y+ = rho y_a + (1 - rho)(2 ybar - y).
// acc[0] += ||y - ybar||^2   (merit R~ of this iteration)
// acc[1] += ||ybar - y_a||^2 (theta~_1 of Algorithm 5)
struct EpiY {
  const double *l, *u, *ya; double *y, *ybar;
  int want_r, want_th;
  double sA, rho;
  static constexpr int NR = 2;
  static constexpr unsigned MAXMASK = 0u;
  __device__ void setup(const DevParams* p, int j) { IterScalars s; s.load(p, j); sA = s.sA; rho = s.rho; }
  __device__ __forceinline__ void operator()(int i, double q, double* acc) const {
    const double yi = ld_stream(y + i), yai = ld_stream(ya + i);
    const double r = q - sA * yi;
    const double yb = (clampd(r, ld_stream(l + i), ld_stream(u + i)) - r) / sA;
    ybar[i] = yb;                                            // gathered next by A^T
    st_stream(y + i, rho * yai + (1.0 - rho) * (2.0 * yb - yi));
    if (want_r) { const double t = yi - yb; acc[0] += t * t; }
    if (want_th) { const double t = yb - yai; acc[1] += t * t; }
  }
};

// A^T-product:  g = A^T ybar;  d = g - A^T y = A^T (ybar - y);
// cache Halpern:  A^T y+ = rho A^T y_a + (1 - rho)(2 g - A^T y).
// At checks also g and e = g - A^T y_a (for theta~ and eta_d).
struct EpiAT {
  double *ATy; const double* ATya; double *d, *g, *e;
  int check;
  double rho;
  static constexpr int NR = 0;
  static constexpr unsigned MAXMASK = 0u;
  __device__ void setup(const DevParams* p, int j) { IterScalars s; s.load(p, j); rho = s.rho; }
  __device__ __forceinline__ void operator()(int i, double q, double*) const {
    const double aty = ld_stream(ATy + i), atya = ld_stream(ATya + i);
    d[i] = q - aty;                                          // gathered next by Q-apply #2
    st_stream(ATy + i, rho * atya + (1.0 - rho) * (2.0 * q - aty));
    if (check) { g[i] = q; e[i] = q - atya; }
  }
};

// Q-apply #2 with the Halpern epilogue and the next iteration's z/x step.
//   q2 = Q d = Q A^T (ybar - y)
//   w_half = (sigma lamQ w + xh)/(1+sigma lamQ);  wbar = w_half + kappa d        ("update-w")
//   Q wbar = (sigma lamQ Qw + q1)/(1+sigma lamQ) + kappa q2
//   Halpern: x+ = rho x_a + (1-rho) xh  (since 2 xbar - x = xh),
//            w+ = rho w_a + (1-rho)(2 wbar - w),  Qw+ likewise.
//   Next z/x step ("update-z", "update-x") with A^T y+ already written by EpiAT:
//            r_z = x+ + sigma(-Qw+ + A^T y+ - c), xbar' = Pi_C(r_z), zbar' = (xbar' - r_z)/sigma,
//            xh' = 2 xbar' - x+.
// Reductions (u - ubar differences, du = u - ubar):
//   acc[0..5] = <dw,Q dw>, <Q dw, A^T dy>, |dx|^2, <A^T dy, Q A^T dy>, <A^T dy, dx>, <Q dw, dx>
//     with A^T dy = -d, Q A^T dy = -q2, dx = xbar - xh;
//   acc[6..8] (checks) with D = ubar - u_a: <Dw, Q Dw>, <Q Dw, e>, |Dx|^2.
// The panel-ordered product loads the Halpern anchors (wa, Qwa, xa) of the
// epilogue below at the start of its last panel (Pre, preload; random QP,
// n = 1e6: 58.1 against 58.6 us; preloading more operands gains nothing more
// and takes registers).  The other products load them in the epilogue.
struct EpiQ2 {
  double *xh, *w, *Qw, *XB, *ZB;
  const double *q1, *d, *wa, *Qwa, *xa, *ATy, *c, *L, *U, *e;
  double *wbar, *qwbar, *x, *xbar_out;
  int want_r, check, xb_next, trace;
  double l1;                      // lambda of phi (0: the box projection)
  double sigma, sQ, kappa, rho;
  static constexpr int NR = 9;
  static constexpr bool PANEL_PREFETCH = true;   // panel-ordered product: prefetch the next chunk
  static constexpr unsigned MAXMASK = 0u;
  __device__ void setup(const DevParams* p, int j) {
    IterScalars s; s.load(p, j);
    sigma = s.sigma; sQ = s.sQ; kappa = s.kappa; rho = s.rho;
  }
  // operands loaded early by the panel-ordered product (before its last panel)
  struct Pre { double wa, Qwa, xa; };
  __device__ __forceinline__ Pre preload(int i) const {
    return Pre{ld_stream(wa + i), ld_stream(Qwa + i), ld_stream(xa + i)};
  }
  __device__ __forceinline__ void operator()(int i, double q2, double* acc, const Pre& pf) const {
    apply(i, q2, acc, [&](double& a, double& b, double& c3) { a = pf.wa; b = pf.Qwa; c3 = pf.xa; });
  }
  __device__ __forceinline__ void operator()(int i, double q2, double* acc) const {
    apply(i, q2, acc, [&](double& a, double& b, double& c3) {
      a = ld_stream(wa + i); b = ld_stream(Qwa + i); c3 = ld_stream(xa + i);
    });
  }
  // anchors(wa_i, Qwa_i, xa_i) supplies the Halpern anchors of entry i
  template <class Anchors>
  __device__ __forceinline__ void apply(int i, double q2, double* acc, Anchors anchors) const {
    const double xhi = ld_stream(xh + i), wi = ld_stream(w + i), Qwi = ld_stream(Qw + i), di = d[i];
    const double inv = 1.0 / (1.0 + sQ);
    const double wb = (sQ * wi + xhi) * inv + kappa * di;
    const double Qwb = (sQ * Qwi + ld_stream(q1 + i)) * inv + kappa * q2;
    double wai, Qwai, xai;
    anchors(wai, Qwai, xai);
    if (want_r || check || trace) {
      const double xb = XB[i];
      if (want_r) {
        const double dw = wi - wb, Qdw = Qwi - Qwb, ATdy = -di, QATdy = -q2, dx = xb - xhi;
        acc[0] += dw * Qdw; acc[1] += Qdw * ATdy; acc[2] += dx * dx;
        acc[3] += ATdy * QATdy; acc[4] += ATdy * dx; acc[5] += Qdw * dx;
      }
      if (check) {
        wbar[i] = wb; qwbar[i] = Qwb;
        const double Dw = wb - wai, QDw = Qwb - Qwai, Dx = xb - xai;
        acc[6] += Dw * QDw; acc[7] += QDw * e[i]; acc[8] += Dx * Dx;
      }
      if (trace) { wbar[i] = wb; xbar_out[i] = xb; }
    }
    const double xn = rho * xai + (1.0 - rho) * xhi;
    const double wn = rho * wai + (1.0 - rho) * (2.0 * wb - wi);
    const double Qwn = rho * Qwai + (1.0 - rho) * (2.0 * Qwb - Qwi);
    st_stream(w + i, wn); st_stream(Qw + i, Qwn);
    if (trace) x[i] = xn;
    const double rz = xn + sigma * (-Qwn + ld_stream(ATy + i) - ld_stream(c + i));
    const double xbn = prox_phi(rz, sigma * l1, ld_stream(L + i), ld_stream(U + i));
    xh[i] = 2.0 * xbn - xn;                                  // gathered next by Q-apply #1
    if (xb_next) { XB[i] = xbn; ZB[i] = (xbn - rz) / sigma; }
  }
};

// Stand-alone z/x step (start of a solve and after a restart):
//   r_z = x + sigma(-Qw + A^T y - c); xbar = Pi_C(r_z); zbar = (xbar - r_z)/sigma; xh = 2 xbar - x.
struct EpiStage1 {
  const double *x, *Qw, *ATy, *c, *L, *U; double *xh, *XB, *ZB;
  double l1;
  double sigma;
  static constexpr int NR = 0;
  static constexpr unsigned MAXMASK = 0u;
  __device__ void setup(const DevParams* p, int) { sigma = p->sigma; }
  __device__ __forceinline__ void operator()(int i, double, double*) const {
    const double xi = x[i];
    const double rz = xi + sigma * (-Qw[i] + ATy[i] - c[i]);
    const double xb = prox_phi(rz, sigma * l1, L[i], U[i]);
    xh[i] = 2.0 * xb - xi; XB[i] = xb; ZB[i] = (xb - rz) / sigma;
  }
};

// Primal residual and the y-part of the dual objective at (x, y) from A x:
//   acc[0] = max |Ax - Pi_K(Ax)|, acc[1] = max |Ax|,
//   acc[2] = sum_i (l_i y_i^+ + u_i y_i^-), acc[3] = #(nonzero y_i against an infinite bound)
// With diagonal preconditioning, ie = 1/E turns the scaled row (A~ x~)_i into
// the given problem's (A x)_i; the objective terms are invariant.
struct EpiResA {
  const double *l, *u, *y;
  const double* ie;   // NULL: no preconditioning
  static constexpr int NR = 4;
  static constexpr unsigned MAXMASK = 0x3u;
  __device__ void setup(const DevParams*, int) {}
  __device__ __forceinline__ void operator()(int i, double ax, double* acc) const {
    const double li = l[i], ui = u[i], yi = y[i];
    const double s = ie ? ie[i] : 1.0;
    acc[0] = fmax(acc[0], fabs(ax - clampd(ax, li, ui)) * s);
    acc[1] = fmax(acc[1], fabs(ax) * s);
    if (yi > 0.0) { if (isinf(li)) acc[3] += 1.0; else acc[2] += li * yi; }
    else if (yi < 0.0) { if (isinf(ui)) acc[3] += 1.0; else acc[2] += ui * yi; }
  }
};

// Dual residual and the rest of the objectives at (x, z) from Q x and g = A^T y:
//   acc[0] = max |-Qx + g + z - c|, acc[1] = max |g|, acc[2] = max |Qx|,
//   acc[3] = <x, Qx>, acc[4] = <c, x> + lambda ||x||_1, acc[5] = -phi^*(-z) (for
//   lambda = 0: sum_j (L_j z_j^+ + U_j z_j^-)), acc[6] = #(z_j making phi^*(-z) infinite).
// Optionally copies x, z to the output buffers.  With diagonal
// preconditioning, id = 1/D maps the scaled dual quantities back (the dual
// residual, A^T y and Q x of the given problem are 1/D times the scaled ones).
struct EpiResQ {
  const double *x, *z, *g, *c, *L, *U; double *xo, *zo;
  const double* id;   // NULL: no preconditioning
  double l1;          // lambda of phi: acc[4] also holds lambda ||x||_1
  static constexpr int NR = 7;
  static constexpr unsigned MAXMASK = 0x7u;
  __device__ void setup(const DevParams*, int) {}
  __device__ __forceinline__ void operator()(int i, double qx, double* acc) const {
    const double xi = x[i], zi = z[i], gi = g ? g[i] : 0.0, ci = c[i];
    const double s = id ? id[i] : 1.0;
    acc[0] = fmax(acc[0], fabs(-qx + gi + zi - ci) * s);
    acc[1] = fmax(acc[1], fabs(gi) * s);
    acc[2] = fmax(acc[2], fabs(qx) * s);
    acc[3] += xi * qx;
    acc[4] += ci * xi + l1 * fabs(xi);
    bool inf = false;
    acc[5] += neg_conj_phi(zi, l1, L[i], U[i], &inf);
    if (inf) acc[6] += 1.0;
    if (xo) { xo[i] = xi; zo[i] = zi; }
  }
};

// acc[0] = max |q_i| s_i (s NULL: 1): the inf-norm of a product, optionally
// rescaled row by row
struct EpiMaxAbs {
  const double* s;
  static constexpr int NR = 1;
  static constexpr unsigned MAXMASK = 0x1u;
  __device__ void setup(const DevParams*, int) {}
  __device__ __forceinline__ void operator()(int i, double q, double* acc) const {
    acc[0] = fmax(acc[0], fabs(q) * (s ? s[i] : 1.0));
  }
};

// theta~_3 = <e, Q e>, e = A^T (ybar - y_a)
struct EpiTheta3 {
  const double* e;
  static constexpr int NR = 1;
  static constexpr unsigned MAXMASK = 0u;
  __device__ void setup(const DevParams*, int) {}
  __device__ __forceinline__ void operator()(int i, double q, double* acc) const { acc[0] += e[i] * q; }
};

// restart: Qw = Qw_a = Q wbar (exact product)
struct EpiStore2 {
  double *a, *b;
  static constexpr int NR = 0;
  static constexpr unsigned MAXMASK = 0u;
  __device__ void setup(const DevParams*, int) {}
  __device__ __forceinline__ void operator()(int i, double q, double*) const { a[i] = q; b[i] = q; }
};

// power method: w = M v stored; acc[0] += v_i w_i (Rayleigh quotient), acc[1] += w_i^2
struct EpiPow {
  const double* v; double* w;
  static constexpr int NR = 2;
  static constexpr unsigned MAXMASK = 0u;
  __device__ void setup(const DevParams*, int) {}
  __device__ __forceinline__ void operator()(int i, double q, double* acc) const {
    w[i] = q; acc[0] += v[i] * q; acc[1] += q * q;
  }
};
