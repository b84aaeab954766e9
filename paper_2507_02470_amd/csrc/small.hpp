// small.hpp -- one workgroup runs a whole check segment of HPR-QP
// (Algorithm 4, Tseg iterations and the check) for a small problem.
//
// At n, m of a few hundred the four products of an iteration are a few
// microseconds of work each, and the per-launch cost of a graph node
// (~7 us) is what an iteration costs.  Here the products are phases of one
// 1024-thread workgroup separated by barriers: each phase runs the same
// fused epilogue as the multi-block kernels (so the arithmetic is that of
// the four-launch path), rows are taken by groups of G lanes (butterfly sum
// in a fixed order), the vectors stay in global memory (they fit the CU's
// caches), and the reductions of a phase go through the block reduction
// into the same slots, with one partial per slot.  Explicit Q (CSR) or
// Q = 0 only.
#pragma once
#include "common.hpp"
#include "epilogues.hpp"

#define HQ_SMALL_BS 1024

struct SmallMat {
  int rows;
  const int* rp;     // nullptr: the zero matrix (q = 0 for every row)
  const int* ci;
  const double* v;
};

struct SmallArgs {
  SmallMat A, AT, Q;
  int n, m;
  const double *l, *u, *c, *L, *U, *iEs, *iDs;
  double *y, *ya, *ybar, *w, *wa, *x, *xa, *ATy, *ATya, *Qw, *Qwa, *xh, *v, *q1, *d, *g, *e, *XB, *ZB, *wbar,
      *qwbar, *xbo, *zbo;
  double l1;
  double* partials;
  int* counts;
  const DevParams* prm;
};

// q_i = (M x)_i for every row, then epi(i, q_i); block reduction of the
// epilogue's accumulators; a barrier makes the epilogue's stores visible to
// the next phase
template <int G, class Epi>
__device__ __forceinline__ void small_phase(const SmallMat& M, const double* __restrict__ x, Epi e,
                                            const DevParams* __restrict__ prm, int j, const RedOut& red) {
  constexpr int NR = Epi::NR;
  e.setup(prm, j);
  double acc[NR > 0 ? NR : 1];
#pragma unroll
  for (int s = 0; s < (NR > 0 ? NR : 1); ++s) acc[s] = 0.0;
  const int gl = threadIdx.x % G, gi = threadIdx.x / G;
  for (int row = gi; row < M.rows; row += HQ_SMALL_BS / G) {
    double sum = 0.0;
    if (M.rp) {
      const int b = M.rp[row], en = M.rp[row + 1];
#pragma unroll 4
      for (int k = b + gl; k < en; k += G) sum += M.v[k] * x[M.ci[k]];
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
    if (gl == 0) e(row, sum, acc);
  }
  if (red.active) block_reduce_store<NR, Epi::MAXMASK>(acc, red);
  __syncthreads();
}

__device__ __forceinline__ RedOut small_red(const SmallArgs& a, int s0, int s1 = -1, int s2 = -1) {
  RedOut r;
  r.partials = a.partials;
  r.counts = a.counts;
  for (int s = 0; s < 16; ++s) r.slot[s] = -1;
  r.slot[0] = (int8_t)s0; r.slot[1] = (int8_t)s1; r.slot[2] = (int8_t)s2;
  r.active = s0 >= 0 || s1 >= 0 || s2 >= 0;
  return r;
}

template <int G>
__global__ __launch_bounds__(HQ_SMALL_BS) void k_small_segment(SmallArgs a, int Tseg) {
  const RedOut none = small_red(a, -1);
  SmallMat zero_n{a.n, nullptr, nullptr, nullptr};
  for (int j = 0; j < Tseg; ++j) {
    const bool check = (j == Tseg - 1);
    const int rgroup = check ? SL_RC : (j == 0 ? SL_RF : -1);
    const bool want_r = rgroup >= 0;
    const bool xb_next = j >= Tseg - 2;
    // a3: q1 = Q xhat, v
    small_phase<G>(a.Q, a.xh, EpiQ1{a.xh, a.Qw, a.v, a.q1, 0.0}, a.prm, j, none);
    if (a.m > 0) {
      // a4: A v, ybar, y+
      small_phase<G>(a.A, a.v, EpiY{a.l, a.u, a.ya, a.y, a.ybar, want_r, check, 0.0, 0.0}, a.prm, j,
                     small_red(a, want_r ? rgroup : -1, check ? SL_TH : -1));
      // a5: A^T ybar, d, A^T y+
      small_phase<G>(a.AT, a.ybar, EpiAT{a.ATy, a.ATya, a.d, a.g, a.e, check, 0.0}, a.prm, j, none);
    }
    if (check) {
      if (a.m > 0) {
        RedOut r = none;
        for (int s = 0; s < 4; ++s) r.slot[s] = (int8_t)(SL_RA + s);
        r.active = 1;
        small_phase<G>(a.A, a.XB, EpiResA{a.l, a.u, a.ybar, a.iEs}, a.prm, j, r);
      }
      RedOut r = none;
      for (int s = 0; s < 7; ++s) r.slot[s] = (int8_t)(SL_RQ + s);
      r.active = 1;
      small_phase<G>(a.Q, a.XB,
                     EpiResQ{a.XB, a.ZB, a.m > 0 ? a.g : nullptr, a.c, a.L, a.U, a.xbo, a.zbo, a.iDs, a.l1}, a.prm, j,
                     r);
    }
    // a6: Q d, wbar, Halpern, next z/x step
    EpiQ2 e6;
    e6.xh = a.xh; e6.w = a.w; e6.Qw = a.Qw; e6.XB = a.XB; e6.ZB = a.ZB;
    e6.q1 = a.q1; e6.d = a.d; e6.wa = a.wa; e6.Qwa = a.Qwa; e6.xa = a.xa; e6.ATy = a.ATy;
    e6.c = a.c; e6.L = a.L; e6.U = a.U; e6.e = a.e;
    e6.wbar = a.wbar; e6.qwbar = a.qwbar; e6.x = a.x; e6.xbar_out = a.xbo;
    e6.want_r = want_r; e6.check = check; e6.xb_next = xb_next; e6.trace = 0;
    e6.l1 = a.l1;
    RedOut r6 = none;
    if (want_r)
      for (int s = 0; s < 6; ++s) r6.slot[s] = (int8_t)(rgroup + 1 + s);
    if (check)
      for (int s = 0; s < 3; ++s) r6.slot[6 + s] = (int8_t)(SL_TH + 1 + s);
    r6.active = want_r || check;
    small_phase<G>(a.m > 0 ? a.Q : zero_n, a.d, e6, a.prm, j, r6);
    if (check && a.m > 0 && a.Q.rp)
      small_phase<G>(a.Q, a.e, EpiTheta3{a.e}, a.prm, j, small_red(a, SL_TH + 4));
  }
}
