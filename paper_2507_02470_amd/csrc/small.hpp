// small.hpp -- one workgroup runs a whole check segment of HPR-QP
// (Algorithm 4, Tseg iterations and the check) for a small problem.
//
// At n, m of a few hundred the four products of an iteration are a few
// microseconds of work each, and the per-launch cost of a graph node
// (~7 us) is what an iteration costs.  Here the products are phases of one
// 1024-thread workgroup separated by barriers: each phase runs the same
// fused epilogue as the multi-block kernels (so the arithmetic is that of
// the four-launch path), rows are taken by groups of G lanes (butterfly sum
// in a fixed order), and the reductions of a phase go through the block
// reduction into the same slots, with one partial per slot.  When the
// matrices and every vector of the iteration fit (dynamic LDS, up to
// HQ_SMALL_LDS bytes; STAGED), they are copied into LDS at the start of the
// segment and the written vectors back at its end, so every gather is an LDS
// access; otherwise they stay in global memory.  The staged kernel derives
// every pointer from the LDS base only (never a global fallback), so the
// compiler addresses them as LDS (ds_read/ds_write) instead of generic flat
// accesses, which go through the vector-memory path and are counted by both
// wait counters.  Explicit Q (CSR) or Q = 0 only.
#pragma once
#include "common.hpp"
#include "epilogues.hpp"
#include "epilogues_primal.hpp"

#ifndef HQ_SMALL_BS
#define HQ_SMALL_BS 1024
#endif
#define HQ_SMALL_LDS (150 * 1024)

struct SmallMat {
  int rows;
  const int* rp;     // nullptr: the zero matrix (q = 0 for every row)
  const int* ci;
  const double* v;
};

// vectors of the iteration, by index
enum : int {
  SV_L, SV_U, SV_C, SV_LB, SV_UB, SV_IE, SV_ID,                 // read only
  SV_YA, SV_WA, SV_XA, SV_ATYA, SV_QWA, SV_PTA,                  // read only during a segment
  SV_Y, SV_YBAR, SV_W, SV_X, SV_ATY, SV_QW, SV_XH, SV_V, SV_Q1, SV_D, SV_G, SV_E, SV_XB, SV_ZB, SV_WBAR,
  SV_QWBAR, SV_XBO, SV_ZBO,                                      // written
  SV_PE, SV_PAX, SV_PDY, SV_PT, SV_PTB, SV_PDT,                  // written (primal methods only)
  SV_COUNT,
  SV_FIRST_WRITTEN = SV_Y
};

struct SmallArgs {
  SmallMat A, AT, Q;
  int n, m;
  double* vec[SV_COUNT];      // global arrays (nullptr: absent)
  int vlen[SV_COUNT];
  double l1;
  double* partials;
  int* counts;
  const DevParams* prm;
  // LDS staging (lds_bytes = 0: none): byte offsets of the vectors and of the
  // matrices' row pointers, columns and values
  int lds_bytes;
  int voff[SV_COUNT];
  int moff[3][3];             // [A, AT, Q][rp, ci, v]
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
    sum = group_sum<G>(sum);   // (a group's lanes share a row: active together)
    if (gl == 0) e(row, sum, acc);
  }
  if (red.active) block_reduce_store<NR, Epi::MAXMASK, true>(acc, red);
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

template <class T>
__device__ __forceinline__ void small_copy(T* __restrict__ dst, const T* __restrict__ src, int count) {
  for (int i = threadIdx.x; i < count; i += HQ_SMALL_BS) dst[i] = src[i];
}

// The arrays the phases use: LDS copies when staged (copied in here), else
// the global ones.  (Loops over the arrays are unrolled so that V and mats
// stay in registers.)
template <bool STAGED>
__device__ __forceinline__ void small_stage_in(const SmallArgs& a, unsigned char* lds, double* (&V)[SV_COUNT],
                                               SmallMat (&mats)[3]) {
#pragma unroll
  for (int s = 0; s < SV_COUNT; ++s) V[s] = STAGED ? nullptr : a.vec[s];
  if (STAGED) {
#pragma unroll
    for (int s = 0; s < SV_COUNT; ++s)
      if (a.vec[s]) {
        double* p = (double*)(lds + a.voff[s]);
        small_copy(p, a.vec[s], a.vlen[s]);
        V[s] = p;
      }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      SmallMat& M = mats[q];
      const SmallMat Mg = M;   // the arrays in global memory (rp == nullptr: the zero matrix)
      M.rp = nullptr; M.ci = nullptr; M.v = nullptr;
      if (Mg.rp) {
        int* rp = (int*)(lds + a.moff[q][0]);
        int* ci = (int*)(lds + a.moff[q][1]);
        double* v = (double*)(lds + a.moff[q][2]);
        small_copy(rp, Mg.rp, Mg.rows + 1);
        __syncthreads();   // the row pointers give the number of nonzeros
        const int nnz = rp[Mg.rows];
        small_copy(ci, Mg.ci, nnz);
        small_copy(v, Mg.v, nnz);
        M.rp = rp; M.ci = ci; M.v = v;
      }
    }
    __syncthreads();
  }
}

// the written vectors back to global memory at the end of a staged segment
template <bool STAGED>
__device__ __forceinline__ void small_stage_out(const SmallArgs& a, double* const (&V)[SV_COUNT]) {
  if (STAGED) {
#pragma unroll
    for (int s = SV_FIRST_WRITTEN; s < SV_COUNT; ++s)
      if (a.vec[s]) small_copy(a.vec[s], V[s], a.vlen[s]);
  }
}

template <int G, bool STAGED>
__global__ __launch_bounds__(HQ_SMALL_BS) void k_small_segment(SmallArgs a, int Tseg) {
  extern __shared__ __align__(16) unsigned char small_lds[];
  double* V[SV_COUNT];
  SmallMat mats[3] = {a.A, a.AT, a.Q};
  small_stage_in<STAGED>(a, small_lds, V, mats);
  // the segment's scalars (sigma, lambda's, t0) are read by every phase: keep a copy in LDS
  __shared__ DevParams sprm;
  if (threadIdx.x == 0) sprm = *a.prm;
  __syncthreads();
  const DevParams* prm = &sprm;
  const SmallMat& A = mats[0];
  const SmallMat& AT = mats[1];
  const SmallMat& Q = mats[2];
  const RedOut none = small_red(a, -1);
  const SmallMat zero_n{a.n, nullptr, nullptr, nullptr};
  for (int j = 0; j < Tseg; ++j) {
    const bool check = (j == Tseg - 1);
    const int rgroup = check ? SL_RC : (j == 0 ? SL_RF : -1);
    const bool want_r = rgroup >= 0;
    const bool xb_next = j >= Tseg - 2;
    // a3: q1 = Q xhat, v
    small_phase<G>(Q, V[SV_XH], EpiQ1{V[SV_XH], V[SV_QW], V[SV_V], V[SV_Q1], 0.0}, prm, j, none);
    if (a.m > 0) {
      // a4: A v, ybar, y+
      small_phase<G>(A, V[SV_V], EpiY{V[SV_L], V[SV_U], V[SV_YA], V[SV_Y], V[SV_YBAR], want_r, check, 0.0, 0.0},
                     prm, j, small_red(a, want_r ? rgroup : -1, check ? SL_TH : -1));
      // a5: A^T ybar, d, A^T y+
      small_phase<G>(AT, V[SV_YBAR], EpiAT{V[SV_ATY], V[SV_ATYA], V[SV_D], V[SV_G], V[SV_E], check, 0.0}, prm, j,
                     none);
    }
    if (check) {
      if (a.m > 0) {
        RedOut r = none;
        for (int s = 0; s < 4; ++s) r.slot[s] = (int8_t)(SL_RA + s);
        r.active = 1;
        small_phase<G>(A, V[SV_XB], EpiResA{V[SV_L], V[SV_U], V[SV_YBAR], V[SV_IE]}, prm, j, r);
      }
      RedOut r = none;
      for (int s = 0; s < 7; ++s) r.slot[s] = (int8_t)(SL_RQ + s);
      r.active = 1;
      small_phase<G>(Q, V[SV_XB],
                     EpiResQ{V[SV_XB], V[SV_ZB], a.m > 0 ? V[SV_G] : nullptr, V[SV_C], V[SV_LB], V[SV_UB], V[SV_XBO],
                             V[SV_ZBO], V[SV_ID], a.l1},
                     prm, j, r);
    }
    // a6: Q d, wbar, Halpern, next z/x step
    EpiQ2 e6;
    e6.xh = V[SV_XH]; e6.w = V[SV_W]; e6.Qw = V[SV_QW]; e6.XB = V[SV_XB]; e6.ZB = V[SV_ZB];
    e6.q1 = V[SV_Q1]; e6.d = V[SV_D]; e6.wa = V[SV_WA]; e6.Qwa = V[SV_QWA]; e6.xa = V[SV_XA]; e6.ATy = V[SV_ATY];
    e6.c = V[SV_C]; e6.L = V[SV_LB]; e6.U = V[SV_UB]; e6.e = V[SV_E];
    e6.wbar = V[SV_WBAR]; e6.qwbar = V[SV_QWBAR]; e6.x = V[SV_X]; e6.xbar_out = V[SV_XBO];
    e6.want_r = want_r; e6.check = check; e6.xb_next = xb_next; e6.trace = 0;
    e6.l1 = a.l1;
    RedOut r6 = none;
    if (want_r)
      for (int s = 0; s < 6; ++s) r6.slot[s] = (int8_t)(rgroup + 1 + s);
    if (check)
      for (int s = 0; s < 3; ++s) r6.slot[6 + s] = (int8_t)(SL_TH + 1 + s);
    r6.active = want_r || check;
    const SmallMat Qd{a.n, a.m > 0 ? Q.rp : nullptr, a.m > 0 ? Q.ci : nullptr, a.m > 0 ? Q.v : nullptr};
    small_phase<G>(Qd, V[SV_D], e6, prm, j, r6);
    if (check && a.m > 0 && Q.rp) small_phase<G>(Q, V[SV_E], EpiTheta3{V[SV_E]}, prm, j, small_red(a, SL_TH + 4));
  }
  small_stage_out<STAGED>(a, V);
}

// HPR on the primal reformulations (Algorithms 6 and 7 of the appendix,
// meth = 1, 2): the products of an iteration as phases, in the order and with
// the epilogues of the multi-launch path.
template <int G, bool STAGED>
__global__ __launch_bounds__(HQ_SMALL_BS) void k_small_primal(SmallArgs a, int Tseg, int meth) {
  extern __shared__ __align__(16) unsigned char small_lds[];
  double* V[SV_COUNT];
  SmallMat mats[3] = {a.A, a.AT, a.Q};
  small_stage_in<STAGED>(a, small_lds, V, mats);
  __shared__ DevParams sprm;
  if (threadIdx.x == 0) sprm = *a.prm;
  __syncthreads();
  const DevParams* prm = &sprm;
  const SmallMat& A = mats[0];
  const SmallMat& AT = mats[1];
  const SmallMat& Q = mats[2];
  const RedOut none = small_red(a, -1);
  const SmallMat zero_n{a.n, nullptr, nullptr, nullptr};
  const bool rows = a.m > 0;
  for (int j = 0; j < Tseg; ++j) {
    const bool check = (j == Tseg - 1);
    const int rgroup = check ? SL_RC : (j == 0 ? SL_RF : -1);
    const bool want_r = rgroup >= 0;
    const int store_bar = want_r || check;
    const auto at = [&](int off) { return want_r ? rgroup + off : -1; };
    // Q x (Algorithm 6) or Q v with the v/t-step (Algorithm 7)
    if (meth == 1) {
      small_phase<G>(Q, V[SV_X], EpiStore{V[SV_Q1]}, prm, j, none);
    } else {
      small_phase<G>(Q, V[SV_W],
                     EpiP2V{V[SV_W], V[SV_X], V[SV_PTA], V[SV_PT], V[SV_WBAR], V[SV_V], V[SV_QW], V[SV_E], V[SV_PDT],
                            V[SV_PTB], want_r, check},
                     prm, j, small_red(a, at(1), at(4), check ? SL_TH + 2 : -1));
    }
    // A x with the s/y-step
    if (rows)
      small_phase<G>(A, V[SV_X],
                     EpiPY{V[SV_L], V[SV_U], V[SV_YA], V[SV_Y], V[SV_YBAR], V[SV_PE], V[SV_PAX], V[SV_PDY], want_r,
                           check, store_bar},
                     prm, j, small_red(a, at(3), check ? SL_TH + 1 : -1));
    // A^T (2 ybar - y) with the x-step
    // (a value, not a reference to one of two locals: that would keep both in scratch)
    const SmallMat ATx{a.n, rows ? AT.rp : nullptr, rows ? AT.ci : nullptr, rows ? AT.v : nullptr};
    if (meth == 1) {
      small_phase<G>(ATx, V[SV_PE],
                     EpiP1X{V[SV_Q1], V[SV_C], V[SV_LB], V[SV_UB], V[SV_XA], V[SV_X], V[SV_XB], V[SV_ZB], V[SV_D],
                            want_r, check, store_bar, a.l1},
                     prm, j, small_red(a, at(0), check ? SL_TH : -1));
    } else {
      small_phase<G>(ATx, V[SV_PE],
                     EpiP2X{V[SV_V], V[SV_C], V[SV_LB], V[SV_UB], V[SV_XA], V[SV_WA], V[SV_WBAR], V[SV_PDT], V[SV_X],
                            V[SV_W], V[SV_XB], V[SV_ZB], V[SV_D], want_r, check, store_bar, a.l1},
                     prm, j, small_red(a, at(0), at(5), check ? SL_TH : -1));
    }
    if (want_r) {
      // <A dx, dy> and <dx, Q dx> (Algorithm 6) or <dv, Q dv> (Algorithm 7)
      if (rows) small_phase<G>(A, V[SV_XB], EpiMeritA{V[SV_PAX], V[SV_PDY]}, prm, j, small_red(a, rgroup + 2));
      if (meth == 1) small_phase<G>(Q, V[SV_XB], EpiMeritQ{V[SV_Q1], V[SV_D]}, prm, j, small_red(a, rgroup + 1));
      else small_phase<G>(Q, V[SV_WBAR], EpiMeritQ{V[SV_QW], V[SV_E]}, prm, j, small_red(a, rgroup + 6));
    }
    if (check) {
      // stopping quantities at (ybar, zbar, xbar): A^T ybar, A xbar, Q xbar
      if (rows) {
        small_phase<G>(AT, V[SV_YBAR], EpiStore{V[SV_G]}, prm, j, none);
        RedOut r = none;
        for (int s = 0; s < 4; ++s) r.slot[s] = (int8_t)(SL_RA + s);
        r.active = 1;
        small_phase<G>(A, V[SV_XB], EpiResA{V[SV_L], V[SV_U], V[SV_YBAR], V[SV_IE]}, prm, j, r);
      }
      RedOut r = none;
      for (int s = 0; s < 7; ++s) r.slot[s] = (int8_t)(SL_RQ + s);
      r.active = 1;
      small_phase<G>(Q, V[SV_XB],
                     EpiResQ{V[SV_XB], V[SV_ZB], rows ? V[SV_G] : nullptr, V[SV_C], V[SV_LB], V[SV_UB], V[SV_XBO],
                             V[SV_ZBO], V[SV_ID], a.l1},
                     prm, j, r);
    }
  }
  small_stage_out<STAGED>(a, V);
}
