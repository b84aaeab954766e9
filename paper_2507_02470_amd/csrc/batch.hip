// batch.hip -- many independent HPR-QPs (Algorithm 4 + Algorithm 5 of arXiv
// 2507.02470) in persistent kernels on one MI355X.
//
// One workgroup owns one instance at a time; instances are pulled from a
// work queue ordered by size (largest first).  The instances are cut into
// size classes (n <= 256, 512, 1024, 2048) and each class runs on a kernel of
// 64, 128, 256 or 512 threads per workgroup (at most 4 entries per thread):
// by default 256 threads up to n = 1024 (two workgroups per CU) and 512 above
// (one per CU); with autotuning, create times every block size that can hold
// a class on a sample of the class's instances and keeps the fastest.  The
// kernels of the block sizes in use run at once on their own streams.
// Thread t of a BS-thread workgroup owns entries t + BS e, e < HB_EPT (so
// n <= BS * HB_EPT): the per-iteration vectors of
// its entries are in registers, and so are its rows of the low-rank factor F
// of Q = diag(d) + F F^T at rank <= 10 (at rank 16 they are read from memory
// at each product); the iterate, its images Q w and A^T y, the Halpern
// anchors and the vectors of length m (<= 64) are in LDS.  The iteration
// is bound by the latency of its dependent steps (a block-wide reduction
// per Q product, the A and A^T products through LDS), not by bandwidth, so
// the loads of each step are issued together and kept to global (not
// generic) addresses.  The whole method runs on the
// device in FP64: power method for lambda_A and lambda_Q, the sigma0 rule,
// the iteration, the merit R~, the stopping test, the restart criteria of
// Section 3.2 and the golden-section sigma update of Algorithm 5 (thread 0,
// broadcast through LDS).  No host round trip until every instance is done.
#include "hprqp.h"
#include "common.hpp"

#include <algorithm>
#include <chrono>
#include <map>
#include <tuple>
#include <type_traits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace hq {
extern thread_local std::string g_err;
}

#define HB_BS 512
#define HB_EPT 4
#define HB_NMAX (HB_BS * HB_EPT)                      // largest n (the 512-thread kernel)
#define HB_NCLASS 4                                    // size classes: n <= 256, 512, 1024, 2048
#define HB_MMAX 64
#define HB_RMAX 16
#define HB_APIECE 256                                  // nonzeros of A per wave work item
#define HB_ATSTEP 3                                    // nonzeros per entry and step of the A^T product

// Per-block sizes of the kernels: BS = 64, 128, 256 or 512 threads for
// n <= 4 BS (512 threads: one block per CU, the LDS holds 156 KB; 256: two per
// CU, so that one block's waits are covered by the other's work; smaller
// blocks let more instances share a CU).  Entry i of a vector belongs to
// thread i mod BS, so NMAX = BS * HB_EPT: the slots of every thread's HB_EPT
// entries exist, also beyond n.
template <int BS>
struct BCfg {
  static_assert(BS == 64 || BS == 128 || BS == 256 || BS == 512, "block sizes");
  static constexpr int WAVES = BS / 64;
  static constexpr int NMAX = BS * HB_EPT;
  // pieces of A at most: a row has at most n nonzeros (checked at create)
  static constexpr int PMAX = HB_MMAX * ((NMAX + HB_APIECE - 1) / HB_APIECE);
  // launch bound: the compiler counts a block's waves per SIMD, so 2 blocks
  // mean 2 waves per SIMD (about 256 VGPRs) at every block size; more small
  // blocks still share a CU when the registers and LDS allow
  static constexpr int MIN_BLOCKS = 2;
};

struct BInst {
  int n, m, r;
  int pad;
  const double *c, *L, *U, *l, *u, *dg, *F;
  const int *arp, *aci;
  const double* aval;
  const int *trp, *tci;   // A^T (n x m) CSR, rows ordered by row of A
  const double* tval;
  const double* FT;       // F with rows padded to the kernel's rank RM (entries k >= r zero)
  long long off_n, off_m;
  long long annz;         // nonzeros of A
};

struct BOpts {
  double tol;
  long long max_iter;
  int check_every;
  double sigma0, lamA, lamQ;
  double alpha1, alpha2, alpha3;
  int enable_restart, enable_sigma_update;
  // time limit: wall-clock ticks (wall_clock64) since *t0, the stamp taken
  // on the stream just before the solve kernels; 0: none
  long long time_ticks;
  const long long* t0;
};

struct BInfo {
  int term, restarts;
  long long iters;
  double sigma, sigma0, lamA, lamQ, eta_p, eta_d, eta_gap, pobj, dobj, R_last;
};

// ---------------------------------------------------------------------------
// LDS of one instance
// ---------------------------------------------------------------------------
#define HB_RED 16   // most values reduced at once

template <int BS>
struct BShared {
  static constexpr int NMAX = BCfg<BS>::NMAX, PMAX = BCfg<BS>::PMAX;
  alignas(16) double red[2][HB_RED][BCfg<BS>::WAVES];   // wave partials, two buffers used in turn
  double vm[NMAX];                   // a length-n vector shared by the block (A v, A xbar)
  // Halpern anchors u^{r,0} and their images (read once per iteration)
  double xa[NMAX], wa[NMAX], Qwa[NMAX], ATya[NMAX];
  // iterate u^{r,t} = (x, w) with the images Q w and A^T y kept by linearity
  double xs[NMAX], ws[NMAX], Qws[NMAX], ATys[NMAX];
  double y[HB_MMAX], ya[HB_MMAX], yb[HB_MMAX], l[HB_MMAX], u[HB_MMAX];
  union {
    double yn[HB_MMAX];              // y^{t+1} (Halpern) until the check is done
    double pw[HB_MMAX];              // power method vector (length m), before the iterations
  };
  // A products: row r of A is cut into pieces of HB_APIECE nonzeros; piece
  // q belongs to row prow[q] and pieces pstart[r] .. pstart[r+1]-1 to row r
  double part[PMAX];
  unsigned char prow[PMAX];          // (m <= 64)
  int pstart[HB_MMAX + 1];
  int arp[HB_MMAX + 1];              // row pointers of A
  int np;
  double ctrl[8];
  int inst;
  BOpts opt;                         // the options, for the out-of-line check decision
};

// DPP move of a double (both 32-bit halves with the same control); lanes
// without a source read 0, the identity of the sums and of the maxima of
// non-negative values reduced here.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp_mov(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Value of lane l of a wave, in scalar registers (l wave-uniform).
__device__ __forceinline__ double readlane_d(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave reduction with DPP (fixed pattern: quad swaps, row shifts by 4 and 8,
// row broadcasts 15 and 31); the result is exact in lane 63 only.
template <bool MX>
__device__ __forceinline__ double wave_reduce63(double v) {
  auto op = [](double a, double b) { return MX ? fmax(a, b) : a + b; };
  v = op(v, dpp_mov<0xb1>(v));          // quad_perm [1,0,3,2]
  v = op(v, dpp_mov<0x4e>(v));          // quad_perm [2,3,0,1]
  v = op(v, dpp_mov<0x114>(v));         // row_shr:4
  v = op(v, dpp_mov<0x118>(v));         // row_shr:8
  v = op(v, dpp_mov<0x142, 0xa>(v));    // row_bcast:15
  v = op(v, dpp_mov<0x143, 0xc>(v));    // row_bcast:31
  return v;
}

// Block-wide reduction of K values (sum, or max where bit s of maxmask is
// set; maxima only of non-negative values) with one barrier: DPP wave
// reductions, lane 63 of each wave stores its partials, then every wave
// combines the W wave partials of value s on lanes Ws..Ws+W-1 with a fixed
// butterfly and reads the result from lane Ws into scalar registers.  Fixed order, deterministic.  The two partial
// buffers alternate between calls, so a buffer is rewritten only after every
// thread has passed the barrier of the call in between.
template <int K, int BS>
__device__ __forceinline__ void bred(BShared<BS>& S, int& par, double (&v)[K], unsigned maxmask) {
  constexpr int W = BCfg<BS>::WAVES;   // partials per value
  static_assert(K <= HB_RED && (W == 1 || W == 2 || W == 4 || W == 8), "reduction layout");
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const double x = ((maxmask >> s) & 1u) ? wave_reduce63<true>(v[s]) : wave_reduce63<false>(v[s]);
    if (lane == 63) S.red[par][s][wv] = x;
  }
  __syncthreads();
  constexpr int VP = 64 / W;   // values combined per pass
#pragma unroll
  for (int s0 = 0; s0 < K; s0 += VP) {
    const int s = s0 + lane / W, w = lane % W;
    const bool mx = (maxmask >> s) & 1u;
    double x = s < K ? S.red[par][s][w] : 0.0;
#pragma unroll
    for (int off = 1; off < W; off <<= 1) {
      // partner lane l ^ off: DPP quad permutations for 1 and 2, a shuffle for 4
      const double y = off == 1 ? dpp_mov<0xb1>(x) : off == 2 ? dpp_mov<0x4e>(x) : __shfl_xor(x, off);
      x = mx ? fmax(x, y) : x + y;
    }
    // every lane of group q holds value q: broadcast it from the group's first lane
#pragma unroll
    for (int q = s0; q < K && q < s0 + VP; ++q) v[q] = readlane_d(x, (q - s0) * W);
  }
  par ^= 1;
}

// ---------------------------------------------------------------------------
// the per-instance operator pieces
// ---------------------------------------------------------------------------
// Load of element i of an instance array.  The arrays are in global memory
// but their pointers are read from memory, so plain indexing would give
// generic (flat) loads, which every wait for an LDS access also waits for.
template <class T>
__device__ __forceinline__ T gld(const T* p, long long i) {
  return ((const __attribute__((address_space(1))) T*)p)[i];
}
__device__ __forceinline__ double2 gld(const double2* p, long long i) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const v2 v = ((const __attribute__((address_space(1))) v2*)p)[i];
  return double2{v.x, v.y};
}

template <int RM, int BS>
struct Elem {
  int n, m, r;
  const double* FT;       // F with rows padded to RM: F(i, k) = FT[i RM + k], zero for k >= r
  const double *c, *L, *U, *dg;
  int tid;                // threadIdx.x, refreshed through an empty asm statement every iteration
  __device__ bool valid(int e) const { return tid + e * BS < n; }
  __device__ int idx(int e) const { return tid + e * BS; }
  // Addresses derived from the thread index are then recomputed in every
  // iteration instead of being hoisted out of the solve loop, where they
  // would outnumber the registers and be spilled.
  __device__ void refresh() {
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    tid = t;
  }
};

// The rows of F that a thread owns, read from the library's copy of F with
// rows padded to RM entries (16-byte loads at fixed offsets from one address
// per entry).  REG: loaded once into registers, so that the products of the
// iteration read only diag(d) from memory (rank 10; at rank 16 the copy would
// take too many registers).  Otherwise read at every product.
template <int RM, bool REG>
struct QRows {
  double f[REG ? HB_EPT : 1][REG ? RM : 2];
  // (the base address passes through an empty asm statement so that the
  // compiler cannot move the loads above the point of the call, which would
  // keep the copy live across a check)
  template <int BS>
  __device__ void load(const Elem<RM, BS>& E) {
    if constexpr (REG) {
      const double* FT = E.FT;
      asm volatile("" : "+s"(FT));
#pragma unroll
      for (int e = 0; e < HB_EPT; ++e) {
        const bool ok = E.valid(e);
        const double2* fr = reinterpret_cast<const double2*>(FT + (size_t)(ok ? E.idx(e) : 0) * RM);
#pragma unroll
        for (int k = 0; k < RM / 2; ++k) {
          const double2 v = ok ? gld(fr, k) : double2{0.0, 0.0};
          f[e][2 * k] = v.x;
          f[e][2 * k + 1] = v.y;
        }
      }
    }
  }
  template <int BS>
  __device__ __forceinline__ double2 row2(const Elem<RM, BS>& E, int e, int k) const {
    if constexpr (REG) return double2{f[e][2 * k], f[e][2 * k + 1]};
    else return gld(reinterpret_cast<const double2*>(E.FT + (size_t)E.idx(e) * RM), k);
  }
  template <int BS>
  __device__ __forceinline__ double diag(const Elem<RM, BS>& E, int e) const { return gld(E.dg, E.idx(e)); }
};

// q = Q p = diag(d) p + F (F^T p)
template <int RM, bool REG, int BS>
__device__ __forceinline__ void q_apply(BShared<BS>& S, int& par, const Elem<RM, BS>& E, const QRows<RM, REG>& Fq,
                                        const double (&p)[HB_EPT], double (&q)[HB_EPT]) {
  static_assert(RM % 2 == 0, "rows are read in pairs");
  double t[RM];
#pragma unroll
  for (int k = 0; k < RM; ++k) t[k] = 0.0;
#pragma unroll
  for (int e = 0; e < HB_EPT; ++e)
    if (E.valid(e)) {
#pragma unroll
      for (int k = 0; k < RM / 2; ++k) {
        const double2 v = Fq.row2(E, e, k);
        t[2 * k] += v.x * p[e];
        t[2 * k + 1] += v.y * p[e];
      }
    }
  double dg[HB_EPT];   // loaded before the reduction's barrier, used after it
#pragma unroll
  for (int e = 0; e < HB_EPT; ++e) dg[e] = E.valid(e) ? Fq.diag(E, e) : 0.0;
  bred<RM>(S, par, t, 0u);
#pragma unroll
  for (int e = 0; e < HB_EPT; ++e) {
    double s = 0.0;
    if (E.valid(e)) {
      s = dg[e] * p[e];
#pragma unroll
      for (int k = 0; k < RM / 2; ++k) {
        const double2 v = Fq.row2(E, e, k);
        s += v.x * t[2 * k];
        s += v.y * t[2 * k + 1];
      }
    }
    q[e] = s;
  }
}

// Pieces of the rows of A for a_apply (thread 0, once per instance).
template <int BS>
__device__ void a_pieces(BShared<BS>& S, const BInst& I) {
  int q = 0;
  for (int r = 0; r < I.m; ++r) {
    S.pstart[r] = q;
    S.arp[r] = I.arp[r];
    const int len = I.arp[r + 1] - I.arp[r];
    for (int c = 0; c * HB_APIECE < len; ++c) S.prow[q++] = (unsigned char)r;
  }
  S.pstart[I.m] = q;
  S.arp[I.m] = I.m > 0 ? I.arp[I.m] : 0;
  S.np = q;
}

// (A p)_row for thread row < m (0 for the other threads), p staged through
// S.vm.  The waves share the pieces of all rows (a dense row does not
// serialise on one wave); thread row < m then adds its row's pieces in order.
template <int RM, int BS>
__device__ __forceinline__ double a_apply(BShared<BS>& S, const Elem<RM, BS>& E, const BInst& I,
                                          const double (&p)[HB_EPT]) {
  constexpr int WAVES = BCfg<BS>::WAVES;
#pragma unroll
  for (int e = 0; e < HB_EPT; ++e)
    if (E.valid(e)) S.vm[E.idx(e)] = p[e];
  __syncthreads();
  // a wave takes pieces q0 and q0 + WAVES together (loads of both in
  // flight); each piece's sum is formed as for one piece at a time
  const int lane = E.tid & 63, wv = E.tid >> 6;
  constexpr int U = HB_APIECE / 64;
  for (int q0 = wv; q0 < S.np; q0 += 2 * WAVES) {
    double av[2][U];
    int ac[2][U];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = q0 + h * WAVES;
      int b = 0, e = 0;
      if (q < S.np) {
        const int row = S.prow[q];
        b = S.arp[row] + (q - S.pstart[row]) * HB_APIECE;
        e = min(S.arp[row + 1], b + HB_APIECE);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = b + lane + 64 * u;
        av[h][u] = k < e ? gld(I.aval, k) : 0.0;
        ac[h][u] = k < e ? gld(I.aci, k) : -1;
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ac[h][u] >= 0) s += av[h][u] * S.vm[ac[h][u]];
      s = wave_reduce63<false>(s);   // exact in lane 63
      const int q = q0 + h * WAVES;
      if (lane == 63 && q < S.np) S.part[q] = s;
    }
  }
  __syncthreads();
  double s = 0.0;
  if (E.tid < E.m)
    for (int q = S.pstart[E.tid]; q < S.pstart[E.tid + 1]; ++q) s += S.part[q];
  return s;
}

// g = A^T yv (yv in LDS, length m); tb/te: the entries' ranges in A^T,
// loaded once per instance.  The thread's entries advance together,
// HB_ATSTEP nonzeros per step, so that their loads are in flight at the same
// time (each entry's sum still runs over its nonzeros in order).
template <int RM, int BS>
__device__ __forceinline__ void at_apply(const Elem<RM, BS>& E, const BInst& I, const int (&tb)[HB_EPT],
                                         const int (&te)[HB_EPT], const double* yv, double (&g)[HB_EPT]) {
  int len = 0;
#pragma unroll
  for (int e = 0; e < HB_EPT; ++e) {
    g[e] = 0.0;
    len = max(len, te[e] - tb[e]);
  }
  constexpr int J = HB_ATSTEP;
  for (int j = 0; j < len; j += J) {
    double v[HB_EPT][J];
    int c[HB_EPT][J];
#pragma unroll
    for (int e = 0; e < HB_EPT; ++e)
#pragma unroll
      for (int u = 0; u < J; ++u) {
        const int k = tb[e] + j + u;
        const bool ok = k < te[e];
        v[e][u] = ok ? gld(I.tval, k) : 0.0;
        c[e][u] = ok ? gld(I.tci, k) : -1;
      }
#pragma unroll
    for (int e = 0; e < HB_EPT; ++e)
#pragma unroll
      for (int u = 0; u < J; ++u)
        if (c[e][u] >= 0) g[e] += v[e][u] * yv[c[e][u]];
  }
}

__device__ double golden_sigma_dev(double th1, double th2, double th3, double lamQ) {
  const double hi = sqrt(th2 / th1);
  if (th3 <= 0.0 || lamQ <= 0.0) return hi;
  const double lo = sqrt(th2 / (th1 + th3 / lamQ));
  double a = log(lo), b = log(hi);
  const double gr = 0.5 * (sqrt(5.0) - 1.0);
  const double stop = log1p(1e-12);
  for (int it = 0; it < 200 && (b - a) > stop; ++it) {
    const double p = b - gr * (b - a), q = a + gr * (b - a);
    const double sp = exp(p), sq = exp(q);
    const double slope = th1 - th2 / (sp * sq) + th3 * (sp + sq + lamQ * sp * sq) / ((1.0 + lamQ * sp) * (1.0 + lamQ * sq));
    if (slope > 0.0) b = q;
    else a = p;
  }
  return exp(0.5 * (a + b));
}

// Halpern step for entry i: u^{r,t+1} = rho u^{r,0} + (1 - rho)(2 ubar - u),
// with Q w and A^T y carried along by linearity
template <int BS>
__device__ __forceinline__ void halpern(BShared<BS>& S, int i, double rho, bool has_rows, double xb, double wb,
                                        double Qwb, double g) {
  const double xn = rho * S.xa[i] + (1.0 - rho) * (2.0 * xb - S.xs[i]);
  const double wn = rho * S.wa[i] + (1.0 - rho) * (2.0 * wb - S.ws[i]);
  const double Qwn = rho * S.Qwa[i] + (1.0 - rho) * (2.0 * Qwb - S.Qws[i]);
  const double ATyn = rho * S.ATya[i] + (1.0 - rho) * (2.0 * g - S.ATys[i]);
  S.xs[i] = xn; S.ws[i] = wn; S.Qws[i] = Qwn; S.ATys[i] = has_rows ? ATyn : 0.0;
}

// Stopping test, restart criteria (Section 3.2) and the sigma update of
// Algorithm 5 at a check; thread 0 only, results in S.ctrl.  Kept out of
// line: it runs once per check and its golden section needs registers the
// iteration does not.
template <int BS>
__device__ __noinline__ void check_decision(BShared<BS>& S, double eta_p, double eta_d, double eta_gap,
                                            double R, double Rr0, double Rprev, long long t, long long k, double lamA,
                                            double lamQ, double thy, double thw, double thq, double th2, double th3,
                                            double sigma, double alpha3, double R0ref) {
  // (read from the LDS copy: a reference to the kernel argument itself would
  // make the compiler keep a copy of it in scratch memory)
  const BOpts& o = S.opt;
  const double kkt = fmax(eta_p, fmax(eta_d, eta_gap));
  int tm = -1, rs = 0;
  if (isnan(kkt) || isnan(R)) tm = HPRQP_NUMERICAL;
  else if (kkt <= o.tol) tm = HPRQP_SOLVED;
  else if (k >= o.max_iter) tm = HPRQP_MAX_ITER;
  else if (o.time_ticks > 0 && (long long)(wall_clock64() - *o.t0) >= o.time_ticks) tm = HPRQP_TIME_LIMIT;
  else if (o.enable_restart) {
    const bool c1 = R <= o.alpha1 * Rr0;                              // eq:restart_1
    const bool c2 = Rprev >= 0.0 && R <= o.alpha2 * Rr0 && R > Rprev; // eq:restart_2
    const bool c3 = (double)t >= alpha3 * (double)k;                  // eq:restart_3
    rs = c1 || c2 || c3;
  }
  double sig = sigma, a3 = alpha3, r0 = R0ref;
  if (tm < 0 && rs) {
    if (r0 < 0.0) r0 = R;
    const double ratio = R / r0;
    if (o.enable_sigma_update) {
      // Algorithm 5
      double th1 = lamA * thy + lamQ * thw - 2.0 * thq;
      th1 = fmax(th1, 1e-12); th2 = fmax(th2, 1e-12); th3 = fmax(th3, 0.0);
      const double snew = golden_sigma_dev(th1, th2, th3, lamQ);
      const double beta = exp(-ratio);
      sig = exp(beta * log(snew) + (1.0 - beta) * log(sig));
    }
    if (ratio <= 0.1) a3 = 0.2;
  }
  S.ctrl[0] = tm; S.ctrl[1] = rs; S.ctrl[2] = sig; S.ctrl[3] = a3; S.ctrl[4] = r0;
}

// ---------------------------------------------------------------------------
// persistent kernel (RM: largest rank of F handled, F rows padded with zeros)
// ---------------------------------------------------------------------------
template <int RM, int BS>
__global__ __launch_bounds__(BS, BCfg<BS>::MIN_BLOCKS) void k_batch_solve(const BInst* __restrict__ insts, const int* __restrict__ order,
                                                      int count, int* __restrict__ queue, BOpts o,
                                                      const double* __restrict__ y0, const double* __restrict__ w0,
                                                      const double* __restrict__ x0, double* __restrict__ yo,
                                                      double* __restrict__ zo, double* __restrict__ wo,
                                                      double* __restrict__ xo, BInfo* __restrict__ infos,
                                                      double* __restrict__ hbuf) {
  constexpr int NM = BCfg<BS>::NMAX;
  __shared__ BShared<BS> S;
  const int tid = threadIdx.x;
  int par = 0;
  if (tid == 0) S.opt = o;   // read after the queue's barriers below
  // the block's check buffer: xbar, wbar, Q wbar, A^T ybar, zbar (entries owned per thread)
  double* const Hx = hbuf + (size_t)blockIdx.x * 5 * NM;
  double* const Hw = Hx + NM;
  double* const HQw = Hx + 2 * NM;
  double* const Hg = Hx + 3 * NM;
  double* const Hz = Hx + 4 * NM;
  for (;;) {
    if (tid == 0) S.inst = atomicAdd(queue, 1);
    __syncthreads();
    const int qi = S.inst;
    __syncthreads();
    if (qi >= count) break;                        // every wave leaves together
    const int ii = order[qi];
    const BInst I = insts[ii];
    Elem<RM, BS> E;
    E.n = I.n; E.m = I.m; E.r = I.r; E.FT = I.FT;
    E.c = I.c; E.L = I.L; E.U = I.U; E.dg = I.dg;
    E.refresh();
    const int n = I.n, m = I.m;
    if (tid < m) { S.l[tid] = I.l[tid]; S.u[tid] = I.u[tid]; }
    if (tid == 0) a_pieces(S, I);
    QRows<RM, false> Fg;   // F from memory: power method and checks (rare)
    int tb[HB_EPT], te[HB_EPT];   // A^T ranges of the thread's entries (empty when invalid)
#pragma unroll
    for (int e = 0; e < HB_EPT; ++e) {
      const int i = E.idx(e);
      tb[e] = i < n ? gld(I.trp, i) : 0;
      te[e] = i < n ? gld(I.trp, i + 1) : 0;
    }
    __syncthreads();

    // ---- lambda_Q: power method on Q from the all-ones start (Section 4.1) ----
    double lamQ = o.lamQ, lamA = o.lamA;
    if (!(lamQ > 0.0)) {
      double pv[HB_EPT], qv[HB_EPT];
      const double s0 = 1.0 / sqrt((double)n);
#pragma unroll
      for (int e = 0; e < HB_EPT; ++e) pv[e] = E.valid(e) ? s0 : 0.0;
      double lam = 0.0, lam_old = 0.0;
      for (int it = 1; it <= 5000; ++it) {
        q_apply(S, par, E, Fg, pv, qv);
        double rr[2] = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < HB_EPT; ++e) { rr[0] += pv[e] * qv[e]; rr[1] += qv[e] * qv[e]; }
        bred<2>(S, par, rr, 0u);
        lam = rr[0];
        if (rr[1] == 0.0) break;
        if (it > 1 && fabs(lam - lam_old) <= 1e-6 * fabs(lam)) break;
        lam_old = lam;
        const double sc = 1.0 / sqrt(rr[1]);
#pragma unroll
        for (int e = 0; e < HB_EPT; ++e) pv[e] = qv[e] * sc;
      }
      lamQ = 1.01 * lam;
    }
    // ---- lambda_A: power method on A A^T from the all-ones start ----
    if (!(lamA > 0.0) && m > 0) {
      double pv[HB_EPT];
      if (tid < m) S.pw[tid] = 1.0 / sqrt((double)m);
      __syncthreads();
      double lam = 0.0, lam_old = 0.0;
      for (int it = 1; it <= 5000; ++it) {
        at_apply(E, I, tb, te, S.pw, pv);          // u = A^T v
        const double au = a_apply(S, E, I, pv);    // w = A u (row tid)
        double rr[2] = {0.0, 0.0};
        if (tid < m) { rr[0] = S.pw[tid] * au; rr[1] = au * au; }
        bred<2>(S, par, rr, 0u);
        lam = rr[0];
        if (rr[1] == 0.0) break;
        if (it > 1 && fabs(lam - lam_old) <= 1e-6 * fabs(lam)) break;
        lam_old = lam;
        if (tid < m) S.pw[tid] = au / sqrt(rr[1]);
        __syncthreads();
      }
      lamA = 1.01 * lam;
    }
    // ---- sigma0 = ||b|| / ||c|| (Section 4.1); ||b||_inf, ||c||_inf ----
    double nrm[4] = {0.0, 0.0, 0.0, 0.0};
    if (tid < m) {
      const double a = isinf(S.l[tid]) ? 0.0 : fabs(S.l[tid]), b = isinf(S.u[tid]) ? 0.0 : fabs(S.u[tid]);
      const double bi = fmax(a, b);
      nrm[0] = bi * bi; nrm[1] = bi;
    }
#pragma unroll
    for (int e = 0; e < HB_EPT; ++e) {
      const double ce = E.valid(e) ? E.c[E.idx(e)] : 0.0;
      nrm[2] += ce * ce; nrm[3] = fmax(nrm[3], fabs(ce));
    }
    bred<4>(S, par, nrm, 0xAu);
    const double binf = nrm[1], cinf = nrm[3];
    double sigma;
    {
      const double nb = sqrt(nrm[0]), nc = sqrt(nrm[2]);
      if (o.sigma0 > 0.0) sigma = o.sigma0;
      else if (nb >= 1e-16 && nb <= 1e16 && nc >= 1e-16 && nc <= 1e16) sigma = nb / nc;
      else sigma = 1.0;
    }
    const double sigma_init = sigma;

    // ---- state: origin or warm start ----
    // the iterate lives in LDS; thread t owns entries t + BS e (no other
    // thread reads them), so updates need no barrier
#pragma unroll
    for (int e = 0; e < HB_EPT; ++e) {
      const int i = E.idx(e);
      const bool ok = i < n;
      S.xs[i] = (ok && x0) ? x0[I.off_n + i] : 0.0;
      S.ws[i] = (ok && w0) ? w0[I.off_n + i] : 0.0;
    }
    if (tid < m) S.y[tid] = y0 ? y0[I.off_m + tid] : 0.0;
    __syncthreads();

    // F in registers for the iteration; not live across a check, which reads
    // F from memory and loads this copy again when it is done
    QRows<RM, (RM <= 10)> Fq;
    Fq.load(E);
    long long k = 0, t = 0;
    int r = 0, term = -1;
    double alpha3 = o.alpha3, R0ref = -1.0, Rr0 = -1.0, Rprev = -1.0, R = 0.0;
    double eta_p = 0, eta_d = 0, eta_gap = 0, pobj = 0, dobj = 0;
    bool new_epoch = true;
    while (term < 0) {
      E.refresh();
      const int tid = E.tid;
      if (new_epoch) {
        // anchor u^{r,0} = u; exact A^T y and Q w.  Each thread keeps the
        // anchors of its own variables in LDS (no other thread reads them).
        if (tid < m) S.ya[tid] = S.y[tid];
        __syncthreads();
        double ATy[HB_EPT], Qw[HB_EPT], w[HB_EPT];
#pragma unroll
        for (int e = 0; e < HB_EPT; ++e) w[e] = S.ws[E.idx(e)];
        at_apply(E, I, tb, te, S.y, ATy);
        q_apply(S, par, E, Fq, w, Qw);
#pragma unroll
        for (int e = 0; e < HB_EPT; ++e) {
          const int i = E.idx(e);
          S.Qws[i] = Qw[e]; S.ATys[i] = ATy[e];
          S.xa[i] = S.xs[i]; S.wa[i] = w[e]; S.Qwa[i] = Qw[e]; S.ATya[i] = ATy[e];
        }
        t = 0; Rprev = -1.0;
        new_epoch = false;
      }
      const double sQ = sigma * lamQ, kappa = sigma / (1.0 + sQ), sA = sigma * lamA;
      const double rho = 1.0 / (double)(t + 2);
      const bool is_check = ((k + 1) % o.check_every == 0) || (k + 1 >= o.max_iter);
      const bool want_r = (t == 0) || is_check;
      // z/x step ("update-z", "update-x"); zbar itself is formed at checks only
      double xh[HB_EPT], xb[HB_EPT];
#pragma unroll
      for (int e = 0; e < HB_EPT; ++e) {
        const int i = E.idx(e);
        const bool ok = E.valid(e);
        const double xe = S.xs[i];
        const double rz = xe + sigma * (-S.Qws[i] + S.ATys[i] - (ok ? gld(E.c, i) : 0.0));
        xb[e] = ok ? clampd(rz, gld(E.L, i), gld(E.U, i)) : 0.0;
        xh[e] = ok ? 2.0 * xb[e] - xe : 0.0;
      }
      // Q xhat, v = xhat + kappa (Qw - Q xhat)
      double q1[HB_EPT];
      q_apply(S, par, E, Fq, xh, q1);
      // y step ("update-y") and its Halpern update
      double dy2 = 0.0, th_y = 0.0;
      if (m > 0) {
        double v[HB_EPT];
#pragma unroll
        for (int e = 0; e < HB_EPT; ++e) v[e] = E.valid(e) ? xh[e] + kappa * (S.Qws[E.idx(e)] - q1[e]) : 0.0;
        const double av = a_apply(S, E, I, v);
        if (tid < m) {
          const double yi = S.y[tid], yai = S.ya[tid];
          const double rr = av - sA * yi;
          const double ybv = (clampd(rr, S.l[tid], S.u[tid]) - rr) / sA;
          S.yb[tid] = ybv;
          dy2 = (yi - ybv) * (yi - ybv);
          th_y = (ybv - yai) * (ybv - yai);
          S.yn[tid] = rho * yai + (1.0 - rho) * (2.0 * ybv - yi);   // Halpern y+ (applied below)
        }
        __syncthreads();
      }
      // g = A^T ybar, d = A^T(ybar - y)
      double d[HB_EPT], g[HB_EPT];
      at_apply(E, I, tb, te, S.yb, g);
#pragma unroll
      for (int e = 0; e < HB_EPT; ++e) d[e] = m > 0 ? g[e] - S.ATys[E.idx(e)] : 0.0;
      double q2[HB_EPT];
      q_apply(S, par, E, Fq, d, q2);
      // wbar ("update-w") and Q wbar
      double wb[HB_EPT], Qwb[HB_EPT];
#pragma unroll
      for (int e = 0; e < HB_EPT; ++e) {
        const double inv = 1.0 / (1.0 + sQ);
        const int i = E.idx(e);
        wb[e] = (sQ * S.ws[i] + xh[e]) * inv + kappa * d[e];
        Qwb[e] = (sQ * S.Qws[i] + q1[e]) * inv + kappa * q2[e];
      }
      // merit R~ = ||u - ubar||_M (theta decomposition of the metric of Algorithm 3)
      if (want_r) {
        double s7[7] = {dy2, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int e = 0; e < HB_EPT; ++e) {
          const int i = E.idx(e);
          const double dw = S.ws[i] - wb[e], Qdw = S.Qws[i] - Qwb[e], ATdy = -d[e], QATdy = -q2[e];
          const double dx = E.valid(e) ? S.xs[i] - xb[e] : 0.0;
          s7[1] += dw * Qdw; s7[2] += Qdw * ATdy; s7[3] += dx * dx;
          s7[4] += ATdy * QATdy; s7[5] += ATdy * dx; s7[6] += Qdw * dx;
        }
        bred<7>(S, par, s7, 0u);
        const double th1 = lamA * s7[0] + lamQ * s7[1] - 2.0 * s7[2];
        const double m2 = sigma * th1 + s7[3] / sigma + sigma * sigma * s7[4] / (1.0 + sQ) + 2.0 * (s7[5] - s7[6]);
        R = sqrt(m2 > 0.0 ? m2 : 0.0);
      }
      t += 1; k += 1;
      if (t == 1) Rr0 = R;
      if (!is_check) {
        // Halpern step: u^{r,t+1} = rho u^{r,0} + (1 - rho)(2 ubar - u)
#pragma unroll
        for (int e = 0; e < HB_EPT; ++e) {
          if (!E.valid(e)) continue;
          const int i = E.idx(e);
          halpern(S, i, rho, m > 0, xb[e], wb[e], Qwb[e], g[e]);
        }
        if (tid < m) S.y[tid] = S.yn[tid];
        __syncthreads();
        continue;
      }

      // ---- check iteration (every check_every iterations): the bar values go
      // to the block's buffer H so that the registers of the loop above are
      // free for the stopping test and Algorithm 5
#pragma unroll
      for (int e = 0; e < HB_EPT; ++e) {
        const int i = E.idx(e);
        Hx[i] = xb[e]; Hw[i] = wb[e]; HQw[i] = Qwb[e]; Hg[i] = g[e];
      }
      // theta~ of Algorithm 5: D = ubar - u^{r,0}; e = A^T (ybar - y_a) = g - ATy_a
      double th[5] = {th_y, 0, 0, 0, 0};
      {
        double ev[HB_EPT], Qe[HB_EPT];
#pragma unroll
        for (int e = 0; e < HB_EPT; ++e) ev[e] = (m > 0 && E.valid(e)) ? Hg[E.idx(e)] - S.ATya[E.idx(e)] : 0.0;
        q_apply(S, par, E, Fg, ev, Qe);
#pragma unroll
        for (int e = 0; e < HB_EPT; ++e) {
          if (!E.valid(e)) continue;
          const int i = E.idx(e);
          const double Dw = Hw[i] - S.wa[i], QDw = HQw[i] - S.Qwa[i];
          const double Dx = Hx[i] - S.xa[i];
          th[1] += Dw * QDw; th[2] += QDw * ev[e]; th[3] += Dx * Dx; th[4] += ev[e] * Qe[e];
        }
        bred<5>(S, par, th, 0u);
      }
      // stopping quantities at (ybar, zbar, xbar) (Section 4.1), with
      // zbar = (xbar - r_z) / sigma formed here
      {
        double res[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        double xbv[HB_EPT], Qx[HB_EPT];
#pragma unroll
        for (int e = 0; e < HB_EPT; ++e) xbv[e] = Hx[E.idx(e)];
        q_apply(S, par, E, Fg, xbv, Qx);
        const double ax = m > 0 ? a_apply(S, E, I, xbv) : 0.0;   // (A xbar)_tid
        // res: 0 max|Ax-PiK|, 1 max|Ax|, 2 sum(l y+ + u y-), 3 #inf, 4 max|dual|, 5 max|g|, 6 max|Qx|,
        //      7 <x,Qx>, 8 <c,x>, 9 sum(L z+ + U z-) (+ #inf folded into 3)
        if (tid < m) {
          const double li = S.l[tid], ui = S.u[tid], yv = S.yb[tid];
          res[0] = fabs(ax - clampd(ax, li, ui));
          res[1] = fabs(ax);
          if (yv > 0.0) { if (isinf(li)) res[3] += 1.0; else res[2] += li * yv; }
          else if (yv < 0.0) { if (isinf(ui)) res[3] += 1.0; else res[2] += ui * yv; }
        }
#pragma unroll
        for (int e = 0; e < HB_EPT; ++e) {
          if (!E.valid(e)) continue;
          const int i = E.idx(e);
          const double ce = gld(E.c, i), Le = gld(E.L, i), Ue = gld(E.U, i), ge = Hg[i];
          const double rz = S.xs[i] + sigma * (-S.Qws[i] + S.ATys[i] - ce);
          const double zbe = (xbv[e] - rz) / sigma;
          Hz[i] = zbe;
          res[4] = fmax(res[4], fabs(-Qx[e] + ge + zbe - ce));
          res[5] = fmax(res[5], fabs(ge));
          res[6] = fmax(res[6], fabs(Qx[e]));
          res[7] += xbv[e] * Qx[e];
          res[8] += ce * xbv[e];
          if (zbe > 0.0) { if (isinf(Le)) res[3] += 1.0; else res[9] += Le * zbe; }
          else if (zbe < 0.0) { if (isinf(Ue)) res[3] += 1.0; else res[9] += Ue * zbe; }
        }
        bred<10>(S, par, res, 0x73u);               // maxes: 0, 1, 4, 5, 6
        eta_p = m > 0 ? res[0] / (1.0 + fmax(binf, res[1])) : 0.0;
        eta_d = res[4] / (1.0 + fmax(cinf, fmax(res[5], res[6])));
        pobj = 0.5 * res[7] + res[8];
        if (res[3] > 0.0) { dobj = -INFINITY; eta_gap = INFINITY; }
        else {
          dobj = -0.5 * res[7] + res[2] + res[9];
          eta_gap = fabs(pobj - dobj) / (1.0 + fmax(fabs(pobj), fabs(dobj)));
        }
      }
      // decisions (thread 0, FP64), broadcast through LDS
      if (tid == 0)
        check_decision(S, eta_p, eta_d, eta_gap, R, Rr0, Rprev, t, k, lamA, lamQ, th[0], th[1], th[2], th[3], th[4],
                       sigma, alpha3, R0ref);
      __syncthreads();
      term = (int)S.ctrl[0];
      const int restart = (term < 0) && (S.ctrl[1] != 0.0);
      sigma = S.ctrl[2]; alpha3 = S.ctrl[3]; R0ref = S.ctrl[4];
      Rprev = R;
      __syncthreads();
      if (term >= 0) {
        // output ubar of the last iteration (Algorithm 4, "Output")
        for (int e = 0; e < HB_EPT; ++e) {
          const int i = E.idx(e);
          if (i < n) {
            xo[I.off_n + i] = Hx[i];
            zo[I.off_n + i] = Hz[i];
            wo[I.off_n + i] = Hw[i];
          }
        }
        break;
      }
      if (restart) {
        // u^{r+1,0} = ubar
        for (int e = 0; e < HB_EPT; ++e) { S.xs[E.idx(e)] = Hx[E.idx(e)]; S.ws[E.idx(e)] = Hw[E.idx(e)]; }
        if (tid < m) S.y[tid] = S.yb[tid];
        __syncthreads();
        r += 1;
        new_epoch = true;
      } else {
        for (int e = 0; e < HB_EPT; ++e) {
          if (!E.valid(e)) continue;
          const int i = E.idx(e);
          halpern(S, i, rho, m > 0, Hx[i], Hw[i], HQw[i], Hg[i]);
        }
        if (tid < m) S.y[tid] = S.yn[tid];
        __syncthreads();
      }
      Fq.load(E);
    }
    if (tid < m) yo[I.off_m + tid] = S.yb[tid];
    if (tid == 0) {
      BInfo f;
      f.term = term; f.restarts = r; f.iters = k; f.sigma = sigma; f.sigma0 = sigma_init;
      f.lamA = lamA; f.lamQ = lamQ; f.eta_p = eta_p; f.eta_d = eta_d; f.eta_gap = eta_gap;
      f.pobj = pobj; f.dobj = dobj; f.R_last = R;
      infos[ii] = f;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------
// per-instance validation: bit 0 bounds / non-finite data, bit 1 CSR structure
__global__ void k_batch_validate(const BInst* __restrict__ insts, int count, int* __restrict__ flags) {
  const int ii = blockIdx.x;
  if (ii >= count) return;
  const BInst I = insts[ii];
  __shared__ int sflag;
  if (threadIdx.x == 0) sflag = 0;
  __syncthreads();
  int f = 0;
  for (int i = threadIdx.x; i < I.n; i += blockDim.x) {
    if (!(I.L[i] <= I.U[i]) || I.L[i] == INFINITY || I.U[i] == -INFINITY || !isfinite(I.c[i]) || !isfinite(I.dg[i]))
      f |= 1;
    for (int k = 0; k < I.r; ++k)
      if (!isfinite(I.F[(size_t)i * I.r + k])) f |= 1;
  }
  for (int i = threadIdx.x; i < I.m; i += blockDim.x) {
    if (!(I.l[i] <= I.u[i]) || I.l[i] == INFINITY || I.u[i] == -INFINITY) f |= 1;
    const int b = I.arp[i], e = I.arp[i + 1];
    if ((i == 0 && b != 0) || b < 0 || e < b || (long long)e > I.annz || (i == I.m - 1 && e != I.annz) || e - b > I.n)
      f |= 2;
  }
  if (f) atomicOr(&sflag, f);
  __syncthreads();
  // columns, only once every row pointer lies in [0, nnz]
  if ((sflag & 2) == 0 && I.m > 0) {
    const int nnz = I.arp[I.m];
    int g = 0;
    for (int k = threadIdx.x; k < nnz; k += blockDim.x)
      if (I.aci[k] < 0 || I.aci[k] >= I.n || !isfinite(I.aval[k])) g |= 2;
    if (g) atomicOr(&sflag, g);
  }
  __syncthreads();
  if (threadIdx.x == 0) flags[ii] = sflag;
}

// A^T of one instance per block (rows of A^T ordered by row of A): LDS
// histogram, then one thread scans and scatters in CSR order (deterministic).
__global__ void k_batch_transpose(const BInst* __restrict__ insts, const int* __restrict__ rep, int nrep,
                                  int* __restrict__ trp_all, int* __restrict__ tci_all, double* __restrict__ tval_all,
                                  const long long* __restrict__ toff) {
  const int q = blockIdx.x;
  if (q >= nrep) return;
  const BInst I = insts[rep[q]];
  __shared__ int cnt[HB_NMAX + 1];
  for (int i = threadIdx.x; i <= I.n; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  const int nnz = I.m > 0 ? I.arp[I.m] : 0;
  for (int k = threadIdx.x; k < nnz; k += blockDim.x) atomicAdd(&cnt[I.aci[k] + 1], 1);
  __syncthreads();
  int* trp = trp_all + toff[2 * q];
  int* tci = tci_all + toff[2 * q + 1];
  double* tv = tval_all + toff[2 * q + 1];
  if (threadIdx.x == 0) {
    for (int i = 0; i < I.n; ++i) cnt[i + 1] += cnt[i];
    for (int i = 0; i <= I.n; ++i) trp[i] = cnt[i];
    for (int row = 0; row < I.m; ++row)
      for (int k = I.arp[row]; k < I.arp[row + 1]; ++k) {
        const int p = cnt[I.aci[k]]++;
        tci[p] = row;
        tv[p] = I.aval[k];
      }
  }
}

// F of every instance with rows padded to the kernel's rank RM:
// FT[i RM + k] = F(i, k) for k < r, 0 for r <= k < RM
// (one block per distinct copy: rep lists one instance of each)
__global__ void k_batch_ft(const BInst* __restrict__ insts, const int* __restrict__ rep, int nrep, int RM,
                           double* __restrict__ ft_all, const long long* __restrict__ ft_off) {
  if ((int)blockIdx.x >= nrep) return;
  const int ii = rep[blockIdx.x];
  const BInst I = insts[ii];
  double* ft = ft_all + ft_off[ii];
  const long long tot = (long long)RM * I.n;
  for (long long q = threadIdx.x; q < tot; q += blockDim.x) {
    const int i = (int)(q / RM), k = (int)(q % RM);
    ft[q] = k < I.r ? I.F[(size_t)i * I.r + k] : 0.0;
  }
}

__global__ void k_zero_ints(int* p, int k) {
  if ((int)threadIdx.x < k) p[threadIdx.x] = 0;
}

// the time-limit stamp of a solve
__global__ void k_stamp(long long* t0) {
  if (threadIdx.x == 0) *t0 = (long long)wall_clock64();
}

// ||Q(w - x)||_inf of every instance at its returned point, Q = diag(d) + F F^T
// (the diagnostic of the shadow w_Q of Proposition 2.4): one workgroup per
// instance, t = F^T (w - x) and the maximum by fixed-order reductions
#define HB_QWX_BS 256
__global__ __launch_bounds__(HB_QWX_BS) void k_batch_qwx(const BInst* __restrict__ insts, int count,
                                                          const double* __restrict__ w, const double* __restrict__ x,
                                                          double* __restrict__ out) {
  constexpr int NW = HB_QWX_BS / 64;
  __shared__ double part[16][NW];
  __shared__ double t[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int ii = blockIdx.x; ii < count; ii += gridDim.x) {
    const BInst I = insts[ii];
    const double* wi = w + I.off_n;
    const double* xi = x + I.off_n;
    double acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.0;
    for (int i = threadIdx.x; i < I.n; i += HB_QWX_BS) {
      const double d = wi[i] - xi[i];
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < I.r) acc[k] += I.F[(size_t)i * I.r + k] * d;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const double v = wave_sum(acc[k]);
      if (lane == 0) part[k][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
      double v = 0.0;
      for (int q = 0; q < NW; ++q) v += part[threadIdx.x][q];
      t[threadIdx.x] = v;
    }
    __syncthreads();
    double mx = 0.0;
    for (int i = threadIdx.x; i < I.n; i += HB_QWX_BS) {
      double q = I.dg[i] * (wi[i] - xi[i]);
      for (int k = 0; k < I.r; ++k) q += I.F[(size_t)i * I.r + k] * t[k];
      mx = fmax(mx, fabs(q));
    }
    mx = wave_max(mx);
    if (lane == 0) part[0][wv] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      double v = part[0][0];
      for (int q = 1; q < NW; ++q) v = fmax(v, part[0][q]);
      out[ii] = v;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct hprqp_batch {
  int count = 0;
  hipStream_t st = nullptr, own_st = nullptr;
  BOpts o{};
  BInst* d_insts = nullptr;
  int* d_order = nullptr;
  int* d_queue = nullptr;
  int* d_flags = nullptr;
  BInfo* d_infos = nullptr;
  double* d_qwx = nullptr;     // ||Q(w - x)||_inf per instance
  long long* d_t0 = nullptr;   // time-limit stamp
  int *trp = nullptr, *tci = nullptr;
  double* tval = nullptr;
  long long* d_toff = nullptr;
  int* d_rep = nullptr;
  double* ft = nullptr;        // F of every instance, rows padded to rank_max
  long long* d_ftoff = nullptr;
  int* d_ftrep = nullptr;      // one instance per distinct F
  // one persistent kernel per block size in use: kernel k takes the
  // instances d_order[first, first + cnt) (largest first) with kern[k].bs
  // threads per workgroup, on its own stream (kernel 0 on the batch stream);
  // d_queue holds one counter per kernel
  struct Kern {
    int bs = 0, first = 0, cnt = 0, grid = 0;
    double* hbuf = nullptr;    // per-block check buffers
    hipStream_t st = nullptr;  // created by the library for kernels 1..
    hipEvent_t ev_join = nullptr;
  } kern[HB_NCLASS];
  int nkern = 0;
  std::vector<int> order_default;   // d_order as built at create
  hipEvent_t ev_fork = nullptr;
  // size classes n <= 256 << c: instances, block size, and (autotuned) the
  // mean kernel time per instance-iteration of each candidate block size
  int class_cnt[HB_NCLASS] = {0, 0, 0, 0};
  int class_bs[HB_NCLASS] = {0, 0, 0, 0};
  double class_us[HB_NCLASS][HB_NCLASS] = {};   // [class][log2(bs / 64)], 0: not timed
  int tuned = 0;
  long long total_n = 0, total_m = 0;
  int rank_max = 0;       // 10 or 16: the kernel instantiation used
  double last_kernel_s = 0.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~hprqp_batch() {
    void* ps[] = {d_insts, d_order, d_queue, d_flags,   d_infos, trp,     tci,     tval,
                  d_toff,  d_rep,   ft,      d_ftoff,   d_ftrep, d_qwx,   d_t0};
    for (void* p : ps)
      if (p) hipFree(p);
    for (auto& k : kern) {
      if (k.hbuf) hipFree(k.hbuf);
      if (k.ev_join) hipEventDestroy(k.ev_join);
      if (k.st) hipStreamDestroy(k.st);
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (ev_fork) hipEventDestroy(ev_fork);
    if (own_st) hipStreamDestroy(own_st);
  }
};

namespace {
struct BErr {
  hprqp_status st;
  std::string msg;
};
[[noreturn]] void bfail(hprqp_status st, const std::string& m) { throw BErr{st, m}; }
void bcheck(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) bfail(HPRQP_ERR_OOM, std::string(what) + ": out of device memory");
    bfail(HPRQP_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  }
}
#define HBC(x) bcheck((x), #x)

// Launch of the persistent solve kernel with bs threads per workgroup.
void batch_launch(int bs, int rank, hipStream_t s, int grid, const BInst* insts, const int* order, int cnt, int* queue,
                  const BOpts& o, const double* y0, const double* w0, const double* x0, double* y, double* z,
                  double* w, double* x, BInfo* infos, double* hbuf) {
#define HB_LAUNCH(RM, BS)                                                                                        \
  k_batch_solve<RM, BS><<<grid, BS, 0, s>>>(insts, order, cnt, queue, o, y0, w0, x0, y, z, w, x, infos, hbuf)
  if (rank == 10) {
    switch (bs) {
      case 64: HB_LAUNCH(10, 64); break;
      case 128: HB_LAUNCH(10, 128); break;
      case 256: HB_LAUNCH(10, 256); break;
      default: HB_LAUNCH(10, 512); break;
    }
  } else {
    switch (bs) {
      case 64: HB_LAUNCH(16, 64); break;
      case 128: HB_LAUNCH(16, 128); break;
      case 256: HB_LAUNCH(16, 256); break;
      default: HB_LAUNCH(16, 512); break;
    }
  }
#undef HB_LAUNCH
  HBC(hipGetLastError());
}

// Workgroups of the solve kernel with bs threads resident on the device at once.
int batch_resident(int bs, int rank, int ncu) {
  const void* k = nullptr;
  if (rank == 10)
    k = bs == 64 ? (const void*)k_batch_solve<10, 64> : bs == 128 ? (const void*)k_batch_solve<10, 128>
        : bs == 256 ? (const void*)k_batch_solve<10, 256> : (const void*)k_batch_solve<10, 512>;
  else
    k = bs == 64 ? (const void*)k_batch_solve<16, 64> : bs == 128 ? (const void*)k_batch_solve<16, 128>
        : bs == 256 ? (const void*)k_batch_solve<16, 256> : (const void*)k_batch_solve<16, 512>;
  int per_cu = 0;
  HBC(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, bs, 0));
  return ncu * std::max(per_cu, 1);
}

// The batched solver's shape autotuner.  For every size class with at least
// 8 instances, each block size that can hold the class (n <= 4 bs) is timed
// on a sample of the class's instances -- evenly spaced over the class, at
// most eight per compute unit, enough to fill the device -- running
// exactly 100 iterations per instance (tolerance 0, lambda's fixed at 1, so
// no power method) into scratch outputs; the default block size is kept
// unless another is at least 5% faster (near ties would otherwise flip
// between runs).  Only the speed is measured: the shapes do not change
// what is computed beyond the order of the block reductions.
void autotune_batch(hprqp_batch* b, const std::vector<BInst>& hi, const std::vector<int> (&cls)[HB_NCLASS], int ncu) {
  BOpts o = b->o;
  o.tol = 0.0; o.max_iter = 100; o.check_every = 100; o.lamA = 1.0; o.lamQ = 1.0; o.sigma0 = 1.0;
  o.time_ticks = 0;
  const long long tn = std::max(1ll, b->total_n), tm = std::max(1ll, b->total_m);
  double *sy = nullptr, *sz = nullptr, *sw = nullptr, *sx = nullptr, *hb = nullptr;
  int *sorder = nullptr, *squeue = nullptr;
  BInfo* sinfo = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  const auto cleanup = [&] {
    for (void* p : {(void*)sy, (void*)sz, (void*)sw, (void*)sx, (void*)hb, (void*)sorder, (void*)squeue, (void*)sinfo})
      if (p) hipFree(p);
    if (t0) hipEventDestroy(t0);
    if (t1) hipEventDestroy(t1);
  };
  try {
    HBC(hipMalloc(&sy, tm * sizeof(double)));
    HBC(hipMalloc(&sz, tn * sizeof(double)));
    HBC(hipMalloc(&sw, tn * sizeof(double)));
    HBC(hipMalloc(&sx, tn * sizeof(double)));
    HBC(hipMalloc(&sinfo, b->count * sizeof(BInfo)));
    HBC(hipMalloc(&squeue, sizeof(int)));
    HBC(hipMalloc(&sorder, b->count * sizeof(int)));
    HBC(hipEventCreate(&t0));
    HBC(hipEventCreate(&t1));
    size_t hb_cap = 0;
    for (int c = 0; c < HB_NCLASS; ++c) {
      const int cnt = (int)cls[c].size();
      if (cnt < 8) continue;
      const int want = std::min(cnt, 8 * ncu);
      std::vector<int> sample;
      for (int q = 0; q < want; ++q) sample.push_back(cls[c][(size_t)q * cnt / want]);
      HBC(hipMemcpyAsync(sorder, sample.data(), sample.size() * sizeof(int), hipMemcpyHostToDevice, b->st));
      double best = 0.0;
      int best_bs = b->class_bs[c];
      for (int lb = 0; lb < HB_NCLASS; ++lb) {
        const int bs = 64 << lb;
        if (HB_EPT * bs < (256 << c)) continue;    // cannot hold the class
        const int grid = std::max(1, std::min(want, batch_resident(bs, b->rank_max, ncu)));
        const size_t need = (size_t)grid * 5 * HB_EPT * bs;
        if (need > hb_cap) {
          if (hb) HBC(hipFree(hb));
          hb = nullptr;
          HBC(hipMalloc(&hb, need * sizeof(double)));
          hb_cap = need;
        }
        float ms = 0.f;
        for (int rep = 0; rep < 2; ++rep) {   // the first launch loads the code
          k_zero_ints<<<1, 64, 0, b->st>>>(squeue, 1);
          HBC(hipEventRecord(t0, b->st));
          batch_launch(bs, b->rank_max, b->st, grid, b->d_insts, sorder, (int)sample.size(), squeue, o, nullptr,
                       nullptr, nullptr, sy, sz, sw, sx, sinfo, hb);
          HBC(hipEventRecord(t1, b->st));
          HBC(hipEventSynchronize(t1));
          HBC(hipEventElapsedTime(&ms, t0, t1));
        }
        const double us = 1e3 * ms / (100.0 * sample.size());   // per instance-iteration
        b->class_us[c][lb] = us;
        if (bs == b->class_bs[c]) best = best > 0.0 ? std::min(best, us) : us;
      }
      // the fastest, unless within 5% of the default
      double dflt = 0.0;
      for (int lb = 0; lb < HB_NCLASS; ++lb)
        if ((64 << lb) == b->class_bs[c]) dflt = b->class_us[c][lb];
      double bu = dflt;
      for (int lb = 0; lb < HB_NCLASS; ++lb) {
        const double us = b->class_us[c][lb];
        if (us > 0.0 && us < 0.95 * dflt && us < bu) { bu = us; best_bs = 64 << lb; }
      }
      b->class_bs[c] = best_bs;
      (void)best;
    }
    b->tuned = 1;
  } catch (...) {
    cleanup();
    throw;
  }
  cleanup();
}

void batch_create_impl(int count, const hprqp_problem* probs, const hprqp_options* opt, hipStream_t st,
                       hprqp_batch** out) {
  if (count <= 0 || !probs || !opt || !out) bfail(HPRQP_ERR_ARG, "bad arguments");
  if (opt->check_every <= 0 || opt->max_iter <= 0 || !(opt->tol >= 0.0)) bfail(HPRQP_ERR_ARG, "bad options");
  auto* b = new hprqp_batch();
  try {
    b->count = count;
    if (!st) {
      HBC(hipStreamCreateWithFlags(&b->own_st, hipStreamNonBlocking));
      HBC(hipDeviceSynchronize());
      st = b->own_st;
    }
    b->st = st;
    b->o.tol = opt->tol; b->o.max_iter = opt->max_iter; b->o.check_every = opt->check_every;
    b->o.sigma0 = opt->sigma0; b->o.lamA = opt->lambda_A; b->o.lamQ = opt->lambda_Q;
    b->o.alpha1 = opt->alpha1; b->o.alpha2 = opt->alpha2; b->o.alpha3 = opt->alpha3;
    b->o.enable_restart = opt->enable_restart; b->o.enable_sigma_update = opt->enable_sigma_update;
    if (!(opt->time_limit_s >= 0.0)) bfail(HPRQP_ERR_ARG, "time_limit_s must be >= 0");
    if (opt->time_limit_s > 0.0) {
      int dev = 0, khz = 0;
      HBC(hipGetDevice(&dev));
      HBC(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
      if (khz <= 0) bfail(HPRQP_ERR_HIP, "device reports no wall-clock rate");
      const double ticks = std::ceil(opt->time_limit_s * 1e3 * (double)khz);
      b->o.time_ticks = ticks >= 9e18 ? (long long)9e18 : std::max(1ll, (long long)ticks);
    }
    std::vector<BInst> hi(count);
    // unique A matrices (instances may share one) -> one A^T each
    std::vector<int> rep_of(count);
    std::vector<int> reps;
    std::map<std::tuple<const void*, const void*, const void*, int, int>, int> rep_index;
    std::vector<long long> toff;
    long long tn = 0, tz = 0;
    for (int i = 0; i < count; ++i) {
      const hprqp_problem& P = probs[i];
      if (P.qkind != HPRQP_Q_LOWRANK) bfail(HPRQP_ERR_UNSUPPORTED, "batched solve supports qkind HPRQP_Q_LOWRANK only");
      if (P.l1_weight != 0.0) bfail(HPRQP_ERR_UNSUPPORTED, "batched solve supports phi = box indicator only (l1_weight 0)");
      if (P.n <= 0 || P.n > HB_NMAX || P.m < 0 || P.m > HB_MMAX || P.lr_rank < 0 || P.lr_rank > HB_RMAX)
        bfail(HPRQP_ERR_UNSUPPORTED, "batched solve needs 0 < n <= 2048, 0 <= m <= 64, lr_rank <= 16 (instance " +
                                         std::to_string(i) + ")");
      if (!P.c || !P.L || !P.U || !P.lr_d || (P.lr_rank > 0 && !P.lr_F) ||
          (P.m > 0 && (!P.l || !P.u || !P.a_rowptr || (P.a_nnz > 0 && (!P.a_col || !P.a_val)))))
        bfail(HPRQP_ERR_ARG, "missing array in instance " + std::to_string(i));
      BInst& I = hi[i];
      std::memset(&I, 0, sizeof(I));
      I.n = P.n; I.m = P.m; I.r = P.lr_rank;
      I.c = P.c; I.L = P.L; I.U = P.U; I.l = P.l; I.u = P.u; I.dg = P.lr_d; I.F = P.lr_F;
      I.arp = P.a_rowptr; I.aci = P.a_col; I.aval = P.a_val;
      I.off_n = b->total_n; I.off_m = b->total_m;
      I.annz = P.m > 0 ? P.a_nnz : 0;
      if (P.a_nnz < 0 || P.a_nnz > (1ll << 30)) bfail(HPRQP_ERR_SHAPE, "bad a_nnz in instance " + std::to_string(i));
      b->total_n += P.n; b->total_m += P.m;
      const auto akey = std::make_tuple((const void*)P.a_rowptr, (const void*)P.a_col, (const void*)P.a_val, P.n, P.m);
      const auto it = rep_index.find(akey);
      int found = it == rep_index.end() ? -1 : it->second;
      if (found < 0) {
        found = (int)reps.size();
        rep_index.emplace(akey, found);
        reps.push_back(i);
        toff.push_back(tn);
        toff.push_back(tz);
        tn += P.n + 1;
        tz += std::max<long long>(P.a_nnz, 0);
      }
      rep_of[i] = found;
    }
    HBC(hipMalloc(&b->trp, std::max<long long>(tn, 1) * sizeof(int)));
    HBC(hipMalloc(&b->tci, std::max<long long>(tz, 1) * sizeof(int)));
    HBC(hipMalloc(&b->tval, std::max<long long>(tz, 1) * sizeof(double)));
    for (int i = 0; i < count; ++i) {
      const int q = rep_of[i];
      hi[i].trp = b->trp + toff[2 * q];
      hi[i].tci = b->tci + toff[2 * q + 1];
      hi[i].tval = b->tval + toff[2 * q + 1];
    }
    // padded copy of F: rank class of the kernel (10 or 16)
    int maxr = 0;
    for (int i = 0; i < count; ++i) maxr = std::max(maxr, hi[i].r);
    b->rank_max = maxr <= 10 ? 10 : 16;
    // (one padded copy per distinct F: instances that share F share the copy)
    std::vector<long long> ftoff(count);
    std::map<std::tuple<const double*, int, int>, long long> ft_index;
    std::vector<int> ft_rep;
    long long tf = 0;
    for (int i = 0; i < count; ++i) {
      const auto key = std::make_tuple(hi[i].F, hi[i].n, hi[i].r);
      const auto it = ft_index.find(key);
      if (it != ft_index.end()) { ftoff[i] = it->second; continue; }
      ftoff[i] = tf;
      ft_index.emplace(key, tf);
      ft_rep.push_back(i);
      tf += (long long)b->rank_max * hi[i].n;
    }
    HBC(hipMalloc(&b->ft, std::max<long long>(tf, 1) * sizeof(double)));
    HBC(hipMalloc(&b->d_ftoff, count * sizeof(long long)));
    HBC(hipMemcpyAsync(b->d_ftoff, ftoff.data(), count * sizeof(long long), hipMemcpyHostToDevice, st));
    for (int i = 0; i < count; ++i) hi[i].FT = b->ft + ftoff[i];
    HBC(hipMalloc(&b->d_insts, count * sizeof(BInst)));
    HBC(hipMemcpyAsync(b->d_insts, hi.data(), count * sizeof(BInst), hipMemcpyHostToDevice, st));
    HBC(hipMalloc(&b->d_flags, count * sizeof(int)));
    HBC(hipMemsetAsync(b->d_flags, 0, count * sizeof(int), st));
    k_batch_validate<<<count, 256, 0, st>>>(b->d_insts, count, b->d_flags);
    std::vector<int> flags(count);
    HBC(hipMemcpyAsync(flags.data(), b->d_flags, count * sizeof(int), hipMemcpyDeviceToHost, st));
    HBC(hipStreamSynchronize(st));
    for (int i = 0; i < count; ++i) {
      if (flags[i] & 2) bfail(HPRQP_ERR_SHAPE, "CSR structure of A invalid in instance " + std::to_string(i));
      if (flags[i] & 1) bfail(HPRQP_ERR_BOUNDS, "invalid bounds or non-finite data in instance " + std::to_string(i));
    }
    HBC(hipMalloc(&b->d_rep, reps.size() * sizeof(int)));
    HBC(hipMalloc(&b->d_toff, toff.size() * sizeof(long long)));
    HBC(hipMemcpyAsync(b->d_rep, reps.data(), reps.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HBC(hipMemcpyAsync(b->d_toff, toff.data(), toff.size() * sizeof(long long), hipMemcpyHostToDevice, st));
    k_batch_transpose<<<(int)reps.size(), 256, 0, st>>>(b->d_insts, b->d_rep, (int)reps.size(), b->trp, b->tci,
                                                         b->tval, b->d_toff);
    HBC(hipMalloc(&b->d_ftrep, ft_rep.size() * sizeof(int)));
    HBC(hipMemcpyAsync(b->d_ftrep, ft_rep.data(), ft_rep.size() * sizeof(int), hipMemcpyHostToDevice, st));
    k_batch_ft<<<(int)ft_rep.size(), 256, 0, st>>>(b->d_insts, b->d_ftrep, (int)ft_rep.size(), b->rank_max, b->ft,
                                                   b->d_ftoff);
    // largest instances first
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return hi[a].n > hi[c].n; });
    HBC(hipMalloc(&b->d_order, count * sizeof(int)));
    HBC(hipMalloc(&b->d_queue, HB_NCLASS * sizeof(int)));
    HBC(hipMalloc(&b->d_infos, count * sizeof(BInfo)));
    HBC(hipEventCreate(&b->e0));
    HBC(hipEventCreate(&b->e1));
    HBC(hipMalloc(&b->d_qwx, count * sizeof(double)));
    HBC(hipMalloc(&b->d_t0, sizeof(long long)));
    b->o.t0 = b->d_t0;
    int dev = 0, ncu = 0;
    HBC(hipGetDevice(&dev));
    HBC(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    // size classes: class c holds the instances with 256 << (c - 1) < n <= 256 << c
    std::vector<int> cls_order[HB_NCLASS];
    for (int i : order) {
      int c = 0;
      while (hi[i].n > (256 << c)) ++c;
      cls_order[c].push_back(i);
    }
    for (int c = 0; c < HB_NCLASS; ++c) {
      b->class_cnt[c] = (int)cls_order[c].size();
      b->class_bs[c] = c == HB_NCLASS - 1 ? 512 : 256;     // default shapes
    }
    const int bt = opt->batch_threads;
    if (bt != 0 && bt != 64 && bt != 128 && bt != 256 && bt != 512)
      bfail(HPRQP_ERR_ARG, "batch_threads must be 0, 64, 128, 256 or 512");
    if (bt != 0) {
      for (int c = 0; c < HB_NCLASS; ++c)
        if (HB_EPT * bt >= (256 << c)) b->class_bs[c] = bt;
    } else if (opt->spmv_autotune == 1) {
      autotune_batch(b, hi, cls_order, ncu);
    }
    // one kernel per block size in use, its instances largest first
    std::vector<int> korder;
    b->nkern = 0;
    for (int bs = 512; bs >= 64; bs /= 2) {
      std::vector<int> mine;
      for (int c = HB_NCLASS - 1; c >= 0; --c)
        if (b->class_bs[c] == bs) mine.insert(mine.end(), cls_order[c].begin(), cls_order[c].end());
      if (mine.empty()) continue;
      hprqp_batch::Kern& K = b->kern[b->nkern];
      K.bs = bs;
      K.first = (int)korder.size();
      K.cnt = (int)mine.size();
      K.grid = std::max(1, std::min(K.cnt, batch_resident(bs, b->rank_max, ncu)));
      HBC(hipMalloc(&K.hbuf, (size_t)K.grid * 5 * HB_EPT * bs * sizeof(double)));
      if (b->nkern > 0) {
        HBC(hipStreamCreateWithFlags(&K.st, hipStreamNonBlocking));
        HBC(hipEventCreateWithFlags(&K.ev_join, hipEventDisableTiming));
      }
      korder.insert(korder.end(), mine.begin(), mine.end());
      ++b->nkern;
    }
    if (b->nkern > 1) HBC(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    b->order_default = korder;
    HBC(hipMemcpyAsync(b->d_order, korder.data(), count * sizeof(int), hipMemcpyHostToDevice, st));
    HBC(hipStreamSynchronize(st));
    *out = b;
  } catch (...) {
    delete b;
    throw;
  }
}

void solve_batch_impl(hprqp_batch* b, const double* y0, const double* w0, const double* x0, double* y, double* z,
                      double* w, double* x, hprqp_info* infos) {
  if (!b || !z || !w || !x || (b->total_m > 0 && !y)) bfail(HPRQP_ERR_ARG, "NULL argument");
  if (b->own_st) HBC(hipDeviceSynchronize());
  k_zero_ints<<<1, 64, 0, b->st>>>(b->d_queue, HB_NCLASS);
  HBC(hipEventRecord(b->e0, b->st));
  k_stamp<<<1, 64, 0, b->st>>>(b->d_t0);
  // one launch per block size in use, kernels 1.. on their own streams
  if (b->nkern > 1) HBC(hipEventRecord(b->ev_fork, b->st));
  for (int k = 0; k < b->nkern; ++k) {
    const hprqp_batch::Kern& K = b->kern[k];
    hipStream_t s = k == 0 ? b->st : K.st;
    if (k > 0) HBC(hipStreamWaitEvent(s, b->ev_fork, 0));
    batch_launch(K.bs, b->rank_max, s, K.grid, b->d_insts, b->d_order + K.first, K.cnt, b->d_queue + k, b->o, y0, w0,
                 x0, y, z, w, x, b->d_infos, K.hbuf);
    if (k > 0) HBC(hipEventRecord(K.ev_join, s));
  }
  for (int k = 1; k < b->nkern; ++k) HBC(hipStreamWaitEvent(b->st, b->kern[k].ev_join, 0));
  HBC(hipEventRecord(b->e1, b->st));
  k_batch_qwx<<<std::min(b->count, 4096), HB_QWX_BS, 0, b->st>>>(b->d_insts, b->count, w, x, b->d_qwx);
  HBC(hipGetLastError());
  std::vector<BInfo> hi(b->count);
  std::vector<double> hq(b->count);
  HBC(hipMemcpyAsync(hi.data(), b->d_infos, b->count * sizeof(BInfo), hipMemcpyDeviceToHost, b->st));
  HBC(hipMemcpyAsync(hq.data(), b->d_qwx, b->count * sizeof(double), hipMemcpyDeviceToHost, b->st));
  HBC(hipStreamSynchronize(b->st));
  float ms = 0.f;
  HBC(hipEventElapsedTime(&ms, b->e0, b->e1));
  b->last_kernel_s = ms * 1e-3;
  if (infos)
    for (int i = 0; i < b->count; ++i) {
      hprqp_info& f = infos[i];
      std::memset(&f, 0, sizeof(f));
      f.term = hi[i].term; f.iters = hi[i].iters; f.restarts = hi[i].restarts;
      f.sigma = hi[i].sigma; f.sigma0 = hi[i].sigma0; f.lambda_A = hi[i].lamA; f.lambda_Q = hi[i].lamQ;
      f.eta_p = hi[i].eta_p; f.eta_d = hi[i].eta_d; f.eta_gap = hi[i].eta_gap;
      f.pobj = hi[i].pobj; f.dobj = hi[i].dobj; f.R_last = hi[i].R_last;
      f.qwx_gap = hq[i];
    }
}
}  // namespace

#define HB_GUARD(...)                 \
  try {                               \
    hq::g_err.clear();                \
    __VA_ARGS__;                      \
    return HPRQP_OK;                  \
  } catch (const BErr& e) {           \
    hq::g_err = e.msg;                \
    return e.st;                      \
  } catch (const std::exception& e) { \
    hq::g_err = e.what();             \
    return HPRQP_ERR_HIP;             \
  }

extern "C" {

hprqp_status hprqp_batch_create(int32_t count, const hprqp_problem* probs, const hprqp_options* opt,
                                hipStream_t stream, hprqp_batch** out) {
  HB_GUARD(batch_create_impl(count, probs, opt, stream, out));
}

hprqp_status hprqp_solve_batch(hprqp_batch* b, const double* y0, const double* w0, const double* x0, double* y,
                               double* z, double* w, double* x, hprqp_info* infos_host) {
  HB_GUARD(solve_batch_impl(b, y0, w0, x0, y, z, w, x, infos_host));
}


hprqp_status hprqp_batch_shapes(hprqp_batch* b, int32_t* class_count_host, int32_t* class_threads_host,
                                double* class_us_host) {
  HB_GUARD(if (!b) bfail(HPRQP_ERR_ARG, "NULL batch");
           for (int c = 0; c < HB_NCLASS; ++c) {
             if (class_count_host) class_count_host[c] = b->class_cnt[c];
             if (class_threads_host) class_threads_host[c] = b->class_bs[c];
             for (int lb = 0; lb < HB_NCLASS; ++lb)
               if (class_us_host) class_us_host[c * HB_NCLASS + lb] = b->class_us[c][lb];
           });
}

hprqp_status hprqp_batch_set_priority(hprqp_batch* b, const float* priority) {
  HB_GUARD(if (!b) bfail(HPRQP_ERR_ARG, "NULL batch");
           std::vector<int> ord = b->order_default;
           if (priority) {
             std::vector<float> pr(b->count);
             HBC(hipMemcpyAsync(pr.data(), priority, b->count * sizeof(float), hipMemcpyDeviceToHost, b->st));
             HBC(hipStreamSynchronize(b->st));
             for (float& v : pr)
               if (!std::isfinite(v)) v = -INFINITY;     // no usable prediction: last
             // each kernel's queue: highest priority first, ties in the default order
             for (int k = 0; k < b->nkern; ++k) {
               auto first = ord.begin() + b->kern[k].first;
               std::stable_sort(first, first + b->kern[k].cnt, [&](int a, int c) { return pr[a] > pr[c]; });
             }
           }
           HBC(hipMemcpyAsync(b->d_order, ord.data(), b->count * sizeof(int), hipMemcpyHostToDevice, b->st));
           HBC(hipStreamSynchronize(b->st)));
}

double hprqp_batch_last_kernel_s(hprqp_batch* b) { return b ? b->last_kernel_s : 0.0; }

void hprqp_batch_destroy(hprqp_batch* b) { delete b; }

}  // extern "C"
