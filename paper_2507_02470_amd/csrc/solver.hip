// solver.hip -- single-instance HPR-QP (Algorithm 4 + Algorithm 5, arXiv
// 2507.02470) on one MI355X: device kernels for every vector/matrix step,
// host C++ for the scalar decisions taken at checks (termination, restart
// criteria of Section 3.2, SigmaUpdate).
//
// Per iteration there are four global dependency points
//   Q xhat  ->  A v  ->  A^T ybar  ->  Q A^T(ybar - y)
// so an iteration is four launches (a3..a6); the z/x step of the next
// iteration is fused into the last one.  A "segment" is the run of
// `check_every` iterations that ends in a check; it can be captured once as
// a HIP graph and replayed, since sigma and the inner counter live in device
// memory.  The host reads back ~30 scalars per segment.
#include "hprqp.h"
#include "common.hpp"
#include "epilogues.hpp"
#include "epilogues_primal.hpp"
#include "qops.hpp"
#include "spmv.hpp"
#include "precond.hpp"
#include "panel.hpp"
#include "split.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

hipError_t hq_build_transpose(int m, int n, int64_t nnz, const int* rowptr, const int* col, const double* val,
                              int* t_rowptr, int* t_col, double* t_val, int* t_perm, hipStream_t st);

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
namespace hq {
thread_local std::string g_err;

struct Error {
  hprqp_status st;
  std::string msg;
};

[[noreturn]] void fail(hprqp_status st, const std::string& msg) { throw Error{st, msg}; }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) fail(HPRQP_ERR_OOM, std::string(what) + ": out of device memory");
    fail(HPRQP_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  }
}
#define HQC(x) ::hq::hip_check((x), #x)

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace hq

extern "C" const char* hprqp_last_error(void) { return hq::g_err.c_str(); }

// ---------------------------------------------------------------------------
// reduction slots (per-block partials -> final reduce -> host)
// ---------------------------------------------------------------------------
enum : int {
  SL_RF = 0,    // merit of the epoch's first iteration: 7 slots
  SL_RC = 7,    // merit at the check: 7 slots
  SL_TH = 14,   // theta~ of Algorithm 5: 5 slots
  SL_RA = 19,   // primal residual part: 4 slots
  SL_RQ = 23,   // dual residual part: 7 slots
  SL_ITER_END = 30,
  SL_POW = 30,  // power method: 2 slots
  SL_NRM = 32,  // norms of b and c: 4 slots
  SL_LR = 36,   // F^T x of the low-rank Q: 16 slots
  SL_QWX = 52,  // ||Q(w - x)||_inf at the returned point: 1 slot
  SL_TOTAL = 53
};
static constexpr unsigned long long kMaxMask =
    (1ull << (SL_RA + 0)) | (1ull << (SL_RA + 1)) | (1ull << (SL_RQ + 0)) | (1ull << (SL_RQ + 1)) |
    (1ull << (SL_RQ + 2)) | (1ull << (SL_NRM + 1)) | (1ull << (SL_NRM + 3)) | (1ull << SL_QWX);

#include "small.hpp"   // uses the reduction slots above


__global__ __launch_bounds__(256) void k_final_reduce(const double* __restrict__ partials, const int* __restrict__ counts,
                                                      int slot0, unsigned long long maxmask, double* __restrict__ out) {
  const int slot = slot0 + blockIdx.x;
  const int cnt = counts[slot];
  const bool mx = (maxmask >> slot) & 1ull;
  double v = 0.0;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const double p = partials[(size_t)slot * HQ_PCAP + i];
    v = mx ? fmax(v, p) : v + p;
  }
  v = mx ? wave_max(v) : wave_sum(v);
  __shared__ double sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = mx ? fmax(r, sh[w]) : r + sh[w];
    out[slot] = r;
  }
}

__global__ void k_zero_ints(int n, int* p) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}
__global__ void k_fill(long long n, double* p, double v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
// o = (a - b) f (f NULL: 1)
__global__ void k_diff(long long n, const double* __restrict__ a, const double* __restrict__ b,
                       const double* __restrict__ f, double* __restrict__ o) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    o[i] = f ? (a[i] - b[i]) * f[i] : a[i] - b[i];
}
__global__ void k_mul(long long n, const double* __restrict__ s, const double* __restrict__ f, double* __restrict__ o) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    o[i] = s[i] * f[i];
}

__global__ void k_recip(long long n, const double* __restrict__ s, double* __restrict__ o) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    o[i] = 1.0 / s[i];
}

__global__ void k_copy(long long n, const double* __restrict__ s, double* __restrict__ a, double* __restrict__ b) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double v = s[i];
    a[i] = v;
    if (b) b[i] = v;
  }
}
// power method: reduce slots (<v,w>, |w|^2) into the history and the next scale
__global__ __launch_bounds__(256) void k_pow_final(const double* __restrict__ partials, const int* __restrict__ counts,
                                                   double* __restrict__ hist, int it, double* __restrict__ scale) {
  __shared__ double sh[2][4];
  for (int s = 0; s < 2; ++s) {
    const int slot = SL_POW + s, cnt = counts[slot];
    double v = 0.0;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) v += partials[(size_t)slot * HQ_PCAP + i];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[s][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double lam = sh[0][0], nw2 = sh[1][0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) { lam += sh[0][w]; nw2 += sh[1][w]; }
    hist[2 * it] = lam;
    hist[2 * it + 1] = nw2;
    *scale = nw2 > 0.0 ? 1.0 / sqrt(nw2) : 0.0;
  }
}
__global__ void k_scale(long long n, const double* __restrict__ in, const double* __restrict__ s, double* __restrict__ out) {
  const double f = *s;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = in[i] * f;
}

struct EpiSumSq {
  const double* v;
  static constexpr int NR = 1;
  static constexpr unsigned MAXMASK = 0u;
  __device__ void setup(const DevParams*, int) {}
  __device__ __forceinline__ void operator()(int i, double, double* acc) const { acc[0] += v[i] * v[i]; }
};
// ||b||^2, ||c||^2, ||b||_inf, ||c||_inf with b_i = max(|l_i|, |u_i|), infinities read as 0 (Section 4.1)
struct EpiNormB {
  const double *l, *u;
  static constexpr int NR = 2;
  static constexpr unsigned MAXMASK = 0x2u;
  __device__ void setup(const DevParams*, int) {}
  __device__ __forceinline__ void operator()(int i, double, double* acc) const {
    const double a = isinf(l[i]) ? 0.0 : fabs(l[i]), b = isinf(u[i]) ? 0.0 : fabs(u[i]);
    const double bi = fmax(a, b);
    acc[0] += bi * bi;
    acc[1] = fmax(acc[1], bi);
  }
};
struct EpiNormC {
  const double* c;
  static constexpr int NR = 2;
  static constexpr unsigned MAXMASK = 0x2u;
  __device__ void setup(const DevParams*, int) {}
  __device__ __forceinline__ void operator()(int i, double, double* acc) const {
    acc[0] += c[i] * c[i];
    acc[1] = fmax(acc[1], fabs(c[i]));
  }
};

// input validation (create): bit 0 -> bounds / non-finite data, bit 1 -> CSR structure
__global__ void k_validate_vec(int n, const double* lo, const double* hi, const double* c, int* flags) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double a = lo[i], b = hi[i];
    bool bad = !(a <= b) || a == INFINITY || b == -INFINITY;
    if (c && !isfinite(c[i])) bad = true;
    if (bad) atomicOr(flags, 1);
  }
}
__global__ void k_validate_finite(long long n, const double* v, int* flags) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    if (!isfinite(v[i])) atomicOr(flags, 1);
}
__global__ void k_max_row_len(int rows, const int* rp, int* out) {
  int mx = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += gridDim.x * blockDim.x) mx = max(mx, rp[i + 1] - rp[i]);
  atomicMax(out, mx);
}
__global__ void k_validate_csr(int rows, int cols, long long nnz, const int* rp, const int* ci, const double* v,
                               int* flags) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += gridDim.x * blockDim.x) {
    const int b = rp[i], e = rp[i + 1];
    // never read columns outside [0, nnz), whatever rowptr holds
    if ((i == 0 && b != 0) || b < 0 || e < b || (long long)e > nnz || (i == rows - 1 && e != nnz)) {
      atomicOr(flags, 2);
      continue;
    }
    for (int k = b; k < e; ++k) {
      if (ci[k] < 0 || ci[k] >= cols) atomicOr(flags, 2);
      if (!isfinite(v[k])) atomicOr(flags, 1);
    }
  }
}

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct Mat {
  int rows = 0, cols = 0;
  const int* rp = nullptr;
  const int* ci = nullptr;
  const double* v = nullptr;
  long long nnz = 0;
  int G = 4;
  int maxlen = -1;    // longest row (-1: not measured)
  PanelMat pm;        // panel-ordered copy (pm.pp == nullptr: not built)
  int G_np = 0;       // kernel used in place of the panel-ordered one under a heavy epilogue
  SplitMat sm;        // column-split copy (sm.off == nullptr: not built)
};

#define HQ_PROF_ITERS 64

struct hprqp_handle {
  int dev = 0;
  int ncu = 256;     // compute units of the device
  hipStream_t st = nullptr;
  int n = 0, m = 0, qkind = 0;
  Mat A, AT, Q;
  int kp = 0, ks = 0;
  const double *kB = nullptr, *kC = nullptr;
  const double *kS = nullptr, *kT = nullptr;   // QAP relaxation: Q = B (x) C - I (x) S - T (x) I
  int small_G = 0;            // > 0: segments run as one workgroup (k_small_segment<small_G>)
  bool small_forced = false;  // small_path = 1: also when the data does not fit the LDS
  int kron_mode = 0;          // 0: k_dgemm16 (K split over waves), 1: LDS-tiled k_dgemm_tile
  int kron_groups = 1;        // split-K groups of the tiled kernel
  int kron_groups_max = 1;    // capacity of kparts (in n-vectors)
  double* kparts = nullptr;
  int lr_r = 0;
  const double *lr_d = nullptr, *lr_F = nullptr;
  Mat G, GT;                 // Q = Ahat^T Ahat: Ahat (p x n) and its stored transpose
  double* gtmp = nullptr;    // Ahat x (p)
  double l1 = 0.0;           // lambda of phi(x) = lambda ||x||_1 + delta_[L,U](x)
  const double *c = nullptr, *L = nullptr, *U = nullptr, *l = nullptr, *u = nullptr;
  // diagonal preconditioning (Section 4.1): the method runs on the scaled data
  // above; A0, AT0, Q0 and c0..u0 are the problem as given
  bool pre = false;
  double *Ds = nullptr, *Es = nullptr, *iDs = nullptr, *iEs = nullptr;
  Mat A0, AT0, Q0;
  const double *c0 = nullptr, *L0 = nullptr, *U0 = nullptr, *l0 = nullptr, *u0 = nullptr;
  int* at_perm = nullptr;
  hprqp_options opt{};
  double lamA = 0, lamQ = 0, sigma0 = 1, binf = 0, cinf = 0;
  double sigma0_primal = 1;  // sigma0 of HPR on the primal reformulations (methods 1, 2)
  double powA_est = 0, powQ_est = 0;
  int powA_it = 0, powQ_it = 0;
  double t_setup = 0, t_precond = 0;
  // owned device memory
  std::vector<void*> owned;
  int *at_rp = nullptr, *at_ci = nullptr;
  double* at_v = nullptr;
  double *y = nullptr, *ya = nullptr, *ybar = nullptr, *tm = nullptr;
  double *w = nullptr, *wa = nullptr, *x = nullptr, *xa = nullptr, *ATy = nullptr, *ATya = nullptr, *Qw = nullptr,
         *Qwa = nullptr, *xh = nullptr, *v = nullptr, *q1 = nullptr, *d = nullptr, *g = nullptr, *e = nullptr,
         *XB = nullptr, *ZB = nullptr, *wbar = nullptr, *qwbar = nullptr, *xbo = nullptr, *zbo = nullptr,
         *t1 = nullptr, *t2 = nullptr, *kronT = nullptr;
  // HPR on the primal reformulations: e = 2 ybar - y, A x and dy at merit
  // iterations (m each); t, its anchor and bar, dt (n each)
  double *pe = nullptr, *pax = nullptr, *pdy = nullptr, *pt = nullptr, *pta = nullptr, *ptb = nullptr,
         *pdt = nullptr;
  double *partials = nullptr, *scalars = nullptr, *hist = nullptr;
  int* counts = nullptr;
  int* dflags = nullptr;
  DevParams* dprm = nullptr;
  // pinned host
  double* hs = nullptr;      // scalars
  DevParams* hp = nullptr;   // params
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_T = 0;
  hipGraphExec_t pgexec = nullptr;   // segment graph of the primal methods
  hipGraph_t pgraph = nullptr;
  int pgraph_T = 0, pgraph_method = 0;
  // kernel timing (profile_kernels): events around the four products of the
  // plain iterations 1..HQ_PROF_ITERS of a timed segment, accumulated over the
  // solve (the first and the check iteration carry extra reductions)
  hipEvent_t pev[HQ_PROF_ITERS][4][2] = {};
  double prof_ms[4] = {0, 0, 0, 0};
  long long prof_n[4] = {0, 0, 0, 0};
  hipStream_t own_st = nullptr;

  template <class T>
  T* dalloc(size_t count) {
    void* p = nullptr;
    HQC(hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)));
    owned.push_back(p);
    return (T*)p;
  }
  ~hprqp_handle() {
    if (gexec) hipGraphExecDestroy(gexec);
    if (graph) hipGraphDestroy(graph);
    if (pgexec) hipGraphExecDestroy(pgexec);
    if (pgraph) hipGraphDestroy(pgraph);
    for (void* p : owned) hipFree(p);
    if (hs) hipHostFree(hs);
    if (hp) hipHostFree(hp);
    if (own_st) hipStreamDestroy(own_st);
    for (auto& a : pev)
      for (auto& b : a)
        for (auto& e : b)
          if (e) hipEventDestroy(e);
  }
};

namespace hq {

inline RedOut no_red(hprqp_handle& h) {
  RedOut r;
  r.partials = h.partials;
  r.counts = h.counts;
  for (int s = 0; s < 16; ++s) r.slot[s] = -1;
  r.active = 0;
  return r;
}
inline RedOut red_seq(hprqp_handle& h, int slot0, int nr) {
  RedOut r = no_red(h);
  for (int s = 0; s < nr; ++s) r.slot[s] = (int8_t)(slot0 + s);
  r.active = 1;
  return r;
}

// A reducing launch stores one partial per workgroup into each of its slots,
// which hold HQ_PCAP partials: every launcher checks its grid against that
// (a larger grid would spill into the next slot).
inline void check_red_grid(long long grid, const RedOut& red) {
  if (red.active && grid > HQ_PCAP)
    fail(HPRQP_ERR_UNSUPPORTED, "reducing launch of " + std::to_string(grid) + " workgroups exceeds the " +
                                    std::to_string(HQ_PCAP) + " partials of a reduction slot");
}

// Lanes-per-row code of the stream kernel that gathers from an LDS copy of the
// input vector (matrices with at most HQ_XLDS_MAX columns).
#define HQ_G_XLDS (-1)
// Lanes-per-row code of the panel-ordered product (Mat::pm built).
#define HQ_G_PANEL (-3)
// Lanes-per-row codes HQ_G_XROW - g: the row-split kernel with g <= 64 lanes
// per row gathering from an LDS copy of the vector (k_csr_xrow).
#define HQ_G_XROW (-100)
inline bool is_xrow(int G) { return G < HQ_G_XROW; }
// Lanes-per-row code of the column-split product (Mat::sm built).
#define HQ_G_SPLIT (-4)

template <class Epi>
void launch_split(hprqp_handle& h, const Mat& M, const double* x, const Epi& epi, int j, const RedOut& red) {
  const SplitMat& S = M.sm;
  const size_t lds = (size_t)S.pw * sizeof(double);
  if (S.pw == HQ_SPLIT_PW) {
    k_split_partial<HQ_BLOCK><<<S.np * S.nrb, HQ_BLOCK, lds, h.st>>>(S, x);
  } else {
    static bool attr_set = false;   // dynamic LDS above 64 KB must be enabled
    if (!attr_set) {
      HQC(hipFuncSetAttribute((const void*)k_split_partial<1024>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(HQ_SPLIT_PW_WIDE * sizeof(double))));
      attr_set = true;
    }
    k_split_partial<1024><<<S.np * S.nrb, 1024, lds, h.st>>>(S, x);
  }
  const int rgrid = std::min((S.rows + HQ_SPLIT_RED_ROWS - 1) / HQ_SPLIT_RED_ROWS, HQ_PCAP);
  check_red_grid(rgrid, red);
  k_split_reduce<Epi><<<rgrid, 4 * HQ_SPLIT_RED_ROWS, 0, h.st>>>(S.rows, S.np, S.partial, epi, h.dprm, j, red);
}

template <int G, class Epi>
void launch_xrow_g(hprqp_handle& h, const Mat& M, const double* x, const Epi& epi, int j, const RedOut& red) {
  constexpr int BS = HQ_XLDS_BLOCK;
  static bool attr_set = false;   // one per instantiation: dynamic LDS above 64 KB must be enabled
  if (!attr_set) {
    HQC(hipFuncSetAttribute((const void*)k_csr_xrow<G, Epi>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(HQ_XLDS_MAX * sizeof(double))));
    attr_set = true;
  }
  const size_t lds = (size_t)M.cols * sizeof(double);
  // persistent grid: as many blocks as fit on the CUs at this LDS size
  const size_t per_block = lds + 16 * 16 * sizeof(double) + 2048;
  const int per_cu = std::max(1, (int)((160 * 1024) / per_block));
  const long long groups = ((long long)M.rows + BS / G - 1) / (BS / G);
  const int grid = (int)std::max(1ll, std::min(groups, (long long)std::min(h.ncu * per_cu, HQ_GRID_CAP)));
  check_red_grid(grid, red);
  k_csr_xrow<G, Epi><<<grid, BS, lds, h.st>>>(M.rows, M.rp, M.ci, M.v, x, epi, h.dprm, j, red, M.cols);
}

template <class Epi>
void launch_csr_xrow(hprqp_handle& h, const Mat& M, const double* x, const Epi& epi, int j, const RedOut& red) {
  if (M.cols > HQ_XLDS_MAX) fail(HPRQP_ERR_UNSUPPORTED, "LDS-gather kernel: vector too long");
  switch (HQ_G_XROW - M.G) {
    case 1: launch_xrow_g<1>(h, M, x, epi, j, red); break;
    case 2: launch_xrow_g<2>(h, M, x, epi, j, red); break;
    case 4: launch_xrow_g<4>(h, M, x, epi, j, red); break;
    case 8: launch_xrow_g<8>(h, M, x, epi, j, red); break;
    case 16: launch_xrow_g<16>(h, M, x, epi, j, red); break;
    case 32: launch_xrow_g<32>(h, M, x, epi, j, red); break;
    default: launch_xrow_g<64>(h, M, x, epi, j, red); break;
  }
}

template <class Epi>
void launch_csr_xlds(hprqp_handle& h, const Mat& M, const double* x, const Epi& epi, int j, const RedOut& red) {
  constexpr int BS = HQ_XLDS_BLOCK;
  const size_t lds = (size_t)M.cols * sizeof(double);
  static bool attr_set = false;   // one per epilogue type: dynamic LDS above 64 KB must be enabled
  if (!attr_set) {
    HQC(hipFuncSetAttribute((const void*)k_csr_stream<Epi, true, BS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(HQ_XLDS_MAX * sizeof(double))));
    attr_set = true;
  }
  // persistent grid of 1024-thread blocks: as many as fit on the CUs at this LDS size
  const size_t per_block = lds + 2 * HQ_STREAM_CHUNK * sizeof(double) + (BS + 1) * sizeof(int) + 2048;
  const int per_cu = std::max(1, (int)((160 * 1024) / per_block));
  const int nblk = (M.rows + BS - 1) / BS;
  const int grid = std::max(1, std::min(nblk, std::min(h.ncu * per_cu, HQ_GRID_CAP)));
  check_red_grid(grid, red);
  k_csr_stream<Epi, true, BS><<<grid, BS, lds, h.st>>>(M.rows, M.rp, M.ci, M.v, x, epi, h.dprm, j, red, M.cols);
}

template <class Epi>
void launch_csr(hprqp_handle& h, const Mat& M, const double* x, const Epi& epi, int j, const RedOut& red) {
  if (M.G == HQ_G_XLDS) { launch_csr_xlds(h, M, x, epi, j, red); return; }
  if (is_xrow(M.G)) { launch_csr_xrow(h, M, x, epi, j, red); return; }
  if (M.G == HQ_G_SPLIT) { launch_split(h, M, x, epi, j, red); return; }
  if (M.G == HQ_G_PANEL) {
    // row blocks per workgroup: the fewest for which the whole grid is
    // resident, by the occupancy of the instantiation that would run (the
    // four differ in registers, so one count does not hold for the others)
    static int per_cu[5] = {0, 0, 0, 0, 0};   // resident workgroups per CU, by row blocks per workgroup
    if (!per_cu[1]) {
      const void* ks[5] = {nullptr, (const void*)k_csr_panel<Epi, 1>, (const void*)k_csr_panel<Epi, 2>,
                           (const void*)k_csr_panel<Epi, 3>, (const void*)k_csr_panel<Epi, 4>};
      for (int b = 1; b <= 4; ++b) {
        HQC(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[b], ks[b], HQ_BLOCK, 0));
        per_cu[b] = std::max(per_cu[b], 1);
      }
    }
    const PanelShape sh = panel_launch_shape(M.rows, h.ncu, per_cu, panel_prefetch<Epi>::value ? 4 : 1);
    check_red_grid(sh.grid, red);
    switch (sh.bpb) {
      case 1: k_csr_panel<Epi, 1><<<sh.grid, HQ_BLOCK, 0, h.st>>>(M.pm, x, epi, h.dprm, j, red); break;
      case 2: k_csr_panel<Epi, 2><<<sh.grid, HQ_BLOCK, 0, h.st>>>(M.pm, x, epi, h.dprm, j, red); break;
      case 3: k_csr_panel<Epi, 3><<<sh.grid, HQ_BLOCK, 0, h.st>>>(M.pm, x, epi, h.dprm, j, red); break;
      default:
        if ((long long)sh.grid * 4 >= (M.rows + HQ_BLOCK - 1) / HQ_BLOCK)
          k_csr_panel<Epi, 4><<<sh.grid, HQ_BLOCK, 0, h.st>>>(M.pm, x, epi, h.dprm, j, red);
        else   // more row blocks than 4 per resident workgroup: grid-stride groups
          k_csr_panel<Epi, 4, true><<<sh.grid, HQ_BLOCK, 0, h.st>>>(M.pm, x, epi, h.dprm, j, red);
        break;
    }
    return;
  }
  // stream kernel: HQ_BLOCK rows per block; row-split kernel: HQ_BLOCK / G rows per block
  const int grid = M.G == 0 ? hq_grid(M.rows, HQ_BLOCK) : hq_grid(M.rows, HQ_BLOCK / M.G);
  check_red_grid(grid, red);
  hipStream_t st = h.st;
  switch (M.G) {
    case 0: k_csr_stream<Epi><<<grid, HQ_BLOCK, 0, st>>>(M.rows, M.rp, M.ci, M.v, x, epi, h.dprm, j, red); break;
    case 1: k_csr<1, Epi><<<grid, HQ_BLOCK, 0, st>>>(M.rows, M.rp, M.ci, M.v, x, epi, h.dprm, j, red); break;
    case 2: k_csr<2, Epi><<<grid, HQ_BLOCK, 0, st>>>(M.rows, M.rp, M.ci, M.v, x, epi, h.dprm, j, red); break;
    case 4: k_csr<4, Epi><<<grid, HQ_BLOCK, 0, st>>>(M.rows, M.rp, M.ci, M.v, x, epi, h.dprm, j, red); break;
    case 8: k_csr<8, Epi><<<grid, HQ_BLOCK, 0, st>>>(M.rows, M.rp, M.ci, M.v, x, epi, h.dprm, j, red); break;
    case 16: k_csr<16, Epi><<<grid, HQ_BLOCK, 0, st>>>(M.rows, M.rp, M.ci, M.v, x, epi, h.dprm, j, red); break;
    case 32: k_csr<32, Epi><<<grid, HQ_BLOCK, 0, st>>>(M.rows, M.rp, M.ci, M.v, x, epi, h.dprm, j, red); break;
    case 64: k_csr<64, Epi><<<grid, HQ_BLOCK, 0, st>>>(M.rows, M.rp, M.ci, M.v, x, epi, h.dprm, j, red); break;
    case 128: k_csr<128, Epi><<<grid, HQ_BLOCK, 0, st>>>(M.rows, M.rp, M.ci, M.v, x, epi, h.dprm, j, red); break;
    default: k_csr<256, Epi><<<grid, HQ_BLOCK, 0, st>>>(M.rows, M.rp, M.ci, M.v, x, epi, h.dprm, j, red); break;
  }
}

template <class Epi>
void launch_elem(hprqp_handle& h, int n, const double* q, const Epi& epi, int j, const RedOut& red) {
  check_red_grid(hq_grid(n, HQ_BLOCK), red);
  k_elem<Epi><<<hq_grid(n, HQ_BLOCK), HQ_BLOCK, 0, h.st>>>(n, q, epi, h.dprm, j, red);
}

void final_reduce(hprqp_handle& h, int slot0, int nslot) {
  k_final_reduce<<<nslot, 256, 0, h.st>>>(h.partials, h.counts, slot0, kMaxMask, h.scalars);
}

// one term list through the tiled GEMM, split-K when h.kron_groups > 1
template <class Epi>
void launch_tile(hprqp_handle& h, int M, int N, const GemmOps& ops, const Epi& epi, int j, const RedOut& red) {
  const int tiles = ((M + HQ_TB - 1) / HQ_TB) * ((N + HQ_TB - 1) / HQ_TB);
  const int G = h.kron_groups;
  if (G <= 1) {
    check_red_grid(std::min(tiles, HQ_GRID_CAP), red);
    k_dgemm_tile<Epi, false><<<std::min(tiles, HQ_GRID_CAP), 256, 0, h.st>>>(M, N, ops, M, epi, h.dprm, j, red, 1,
                                                                          nullptr);
  } else {
    k_dgemm_tile<Epi, true><<<std::min(tiles * G, HQ_GRID_CAP), 256, 0, h.st>>>(M, N, ops, M, epi, h.dprm, j,
                                                                             no_red(h), G, h.kparts);
    const long long cnt = (long long)M * N;
    check_red_grid(hq_grid(cnt, HQ_BLOCK), red);
    k_gemm_sum<Epi><<<hq_grid(cnt, HQ_BLOCK), HQ_BLOCK, 0, h.st>>>(cnt, G, h.kparts, epi, h.dprm, j, red);
  }
}

// Kronecker / QAP-relaxation Q through the tiled GEMM: T1 = C X, then
// Y = T1 B^T (- X T^T - S X) with the epilogue
template <class Epi>
void kron_tiled(hprqp_handle& h, const double* x, const Epi& epi, int j, const RedOut& red) {
  const int s = h.ks, p = h.kp;
  GemmOps g1{};
  g1.nt = 1;
  g1.A[0] = h.kC; g1.lda[0] = s; g1.B[0] = x; g1.ldb[0] = s; g1.K[0] = s; g1.transb[0] = 0; g1.sign[0] = 1.0;
  launch_tile(h, s, p, g1, EpiStore{h.kronT}, j, no_red(h));
  GemmOps g2{};
  g2.nt = 1;
  g2.A[0] = h.kronT; g2.lda[0] = s; g2.B[0] = h.kB; g2.ldb[0] = p; g2.K[0] = p; g2.transb[0] = 1; g2.sign[0] = 1.0;
  if (h.kT) {
    const int t = g2.nt++;
    g2.A[t] = x; g2.lda[t] = s; g2.B[t] = h.kT; g2.ldb[t] = p; g2.K[t] = p; g2.transb[t] = 1; g2.sign[t] = -1.0;
  }
  if (h.kS) {
    const int t = g2.nt++;
    g2.A[t] = h.kS; g2.lda[t] = s; g2.B[t] = x; g2.ldb[t] = s; g2.K[t] = s; g2.transb[t] = 0; g2.sign[t] = -1.0;
  }
  launch_tile(h, s, p, g2, epi, j, red);
}

// out-of-place Q product with a fused epilogue: epi(i, (Q x)_i).  heavy: the
// epilogue streams many vectors; the panel-ordered product, whose epilogues all
// run at the end of the launch, then gives way to the best other kernel
template <class Epi>
void q_apply(hprqp_handle& h, const double* x, const Epi& epi, int j, const RedOut& red, bool heavy = false) {
  switch (h.qkind) {
    case HPRQP_Q_ZERO:
      launch_elem(h, h.n, nullptr, epi, j, red);
      break;
    case HPRQP_Q_CSR:
      if (heavy && h.Q.G == HQ_G_PANEL) {
        Mat M = h.Q;
        M.G = h.Q.G_np;
        launch_csr(h, M, x, epi, j, red);
      } else {
        launch_csr(h, h.Q, x, epi, j, red);
      }
      break;
    case HPRQP_Q_KRON: {
      // Q vec(X) = vec(C X B^T): T = C X, then Y = T B^T with the epilogue
      const int s = h.ks, p = h.kp;
      if (h.kron_mode == 1) {
        kron_tiled(h, x, epi, j, red);
        break;
      }
      const int tiles = ((s + 15) / 16) * ((p + 15) / 16);
      const int grid = std::min(tiles, HQ_GRID_CAP);
      check_red_grid(grid, red);
      k_dgemm16<false, EpiStore><<<grid, 64 * HQ_KSPLIT, 0, h.st>>>(s, p, s, h.kC, s, x, s, s, EpiStore{h.kronT},
                                                                    h.dprm, j, no_red(h));
      if (!h.kS && !h.kT) {
        k_dgemm16<true, Epi><<<grid, 64 * HQ_KSPLIT, 0, h.st>>>(s, p, p, h.kronT, s, h.kB, p, s, epi, h.dprm, j, red);
      } else {
        // QAP relaxation: Y = T1 B^T - X T^T - S X in one accumulation
        GemmTerms ex{};
        if (h.kT) {
          const int t = ex.nt++;
          ex.A[t] = x; ex.lda[t] = s; ex.B[t] = h.kT; ex.ldb[t] = p; ex.K[t] = p; ex.transb[t] = 1; ex.sign[t] = -1.0;
        }
        if (h.kS) {
          const int t = ex.nt++;
          ex.A[t] = h.kS; ex.lda[t] = s; ex.B[t] = x; ex.ldb[t] = s; ex.K[t] = s; ex.transb[t] = 0; ex.sign[t] = -1.0;
        }
        k_dgemm16<true, Epi, true><<<grid, 64 * HQ_KSPLIT, 0, h.st>>>(s, p, p, h.kronT, s, h.kB, p, s, epi, h.dprm,
                                                                      j, red, ex);
      }
      break;
    }
    case HPRQP_Q_GRAM:
      // Q x = Ahat^T (Ahat x): a plain product into gtmp, then the epilogue product
      launch_csr(h, h.G, x, EpiStore{h.gtmp}, j, no_red(h));
      launch_csr(h, h.GT, h.gtmp, epi, j, red);
      break;
    case HPRQP_Q_LOWRANK: {
      const int grid = hq_grid(h.n, HQ_BLOCK);
      RedOut lr = no_red(h);
      for (int k = 0; k < h.lr_r; ++k) lr.slot[k] = (int8_t)(SL_LR + k);
      lr.active = 1;
      check_red_grid(grid, lr);
      check_red_grid(grid, red);
      k_lr_partial<<<grid, HQ_BLOCK, 0, h.st>>>(h.n, h.lr_r, h.lr_F, x, lr);
      final_reduce(h, SL_LR, h.lr_r);
      k_lr_apply<Epi><<<grid, HQ_BLOCK, 0, h.st>>>(h.n, h.lr_r, h.lr_d, h.lr_F, x, h.scalars + SL_LR, epi, h.dprm, j,
                                                   red);
      break;
    }
    default:
      fail(HPRQP_ERR_UNSUPPORTED, "unknown qkind");
  }
}

// ||Q(w - x)||_inf of the problem as given, for (w, x) in the variables the
// method runs on (the scaled ones when preconditioned: Q D (w~ - x~) =
// D^-1 Q~ (w~ - x~)).  At a solution the shadow w_Q and x differ by an
// element of ker Q (Proposition 2.4), so this is 0 up to rounding there.
double qwx_norm(hprqp_handle& h, const double* wv, const double* xv) {
  k_diff<<<hq_grid(h.n, 256), 256, 0, h.st>>>(h.n, wv, xv, nullptr, h.t1);
  q_apply(h, h.t1, EpiMaxAbs{h.pre ? h.iDs : nullptr}, 0, red_seq(h, SL_QWX, 1));
  final_reduce(h, SL_QWX, 1);
  HQC(hipMemcpyAsync(h.hs + SL_QWX, h.scalars + SL_QWX, sizeof(double), hipMemcpyDeviceToHost, h.st));
  HQC(hipStreamSynchronize(h.st));
  return h.hs[SL_QWX];
}

void write_params(hprqp_handle& h, double sigma, long long t0) {
  h.hp->sigma = sigma;
  h.hp->lamA = h.lamA;
  h.hp->lamQ = h.lamQ;
  h.hp->t0 = t0;
  HQC(hipMemcpyAsync(h.dprm, h.hp, sizeof(DevParams), hipMemcpyHostToDevice, h.st));
}

// One iteration (index j of a segment of Tseg iterations; the last one is a check).
void enqueue_iter(hprqp_handle& h, int j, int Tseg, bool trace, bool prof) {
  const bool check = (j == Tseg - 1);
  const int rgroup = check ? SL_RC : (j == 0 ? SL_RF : -1);
  const bool want_r = rgroup >= 0;
  const bool xb_next = trace || (j >= Tseg - 2);
  int ps = -1;  // timing sample index of this iteration
  if (prof && !trace && j >= 1 && j <= HQ_PROF_ITERS && j < Tseg - 1) ps = j - 1;
  auto mark = [&](int kind, int edge) {
    if (ps >= 0) HQC(hipEventRecord(h.pev[ps][kind][edge], h.st));
  };
  // a3: q1 = Q xhat, v
  mark(0, 0);
  q_apply(h, h.xh, EpiQ1{h.xh, h.Qw, h.v, h.q1, 0.0}, j, no_red(h));
  mark(0, 1);
  if (h.m > 0) {
    // a4: A v, ybar, y+
    RedOut r4 = no_red(h);
    if (want_r) r4.slot[0] = (int8_t)rgroup;
    if (check) r4.slot[1] = (int8_t)SL_TH;
    r4.active = want_r || check;
    mark(1, 0);
    launch_csr(h, h.A, h.v, EpiY{h.l, h.u, h.ya, h.y, h.ybar, want_r, check, 0.0, 0.0}, j, r4);
    mark(1, 1);
    // a5: A^T ybar, d, A^T y+
    mark(2, 0);
    launch_csr(h, h.AT, h.ybar, EpiAT{h.ATy, h.ATya, h.d, h.g, h.e, check, 0.0}, j, no_red(h));
    mark(2, 1);
  }
  if (check) {
    // stopping quantities at ubar = (ybar, zbar, xbar) (Section 4.1)
    if (h.m > 0) launch_csr(h, h.A, h.XB, EpiResA{h.l, h.u, h.ybar, h.iEs}, j, red_seq(h, SL_RA, 4));
    q_apply(h, h.XB, EpiResQ{h.XB, h.ZB, h.m > 0 ? h.g : nullptr, h.c, h.L, h.U, h.xbo, h.zbo, h.iDs, h.l1}, j,
            red_seq(h, SL_RQ, 7));
  }
  // a6: Q d, wbar, Halpern, next z/x step
  EpiQ2 e6;
  e6.xh = h.xh; e6.w = h.w; e6.Qw = h.Qw; e6.XB = h.XB; e6.ZB = h.ZB;
  e6.q1 = h.q1; e6.d = h.d; e6.wa = h.wa; e6.Qwa = h.Qwa; e6.xa = h.xa; e6.ATy = h.ATy;
  e6.c = h.c; e6.L = h.L; e6.U = h.U; e6.e = h.e;
  e6.wbar = h.wbar; e6.qwbar = h.qwbar; e6.x = h.x; e6.xbar_out = h.xbo;
  e6.want_r = want_r; e6.check = check; e6.xb_next = xb_next; e6.trace = trace;
  e6.l1 = h.l1;
  RedOut r6 = no_red(h);
  if (want_r)
    for (int s = 0; s < 6; ++s) r6.slot[s] = (int8_t)(rgroup + 1 + s);
  if (check)
    for (int s = 0; s < 3; ++s) r6.slot[6 + s] = (int8_t)(SL_TH + 1 + s);
  r6.active = want_r || check;
  mark(3, 0);
  if (h.m > 0) q_apply(h, h.d, e6, j, r6, true);
  else launch_elem(h, h.n, nullptr, e6, j, r6);  // Q A^T(ybar - y) = 0 without constraints
  mark(3, 1);
  if (check && h.m > 0 && h.qkind != HPRQP_Q_ZERO)
    q_apply(h, h.e, EpiTheta3{h.e}, j, red_seq(h, SL_TH + 4, 1));
}

// the whole segment in one workgroup (small explicit-Q problems)
SmallArgs small_args(hprqp_handle& h) {
  SmallArgs a{};
  a.A = SmallMat{h.m, h.A.rp, h.A.ci, h.A.v};
  a.AT = SmallMat{h.n, h.AT.rp, h.AT.ci, h.AT.v};
  a.Q = h.qkind == HPRQP_Q_CSR ? SmallMat{h.n, h.Q.rp, h.Q.ci, h.Q.v} : SmallMat{h.n, nullptr, nullptr, nullptr};
  if (h.m == 0) { a.A = SmallMat{0, nullptr, nullptr, nullptr}; a.AT = SmallMat{h.n, nullptr, nullptr, nullptr}; }
  a.n = h.n; a.m = h.m;
  const int n = h.n, m = h.m;
  auto set = [&](int s, const double* p, int len) { a.vec[s] = const_cast<double*>(p); a.vlen[s] = p ? len : 0; };
  set(SV_L, h.l, m); set(SV_U, h.u, m); set(SV_C, h.c, n); set(SV_LB, h.L, n); set(SV_UB, h.U, n);
  set(SV_IE, h.iEs, m); set(SV_ID, h.iDs, n);
  set(SV_YA, h.ya, m); set(SV_WA, h.wa, n); set(SV_XA, h.xa, n); set(SV_ATYA, h.ATya, n); set(SV_QWA, h.Qwa, n);
  set(SV_Y, h.y, m); set(SV_YBAR, h.ybar, m); set(SV_W, h.w, n); set(SV_X, h.x, n); set(SV_ATY, h.ATy, n);
  set(SV_QW, h.Qw, n); set(SV_XH, h.xh, n); set(SV_V, h.v, n); set(SV_Q1, h.q1, n); set(SV_D, h.d, n);
  set(SV_G, h.g, n); set(SV_E, h.e, n); set(SV_XB, h.XB, n); set(SV_ZB, h.ZB, n); set(SV_WBAR, h.wbar, n);
  set(SV_QWBAR, h.qwbar, n); set(SV_XBO, h.xbo, n); set(SV_ZBO, h.zbo, n);
  if (h.opt.method != 0) {   // the primal methods' own vectors
    set(SV_PTA, h.pta, n); set(SV_PT, h.pt, n); set(SV_PTB, h.ptb, n); set(SV_PDT, h.pdt, n);
    set(SV_PE, h.pe, m); set(SV_PAX, h.pax, m); set(SV_PDY, h.pdy, m);
  }
  a.l1 = h.l1;
  a.partials = h.partials; a.counts = h.counts; a.prm = h.dprm;
  // LDS layout: every vector, then row pointers, columns and values of A, A^T, Q
  long long off = 0;
  auto take = [&](long long bytes) { const long long o = off; off += (bytes + 15) / 16 * 16; return (int)o; };
  for (int s = 0; s < SV_COUNT; ++s) a.voff[s] = a.vec[s] ? take(8ll * a.vlen[s]) : 0;
  const Mat* ms[3] = {&h.A, &h.AT, &h.Q};
  const SmallMat sm[3] = {a.A, a.AT, a.Q};
  for (int q = 0; q < 3; ++q) {
    if (!sm[q].rp) { a.moff[q][0] = a.moff[q][1] = a.moff[q][2] = 0; continue; }
    a.moff[q][0] = take(4ll * (sm[q].rows + 1));
    a.moff[q][1] = take(4ll * ms[q]->nnz);
    a.moff[q][2] = take(8ll * ms[q]->nnz);
  }
  a.lds_bytes = off <= HQ_SMALL_LDS ? (int)off : 0;
  return a;
}

template <int G>
void launch_small(hprqp_handle& h, const SmallArgs& a, int Tseg) {
  const int meth = h.opt.method;
  if (meth == 0) {
    if (a.lds_bytes > 0) k_small_segment<G, true><<<1, HQ_SMALL_BS, a.lds_bytes, h.st>>>(a, Tseg);
    else k_small_segment<G, false><<<1, HQ_SMALL_BS, 0, h.st>>>(a, Tseg);
  } else {
    if (a.lds_bytes > 0) k_small_primal<G, true><<<1, HQ_SMALL_BS, a.lds_bytes, h.st>>>(a, Tseg, meth);
    else k_small_primal<G, false><<<1, HQ_SMALL_BS, 0, h.st>>>(a, Tseg, meth);
  }
}

// dynamic LDS above 64 KB must be enabled per kernel (at create, outside any capture)
void small_attrs() {
  const void* ks[] = {(const void*)k_small_segment<1, true>, (const void*)k_small_segment<2, true>,
                      (const void*)k_small_segment<4, true>,  (const void*)k_small_segment<8, true>,
                      (const void*)k_small_segment<16, true>, (const void*)k_small_primal<1, true>,
                      (const void*)k_small_primal<2, true>,   (const void*)k_small_primal<4, true>,
                      (const void*)k_small_primal<8, true>,   (const void*)k_small_primal<16, true>};
  for (const void* k : ks) HQC(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, HQ_SMALL_LDS));
}

void enqueue_small_segment(hprqp_handle& h, int Tseg) {
  const SmallArgs a = small_args(h);
  switch (h.small_G) {
    case 1: launch_small<1>(h, a, Tseg); break;
    case 2: launch_small<2>(h, a, Tseg); break;
    case 4: launch_small<4>(h, a, Tseg); break;
    case 8: launch_small<8>(h, a, Tseg); break;
    default: launch_small<16>(h, a, Tseg); break;
  }
  final_reduce(h, 0, SL_ITER_END);
  HQC(hipMemcpyAsync(h.hs, h.scalars, SL_ITER_END * sizeof(double), hipMemcpyDeviceToHost, h.st));
}

// one workgroup per segment: chosen at create, and used while the data of
// the current method fits the LDS (a method switched to later may need more)
bool use_small(hprqp_handle& h) { return h.small_G > 0 && (h.small_forced || small_args(h).lds_bytes > 0); }

void enqueue_segment(hprqp_handle& h, int Tseg, bool prof) {
  if (!prof && use_small(h)) {
    enqueue_small_segment(h, Tseg);
    return;
  }
  for (int j = 0; j < Tseg; ++j) enqueue_iter(h, j, Tseg, false, prof);
  final_reduce(h, 0, SL_ITER_END);
  HQC(hipMemcpyAsync(h.hs, h.scalars, SL_ITER_END * sizeof(double), hipMemcpyDeviceToHost, h.st));
}

void stage1(hprqp_handle& h) {
  launch_elem(h, h.n, nullptr, EpiStage1{h.x, h.Qw, h.ATy, h.c, h.L, h.U, h.xh, h.XB, h.ZB, h.l1, 0.0}, 0,
              no_red(h));
}

// anchor/state <- (y, w, x) buffers; exact A^T y and Q w; z/x step
void reset_epoch(hprqp_handle& h) {
  const long long n = h.n, m = h.m;
  if (m > 0) {
    k_copy<<<hq_grid(m, 256), 256, 0, h.st>>>(m, h.y, h.ya, nullptr);
    launch_csr(h, h.AT, h.y, EpiStore2{h.ATy, h.ATya}, 0, no_red(h));
  }
  k_copy<<<hq_grid(n, 256), 256, 0, h.st>>>(n, h.w, h.wa, nullptr);
  k_copy<<<hq_grid(n, 256), 256, 0, h.st>>>(n, h.x, h.xa, nullptr);
  q_apply(h, h.w, EpiStore2{h.Qw, h.Qwa}, 0, no_red(h));
  stage1(h);
}

// ||du||_M^2 from the seven merit slots (theta decomposition of the metric of Algorithm 3)
double mnorm(const hprqp_handle& h, const double* S, double sigma) {
  const double th1 = h.lamA * S[0] + h.lamQ * S[1] - 2.0 * S[2];
  const double th2 = S[3], th3 = S[4], cross = S[5] - S[6];
  const double m2 = sigma * th1 + th2 / sigma + sigma * sigma * th3 / (1.0 + sigma * h.lamQ) + 2.0 * cross;
  return std::sqrt(m2 > 0.0 ? m2 : 0.0);
}

struct Resid {
  double eta_p, eta_d, eta_gap, pobj, dobj;
};
Resid residuals_from(const hprqp_handle& h, const double* S) {
  Resid r;
  r.eta_p = (h.m > 0) ? S[SL_RA + 0] / (1.0 + std::max(h.binf, S[SL_RA + 1])) : 0.0;
  r.eta_d = S[SL_RQ + 0] / (1.0 + std::max(h.cinf, std::max(S[SL_RQ + 1], S[SL_RQ + 2])));
  const double xQx = S[SL_RQ + 3];
  r.pobj = 0.5 * xQx + S[SL_RQ + 4];
  const double dinf = (h.m > 0 ? S[SL_RA + 3] : 0.0) + S[SL_RQ + 6];
  if (dinf > 0.0) {
    r.dobj = -INFINITY;
    r.eta_gap = INFINITY;
  } else {
    r.dobj = -0.5 * xQx + (h.m > 0 ? S[SL_RA + 2] : 0.0) + S[SL_RQ + 5];
    r.eta_gap = std::fabs(r.pobj - r.dobj) / (1.0 + std::max(std::fabs(r.pobj), std::fabs(r.dobj)));
  }
  return r;
}

// Algorithm 5, step 4: argmin of f(s) = th1 s + th2/s + s^2 th3/(1 + lamQ s) by a
// golden-section search on log s over the interval where f' changes sign; the
// comparison of f at the two probes uses the divided difference of f.
double golden_sigma(double th1, double th2, double th3, double lamQ) {
  const double hi = std::sqrt(th2 / th1);
  if (th3 <= 0.0 || lamQ <= 0.0) return hi;
  const double lo = std::sqrt(th2 / (th1 + th3 / lamQ));
  double a = std::log(lo), b = std::log(hi);
  const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
  const double stop = std::log1p(1e-12);
  for (int it = 0; it < 200 && (b - a) > stop; ++it) {
    const double p = b - gr * (b - a), q = a + gr * (b - a);
    const double sp = std::exp(p), sq = std::exp(q);
    const double slope = th1 - th2 / (sp * sq) + th3 * (sp + sq + lamQ * sp * sq) / ((1.0 + lamQ * sp) * (1.0 + lamQ * sq));
    if (slope > 0.0) b = q;   // f(p) < f(q)
    else a = p;
  }
  return std::exp(0.5 * (a + b));
}

// ---------------------------------------------------------------------------
// setup pieces
// ---------------------------------------------------------------------------
// Power method on A A^T (which = 0, vectors of length m) or Q (which = 1, length n):
// v <- start/|start|; repeat w = M v, lambda = <v, w>, v <- w/|w|; stop at the first
// iteration whose Rayleigh quotient changes by <= tol relative (Section 4.1).
double power_method(hprqp_handle& h, int which, const double* start, int maxit, double tol, int* iters_out) {
  const long long k = which == 0 ? h.m : h.n;
  if (k == 0) { if (iters_out) *iters_out = 0; return 0.0; }
  double* v = h.t1;   // current unit vector
  double* wv = h.t2;  // product
  double* tmpn = h.kronT ? nullptr : nullptr;
  (void)tmpn;
  double* mid = (which == 0) ? h.xh : nullptr;  // A^T v (n) for the A A^T case; xh is free at setup
  if (start) k_copy<<<hq_grid(k, 256), 256, 0, h.st>>>(k, start, v, nullptr);
  else k_fill<<<hq_grid(k, 256), 256, 0, h.st>>>(k, v, 1.0);
  launch_elem(h, (int)k, nullptr, EpiSumSq{v}, 0, red_seq(h, SL_POW, 1));
  final_reduce(h, SL_POW, 1);
  HQC(hipMemcpyAsync(h.hs, h.scalars + SL_POW, sizeof(double), hipMemcpyDeviceToHost, h.st));
  HQC(hipStreamSynchronize(h.st));
  const double s0 = h.hs[0] > 0.0 ? 1.0 / std::sqrt(h.hs[0]) : 0.0;
  h.hs[1] = s0;
  HQC(hipMemcpyAsync(h.scalars + SL_TOTAL, h.hs + 1, sizeof(double), hipMemcpyHostToDevice, h.st));
  k_scale<<<hq_grid(k, 256), 256, 0, h.st>>>(k, v, h.scalars + SL_TOTAL, v);
  const int chunk = 16;
  std::vector<double> hist;
  double lam = 0.0;
  int stop_it = -1;
  for (int it0 = 1; it0 <= maxit && stop_it < 0; it0 += chunk) {
    const int it1 = std::min(maxit, it0 + chunk - 1);
    for (int it = it0; it <= it1; ++it) {
      if (which == 0) {
        launch_csr(h, h.AT, v, EpiStore{mid}, 0, no_red(h));
        launch_csr(h, h.A, mid, EpiPow{v, wv}, 0, red_seq(h, SL_POW, 2));
      } else {
        q_apply(h, v, EpiPow{v, wv}, 0, red_seq(h, SL_POW, 2));
      }
      k_pow_final<<<1, 256, 0, h.st>>>(h.partials, h.counts, h.hist, it, h.scalars + SL_TOTAL);
      k_scale<<<hq_grid(k, 256), 256, 0, h.st>>>(k, wv, h.scalars + SL_TOTAL, v);
    }
    std::vector<double> hh(2 * (it1 + 1));
    HQC(hipMemcpyAsync(hh.data(), h.hist, hh.size() * sizeof(double), hipMemcpyDeviceToHost, h.st));
    HQC(hipStreamSynchronize(h.st));
    for (int it = it0; it <= it1; ++it) {
      lam = hh[2 * it];
      const double nw2 = hh[2 * it + 1];
      if (nw2 == 0.0) { stop_it = it; break; }
      if (it > 1 && std::fabs(lam - hh[2 * (it - 1)]) <= tol * std::fabs(lam)) { stop_it = it; break; }
    }
  }
  if (iters_out) *iters_out = stop_it < 0 ? maxit : stop_it;
  return lam;
}

// Panel-ordered copy of M (panel.hpp); false when a chunk would need more than
// 16-bit local offsets or the matrix is too small to gain from it
bool build_panel(hprqp_handle& h, Mat& M, bool any_size = false) {
  if (M.pm.pp) return true;
  if (M.rows == 0 || M.nnz == 0 || M.cols < HQ_PANELS) return false;
  if (!any_size && M.cols < 262144) return false;   // a vector of 2 MB or less stays in the L2 anyway
  const int nblk = (M.rows + HQ_BLOCK - 1) / HQ_BLOCK;
  const long long nch = (long long)nblk * HQ_PANELS;
  int *cnt = nullptr, *size = nullptr;
  HQC(hipMalloc(&cnt, sizeof(int) * (size_t)M.rows * HQ_PANELS));
  HQC(hipMalloc(&size, sizeof(int) * (size_t)nch));
  unsigned short* lrp = h.dalloc<unsigned short>((size_t)nch * (HQ_BLOCK + 1));
  k_panel_count<<<hq_grid(M.rows, 256), 256, 0, h.st>>>(M.rows, M.cols, M.rp, M.ci, cnt);
  k_panel_offsets<<<hq_grid(nch, 256), 256, 0, h.st>>>(M.rows, cnt, lrp, size);
  std::vector<int> hs((size_t)nch), hp((size_t)nch + 1, 0);
  HQC(hipMemcpyAsync(hs.data(), size, sizeof(int) * (size_t)nch, hipMemcpyDeviceToHost, h.st));
  HQC(hipStreamSynchronize(h.st));
  hipFree(cnt);
  hipFree(size);
  for (long long c = 0; c < nch; ++c) {
    if (hs[c] > 65535) return false;   // local offsets are 16-bit
    hp[c + 1] = hp[c] + hs[c];
  }
  if (hp[nch] != M.nnz) fail(HPRQP_ERR_HIP, "panel layout: nonzero count mismatch");
  int* pp = h.dalloc<int>((size_t)nch + 1);
  int* pci = h.dalloc<int>((size_t)M.nnz);
  double* pv = h.dalloc<double>((size_t)M.nnz);
  HQC(hipMemcpyAsync(pp, hp.data(), sizeof(int) * ((size_t)nch + 1), hipMemcpyHostToDevice, h.st));
  k_panel_scatter<<<hq_grid(M.rows, 256), 256, 0, h.st>>>(M.rows, M.cols, M.rp, M.ci, M.v, pp, lrp, pci, pv);
  HQC(hipStreamSynchronize(h.st));
  M.pm = PanelMat{M.rows, M.cols, pp, lrp, pci, pv};
  return true;
}

// Column-split copy of M (split.hpp); false when the matrix does not have the
// shape it serves: a vector too long for LDS, and rows long enough that the
// per-(panel, row) starts and partial sums stay small beside the matrix: on
// average at least 8 nonzeros per row in a panel of 2,048 columns, else at
// least 2 in a panel of 16,384
bool build_split(hprqp_handle& h, Mat& M) {
  if (M.sm.off) return true;
  if (M.rows == 0 || M.nnz == 0 || M.cols <= HQ_XLDS_MAX) return false;
  int pw = 0;
  long long np = 0, cells = 0;
  for (int w : {HQ_SPLIT_PW, HQ_SPLIT_PW_WIDE}) {
    np = (M.cols + w - 1) / w;
    cells = np * M.rows;
    if (cells * (w == HQ_SPLIT_PW ? 8 : 2) <= M.nnz) { pw = w; break; }
  }
  if (!pw || cells + 1 >= (1ll << 31)) return false;
  // workgroups per panel: one pass of 1,024 rows each for the narrow panels; for
  // the wide ones (one workgroup per CU) as few as keep the copies of x under an
  // eighth of the matrix's bytes, chosen to fill the last round of workgroups
  int nrb = (M.rows + HQ_SPLIT_ROWS - 1) / HQ_SPLIT_ROWS;
  if (pw == HQ_SPLIT_PW_WIDE) {
    const long long cap = std::max(1ll, (M.nnz * 10) / (8ll * 8 * M.cols));
    const int most = (int)std::min<long long>(std::min<long long>(cap, 16), nrb);
    double best = -1.0;
    int pick = 1;
    for (int r = 1; r <= most; ++r) {
      const long long blocks = np * r, rounds = (blocks + h.ncu - 1) / h.ncu;
      const double fill = (double)blocks / (double)(rounds * h.ncu);
      if (fill > best + 1e-9) { best = fill; pick = r; }
    }
    nrb = pick;
  }
  const int rpb = (int)((((long long)M.rows + nrb - 1) / nrb + HQ_SPLIT_ROWS - 1) / HQ_SPLIT_ROWS) * HQ_SPLIT_ROWS;
  nrb = (M.rows + rpb - 1) / rpb;
  if (np * nrb >= (1ll << 31)) return false;
  int* cnt = nullptr;
  HQC(hipMalloc(&cnt, sizeof(int) * (size_t)cells));
  HQC(hipMemsetAsync(cnt, 0, sizeof(int) * (size_t)cells, h.st));   // (setup, never captured)
  k_split_count<<<hq_grid(M.rows, 256), 256, 0, h.st>>>(M.rows, pw, M.rp, M.ci, cnt);
  std::vector<int> hc((size_t)cells), ho((size_t)cells + 1, 0);
  HQC(hipMemcpyAsync(hc.data(), cnt, sizeof(int) * (size_t)cells, hipMemcpyDeviceToHost, h.st));
  HQC(hipStreamSynchronize(h.st));
  for (long long c = 0; c < cells; ++c) ho[c + 1] = ho[c] + hc[c];
  if (ho[cells] != M.nnz) { hipFree(cnt); fail(HPRQP_ERR_HIP, "column-split layout: nonzero count mismatch"); }
  int* off = h.dalloc<int>((size_t)cells + 1);
  unsigned short* lci = h.dalloc<unsigned short>((size_t)M.nnz);
  double* sv = h.dalloc<double>((size_t)M.nnz);
  double* part = h.dalloc<double>((size_t)cells);
  HQC(hipMemcpyAsync(off, ho.data(), sizeof(int) * ((size_t)cells + 1), hipMemcpyHostToDevice, h.st));
  HQC(hipMemcpyAsync(cnt, ho.data(), sizeof(int) * (size_t)cells, hipMemcpyHostToDevice, h.st));   // cursors
  k_split_scatter<<<hq_grid(M.rows, 256), 256, 0, h.st>>>(M.rows, pw, M.rp, M.ci, M.v, cnt, lci, sv);
  HQC(hipStreamSynchronize(h.st));
  hipFree(cnt);
  SplitMat S;
  S.rows = M.rows; S.cols = M.cols; S.pw = pw; S.np = (int)np; S.rpb = rpb; S.nrb = nrb;
  S.off = off; S.lci = lci; S.v = sv; S.partial = part;
  M.sm = S;
  return true;
}

void autotune_csr(hprqp_handle& h, Mat& M, const double* x, double* out) {
  if (M.rows == 0 || M.nnz == 0) return;
  const int Gs[] = {0, HQ_G_XLDS, HQ_G_PANEL, HQ_G_SPLIT, 2, 4, 8, 16, 32, 64, 128, 256,
                    HQ_G_XROW - 2, HQ_G_XROW - 4, HQ_G_XROW - 8, HQ_G_XROW - 16, HQ_G_XROW - 32, HQ_G_XROW - 64};
  hipEvent_t e0, e1;
  HQC(hipEventCreate(&e0));
  HQC(hipEventCreate(&e1));
  // the default choice is kept unless another is at least 5% faster, so that
  // near-ties do not flip between runs
  const int G0 = M.G;
  float best = 1e30f, t_default = 1e30f, best_np = 1e30f;
  int bestG = G0, bestG_np = G0;
  for (int G : Gs) {
    // the CSR-stream kernels add a row serially: not candidates for very long rows
    if ((G == 0 || G == HQ_G_XLDS) && M.maxlen > 4096 && G0 != 0) continue;
    if ((G == HQ_G_XLDS || is_xrow(G)) && M.cols > HQ_XLDS_MAX) continue;
    const int lanes = is_xrow(G) ? HQ_G_XROW - G : G;   // lanes per row of a row-split kernel
    if (G == HQ_G_PANEL && (M.maxlen > 4096 || !build_panel(h, M))) continue;
    if (G == HQ_G_SPLIT && !build_split(h, M)) continue;
    // row-split groups much wider than the rows only idle their lanes: skip them
    if (lanes > 1 && M.maxlen >= 0 && M.maxlen <= 4096 && (double)lanes > 4.0 * ((double)M.nnz / M.rows) &&
        lanes > 8)
      continue;
    M.G = G;
    launch_csr(h, M, x, EpiStore{out}, 0, no_red(h));
    // one timed launch first: a candidate already twice as slow as the best
    // so far is not timed further (its single launch, times 5, stands in;
    // large matrices spend most of create here otherwise)
    float ms = 0, ms1 = 0;
    HQC(hipEventRecord(e0, h.st));
    launch_csr(h, M, x, EpiStore{out}, 0, no_red(h));
    HQC(hipEventRecord(e1, h.st));
    HQC(hipEventSynchronize(e1));
    HQC(hipEventElapsedTime(&ms1, e0, e1));
    if (G != G0 && 5.0f * ms1 > 2.0f * best) {
      ms = 5.0f * ms1;
    } else {
      HQC(hipEventRecord(e0, h.st));
      for (int r = 0; r < 4; ++r) launch_csr(h, M, x, EpiStore{out}, 0, no_red(h));
      HQC(hipEventRecord(e1, h.st));
      HQC(hipEventSynchronize(e1));
      HQC(hipEventElapsedTime(&ms, e0, e1));
      ms += ms1;
    }
    if (G == G0) t_default = ms;
    if (ms < best) { best = ms; bestG = G; }
    if (G != HQ_G_PANEL && G != HQ_G_SPLIT && ms < best_np) { best_np = ms; bestG_np = G; }
  }
  M.G = best < 0.95f * t_default ? bestG : G0;
  M.G_np = best_np < 0.95f * t_default ? bestG_np : G0;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
}

// Kronecker Q: the K-split kernel for small factors (latency-bound, d ~ 300),
// the LDS-tiled kernel above that, with split-K groups until there are 4
// blocks per compute unit (one 4-wave block per CU leaves the MFMA pipes
// waiting on LDS and L2; measured: d = 1024, 236 us with 4 groups against
// 484 us with 1)
void default_kron(hprqp_handle& h) {
  const int tiles = ((h.ks + HQ_TB - 1) / HQ_TB) * ((h.kp + HQ_TB - 1) / HQ_TB);
  if (std::max(h.ks, h.kp) <= 384) { h.kron_mode = 0; h.kron_groups = 1; return; }
  h.kron_mode = 1;
  int G = 1;
  while (G < h.kron_groups_max && tiles * G < 4 * h.ncu) G *= 2;
  h.kron_groups = G;
}

// time the Kronecker variants on a full Q product; keep the default unless
// another is at least 5% faster
void autotune_kron(hprqp_handle& h, const double* x, double* out) {
  hipEvent_t e0, e1;
  HQC(hipEventCreate(&e0));
  HQC(hipEventCreate(&e1));
  const int m0 = h.kron_mode, g0 = h.kron_groups;
  float best = 1e30f, t_default = 1e30f;
  int bm = m0, bg = g0;
  for (int mode = 0; mode < 2; ++mode)
    for (int G = 1; G <= (mode ? h.kron_groups_max : 1); G *= 2) {
      h.kron_mode = mode; h.kron_groups = G;
      q_apply(h, x, EpiStore{out}, 0, no_red(h));
      HQC(hipEventRecord(e0, h.st));
      for (int r = 0; r < 5; ++r) q_apply(h, x, EpiStore{out}, 0, no_red(h));
      HQC(hipEventRecord(e1, h.st));
      HQC(hipEventSynchronize(e1));
      float ms = 0;
      HQC(hipEventElapsedTime(&ms, e0, e1));
      if (mode == m0 && G == g0) t_default = ms;
      if (ms < best) { best = ms; bm = mode; bg = G; }
    }
  if (best < 0.95f * t_default) { h.kron_mode = bm; h.kron_groups = bg; }
  else { h.kron_mode = m0; h.kron_groups = g0; }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
}

// The Q d product carries the heaviest epilogue (11 vectors read, 3 written),
// which the panel-ordered kernel runs only after its last panel: time that
// product both ways (on the workspace as it is; every solve resets the state)
// and keep the panel-ordered kernel for it only if it is at least 5% faster.
void autotune_heavy_q(hprqp_handle& h) {
  if (h.Q.G != HQ_G_PANEL || h.m == 0) return;
  EpiQ2 e6{};
  e6.xh = h.xh; e6.w = h.w; e6.Qw = h.Qw; e6.XB = h.XB; e6.ZB = h.ZB;
  e6.q1 = h.q1; e6.d = h.d; e6.wa = h.wa; e6.Qwa = h.Qwa; e6.xa = h.xa; e6.ATy = h.ATy;
  e6.c = h.c; e6.L = h.L; e6.U = h.U; e6.e = h.e;
  e6.wbar = h.wbar; e6.qwbar = h.qwbar; e6.x = h.x; e6.xbar_out = h.xbo;
  e6.l1 = h.l1;
  hipEvent_t e0, e1;
  HQC(hipEventCreate(&e0));
  HQC(hipEventCreate(&e1));
  // the other kernel: the autotuner's best non-panel choice (the CSR-stream kernel by default)
  const int g_np = h.Q.G_np == HQ_G_PANEL ? 0 : h.Q.G_np;
  float t[2] = {0.f, 0.f};
  for (int v = 0; v < 2; ++v) {
    h.Q.G_np = v ? HQ_G_PANEL : g_np;
    q_apply(h, h.d, e6, 0, no_red(h), true);
    HQC(hipEventRecord(e0, h.st));
    for (int r = 0; r < 5; ++r) q_apply(h, h.d, e6, 0, no_red(h), true);
    HQC(hipEventRecord(e1, h.st));
    HQC(hipEventSynchronize(e1));
    HQC(hipEventElapsedTime(&t[v], e0, e1));
  }
  // the panel-ordered kernel is the default: the other one must be 5% faster
  h.Q.G_np = t[0] < 0.95f * t[1] ? g_np : HQ_G_PANEL;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
}

// Lanes per row of the row-split kernel, or 0 for the CSR-stream kernel
// (short rows: average up to 32 nonzeros and none longer than 4096).  The
// variant gathering from an LDS copy of the vector is left to the autotuner:
// measured on a 5e7-nonzero A^T with an 80 KB vector it was slower (322 us vs
// 262 us) than gathering through the L2.
int default_G(long long nnz, int rows, int maxlen, int cols) {
  const double avg = rows > 0 ? (double)nnz / rows : 1.0;
  (void)cols;
  if (avg <= 32.0 && maxlen <= 4096) return 0;
  // up to one wave per row for rows of up to 4096 entries on average (the
  // Kronecker QP's A, 300 per row: 64 lanes 7.5 us, 128 8.9 us, 256 9.3 us)
  const int cap = avg <= 4096.0 ? 64 : HQ_BLOCK;
  int G = 1;
  while (G < cap && G * 2 <= avg) G *= 2;
  return G;
}

void create_impl(const hprqp_problem* P, const hprqp_options* opt, hipStream_t st, hprqp_handle** out) {
  const double t0 = now_s();
  if (!P || !opt || !out) fail(HPRQP_ERR_ARG, "NULL argument");
  if (P->n <= 0 || P->m < 0) fail(HPRQP_ERR_SHAPE, "n must be > 0 and m >= 0");
  if (!P->c || !P->L || !P->U) fail(HPRQP_ERR_ARG, "c, L, U are required");
  if (P->m > 0 && (!P->a_rowptr || !P->l || !P->u || (P->a_nnz > 0 && (!P->a_col || !P->a_val))))
    fail(HPRQP_ERR_ARG, "A, l, u are required when m > 0");
  if (opt->check_every <= 0 || opt->max_iter <= 0 || !(opt->tol >= 0.0)) fail(HPRQP_ERR_ARG, "bad options");
  if (opt->method < 0 || opt->method > 2) fail(HPRQP_ERR_ARG, "method must be 0, 1 or 2");
  if (P->a_nnz < 0 || P->a_nnz >= (1ll << 31) || P->q_nnz < 0 || P->q_nnz >= (1ll << 31))
    fail(HPRQP_ERR_SHAPE, "nnz must fit int32");
  auto hp = new hprqp_handle();
  try {
    hprqp_handle& h = *hp;
    HQC(hipGetDevice(&h.dev));
    HQC(hipDeviceGetAttribute(&h.ncu, hipDeviceAttributeMultiprocessorCount, h.dev));
    if (!st) {
      // graphs cannot be captured on the legacy null stream: use a private one
      HQC(hipStreamCreateWithFlags(&h.own_st, hipStreamNonBlocking));
      HQC(hipDeviceSynchronize());
      st = h.own_st;
    }
    h.st = st;
    h.n = P->n; h.m = P->m; h.qkind = P->qkind;
    h.opt = *opt;
    if (opt->profile_kernels)
      for (auto& a : h.pev)
        for (auto& b : a)
          for (auto& e : b) HQC(hipEventCreate(&e));
    h.c = P->c; h.L = P->L; h.U = P->U; h.l = P->l; h.u = P->u;
    if (!(P->l1_weight >= 0.0) || std::isinf(P->l1_weight)) fail(HPRQP_ERR_ARG, "l1_weight must be finite and >= 0");
    h.l1 = P->l1_weight;
    const int n = h.n, m = h.m;
    switch (P->qkind) {
      case HPRQP_Q_ZERO: break;
      case HPRQP_Q_CSR:
        if (!P->q_rowptr || (P->q_nnz > 0 && (!P->q_col || !P->q_val))) fail(HPRQP_ERR_ARG, "Q CSR arrays required");
        h.Q = Mat{n, n, P->q_rowptr, P->q_col, P->q_val, P->q_nnz, 0};
        break;
      case HPRQP_Q_KRON:
        if (!P->kron_B || !P->kron_C || P->kron_p <= 0 || P->kron_s <= 0) fail(HPRQP_ERR_ARG, "Kronecker factors required");
        if ((long long)P->kron_p * P->kron_s != n) fail(HPRQP_ERR_SHAPE, "n must equal kron_p * kron_s");
        h.kp = P->kron_p; h.ks = P->kron_s; h.kB = P->kron_B; h.kC = P->kron_C;
        h.kS = P->kron_S; h.kT = P->kron_T;
        break;
      case HPRQP_Q_GRAM:
        if (P->gram_p <= 0 || !P->gram_rowptr || (P->gram_nnz > 0 && (!P->gram_col || !P->gram_val)))
          fail(HPRQP_ERR_ARG, "Gram factor Ahat (gram_p > 0, CSR arrays) required");
        if (P->gram_nnz < 0 || P->gram_nnz >= (1ll << 31)) fail(HPRQP_ERR_SHAPE, "gram_nnz must fit int32");
        h.G = Mat{P->gram_p, n, P->gram_rowptr, P->gram_col, P->gram_val, P->gram_nnz, 0};
        break;
      case HPRQP_Q_LOWRANK:
        if (!P->lr_d || (P->lr_rank > 0 && !P->lr_F)) fail(HPRQP_ERR_ARG, "low-rank arrays required");
        if (P->lr_rank < 0 || P->lr_rank > 16) fail(HPRQP_ERR_UNSUPPORTED, "lr_rank must be in [0, 16]");
        h.lr_r = P->lr_rank; h.lr_d = P->lr_d; h.lr_F = P->lr_F;
        break;
      default: fail(HPRQP_ERR_ARG, "unknown qkind");
    }
    // workspace
    h.partials = h.dalloc<double>((size_t)SL_TOTAL * HQ_PCAP);
    h.counts = h.dalloc<int>(SL_TOTAL);
    h.scalars = h.dalloc<double>(SL_TOTAL + 8);
    h.hist = h.dalloc<double>(2 * 5002);
    h.dflags = h.dalloc<int>(1);
    h.dprm = h.dalloc<DevParams>(1);
    HQC(hipHostMalloc((void**)&h.hs, 64 * sizeof(double), hipHostMallocDefault));
    HQC(hipHostMalloc((void**)&h.hp, sizeof(DevParams), hipHostMallocDefault));
    k_zero_ints<<<1, 64, 0, st>>>(SL_TOTAL, h.counts);
    k_zero_ints<<<1, 64, 0, st>>>(1, h.dflags);
    double** nv[] = {&h.w, &h.wa, &h.x, &h.xa, &h.ATy, &h.ATya, &h.Qw, &h.Qwa, &h.xh, &h.v, &h.q1, &h.d, &h.g,
                     &h.e, &h.XB, &h.ZB, &h.wbar, &h.qwbar, &h.xbo, &h.zbo, &h.t1, &h.t2,
                     &h.pt, &h.pta, &h.ptb, &h.pdt};
    for (double** p : nv) *p = h.dalloc<double>(n);
    if (h.qkind == HPRQP_Q_KRON) {
      h.kronT = h.dalloc<double>(n);
      // split-K workspace of the tiled GEMM while its tiles are fewer than 4 per CU
      const int tiles = ((h.ks + HQ_TB - 1) / HQ_TB) * ((h.kp + HQ_TB - 1) / HQ_TB);
      h.kron_groups_max = tiles < 4 * h.ncu ? 8 : 1;
      if (h.kron_groups_max > 1) h.kparts = h.dalloc<double>((size_t)h.kron_groups_max * n);
      default_kron(h);
    }
    double** mv[] = {&h.y, &h.ya, &h.ybar, &h.tm, &h.pe, &h.pax, &h.pdy};
    for (double** p : mv) *p = h.dalloc<double>(std::max(m, 1));
    for (double** p : nv) k_fill<<<hq_grid(n, 256), 256, 0, st>>>(n, *p, 0.0);
    for (double** p : mv) k_fill<<<hq_grid(std::max(m, 1), 256), 256, 0, st>>>(std::max(m, 1), *p, 0.0);
    // validation
    k_validate_vec<<<hq_grid(n, 256), 256, 0, st>>>(n, h.L, h.U, h.c, h.dflags);
    if (m > 0) {
      k_validate_vec<<<hq_grid(m, 256), 256, 0, st>>>(m, h.l, h.u, nullptr, h.dflags);
      k_validate_csr<<<hq_grid(m, 256), 256, 0, st>>>(m, n, P->a_nnz, P->a_rowptr, P->a_col, P->a_val, h.dflags);
    }
    if (h.qkind == HPRQP_Q_CSR)
      k_validate_csr<<<hq_grid(n, 256), 256, 0, st>>>(n, n, P->q_nnz, P->q_rowptr, P->q_col, P->q_val, h.dflags);
    if (h.qkind == HPRQP_Q_KRON) {
      k_validate_finite<<<64, 256, 0, st>>>((long long)h.kp * h.kp, h.kB, h.dflags);
      k_validate_finite<<<64, 256, 0, st>>>((long long)h.ks * h.ks, h.kC, h.dflags);
      if (h.kS) k_validate_finite<<<64, 256, 0, st>>>((long long)h.ks * h.ks, h.kS, h.dflags);
      if (h.kT) k_validate_finite<<<64, 256, 0, st>>>((long long)h.kp * h.kp, h.kT, h.dflags);
    }
    if (h.qkind == HPRQP_Q_LOWRANK) {
      k_validate_finite<<<64, 256, 0, st>>>(n, h.lr_d, h.dflags);
      k_validate_finite<<<256, 256, 0, st>>>((long long)n * h.lr_r, h.lr_F, h.dflags);
    }
    if (h.qkind == HPRQP_Q_GRAM)
      k_validate_csr<<<hq_grid(h.G.rows, 256), 256, 0, st>>>(h.G.rows, n, P->gram_nnz, P->gram_rowptr, P->gram_col,
                                                             P->gram_val, h.dflags);
    int flags = 0;
    HQC(hipMemcpyAsync(&flags, h.dflags, sizeof(int), hipMemcpyDeviceToHost, st));
    HQC(hipStreamSynchronize(st));
    if (flags & 2) fail(HPRQP_ERR_SHAPE, "CSR structure invalid (rowptr not monotone / not ending at nnz, or column out of range)");
    if (flags & 1) fail(HPRQP_ERR_BOUNDS, "invalid bounds (l > u, L > U, NaN, wrong-sided infinity) or non-finite data");
    // A and explicit A^T
    if (m > 0) {
      h.A = Mat{m, n, P->a_rowptr, P->a_col, P->a_val, P->a_nnz, 0};
      h.at_rp = h.dalloc<int>(n + 1);
      h.at_ci = h.dalloc<int>(P->a_nnz);
      h.at_v = h.dalloc<double>(P->a_nnz);
      const bool want_perm = opt->precondition && (h.qkind == HPRQP_Q_CSR || h.qkind == HPRQP_Q_ZERO) && h.l1 == 0.0;
      if (want_perm) h.at_perm = h.dalloc<int>(P->a_nnz);
      HQC(hq_build_transpose(m, n, P->a_nnz, P->a_rowptr, P->a_col, P->a_val, h.at_rp, h.at_ci, h.at_v, h.at_perm,
                             st));
      h.AT = Mat{n, m, h.at_rp, h.at_ci, h.at_v, P->a_nnz, 0};
    }
    // Gram factor: explicit Ahat^T for the second product of Q x = Ahat^T (Ahat x)
    if (h.qkind == HPRQP_Q_GRAM) {
      const int p = h.G.rows;
      int* grp = h.dalloc<int>(n + 1);
      int* gci = h.dalloc<int>(std::max<long long>(P->gram_nnz, 1));
      double* gv = h.dalloc<double>(std::max<long long>(P->gram_nnz, 1));
      HQC(hq_build_transpose(p, n, P->gram_nnz, P->gram_rowptr, P->gram_col, P->gram_val, grp, gci, gv, nullptr, st));
      h.GT = Mat{n, p, grp, gci, gv, P->gram_nnz, 0};
      h.gtmp = h.dalloc<double>(p);
    }
    h.A0 = h.A; h.AT0 = h.AT; h.Q0 = h.Q;
    h.c0 = h.c; h.L0 = h.L; h.U0 = h.U; h.l0 = h.l; h.u0 = h.u;
    // diagonal preconditioning (Section 4.1): explicit Q and phi a box indicator
    // only (a scaled ||x||_1 would need per-variable weights)
    if (opt->precondition && (h.qkind == HPRQP_Q_CSR || h.qkind == HPRQP_Q_ZERO) && h.l1 == 0.0) {
      if (opt->ruiz_iters < 0) fail(HPRQP_ERR_ARG, "ruiz_iters must be >= 0");
      h.pre = true;
      h.Ds = h.dalloc<double>(n); h.iDs = h.dalloc<double>(n);
      h.Es = h.dalloc<double>(std::max(m, 1)); h.iEs = h.dalloc<double>(std::max(m, 1));
      HqPrecondIn pin{};
      pin.m = m; pin.n = n;
      pin.a_rp = P->a_rowptr; pin.a_ci = P->a_col; pin.a_v = P->a_val; pin.a_nnz = m > 0 ? P->a_nnz : 0;
      pin.at_rp = h.at_rp; pin.at_ci = h.at_ci; pin.at_perm = h.at_perm; pin.at_v = h.at_v;
      if (h.qkind == HPRQP_Q_CSR) { pin.q_rp = P->q_rowptr; pin.q_ci = P->q_col; pin.q_v = P->q_val; }
      pin.c = P->c; pin.L = P->L; pin.U = P->U; pin.l = P->l; pin.u = P->u;
      pin.ruiz_iters = opt->ruiz_iters;
      HqPrecondOut pout{};
      pout.D = h.Ds; pout.E = h.Es;
      pout.q_v = h.qkind == HPRQP_Q_CSR ? h.dalloc<double>(std::max<long long>(P->q_nnz, 1)) : nullptr;
      pout.a_v = m > 0 ? h.dalloc<double>(std::max<long long>(P->a_nnz, 1)) : nullptr;
      pout.at_v = m > 0 ? h.dalloc<double>(std::max<long long>(P->a_nnz, 1)) : nullptr;
      pout.c = h.dalloc<double>(n); pout.L = h.dalloc<double>(n); pout.U = h.dalloc<double>(n);
      pout.l = m > 0 ? h.dalloc<double>(m) : nullptr; pout.u = m > 0 ? h.dalloc<double>(m) : nullptr;
      pout.work_n = h.t1; pout.work_n2 = h.t2; pout.work_m = h.tm;
      HQC(hipStreamSynchronize(st));
      const double tp = now_s();
      HQC(hq_precondition(pin, pout, st));
      k_recip<<<hq_grid(n, 256), 256, 0, st>>>(n, h.Ds, h.iDs);
      if (m > 0) k_recip<<<hq_grid(m, 256), 256, 0, st>>>(m, h.Es, h.iEs);
      if (h.qkind == HPRQP_Q_CSR) h.Q.v = pout.q_v;
      if (m > 0) { h.A.v = pout.a_v; h.AT.v = pout.at_v; h.l = pout.l; h.u = pout.u; }
      h.c = pout.c; h.L = pout.L; h.U = pout.U;
      HQC(hipStreamSynchronize(st));
      h.t_precond = now_s() - tp;
    }
    // product kernel per matrix from the row-length profile (autotuning may refine it)
    auto pick = [&](Mat& M) {
      if (M.rows == 0) return;
      k_zero_ints<<<1, 64, 0, st>>>(1, h.dflags);
      k_max_row_len<<<hq_grid(M.rows, 256), 256, 0, st>>>(M.rows, M.rp, h.dflags);
      int mx = 0;
      HQC(hipMemcpyAsync(&mx, h.dflags, sizeof(int), hipMemcpyDeviceToHost, st));
      HQC(hipStreamSynchronize(st));
      M.G = default_G(M.nnz, M.rows, mx, M.cols);
      M.G_np = M.G;
      M.maxlen = mx;
      if (M.G > 0 && M.cols <= HQ_XLDS_MAX && M.rows >= 65536) {
        // many long rows over a vector that fits LDS: the row-split kernel
        // gathering from LDS, about six nonzeros per lane (the Lasso's
        // Ahat^T, 100 per row: 173 us with 16 lanes against 350 us through
        // the L2 and 250 us with 64 lanes from LDS)
        const double avg = (double)M.nnz / M.rows;
        int g = 1;
        while (g < HQ_WAVE && 6.0 * 2 * g <= avg) g *= 2;
        M.G = HQ_G_XROW - g;
        M.G_np = M.G;
      } else if (M.G > 0 && (long long)M.cols * 8 > (3ll << 20) && build_split(h, M)) {
        // long rows over a vector larger than three quarters of an XCD's L2:
        // the column-split product (the Lasso's Ahat, 1e4 rows of 5000 over a
        // 4 MB vector: 145 us against 326 us; 2e5 rows of 1000 over 40 MB:
        // 1.30 ms against 3.0 ms panel-ordered).  Over a vector that stays in
        // the L2 its partial sums cost more than the gathers (Ahat^T of the
        // latter, 5e6 rows of 40 over 1.6 MB: 1.59 ms against 1.18 ms)
        M.G = HQ_G_SPLIT;
      }
      // short rows gathering from a vector larger than three quarters of an
      // XCD's 4 MiB L2 (which the matrix streams through as well): the
      // panel-ordered product, also under heavy epilogues (measured on 5e6
      // random gathers: 20% faster from an 8 MB vector, 1.8% from a 4 MB one,
      // A^T ybar of the random QP with n = 1e6, m = 5e5)
      if (M.G == 0 && (long long)M.cols * 8 > (3ll << 20) && build_panel(h, M)) {
        M.G = HQ_G_PANEL;
        M.G_np = HQ_G_PANEL;
      }
    };
    if (m > 0) { pick(h.A); pick(h.AT); }
    if (h.qkind == HPRQP_Q_CSR) pick(h.Q);
    if (h.qkind == HPRQP_Q_GRAM) { pick(h.G); pick(h.GT); }
    // lambda's: needed by the params of every kernel, also during the power method
    h.lamA = 0; h.lamQ = 0;
    write_params(h, 1.0, 0);
    if (opt->spmv_autotune) {
      if (m > 0) {
        autotune_csr(h, h.A, h.t1, h.tm);
        autotune_csr(h, h.AT, h.tm, h.t1);
      }
      if (h.qkind == HPRQP_Q_CSR) autotune_csr(h, h.Q, h.t1, h.t2);
      if (h.qkind == HPRQP_Q_KRON && opt->kron_kernel < 0) autotune_kron(h, h.t1, h.t2);
      if (h.qkind == HPRQP_Q_CSR) autotune_heavy_q(h);
      if (h.qkind == HPRQP_Q_GRAM) {
        autotune_csr(h, h.G, h.t1, h.gtmp);
        autotune_csr(h, h.GT, h.gtmp, h.t1);
      }
    }
    // one-workgroup segments for small explicit-Q problems (a launch per product
    // would cost more than the product)
    {
      const bool ok = (h.qkind == HPRQP_Q_CSR || h.qkind == HPRQP_Q_ZERO);
      if (opt->small_path < -1 || opt->small_path > 1) fail(HPRQP_ERR_ARG, "small_path must be -1, 0 or 1");
      if (opt->small_path == 1 && !ok) fail(HPRQP_ERR_UNSUPPORTED, "small_path needs an explicit or zero Q");
      // automatic: when the matrices and the vectors fit the workgroup's LDS
      const bool on = ok && (opt->small_path == 1 || (opt->small_path == -1 && small_args(h).lds_bytes > 0));
      if (on) {
        // the most lanes per row with which one pass of the workgroup covers
        // every row (small CCQP, n = 200: 4 lanes 6.9 us/iteration, 2 lanes
        // 7.3, 8 lanes 7.9)
        int G = 1;
        while (G < 16 && (long long)std::max(n, m) * G * 2 <= HQ_SMALL_BS) G *= 2;
        h.small_G = G;
        h.small_forced = opt->small_path == 1;
        small_attrs();
      }
    }
    if (h.qkind == HPRQP_Q_KRON && opt->kron_kernel >= 0) {
      const int kk = opt->kron_kernel;
      if (kk != 0 && kk != 1 && kk != 2 && kk != 4 && kk != 8)
        fail(HPRQP_ERR_ARG, "kron_kernel must be -1, 0, 1, 2, 4 or 8");
      if (kk > h.kron_groups_max) fail(HPRQP_ERR_ARG, "kron_kernel: split-K groups need fewer than 4 tiles per CU");
      h.kron_mode = kk == 0 ? 0 : 1;
      h.kron_groups = kk == 0 ? 1 : kk;
    }
    if (opt->spmv_lanes == HQ_G_SPLIT) {
      // the column-split product wherever its layout applies, else the default kernel
      for (Mat* M : {&h.A, &h.AT, &h.Q, &h.G, &h.GT})
        if (build_split(h, *M)) { M->G_np = M->G; M->G = HQ_G_SPLIT; }
    } else if (opt->spmv_lanes == -3) {
      // panel-ordered products wherever the layout applies, else the default kernel
      for (Mat* M : {&h.A, &h.AT, &h.Q, &h.G, &h.GT})
        if (M->rows > 0 && M->maxlen <= 4096 && build_panel(h, *M, true)) { M->G_np = M->G; M->G = HQ_G_PANEL; }
    } else if (opt->spmv_lanes >= 0 || opt->spmv_lanes == -2) {
      const int g = opt->spmv_lanes == -2 ? HQ_G_XLDS : opt->spmv_lanes;
      if (g != HQ_G_XLDS && (g > HQ_BLOCK || (g & (g - 1)) != 0))
        fail(HPRQP_ERR_ARG, "spmv_lanes must be -4, -3, -2, -1, 0, a power of 2 <= 256 or -100 - g (g <= 64)");
      for (Mat* M : {&h.A, &h.AT, &h.Q, &h.G, &h.GT}) {
        M->G = (g == HQ_G_XLDS && M->cols > HQ_XLDS_MAX) ? 0 : g;   // the LDS copy needs a small vector
        M->G_np = M->G;
      }
    } else if (opt->spmv_lanes < HQ_G_XROW) {
      const int g = HQ_G_XROW - opt->spmv_lanes;
      if (g > HQ_WAVE || (g & (g - 1)) != 0)
        fail(HPRQP_ERR_ARG, "spmv_lanes below -100 must be -100 - g with g a power of 2 <= 64");
      for (Mat* M : {&h.A, &h.AT, &h.Q, &h.G, &h.GT}) {
        // the LDS copy needs a small vector: the row-split kernel with g lanes otherwise
        M->G = M->cols > HQ_XLDS_MAX ? g : opt->spmv_lanes;
        M->G_np = M->G;
      }
    } else if (opt->spmv_lanes != -1) {
      fail(HPRQP_ERR_ARG, "spmv_lanes must be -4, -3, -2, -1, 0, a power of 2 <= 256 or -100 - g (g <= 64)");
    }
    // the operators as given (hprqp_apply, and the residuals of a preconditioned
    // handle) take the kernel chosen for the method's copy: the same arrays
    // without preconditioning; with it the unscaled arrays have the same
    // structure, but the panel-ordered copy holds scaled values
    auto inherit = [&](Mat& M0, const Mat& M) {
      if (!h.pre) { M0 = M; return; }
      const auto layout = [](int G) { return G == HQ_G_PANEL || G == HQ_G_SPLIT; };
      M0.maxlen = M.maxlen;
      M0.G = layout(M.G) ? (layout(M.G_np) ? 0 : M.G_np) : M.G;
      M0.G_np = M0.G;
    };
    inherit(h.A0, h.A); inherit(h.AT0, h.AT); inherit(h.Q0, h.Q);
    if (opt->lambda_A > 0) h.lamA = opt->lambda_A;
    else if (m > 0) {
      h.powA_est = power_method(h, 0, opt->power_start_A, 5000, 1e-6, &h.powA_it);
      h.lamA = 1.01 * h.powA_est;
    }
    if (opt->lambda_Q > 0) h.lamQ = opt->lambda_Q;
    else if (h.qkind != HPRQP_Q_ZERO) {
      h.powQ_est = power_method(h, 1, opt->power_start_Q, 5000, 1e-6, &h.powQ_it);
      h.lamQ = 1.01 * h.powQ_est;
    }
    if (m > 0 && !(h.lamA > 0.0)) fail(HPRQP_ERR_ARG, "lambda_A must be positive (A = 0?)");
    // norms of b and c: sigma0 rule and the denominators of eta_p, eta_d
    if (m > 0) launch_elem(h, m, nullptr, EpiNormB{h.l, h.u}, 0, red_seq(h, SL_NRM, 2));
    launch_elem(h, n, nullptr, EpiNormC{h.c}, 0, red_seq(h, SL_NRM + 2, 2));
    // EpiNormC writes (sum c^2, max|c|) into slots NRM+2, NRM+3
    final_reduce(h, SL_NRM, 4);
    HQC(hipMemcpyAsync(h.hs, h.scalars + SL_NRM, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    HQC(hipStreamSynchronize(st));
    const double nb = m > 0 ? std::sqrt(h.hs[0]) : 0.0, nc = std::sqrt(h.hs[2]);
    h.binf = m > 0 ? h.hs[1] : 0.0;
    h.cinf = h.hs[3];
    if (h.pre) {
      // sigma0 uses the scaled b and c (the problem the method runs on); the
      // stopping test uses the norms of the given problem
      if (m > 0) launch_elem(h, m, nullptr, EpiNormB{h.l0, h.u0}, 0, red_seq(h, SL_NRM, 2));
      launch_elem(h, n, nullptr, EpiNormC{h.c0}, 0, red_seq(h, SL_NRM + 2, 2));
      final_reduce(h, SL_NRM, 4);
      HQC(hipMemcpyAsync(h.hs, h.scalars + SL_NRM, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
      HQC(hipStreamSynchronize(st));
      h.binf = m > 0 ? h.hs[1] : 0.0;
      h.cinf = h.hs[3];
    }
    const bool norms_ok = nb >= 1e-16 && nb <= 1e16 && nc >= 1e-16 && nc <= 1e16;
    if (opt->sigma0 > 0) h.sigma0 = opt->sigma0;
    else h.sigma0 = norms_ok ? nb / nc : 1.0;
    // the primal methods' sigma multiplies the primal residual: the reciprocal rule
    if (opt->sigma0 > 0) h.sigma0_primal = opt->sigma0;
    else h.sigma0_primal = norms_ok ? nc / nb : 1.0;
    HQC(hipStreamSynchronize(st));
    h.t_setup = now_s() - t0;
    *out = hp;
  } catch (...) {
    delete hp;
    throw;
  }
}

// dst = src (times f elementwise when f is given), or 0 without src
void copy_or_zero(hprqp_handle& h, long long k, const double* src, double* dst, const double* f = nullptr) {
  if (src && f) k_mul<<<hq_grid(k, 256), 256, 0, h.st>>>(k, src, f, dst);
  else if (src) k_copy<<<hq_grid(k, 256), 256, 0, h.st>>>(k, src, dst, nullptr);
  else k_fill<<<hq_grid(k, 256), 256, 0, h.st>>>(k, dst, 0.0);
}

void trace_row(hprqp_handle& h, double* row) {
  const int n = h.n, m = h.m;
  HQC(hipStreamSynchronize(h.st));
  HQC(hipMemcpy(row, h.y, m * sizeof(double), hipMemcpyDeviceToHost)); row += m;
  HQC(hipMemcpy(row, h.w, n * sizeof(double), hipMemcpyDeviceToHost)); row += n;
  HQC(hipMemcpy(row, h.x, n * sizeof(double), hipMemcpyDeviceToHost)); row += n;
  HQC(hipMemcpy(row, h.ybar, m * sizeof(double), hipMemcpyDeviceToHost)); row += m;
  HQC(hipMemcpy(row, h.wbar, n * sizeof(double), hipMemcpyDeviceToHost)); row += n;
  HQC(hipMemcpy(row, h.xbo, n * sizeof(double), hipMemcpyDeviceToHost));
}

void solve_impl(hprqp_handle& h, const double* y0, const double* w0, const double* x0, double* yo, double* zo,
                double* wo, double* xo, hprqp_info* info, const hprqp_state* rs = nullptr,
                hprqp_state* sv = nullptr) {
  const double tstart = now_s();
  if (h.own_st) HQC(hipDeviceSynchronize());   // inputs written on other streams
  for (int kind = 0; kind < 4; ++kind) { h.prof_ms[kind] = 0.0; h.prof_n[kind] = 0; }
  const hprqp_options& o = h.opt;
  const int n = h.n, m = h.m;
  const int T = o.check_every;
  const bool tracing = o.trace_iters > 0 && o.trace_host;
  if (!yo && m > 0) fail(HPRQP_ERR_ARG, "output y required");
  if (!zo || !wo || !xo) fail(HPRQP_ERR_ARG, "outputs z, w, x required");
  if (sv && ((m > 0 && !sv->y) || !sv->w || !sv->x)) fail(HPRQP_ERR_ARG, "save: arrays y, w, x required");
  double sigma = h.sigma0;
  long long k = 0, t = 0;
  int r = 0, term = -1, nlog = 0;
  double alpha3 = o.alpha3, R0ref = -1.0, Rr0 = -1.0, Rprev = -1.0, R = 0.0;
  if (rs) {
    // an epoch start saved by an earlier solve, already in the internal variables
    if ((m > 0 && !rs->y) || !rs->w || !rs->x) fail(HPRQP_ERR_ARG, "resume: arrays y, w, x required");
    if (rs->k < 0 || rs->k >= o.max_iter) fail(HPRQP_ERR_ARG, "resume: k must lie in [0, max_iter)");
    if (rs->restarts < 0 || !(rs->sigma > 0.0) || !std::isfinite(rs->sigma) || !(rs->alpha3 > 0.0) ||
        !std::isfinite(rs->R0ref))
      fail(HPRQP_ERR_ARG, "resume: restarts >= 0, finite sigma > 0, alpha3 > 0 and finite R0ref required");
    if (m > 0) copy_or_zero(h, m, rs->y, h.y);
    copy_or_zero(h, n, rs->w, h.w);
    copy_or_zero(h, n, rs->x, h.x);
    k = rs->k; r = rs->restarts; sigma = rs->sigma; alpha3 = rs->alpha3; R0ref = rs->R0ref;
  } else {
    // a warm start in the given variables enters scaled: y/E, w/D, x/D
    if (m > 0) copy_or_zero(h, m, y0, h.y, h.pre ? h.iEs : nullptr);
    copy_or_zero(h, n, w0, h.w, h.pre ? h.iDs : nullptr);
    copy_or_zero(h, n, x0, h.x, h.pre ? h.iDs : nullptr);
  }
  write_params(h, sigma, 0);
  reset_epoch(h);
  // the state at the start of the current epoch (its point is the anchor ya, wa, xa)
  hprqp_state ep{k, r, 0, sigma, R0ref, alpha3, nullptr, nullptr, nullptr};
  Resid res{};
  const int rowlen = 2 * m + 4 * n;
  long long seg = 0;
  while (term < 0) {
    const int Tseg = (int)std::min<long long>(T, o.max_iter - k);
    // kernel timing: every 4th segment is launched directly with HIP events
    // around the four products (event nodes inside a replayed graph cannot be
    // read back); the other segments replay the captured graph
    const bool prof = o.profile_kernels && Tseg >= 4 && (seg++ % 4) == 1 && !(tracing && k < o.trace_iters);
    write_params(h, sigma, t);
    if (tracing && k < o.trace_iters) {
      for (int j = 0; j < Tseg; ++j) {
        enqueue_iter(h, j, Tseg, true, false);
        if (j < Tseg - 1 && k + j + 1 <= o.trace_iters) trace_row(h, o.trace_host + (size_t)(k + j) * rowlen);
      }
      final_reduce(h, 0, SL_ITER_END);
      HQC(hipMemcpyAsync(h.hs, h.scalars, SL_ITER_END * sizeof(double), hipMemcpyDeviceToHost, h.st));
    } else if (o.use_graph && Tseg == T && !prof) {
      if (!h.gexec || h.graph_T != T) {
        if (h.gexec) { hipGraphExecDestroy(h.gexec); h.gexec = nullptr; }
        if (h.graph) { hipGraphDestroy(h.graph); h.graph = nullptr; }
        HQC(hipStreamBeginCapture(h.st, hipStreamCaptureModeThreadLocal));
        enqueue_segment(h, T, false);
        HQC(hipStreamEndCapture(h.st, &h.graph));
        HQC(hipGraphInstantiate(&h.gexec, h.graph, nullptr, nullptr, 0));
        h.graph_T = T;
      }
      HQC(hipGraphLaunch(h.gexec, h.st));
    } else {
      enqueue_segment(h, Tseg, prof);
    }
    HQC(hipStreamSynchronize(h.st));
    if (prof) {
      for (int ps = 0; ps < HQ_PROF_ITERS && ps + 1 < Tseg - 1; ++ps)
        for (int kind = 0; kind < 4; ++kind) {
          if (m == 0 && (kind == 1 || kind == 2)) continue;
          float ms = 0.f;
          HQC(hipEventElapsedTime(&ms, h.pev[ps][kind][0], h.pev[ps][kind][1]));
          h.prof_ms[kind] += ms;
          h.prof_n[kind] += 1;
        }
    }
    const double* S = h.hs;
    if (t == 0) Rr0 = mnorm(h, S + (Tseg == 1 ? SL_RC : SL_RF), sigma);
    R = mnorm(h, S + SL_RC, sigma);
    res = residuals_from(h, S);
    const double th_slots[5] = {S[SL_TH], S[SL_TH + 1], S[SL_TH + 2], S[SL_TH + 3], S[SL_TH + 4]};
    k += Tseg;
    t += Tseg;
    const long long t_check = t;
    const double kkt = std::max(res.eta_p, std::max(res.eta_d, res.eta_gap));
    const double sigma_used = sigma;
    int restarted = 0;
    bool do_restart = false;
    if (std::isnan(kkt) || std::isnan(R)) term = HPRQP_NUMERICAL;
    else if (kkt <= o.tol) term = HPRQP_SOLVED;
    else if (k >= o.max_iter) term = HPRQP_MAX_ITER;
    else if (o.time_limit_s > 0 && now_s() - tstart >= o.time_limit_s) term = HPRQP_TIME_LIMIT;
    else if (o.enable_restart) {
      const bool c1 = R <= o.alpha1 * Rr0;                                   // eq:restart_1
      const bool c2 = Rprev >= 0.0 && R <= o.alpha2 * Rr0 && R > Rprev;      // eq:restart_2
      const bool c3 = (double)t >= alpha3 * (double)k;                       // eq:restart_3
      do_restart = c1 || c2 || c3;
    }
    Rprev = R;
    if (term < 0 && do_restart) {
      if (R0ref < 0.0) R0ref = R;
      const double ratio = R / R0ref;
      if (o.enable_sigma_update) {
        double th1 = h.lamA * th_slots[0] + h.lamQ * th_slots[1] - 2.0 * th_slots[2];
        double th2 = th_slots[3], th3 = th_slots[4];
        th1 = std::max(th1, 1e-12);
        th2 = std::max(th2, 1e-12);
        th3 = std::max(th3, 0.0);
        const double snew = golden_sigma(th1, th2, th3, h.lamQ);
        const double beta = std::exp(-ratio);
        sigma = std::exp(beta * std::log(snew) + (1.0 - beta) * std::log(sigma));
      }
      if (ratio <= 0.1) alpha3 = 0.2;
      // u^{r+1,0} = ubar
      if (m > 0) k_copy<<<hq_grid(m, 256), 256, 0, h.st>>>(m, h.ybar, h.y, nullptr);
      k_copy<<<hq_grid(n, 256), 256, 0, h.st>>>(n, h.wbar, h.w, nullptr);
      k_copy<<<hq_grid(n, 256), 256, 0, h.st>>>(n, h.xbo, h.x, nullptr);
      write_params(h, sigma, 0);
      reset_epoch(h);
      t = 0;
      Rprev = -1.0;
      r += 1;
      restarted = 1;
      ep = hprqp_state{k, r, 0, sigma, R0ref, alpha3, nullptr, nullptr, nullptr};
    }
    if (tracing && k <= o.trace_iters) trace_row(h, o.trace_host + (size_t)(k - 1) * rowlen);
    if (o.check_log_host && nlog < o.log_cap) {
      double* row = o.check_log_host + 10 * (size_t)nlog;
      row[0] = (double)k; row[1] = (double)t_check;
      row[2] = R; row[3] = res.eta_p; row[4] = res.eta_d; row[5] = res.eta_gap;
      row[6] = sigma_used; row[7] = restarted; row[8] = sigma; row[9] = r;
      ++nlog;
    }
  }
  // output ubar of the last iteration, in the given variables when
  // preconditioned: y = E y~, z = z~ / D, w = D w~, x = D x~
  if (m > 0) copy_or_zero(h, m, h.ybar, yo, h.pre ? h.Es : nullptr);
  copy_or_zero(h, n, h.zbo, zo, h.pre ? h.iDs : nullptr);
  copy_or_zero(h, n, h.wbar, wo, h.pre ? h.Ds : nullptr);
  copy_or_zero(h, n, h.xbo, xo, h.pre ? h.Ds : nullptr);
  if (sv) {
    if (m > 0) copy_or_zero(h, m, h.ya, sv->y);
    copy_or_zero(h, n, h.wa, sv->w);
    copy_or_zero(h, n, h.xa, sv->x);
    ep.y = sv->y; ep.w = sv->w; ep.x = sv->x;
  }
  HQC(hipStreamSynchronize(h.st));
  if (sv) *sv = ep;
  if (info) {
    const double tsolve = now_s() - tstart;
    info->term = term; info->iters = k; info->restarts = r; info->n_log = nlog;
    info->sigma = sigma; info->sigma0 = h.sigma0; info->lambda_A = h.lamA; info->lambda_Q = h.lamQ;
    info->eta_p = res.eta_p; info->eta_d = res.eta_d; info->eta_gap = res.eta_gap;
    info->pobj = res.pobj; info->dobj = res.dobj; info->R_last = R;
    info->t_setup_s = h.t_setup; info->t_solve_s = tsolve; info->t_precond_s = h.t_precond;
    info->qwx_gap = qwx_norm(h, h.wbar, h.xbo);   // diagnostic of the shadow w_Q, after the timed solve
  }
}

// ---------------------------------------------------------------------------
// HPR on the primal reformulations (Appendix A: Algorithm 6, method 1;
// Algorithm 7, method 2), the baselines of Table 1.  Same check segments,
// graphs, stopping test and restart criteria as HPR-QP; the merit uses the
// metric of the reformulation and needs two extra products (A xbar and
// Q xbar / Q vbar) at the first iteration of a segment and at its check.
// ---------------------------------------------------------------------------
void enqueue_primal_iter(hprqp_handle& h, int j, int Tseg, bool trace, bool prof) {
  const int meth = h.opt.method;
  const bool check = (j == Tseg - 1);
  const int rgroup = check ? SL_RC : (j == 0 ? SL_RF : -1);
  const bool want_r = rgroup >= 0;
  const bool store_bar = want_r || check || trace;
  int ps = -1;
  if (prof && !trace && j >= 1 && j <= HQ_PROF_ITERS && j < Tseg - 1) ps = j - 1;
  auto mark = [&](int kind, int edge) {
    if (ps >= 0) HQC(hipEventRecord(h.pev[ps][kind][edge], h.st));
  };
  auto slots = [&](std::initializer_list<int> s) {
    RedOut r = no_red(h);
    int k = 0;
    for (int v : s) r.slot[k++] = (int8_t)v;
    r.active = 0;
    for (int q = 0; q < k; ++q) r.active |= r.slot[q] >= 0;
    return r;
  };
  auto at = [&](int off) { return want_r ? rgroup + off : -1; };
  // Q x (Algorithm 6) or Q v with the v/t-step (Algorithm 7)
  mark(0, 0);
  if (meth == 1) {
    q_apply(h, h.x, EpiStore{h.q1}, j, no_red(h));
  } else {
    EpiP2V ev{h.w, h.x, h.pta, h.pt, h.wbar, h.v, h.Qw, h.e, h.pdt, h.ptb, want_r, check};
    q_apply(h, h.w, ev, j, slots({at(1), at(4), check ? SL_TH + 2 : -1}));
  }
  mark(0, 1);
  // A x with the s/y-step
  if (h.m > 0) {
    mark(1, 0);
    EpiPY ey{h.l, h.u, h.ya, h.y, h.ybar, h.pe, h.pax, h.pdy, want_r, check, store_bar};
    launch_csr(h, h.A, h.x, ey, j, slots({at(3), check ? SL_TH + 1 : -1}));
    mark(1, 1);
  }
  // A^T (2 ybar - y) with the x-step.  Its epilogue reads and writes a dozen
  // vectors, which the panel-ordered kernel runs only after its last panel:
  // like the Q d product of HPR-QP, this product takes the best other kernel
  // (random QP, Algorithm 6: 64.7 us on the panel kernel, 6,423 iterations/s;
  // the CSR-stream kernel, 6,518 iterations/s)
  mark(2, 0);
  Mat ATx = h.AT;
  if (ATx.G == HQ_G_PANEL) ATx.G = h.AT.G_np == HQ_G_PANEL ? 0 : h.AT.G_np;
  if (meth == 1) {
    EpiP1X ex{h.q1, h.c, h.L, h.U, h.xa, h.x, h.XB, h.ZB, h.d, want_r, check, store_bar, h.l1};
    RedOut rx = slots({at(0), check ? SL_TH : -1});
    if (h.m > 0) launch_csr(h, ATx, h.pe, ex, j, rx);
    else launch_elem(h, h.n, nullptr, ex, j, rx);
  } else {
    EpiP2X ex{h.v, h.c, h.L, h.U, h.xa, h.wa, h.wbar, h.pdt, h.x, h.w, h.XB, h.ZB, h.d, want_r, check, store_bar,
              h.l1};
    RedOut rx = slots({at(0), at(5), check ? SL_TH : -1});
    if (h.m > 0) launch_csr(h, ATx, h.pe, ex, j, rx);
    else launch_elem(h, h.n, nullptr, ex, j, rx);
  }
  mark(2, 1);
  if (want_r) {
    // <A dx, dy> and <dx, Q dx> (Algorithm 6) or <dv, Q dv> (Algorithm 7)
    if (h.m > 0) launch_csr(h, h.A, h.XB, EpiMeritA{h.pax, h.pdy}, j, slots({rgroup + 2}));
    if (meth == 1) q_apply(h, h.XB, EpiMeritQ{h.q1, h.d}, j, slots({rgroup + 1}));
    else q_apply(h, h.wbar, EpiMeritQ{h.Qw, h.e}, j, slots({rgroup + 6}));
  }
  if (check) {
    // stopping quantities at (ybar, zbar, xbar): A^T ybar, A xbar, Q xbar
    if (h.m > 0) {
      launch_csr(h, h.AT, h.ybar, EpiStore{h.g}, j, no_red(h));
      launch_csr(h, h.A, h.XB, EpiResA{h.l, h.u, h.ybar, h.iEs}, j, red_seq(h, SL_RA, 4));
    }
    q_apply(h, h.XB, EpiResQ{h.XB, h.ZB, h.m > 0 ? h.g : nullptr, h.c, h.L, h.U, h.xbo, h.zbo, h.iDs, h.l1}, j,
            red_seq(h, SL_RQ, 7));
  }
}

void enqueue_primal_segment(hprqp_handle& h, int Tseg, bool prof) {
  if (!prof && use_small(h)) {
    enqueue_small_segment(h, Tseg);   // the primal kernel: launch_small dispatches on the method
    return;
  }
  for (int j = 0; j < Tseg; ++j) enqueue_primal_iter(h, j, Tseg, false, prof);
  final_reduce(h, 0, SL_ITER_END);
  HQC(hipMemcpyAsync(h.hs, h.scalars, SL_ITER_END * sizeof(double), hipMemcpyDeviceToHost, h.st));
}

// ||du||_M from the merit slots, metric of Algorithm 6 / 7
double primal_mnorm(const hprqp_handle& h, const double* S, double sigma) {
  double m2;
  if (h.opt.method == 1)
    m2 = (h.lamQ + sigma * h.lamA) * S[0] - S[1] - 2.0 * S[2] + S[3] / sigma;
  else
    m2 = sigma * (1.0 + h.lamA) * S[0] - 2.0 * S[2] - 2.0 * S[5] + (S[3] + S[4]) / sigma + h.lamQ * S[1] - S[6];
  return std::sqrt(m2 > 0.0 ? m2 : 0.0);
}

// trace row [y, v, x, ybar, vbar, xbar] (Algorithm 6 has no v: x stands in)
void primal_trace_row(hprqp_handle& h, double* row) {
  const int n = h.n, m = h.m;
  const bool two = h.opt.method == 2;
  HQC(hipStreamSynchronize(h.st));
  HQC(hipMemcpy(row, h.y, m * sizeof(double), hipMemcpyDeviceToHost)); row += m;
  HQC(hipMemcpy(row, two ? h.w : h.x, n * sizeof(double), hipMemcpyDeviceToHost)); row += n;
  HQC(hipMemcpy(row, h.x, n * sizeof(double), hipMemcpyDeviceToHost)); row += n;
  HQC(hipMemcpy(row, h.ybar, m * sizeof(double), hipMemcpyDeviceToHost)); row += m;
  HQC(hipMemcpy(row, two ? h.wbar : h.XB, n * sizeof(double), hipMemcpyDeviceToHost)); row += n;
  HQC(hipMemcpy(row, h.XB, n * sizeof(double), hipMemcpyDeviceToHost));
}

// anchor <- state
void primal_reset_epoch(hprqp_handle& h) {
  const long long n = h.n, m = h.m;
  if (m > 0) k_copy<<<hq_grid(m, 256), 256, 0, h.st>>>(m, h.y, h.ya, nullptr);
  k_copy<<<hq_grid(n, 256), 256, 0, h.st>>>(n, h.x, h.xa, nullptr);
  if (h.opt.method == 2) {
    k_copy<<<hq_grid(n, 256), 256, 0, h.st>>>(n, h.w, h.wa, nullptr);
    k_copy<<<hq_grid(n, 256), 256, 0, h.st>>>(n, h.pt, h.pta, nullptr);
  }
}

void solve_primal_impl(hprqp_handle& h, const double* y0, const double* w0, const double* x0, double* yo,
                       double* zo, double* wo, double* xo, hprqp_info* info) {
  const double tstart = now_s();
  if (h.own_st) HQC(hipDeviceSynchronize());
  for (int kind = 0; kind < 4; ++kind) { h.prof_ms[kind] = 0.0; h.prof_n[kind] = 0; }
  const hprqp_options& o = h.opt;
  const int n = h.n, m = h.m, meth = o.method;
  const int T = o.check_every;
  const bool tracing = o.trace_iters > 0 && o.trace_host;
  if (!yo && m > 0) fail(HPRQP_ERR_ARG, "output y required");
  if (!zo || !wo || !xo) fail(HPRQP_ERR_ARG, "outputs z, w, x required");
  // state (x, v, y, t) from (x0, w0, y0, 0), scaled when preconditioned
  if (m > 0) copy_or_zero(h, m, y0, h.y, h.pre ? h.iEs : nullptr);
  copy_or_zero(h, n, x0, h.x, h.pre ? h.iDs : nullptr);
  copy_or_zero(h, n, meth == 2 ? w0 : nullptr, h.w, h.pre ? h.iDs : nullptr);
  copy_or_zero(h, n, nullptr, h.pt);
  double sigma = h.sigma0_primal;
  primal_reset_epoch(h);
  long long k = 0, t = 0;
  int r = 0, term = -1, nlog = 0;
  double alpha3 = o.alpha3, R0ref = -1.0, Rr0 = -1.0, Rprev = -1.0, R = 0.0;
  Resid res{};
  const int rowlen = 2 * m + 4 * n;
  long long seg = 0;
  while (term < 0) {
    const int Tseg = (int)std::min<long long>(T, o.max_iter - k);
    const bool prof = o.profile_kernels && Tseg >= 4 && (seg++ % 4) == 1 && !(tracing && k < o.trace_iters);
    write_params(h, sigma, t);
    if (tracing && k < o.trace_iters) {
      for (int j = 0; j < Tseg; ++j) {
        enqueue_primal_iter(h, j, Tseg, true, false);
        if (j < Tseg - 1 && k + j + 1 <= o.trace_iters) primal_trace_row(h, o.trace_host + (size_t)(k + j) * rowlen);
      }
      final_reduce(h, 0, SL_ITER_END);
      HQC(hipMemcpyAsync(h.hs, h.scalars, SL_ITER_END * sizeof(double), hipMemcpyDeviceToHost, h.st));
    } else if (o.use_graph && Tseg == T && !prof) {
      if (!h.pgexec || h.pgraph_T != T || h.pgraph_method != meth) {
        if (h.pgexec) { hipGraphExecDestroy(h.pgexec); h.pgexec = nullptr; }
        if (h.pgraph) { hipGraphDestroy(h.pgraph); h.pgraph = nullptr; }
        HQC(hipStreamBeginCapture(h.st, hipStreamCaptureModeThreadLocal));
        enqueue_primal_segment(h, T, false);
        HQC(hipStreamEndCapture(h.st, &h.pgraph));
        HQC(hipGraphInstantiate(&h.pgexec, h.pgraph, nullptr, nullptr, 0));
        h.pgraph_T = T;
        h.pgraph_method = meth;
      }
      HQC(hipGraphLaunch(h.pgexec, h.st));
    } else {
      enqueue_primal_segment(h, Tseg, prof);
    }
    HQC(hipStreamSynchronize(h.st));
    if (prof) {
      for (int ps = 0; ps < HQ_PROF_ITERS && ps + 1 < Tseg - 1; ++ps)
        for (int kind = 0; kind < 3; ++kind) {
          if (m == 0 && kind == 1) continue;
          float ms = 0.f;
          HQC(hipEventElapsedTime(&ms, h.pev[ps][kind][0], h.pev[ps][kind][1]));
          h.prof_ms[kind] += ms;
          h.prof_n[kind] += 1;
        }
    }
    const double* S = h.hs;
    if (t == 0) Rr0 = primal_mnorm(h, S + (Tseg == 1 ? SL_RC : SL_RF), sigma);
    R = primal_mnorm(h, S + SL_RC, sigma);
    res = residuals_from(h, S);
    const double nDx = S[SL_TH], nDy = m > 0 ? S[SL_TH + 1] : 0.0, nDt = meth == 2 ? S[SL_TH + 2] : 0.0;
    k += Tseg;
    t += Tseg;
    const long long t_check = t;
    const double kkt = std::max(res.eta_p, std::max(res.eta_d, res.eta_gap));
    const double sigma_used = sigma;
    int restarted = 0;
    bool do_restart = false;
    if (std::isnan(kkt) || std::isnan(R)) term = HPRQP_NUMERICAL;
    else if (kkt <= o.tol) term = HPRQP_SOLVED;
    else if (k >= o.max_iter) term = HPRQP_MAX_ITER;
    else if (o.time_limit_s > 0 && now_s() - tstart >= o.time_limit_s) term = HPRQP_TIME_LIMIT;
    else if (o.enable_restart) {
      const bool c1 = R <= o.alpha1 * Rr0;
      const bool c2 = Rprev >= 0.0 && R <= o.alpha2 * Rr0 && R > Rprev;
      const bool c3 = (double)t >= alpha3 * (double)k;
      do_restart = c1 || c2 || c3;
    }
    Rprev = R;
    if (term < 0 && do_restart) {
      if (R0ref < 0.0) R0ref = R;
      const double ratio = R / R0ref;
      if (o.enable_sigma_update && !(meth == 1 && m == 0)) {
        // minimiser of the sigma-dependent part of ||ubar - u_a||_M^2, smoothed as in Algorithm 5
        const double th1 = std::max((meth == 1 ? h.lamA : 1.0 + h.lamA) * nDx, 1e-12);
        const double th2 = std::max(nDy + nDt, 1e-12);
        const double snew = std::sqrt(th2 / th1);
        const double beta = std::exp(-ratio);
        sigma = std::exp(beta * std::log(snew) + (1.0 - beta) * std::log(sigma));
      }
      if (ratio <= 0.1) alpha3 = 0.2;
      // u^{r+1,0} = ubar
      if (m > 0) k_copy<<<hq_grid(m, 256), 256, 0, h.st>>>(m, h.ybar, h.y, nullptr);
      k_copy<<<hq_grid(n, 256), 256, 0, h.st>>>(n, h.XB, h.x, nullptr);
      if (meth == 2) {
        k_copy<<<hq_grid(n, 256), 256, 0, h.st>>>(n, h.wbar, h.w, nullptr);
        k_copy<<<hq_grid(n, 256), 256, 0, h.st>>>(n, h.ptb, h.pt, nullptr);
      }
      primal_reset_epoch(h);
      t = 0;
      Rprev = -1.0;
      r += 1;
      restarted = 1;
    }
    if (tracing && k <= o.trace_iters) primal_trace_row(h, o.trace_host + (size_t)(k - 1) * rowlen);
    if (o.check_log_host && nlog < o.log_cap) {
      double* row = o.check_log_host + 10 * (size_t)nlog;
      row[0] = (double)k; row[1] = (double)t_check;
      row[2] = R; row[3] = res.eta_p; row[4] = res.eta_d; row[5] = res.eta_gap;
      row[6] = sigma_used; row[7] = restarted; row[8] = sigma; row[9] = r;
      ++nlog;
    }
  }
  // output ubar of the last (check) iteration; w = xbar (Algorithm 6) or vbar (7)
  if (m > 0) copy_or_zero(h, m, h.ybar, yo, h.pre ? h.Es : nullptr);
  copy_or_zero(h, n, h.zbo, zo, h.pre ? h.iDs : nullptr);
  copy_or_zero(h, n, meth == 2 ? h.wbar : h.xbo, wo, h.pre ? h.Ds : nullptr);
  copy_or_zero(h, n, h.xbo, xo, h.pre ? h.Ds : nullptr);
  HQC(hipStreamSynchronize(h.st));
  if (info) {
    info->term = term; info->iters = k; info->restarts = r; info->n_log = nlog;
    info->sigma = sigma; info->sigma0 = h.sigma0_primal; info->lambda_A = h.lamA; info->lambda_Q = h.lamQ;
    info->eta_p = res.eta_p; info->eta_d = res.eta_d; info->eta_gap = res.eta_gap;
    info->pobj = res.pobj; info->dobj = res.dobj; info->R_last = R;
    info->t_setup_s = h.t_setup; info->t_solve_s = now_s() - tstart; info->t_precond_s = h.t_precond;
    // w = xbar (Algorithm 6: 0) or vbar (Algorithm 7)
    info->qwx_gap = qwx_norm(h, meth == 2 ? h.wbar : h.xbo, h.xbo);
  }
}

void residuals_impl(hprqp_handle& h, const double* y, const double* z, const double* w, const double* x,
                    hprqp_info* info) {
  if (!z || !x || (h.m > 0 && !y) || !info) fail(HPRQP_ERR_ARG, "NULL argument");
  const double* const x_given = x;   // x below becomes the scaled copy when preconditioned
  write_params(h, h.sigma0, 0);
  k_zero_ints<<<1, 64, 0, h.st>>>(SL_ITER_END, h.counts);
  if (h.pre) {
    // the point is given in the original variables: scale it (y/E, z D, x/D)
    // and take the stopping quantities as at a check
    if (h.m > 0) k_mul<<<hq_grid(h.m, 256), 256, 0, h.st>>>(h.m, y, h.iEs, h.tm);
    k_mul<<<hq_grid(h.n, 256), 256, 0, h.st>>>(h.n, z, h.Ds, h.q1);
    k_mul<<<hq_grid(h.n, 256), 256, 0, h.st>>>(h.n, x, h.iDs, h.v);
    y = h.m > 0 ? h.tm : y; z = h.q1; x = h.v;
  }
  if (h.m > 0) {
    launch_csr(h, h.AT, y, EpiStore{h.t2}, 0, no_red(h));
    launch_csr(h, h.A, x, EpiResA{h.l, h.u, y, h.iEs}, 0, red_seq(h, SL_RA, 4));
  }
  q_apply(h, x, EpiResQ{x, z, h.m > 0 ? h.t2 : nullptr, h.c, h.L, h.U, nullptr, nullptr, h.iDs, h.l1}, 0,
          red_seq(h, SL_RQ, 7));
  final_reduce(h, 0, SL_ITER_END);
  HQC(hipMemcpyAsync(h.hs, h.scalars, SL_ITER_END * sizeof(double), hipMemcpyDeviceToHost, h.st));
  HQC(hipStreamSynchronize(h.st));
  const Resid r = residuals_from(h, h.hs);
  std::memset(info, 0, sizeof(*info));
  info->eta_p = r.eta_p; info->eta_d = r.eta_d; info->eta_gap = r.eta_gap; info->pobj = r.pobj; info->dobj = r.dobj;
  info->qwx_gap = std::numeric_limits<double>::quiet_NaN();
  if (w) {
    // Q (w - x) of the given problem: with preconditioning, (w - x)/D in the scaled variables
    k_diff<<<hq_grid(h.n, 256), 256, 0, h.st>>>(h.n, w, x_given, h.pre ? h.iDs : nullptr, h.t2);
    q_apply(h, h.t2, EpiMaxAbs{h.pre ? h.iDs : nullptr}, 0, red_seq(h, SL_QWX, 1));
    final_reduce(h, SL_QWX, 1);
    HQC(hipMemcpyAsync(h.hs + SL_QWX, h.scalars + SL_QWX, sizeof(double), hipMemcpyDeviceToHost, h.st));
    HQC(hipStreamSynchronize(h.st));
    info->qwx_gap = h.hs[SL_QWX];
  }
}

void apply_impl(hprqp_handle& h, int op, const double* in, double* out) {
  if (!in || !out) fail(HPRQP_ERR_ARG, "NULL argument");
  write_params(h, h.sigma0, 0);
  // the operators of the problem as given (the unscaled copies when preconditioned)
  if (op == 0 && h.pre && h.qkind == HPRQP_Q_CSR) launch_csr(h, h.Q0, in, EpiStore{out}, 0, no_red(h));
  else if (op == 0) q_apply(h, in, EpiStore{out}, 0, no_red(h));
  else if (op == 1 && h.m > 0) launch_csr(h, h.A0, in, EpiStore{out}, 0, no_red(h));
  else if (op == 2 && h.m > 0) launch_csr(h, h.AT0, in, EpiStore{out}, 0, no_red(h));
  else if (op == 2) k_fill<<<hq_grid(h.n, 256), 256, 0, h.st>>>(h.n, out, 0.0);
  else if (op != 1) fail(HPRQP_ERR_ARG, "op must be 0 (Q), 1 (A) or 2 (A^T)");
  HQC(hipStreamSynchronize(h.st));
}

}  // namespace hq

// ---------------------------------------------------------------------------
// Stopping quantities with no handle and no allocation (hprqp_residuals_noalloc)
// ---------------------------------------------------------------------------
// Workspace: one file-scope device array, which every GPU the library runs on
// holds until the process ends.  Host code never uses its name as an address:
// the device address comes from hipGetSymbolAddress, once per device.
#define HQ_NOALLOC_BYTES (32ll << 20)
static __device__ __align__(256) double scratch[HQ_NOALLOC_BYTES / sizeof(double)];

// g += A^T y without a stored transpose: one nonzero per thread (its row
// found by bisection of rowptr), added with FP64 atomics, so the order of the
// additions, and the rounding of g, can differ between calls
__global__ void k_csr_t_scatter(int rows, long long nnz, const int* __restrict__ rp, const int* __restrict__ ci,
                                const double* __restrict__ v, const double* __restrict__ y, double* __restrict__ g) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (long long)gridDim.x * blockDim.x) {
    int lo = 0, hi = rows - 1;   // the last row r with rp[r] <= k: the row holding k
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rp[mid] <= k) lo = mid;
      else hi = mid - 1;
    }
    const double p = v[k] * y[lo];
    if (p != 0.0) atomicAdd(g + ci[k], p);
  }
}

namespace hq {

#define HQ_NOALLOC_MAXDEV 64
std::mutex g_noalloc_mu[HQ_NOALLOC_MAXDEV];        // one call at a time per device
double* g_noalloc_ptr[HQ_NOALLOC_MAXDEV] = {};     // device address of `scratch`, per device

// Fixed part of the workspace, in doubles: block partials, scalars, counters
// and flags, the parameter block; the vectors follow.
constexpr long long kNaPartials = (long long)SL_TOTAL * HQ_PCAP;
constexpr long long kNaScalars = kNaPartials;            // 64 doubles
constexpr long long kNaInts = kNaScalars + 64;           // 64 ints (32 doubles): counts, then flags
constexpr long long kNaParams = kNaInts + 32;            // DevParams (32 doubles reserved)
constexpr long long kNaVectors = kNaParams + 32;
constexpr long long kNaCapacity = HQ_NOALLOC_BYTES / (long long)sizeof(double);
static_assert(SL_TOTAL <= 60, "counts and flags share 64 ints");
static_assert(sizeof(DevParams) <= 32 * sizeof(double), "parameter block");

// Q v through the epilogue; the Gram Q = Ahat^T (Ahat v) takes Ahat v into
// tp (p) and scatters Ahat^T of it into tq (n), then runs the epilogue on tq
template <class Epi>
void noalloc_q(hprqp_handle& h, const double* v, const Epi& epi, const RedOut& red, double* tp, double* tq) {
  if (h.qkind != HPRQP_Q_GRAM) {
    q_apply(h, v, epi, 0, red);
    return;
  }
  launch_csr(h, h.G, v, EpiStore{tp}, 0, no_red(h));
  k_fill<<<hq_grid(h.n, 256), 256, 0, h.st>>>(h.n, tq, 0.0);
  if (h.G.nnz > 0)
    k_csr_t_scatter<<<hq_grid(h.G.nnz, 256), 256, 0, h.st>>>(h.G.rows, h.G.nnz, h.G.rp, h.G.ci, h.G.v, tp, tq);
  launch_elem(h, h.n, tq, epi, 0, red);
}

void residuals_noalloc_impl(const hprqp_problem* P, const double* y, const double* z, const double* w,
                            const double* x, hprqp_info* info, hipStream_t st) {
  if (!P || !info || !z || !x) fail(HPRQP_ERR_ARG, "NULL argument");
  if (P->n <= 0 || P->m < 0) fail(HPRQP_ERR_SHAPE, "n must be > 0 and m >= 0");
  if (!P->c || !P->L || !P->U) fail(HPRQP_ERR_ARG, "c, L, U are required");
  if (P->m > 0 && (!y || !P->a_rowptr || !P->l || !P->u || (P->a_nnz > 0 && (!P->a_col || !P->a_val))))
    fail(HPRQP_ERR_ARG, "y, A, l, u are required when m > 0");
  if (P->a_nnz < 0 || P->a_nnz >= (1ll << 31) || P->q_nnz < 0 || P->q_nnz >= (1ll << 31))
    fail(HPRQP_ERR_SHAPE, "nnz must fit int32");
  if (!(P->l1_weight >= 0.0) || std::isinf(P->l1_weight)) fail(HPRQP_ERR_ARG, "l1_weight must be finite and >= 0");
  const int n = P->n, m = P->m;
  // the workspace this call needs: A^T y (n), the Kronecker or Gram
  // intermediates, w - x (n)
  long long need = (m > 0 ? n : 0) + (w ? n : 0);
  switch (P->qkind) {
    case HPRQP_Q_ZERO: break;
    case HPRQP_Q_CSR:
      if (!P->q_rowptr || (P->q_nnz > 0 && (!P->q_col || !P->q_val))) fail(HPRQP_ERR_ARG, "Q CSR arrays required");
      break;
    case HPRQP_Q_KRON:
      if (!P->kron_B || !P->kron_C || P->kron_p <= 0 || P->kron_s <= 0) fail(HPRQP_ERR_ARG, "Kronecker factors required");
      if ((long long)P->kron_p * P->kron_s != n) fail(HPRQP_ERR_SHAPE, "n must equal kron_p * kron_s");
      need += n;
      break;
    case HPRQP_Q_GRAM:
      if (P->gram_p <= 0 || !P->gram_rowptr || (P->gram_nnz > 0 && (!P->gram_col || !P->gram_val)))
        fail(HPRQP_ERR_ARG, "Gram factor Ahat (gram_p > 0, CSR arrays) required");
      if (P->gram_nnz < 0 || P->gram_nnz >= (1ll << 31)) fail(HPRQP_ERR_SHAPE, "gram_nnz must fit int32");
      need += (long long)P->gram_p + n;
      break;
    case HPRQP_Q_LOWRANK:
      if (!P->lr_d || (P->lr_rank > 0 && !P->lr_F)) fail(HPRQP_ERR_ARG, "low-rank arrays required");
      if (P->lr_rank < 0 || P->lr_rank > 16) fail(HPRQP_ERR_UNSUPPORTED, "lr_rank must be in [0, 16]");
      break;
    default: fail(HPRQP_ERR_ARG, "unknown qkind");
  }
  if (need > kNaCapacity - kNaVectors)
    fail(HPRQP_ERR_UNSUPPORTED, "problem needs " + std::to_string(need * 8) + " bytes of workspace; the allocation-free "
                                "residuals hold " + std::to_string((kNaCapacity - kNaVectors) * 8));
  int dev = 0;
  HQC(hipGetDevice(&dev));
  if (dev < 0 || dev >= HQ_NOALLOC_MAXDEV) fail(HPRQP_ERR_UNSUPPORTED, "device index beyond the workspace table");
  std::lock_guard<std::mutex> lock(g_noalloc_mu[dev]);
  if (!g_noalloc_ptr[dev]) {
    void* addr = nullptr;
    HQC(hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)));
    g_noalloc_ptr[dev] = (double*)addr;
  }
  double* const ws = g_noalloc_ptr[dev];

  // a handle on the stack whose workspace pointers point into `scratch`
  // (it owns nothing: its destructor frees nothing)
  hprqp_handle h;
  h.dev = dev;
  HQC(hipDeviceGetAttribute(&h.ncu, hipDeviceAttributeMultiprocessorCount, dev));
  h.st = st;
  h.n = n; h.m = m; h.qkind = P->qkind; h.l1 = P->l1_weight;
  h.c = P->c; h.L = P->L; h.U = P->U; h.l = P->l; h.u = P->u;
  h.partials = ws;
  h.scalars = ws + kNaScalars;
  h.counts = (int*)(ws + kNaInts);
  int* flags = h.counts + 60;                  // [0] validation, [1..3] longest row of A, Q, Ahat
  h.dprm = (DevParams*)(ws + kNaParams);
  double* vec = ws + kNaVectors;
  double* g = nullptr;
  if (m > 0) { g = vec; vec += n; }
  double* d = nullptr;
  if (w) { d = vec; vec += n; }
  double *tp = nullptr, *tq = nullptr;
  if (P->qkind == HPRQP_Q_KRON) { h.kronT = vec; vec += n; }
  if (P->qkind == HPRQP_Q_GRAM) { tp = vec; vec += P->gram_p; tq = vec; vec += n; }
  k_zero_ints<<<1, 64, 0, st>>>(64, h.counts);    // counts of every slot and the flags start at 0
  k_fill<<<1, 64, 0, st>>>(32, ws + kNaParams, 0.0);
  // validation (as at create) and the longest row of each CSR matrix
  k_validate_vec<<<hq_grid(n, 256), 256, 0, st>>>(n, P->L, P->U, P->c, flags);
  if (m > 0) {
    k_validate_vec<<<hq_grid(m, 256), 256, 0, st>>>(m, P->l, P->u, nullptr, flags);
    k_validate_csr<<<hq_grid(m, 256), 256, 0, st>>>(m, n, P->a_nnz, P->a_rowptr, P->a_col, P->a_val, flags);
    k_max_row_len<<<hq_grid(m, 256), 256, 0, st>>>(m, P->a_rowptr, flags + 1);
  }
  switch (P->qkind) {
    case HPRQP_Q_CSR:
      k_validate_csr<<<hq_grid(n, 256), 256, 0, st>>>(n, n, P->q_nnz, P->q_rowptr, P->q_col, P->q_val, flags);
      k_max_row_len<<<hq_grid(n, 256), 256, 0, st>>>(n, P->q_rowptr, flags + 2);
      break;
    case HPRQP_Q_KRON:
      k_validate_finite<<<64, 256, 0, st>>>((long long)P->kron_p * P->kron_p, P->kron_B, flags);
      k_validate_finite<<<64, 256, 0, st>>>((long long)P->kron_s * P->kron_s, P->kron_C, flags);
      if (P->kron_S) k_validate_finite<<<64, 256, 0, st>>>((long long)P->kron_s * P->kron_s, P->kron_S, flags);
      if (P->kron_T) k_validate_finite<<<64, 256, 0, st>>>((long long)P->kron_p * P->kron_p, P->kron_T, flags);
      break;
    case HPRQP_Q_LOWRANK:
      k_validate_finite<<<64, 256, 0, st>>>(n, P->lr_d, flags);
      if (P->lr_rank > 0) k_validate_finite<<<256, 256, 0, st>>>((long long)n * P->lr_rank, P->lr_F, flags);
      break;
    case HPRQP_Q_GRAM:
      k_validate_csr<<<hq_grid(P->gram_p, 256), 256, 0, st>>>(P->gram_p, n, P->gram_nnz, P->gram_rowptr, P->gram_col,
                                                              P->gram_val, flags);
      k_max_row_len<<<hq_grid(P->gram_p, 256), 256, 0, st>>>(P->gram_p, P->gram_rowptr, flags + 3);
      break;
    default: break;
  }
  int hf[4] = {0, 0, 0, 0};
  HQC(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st));
  HQC(hipStreamSynchronize(st));
  if (hf[0] & 2) fail(HPRQP_ERR_SHAPE, "CSR structure invalid (rowptr not monotone / not ending at nnz, or column out of range)");
  if (hf[0] & 1) fail(HPRQP_ERR_BOUNDS, "invalid bounds (l > u, L > U, NaN, wrong-sided infinity) or non-finite data");
  if (m > 0) h.A = Mat{m, n, P->a_rowptr, P->a_col, P->a_val, P->a_nnz, default_G(P->a_nnz, m, hf[1], n)};
  if (P->qkind == HPRQP_Q_CSR) h.Q = Mat{n, n, P->q_rowptr, P->q_col, P->q_val, P->q_nnz, default_G(P->q_nnz, n, hf[2], n)};
  if (P->qkind == HPRQP_Q_KRON) {
    h.kp = P->kron_p; h.ks = P->kron_s; h.kB = P->kron_B; h.kC = P->kron_C; h.kS = P->kron_S; h.kT = P->kron_T;
    h.kron_mode = 0;
  }
  if (P->qkind == HPRQP_Q_LOWRANK) { h.lr_r = P->lr_rank; h.lr_d = P->lr_d; h.lr_F = P->lr_F; }
  if (P->qkind == HPRQP_Q_GRAM)
    h.G = Mat{P->gram_p, n, P->gram_rowptr, P->gram_col, P->gram_val, P->gram_nnz,
              default_G(P->gram_nnz, P->gram_p, hf[3], n)};
  // norms of b and c (denominators of eta_p, eta_d)
  if (m > 0) launch_elem(h, m, nullptr, EpiNormB{P->l, P->u}, 0, red_seq(h, SL_NRM, 2));
  launch_elem(h, n, nullptr, EpiNormC{P->c}, 0, red_seq(h, SL_NRM + 2, 2));
  // A^T y, then A x with the primal part, Q x with the dual part
  if (m > 0) {
    k_fill<<<hq_grid(n, 256), 256, 0, st>>>(n, g, 0.0);
    if (P->a_nnz > 0)
      k_csr_t_scatter<<<hq_grid(P->a_nnz, 256), 256, 0, st>>>(m, P->a_nnz, P->a_rowptr, P->a_col, P->a_val, y, g);
    launch_csr(h, h.A, x, EpiResA{P->l, P->u, y, nullptr}, 0, red_seq(h, SL_RA, 4));
  }
  noalloc_q(h, x, EpiResQ{x, z, g, P->c, P->L, P->U, nullptr, nullptr, nullptr, h.l1}, red_seq(h, SL_RQ, 7), tp, tq);
  if (w) {
    k_diff<<<hq_grid(n, 256), 256, 0, st>>>(n, w, x, nullptr, d);
    noalloc_q(h, d, EpiMaxAbs{nullptr}, red_seq(h, SL_QWX, 1), tp, tq);
  }
  final_reduce(h, 0, SL_TOTAL);
  double hs[64];
  HQC(hipMemcpyAsync(hs, h.scalars, SL_TOTAL * sizeof(double), hipMemcpyDeviceToHost, st));
  HQC(hipStreamSynchronize(st));
  h.binf = m > 0 ? hs[SL_NRM + 1] : 0.0;
  h.cinf = hs[SL_NRM + 3];
  const Resid r = residuals_from(h, hs);
  std::memset(info, 0, sizeof(*info));
  info->eta_p = r.eta_p; info->eta_d = r.eta_d; info->eta_gap = r.eta_gap; info->pobj = r.pobj; info->dobj = r.dobj;
  info->qwx_gap = w ? hs[SL_QWX] : std::numeric_limits<double>::quiet_NaN();
}

}  // namespace hq

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
#define HQ_GUARD(...)                                    \
  try {                                                  \
    hq::g_err.clear();                                   \
    __VA_ARGS__;                                         \
    return HPRQP_OK;                                     \
  } catch (const hq::Error& e) {                         \
    hq::g_err = e.msg;                                   \
    return e.st;                                         \
  } catch (const std::exception& e) {                    \
    hq::g_err = e.what();                                \
    return HPRQP_ERR_HIP;                                \
  }

extern "C" {

void hprqp_default_options(hprqp_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-8;
  o->max_iter = 1000000;
  o->time_limit_s = 3600.0;
  o->check_every = 100;
  o->alpha1 = 0.2; o->alpha2 = 0.8; o->alpha3 = 0.5;
  o->enable_restart = 1;
  o->enable_sigma_update = 1;
  o->use_graph = 1;
  o->spmv_autotune = 0;
  o->precondition = 0;
  o->ruiz_iters = 10;
  o->spmv_lanes = -1;
  o->method = 0;
  o->kron_kernel = -1;
  o->small_path = -1;
  o->batch_threads = 0;
}

hprqp_status hprqp_create(const hprqp_problem* prob, const hprqp_options* opt, hipStream_t stream,
                          hprqp_handle** out) {
  HQ_GUARD(hq::create_impl(prob, opt, stream, out));
}

hprqp_status hprqp_solve(hprqp_handle* h, const double* y0, const double* w0, const double* x0, double* y, double* z,
                         double* w, double* x, hprqp_info* info) {
  HQ_GUARD(if (!h) hq::fail(HPRQP_ERR_ARG, "NULL handle");
           if (h->opt.method == 0) hq::solve_impl(*h, y0, w0, x0, y, z, w, x, info);
           else hq::solve_primal_impl(*h, y0, w0, x0, y, z, w, x, info));
}

hprqp_status hprqp_solve_resume(hprqp_handle* h, const hprqp_state* resume, hprqp_state* save, double* y, double* z,
                                double* w, double* x, hprqp_info* info) {
  HQ_GUARD(if (!h) hq::fail(HPRQP_ERR_ARG, "NULL handle");
           if (h->opt.method != 0) hq::fail(HPRQP_ERR_UNSUPPORTED, "resume: method 0 (HPR-QP) only");
           hq::solve_impl(*h, nullptr, nullptr, nullptr, y, z, w, x, info, resume, save));
}

hprqp_status hprqp_residuals(hprqp_handle* h, const double* y, const double* z, const double* w, const double* x,
                             hprqp_info* info_host) {
  HQ_GUARD(if (!h) hq::fail(HPRQP_ERR_ARG, "NULL handle"); hq::residuals_impl(*h, y, z, w, x, info_host));
}

hprqp_status hprqp_residuals_noalloc(const hprqp_problem* prob, const double* y, const double* z, const double* w,
                                     const double* x, hprqp_info* info_host, hipStream_t stream) {
  HQ_GUARD(hq::residuals_noalloc_impl(prob, y, z, w, x, info_host, stream));
}

hprqp_status hprqp_apply(hprqp_handle* h, int32_t op, const double* in, double* out) {
  HQ_GUARD(if (!h) hq::fail(HPRQP_ERR_ARG, "NULL handle"); hq::apply_impl(*h, op, in, out));
}

hprqp_status hprqp_power_info(hprqp_handle* h, double* est_A, int32_t* it_A, double* est_Q, int32_t* it_Q) {
  HQ_GUARD(if (!h) hq::fail(HPRQP_ERR_ARG, "NULL handle"); if (est_A) *est_A = h->powA_est;
           if (it_A) *it_A = h->powA_it; if (est_Q) *est_Q = h->powQ_est; if (it_Q) *it_Q = h->powQ_it);
}

hprqp_status hprqp_set_options(hprqp_handle* h, const hprqp_options* opt) {
  HQ_GUARD(
      if (!h || !opt) hq::fail(HPRQP_ERR_ARG, "NULL argument");
      if (opt->check_every <= 0 || opt->max_iter <= 0 || !(opt->tol >= 0.0)) hq::fail(HPRQP_ERR_ARG, "bad options");
      if (opt->method < 0 || opt->method > 2) hq::fail(HPRQP_ERR_ARG, "method must be 0, 1 or 2");
      if (opt->profile_kernels && !h->pev[0][0][0])
        for (auto& a : h->pev)
          for (auto& b : a)
            for (auto& e : b) HQC(hipEventCreate(&e));
      // setup-time choices (lambda's, sigma0, power start, autotune, preconditioning) keep their values
      const double la = h->opt.lambda_A, lq = h->opt.lambda_Q, s0 = h->opt.sigma0;
      const double *pa = h->opt.power_start_A, *pq = h->opt.power_start_Q;
      const int at = h->opt.spmv_autotune, pc = h->opt.precondition, ri = h->opt.ruiz_iters;
      const int kk = h->opt.kron_kernel, sp = h->opt.small_path;
      // the captured segment depends on the options (length, timing events): capture again
      if (h->gexec) { hipGraphExecDestroy(h->gexec); h->gexec = nullptr; }
      if (h->graph) { hipGraphDestroy(h->graph); h->graph = nullptr; }
      h->graph_T = 0;
      if (h->pgexec) { hipGraphExecDestroy(h->pgexec); h->pgexec = nullptr; }
      if (h->pgraph) { hipGraphDestroy(h->pgraph); h->pgraph = nullptr; }
      h->pgraph_T = 0;
      h->opt = *opt;
      h->opt.lambda_A = la; h->opt.lambda_Q = lq; h->opt.sigma0 = s0;
      h->opt.power_start_A = pa; h->opt.power_start_Q = pq; h->opt.spmv_autotune = at;
      h->opt.precondition = pc; h->opt.ruiz_iters = ri; h->opt.kron_kernel = kk; h->opt.small_path = sp);
}

hprqp_status hprqp_scaling(hprqp_handle* h, double* D, double* E) {
  HQ_GUARD(if (!h) hq::fail(HPRQP_ERR_ARG, "NULL handle");
           if (D) {
             if (h->pre) HQC(hipMemcpyAsync(D, h->Ds, h->n * sizeof(double), hipMemcpyDeviceToDevice, h->st));
             else k_fill<<<hq_grid(h->n, 256), 256, 0, h->st>>>(h->n, D, 1.0);
           }
           if (E && h->m > 0) {
             if (h->pre) HQC(hipMemcpyAsync(E, h->Es, h->m * sizeof(double), hipMemcpyDeviceToDevice, h->st));
             else k_fill<<<hq_grid(h->m, 256), 256, 0, h->st>>>(h->m, E, 1.0);
           }
           HQC(hipStreamSynchronize(h->st)));
}

hprqp_status hprqp_kernel_stats(hprqp_handle* h, double* avg_ms, int64_t* launches, int32_t* g) {
  HQ_GUARD(if (!h || !avg_ms || !launches) hq::fail(HPRQP_ERR_ARG, "NULL argument");
           for (int k = 0; k < 4; ++k) {
             launches[k] = h->prof_n[k];
             avg_ms[k] = h->prof_n[k] ? h->prof_ms[k] / (double)h->prof_n[k] : 0.0;
           } if (g) { g[0] = h->A.G; g[1] = h->AT.G; g[2] = h->Q.G; });
}

void hprqp_destroy(hprqp_handle* h) { delete h; }

}  // extern "C"
