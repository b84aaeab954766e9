// qops.hpp -- matrix-free Q products: Kronecker (FP64 MFMA) and diag + low rank.
#pragma once
#include "common.hpp"

typedef double hq_dx4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// D (M x N) = A (M x K, col-major, lda) * op(B); op(B)[k][j] = B[k + ldb j]
// (TRANSB = false) or B[j + ldb k] (TRANSB = true).  Output element (i, j)
// goes to the epilogue as vector index i + ldo j.
//
// One 16 x 16 output tile per block of HQ_KSPLIT waves; the waves split K
// into HQ_KSPLIT ranges, each accumulating with v_mfma_f64_16x16x4f64, and
// the partial tiles are summed in LDS in a fixed order (deterministic).  A
// short K range per wave keeps the chain of loads and MFMAs short:
// at these sizes (d ~ 300) the product is latency-bound, not MFMA-bound.
// Operand layout of the 16x16x4 f64 MFMA (measured on gfx950): lane l
// supplies A[l%16][l/16] and B[l/16][l%16]; accumulator register v of lane l
// holds D[l/16 + 4v][l%16], v = 0..3.
// ---------------------------------------------------------------------------
//
// EXTRA: up to two more terms sign_t * A_t op_t(B_t) (same M x N output, own
// K_t, lda, ldb, transpose flag) are added to the same accumulator; their
// k-steps follow those of the main term, and the waves split all of them.
// Used for the QAP-relaxation operator C X B^T - X T^T - S X.
#define HQ_KSPLIT 8
#define HQ_KUNROLL 5
struct GemmTerms {
  const double* A[2];
  const double* B[2];
  int lda[2], ldb[2], K[2], transb[2];
  double sign[2];
  int nt;   // extra terms used (0..2)
};
template <bool TRANSB, class Epi, bool EXTRA = false>
__global__ __launch_bounds__(64 * HQ_KSPLIT) void k_dgemm16(int M, int N, int K, const double* __restrict__ A, int lda,
                                                            const double* __restrict__ B, int ldb, int ldo, Epi epi,
                                                            const DevParams* __restrict__ prm, int jit, RedOut red,
                                                            GemmTerms ex = GemmTerms{}) {
  constexpr int NR = Epi::NR;
  __shared__ double part[HQ_KSPLIT][16][17];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tiles_m = (M + 15) >> 4, tiles_n = (N + 15) >> 4;
  const int ks_main = (K + 3) >> 2;
  int ksteps = ks_main;
  int ks_t1 = 0;   // first k-step of the second extra term
  if constexpr (EXTRA) {
    const int k0 = ex.nt > 0 ? (ex.K[0] + 3) >> 2 : 0, k1 = ex.nt > 1 ? (ex.K[1] + 3) >> 2 : 0;
    ks_t1 = ks_main + k0;
    ksteps = ks_t1 + k1;
  }
  const int per = (ksteps + HQ_KSPLIT - 1) / HQ_KSPLIT;
  const int ks0 = wv * per;
  const int ks1 = (ks0 + per < ksteps) ? ks0 + per : ksteps;
  Epi e = epi;
  e.setup(prm, jit);
  double acc[NR > 0 ? NR : 1];
#pragma unroll
  for (int s = 0; s < (NR > 0 ? NR : 1); ++s) acc[s] = 0.0;
  for (int tile = blockIdx.x; tile < tiles_m * tiles_n; tile += gridDim.x) {
    const int i0 = (tile % tiles_m) << 4, j0 = (tile / tiles_m) << 4;
    const int ia = i0 + li, jb = j0 + li;
    hq_dx4 d = {0.0, 0.0, 0.0, 0.0};
    // the operands of HQ_KUNROLL k-steps are loaded first (all in flight at
    // once: the MFMA chain would otherwise wait a full load latency per
    // step), then multiplied; out-of-range operands are read from a clamped
    // index and replaced by 0
    for (int kc = ks0; kc < ks1; kc += HQ_KUNROLL) {
      double av[HQ_KUNROLL], bv[HQ_KUNROLL];
#pragma unroll
      for (int u = 0; u < HQ_KUNROLL; ++u) {
        const int ks = kc + u;
        const int ic = ia < M ? ia : M - 1, jc = jb < N ? jb : N - 1;
        if (!EXTRA || ks < ks_main) {
          const int k = (ks << 2) + lk;
          const bool kin = ks < ks1 && k < K;
          const int kk = kin ? k : 0;
          const double a = A[ic + (size_t)lda * kk];
          const double b = TRANSB ? B[jc + (size_t)ldb * kk] : B[kk + (size_t)ldb * jc];
          av[u] = (ia < M && kin) ? a : 0.0;
          bv[u] = (jb < N && kin) ? b : 0.0;
        } else if (ks >= ks1) {
          av[u] = 0.0;
          bv[u] = 0.0;
        } else {
          // extra term t (a wave-uniform choice; t = 1 only when two are given)
          const int t = ks < ks_t1 ? 0 : 1;
          const int k = ((ks - (t ? ks_t1 : ks_main)) << 2) + lk;
          const bool kin = ks < ks1 && k < ex.K[t];
          const int kk = kin ? k : 0;
          const double a = ex.A[t][ic + (size_t)ex.lda[t] * kk];
          const double b = ex.transb[t] ? ex.B[t][jc + (size_t)ex.ldb[t] * kk] : ex.B[t][kk + (size_t)ex.ldb[t] * jc];
          av[u] = (ia < M && kin) ? a : 0.0;
          bv[u] = (jb < N && kin) ? ex.sign[t] * b : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < HQ_KUNROLL; ++u) d = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], d, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) part[wv][lk + 4 * v][li] = d[v];
    __syncthreads();
    if (threadIdx.x < 256) {
      const int r = threadIdx.x & 15, cc = threadIdx.x >> 4;
      double q = part[0][r][cc];
#pragma unroll
      for (int w = 1; w < HQ_KSPLIT; ++w) q += part[w][r][cc];
      const int gi = i0 + r, gj = j0 + cc;
      if (gi < M && gj < N) e(gi + ldo * gj, q, acc);
    }
    __syncthreads();
  }
  if (red.active) block_reduce_store<NR, Epi::MAXMASK>(acc, red);
}

// ---------------------------------------------------------------------------
// Q = diag(d) + F F^T, F n x r row-major (r <= 16).
// Stage 1: per-block partial sums of t = F^T x (slots red.slot[0..r-1]).
// Stage 2 (after the final reduction): (Q x)_i = d_i x_i + sum_k F_ik t_k.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(HQ_BLOCK) void k_lr_partial(int n, int r, const double* __restrict__ F,
                                                         const double* __restrict__ x, RedOut red) {
  double acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  for (long long i = (long long)blockIdx.x * HQ_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * HQ_BLOCK) {
    const double xi = x[i];
    const double* Fi = F + (size_t)i * r;
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (k < r) acc[k] += Fi[k] * xi;
  }
  block_reduce_store<16, 0u>(acc, red);
}

template <class Epi>
__global__ __launch_bounds__(HQ_BLOCK) void k_lr_apply(int n, int r, const double* __restrict__ dg,
                                                       const double* __restrict__ F,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ t, Epi epi,
                                                       const DevParams* __restrict__ prm, int jit, RedOut red) {
  constexpr int NR = Epi::NR;
  Epi e = epi;
  e.setup(prm, jit);
  double acc[NR > 0 ? NR : 1];
#pragma unroll
  for (int s = 0; s < (NR > 0 ? NR : 1); ++s) acc[s] = 0.0;
  double tk[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) tk[k] = (k < r) ? t[k] : 0.0;
  for (long long i = (long long)blockIdx.x * HQ_BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * HQ_BLOCK) {
    const double* Fi = F + (size_t)i * r;
    double q = dg[i] * x[i];
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (k < r) q += Fi[k] * tk[k];
    e((int)i, q, acc);
  }
  if (red.active) block_reduce_store<NR, Epi::MAXMASK>(acc, red);
}
