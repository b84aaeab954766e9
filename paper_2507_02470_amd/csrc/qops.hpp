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
// LDS-tiled FP64 MFMA GEMM for large Kronecker factors (d >~ 400), same
// operation as k_dgemm16 with up to three terms:
//   D (M x N) = sum_t sign_t A_t (M x K_t, col-major) op_t(B_t).
// A block of 256 threads (4 waves, 2 x 2) owns a 64 x 64 output tile, each
// wave a 32 x 32 part (2 x 2 MFMA 16 x 16 tiles, every operand fragment used
// twice).  K runs in chunks of 16: the 64 x 16 slice of A and the 16 x 64 slice
// of op(B) are loaded with coalesced global reads into registers while the
// previous chunk is multiplied out of LDS (two LDS buffers, one barrier per
// chunk).  The MFMA is fed op(B)^T as its A operand and A^T as its B operand,
// so it produces D^T: lane l then holds rows l%16 of the tile for columns
// l/16 + 4v, and the epilogue's vector accesses (index i + ldo j) are 16
// consecutive rows per column.
// Split-K (PART): the chunks of all terms are divided among `kgroups` groups
// (grid = tiles x kgroups); group g writes its partial tile to
// parts + g * M * N and k_gemm_sum adds the groups in order and runs the
// epilogue.  Deterministic either way.
// ---------------------------------------------------------------------------
#define HQ_TB 64
#define HQ_TKC 16
#define HQ_TPITCH (HQ_TB + 2)
struct GemmOps {
  const double* A[3];
  const double* B[3];
  int lda[3], ldb[3], K[3], transb[3];
  double sign[3];
  int nt;
};

template <class Epi, bool PART>
__global__ __launch_bounds__(256) void k_dgemm_tile(int M, int N, GemmOps op, int ldo, Epi epi,
                                                    const DevParams* __restrict__ prm, int jit, RedOut red,
                                                    int kgroups, double* __restrict__ parts) {
  constexpr int NR = Epi::NR;
  __shared__ double As[2][HQ_TKC][HQ_TPITCH];
  __shared__ double Bs[2][HQ_TKC][HQ_TPITCH];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv & 1, wn = wv >> 1;
  const int li = lane & 15, lk = lane >> 4;
  const int tiles_m = (M + HQ_TB - 1) / HQ_TB, tiles_n = (N + HQ_TB - 1) / HQ_TB;
  const int tiles = tiles_m * tiles_n;
  const int n0 = (op.K[0] + HQ_TKC - 1) / HQ_TKC;
  const int n1 = op.nt > 1 ? (op.K[1] + HQ_TKC - 1) / HQ_TKC : 0;
  const int n2 = op.nt > 2 ? (op.K[2] + HQ_TKC - 1) / HQ_TKC : 0;
  const int total = n0 + n1 + n2;
  const int per = (total + kgroups - 1) / kgroups;
  Epi e = epi;
  e.setup(prm, jit);
  double acc[NR > 0 ? NR : 1];
#pragma unroll
  for (int q = 0; q < (NR > 0 ? NR : 1); ++q) acc[q] = 0.0;
  for (int w = blockIdx.x; w < tiles * kgroups; w += gridDim.x) {
    const int tile = w % tiles, grp = w / tiles;
    const int i0 = (tile % tiles_m) * HQ_TB, j0 = (tile / tiles_m) * HQ_TB;
    const int c0 = grp * per, c1 = min(total, c0 + per);
    constexpr int NQ = HQ_TKC / 4;      // loads per thread and operand per chunk
    double ra[NQ], rb[NQ];
    // global -> registers for chunk c (term t, first k k0); out-of-range -> 0
    auto load = [&](int c) {
      int t = 0, cc = c;      // chunk c -> (term t, chunk cc of that term); wave-uniform
      if (cc >= n0) { cc -= n0; t = 1; if (cc >= n1) { cc -= n1; t = 2; } }
      const int k0 = cc * HQ_TKC, Kt = op.K[t];
      const double* __restrict__ Ap = op.A[t];
      const double* __restrict__ Bp = op.B[t];
      const int lda = op.lda[t], ldb = op.ldb[t];
      const double sg = op.sign[t];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int r = tid & 63, kk = (tid >> 6) + 4 * q;
        const int gi = i0 + r, gk = k0 + kk;
        const bool ok = gi < M && gk < Kt;
        const double v = Ap[(size_t)(ok ? gi : 0) + (size_t)lda * (ok ? gk : 0)];
        ra[q] = ok ? v : 0.0;
      }
      if (op.transb[t]) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int c = tid & 63, kk = (tid >> 6) + 4 * q;
          const int gj = j0 + c, gk = k0 + kk;
          const bool ok = gj < N && gk < Kt;
          const double v = Bp[(size_t)(ok ? gj : 0) + (size_t)ldb * (ok ? gk : 0)];
          rb[q] = ok ? sg * v : 0.0;
        }
      } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int kk = tid % HQ_TKC, c = tid / HQ_TKC + (256 / HQ_TKC) * q;
          const int gj = j0 + c, gk = k0 + kk;
          const bool ok = gj < N && gk < Kt;
          const double v = Bp[(size_t)(ok ? gk : 0) + (size_t)ldb * (ok ? gj : 0)];
          rb[q] = ok ? sg * v : 0.0;
        }
      }
      return (int)op.transb[t];
    };
    auto store = [&](int buf, int tb) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) As[buf][(tid >> 6) + 4 * q][tid & 63] = ra[q];
      if (tb) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) Bs[buf][(tid >> 6) + 4 * q][tid & 63] = rb[q];
      } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) Bs[buf][tid % HQ_TKC][tid / HQ_TKC + (256 / HQ_TKC) * q] = rb[q];
      }
    };
    hq_dx4 d[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) d[a][b] = hq_dx4{0.0, 0.0, 0.0, 0.0};
    int buf = 0;
    if (c0 < c1) {
      const int tb = load(c0);
      store(0, tb);
    }
    __syncthreads();
    for (int c = c0; c < c1; ++c) {
      int tb = 0;
      if (c + 1 < c1) tb = load(c + 1);
#pragma unroll
      for (int ks = 0; ks < HQ_TKC / 4; ++ks) {
        const int kr = ks * 4 + lk;
        double fa[2], fb[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) fb[a] = As[buf][kr][wm * 32 + a * 16 + li];   // A^T: rows of D
#pragma unroll
        for (int b = 0; b < 2; ++b) fa[b] = Bs[buf][kr][wn * 32 + b * 16 + li];   // op(B)^T: columns
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) d[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[b], fb[a], d[a][b], 0, 0, 0);
      }
      if (c + 1 < c1) store(buf ^ 1, tb);
      __syncthreads();
      buf ^= 1;
    }
    // lane l holds D[i0 + wm*32 + a*16 + l%16][j0 + wn*32 + b*16 + l/16 + 4v]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int gi = i0 + wm * 32 + a * 16 + li, gj = j0 + wn * 32 + b * 16 + lk + 4 * v;
          if (gi < M && gj < N) {
            if constexpr (PART) parts[(size_t)grp * M * N + gi + (size_t)M * gj] = d[a][b][v];
            else e(gi + ldo * gj, d[a][b][v], acc);
          }
        }
  }
  if constexpr (!PART) {
    if (red.active) block_reduce_store<NR, Epi::MAXMASK>(acc, red);
  }
}

// out(i) = sum over the kgroups partial products in group order -> epilogue
template <class Epi>
__global__ __launch_bounds__(HQ_BLOCK) void k_gemm_sum(long long count, int kgroups, const double* __restrict__ parts,
                                                       Epi epi, const DevParams* __restrict__ prm, int jit,
                                                       RedOut red) {
  constexpr int NR = Epi::NR;
  Epi e = epi;
  e.setup(prm, jit);
  double acc[NR > 0 ? NR : 1];
#pragma unroll
  for (int q = 0; q < (NR > 0 ? NR : 1); ++q) acc[q] = 0.0;
  for (long long i = (long long)blockIdx.x * HQ_BLOCK + threadIdx.x; i < count; i += (long long)gridDim.x * HQ_BLOCK) {
    double q = parts[i];
    for (int g = 1; g < kgroups; ++g) q += parts[(size_t)g * count + i];
    e((int)i, q, acc);
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
