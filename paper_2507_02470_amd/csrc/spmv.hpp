// spmv.hpp -- CSR SpMV kernels for gfx950 with a fused per-row epilogue.
#pragma once
#include "common.hpp"

// Row-split kernel for long rows: groups of G lanes each own one row (a
// block covers HQ_BLOCK / G rows per pass); the lanes stride over the row's
// nonzeros, the group's partial sums are added by a butterfly (G <= 64) or by
// wave sums combined in LDS in wave order (G = 128, 256: one row spans 2 or 4
// waves), and the group's first lane runs the epilogue.  Rows are dealt out
// in grid-stride order, so a matrix with a few hundred long rows still
// spreads over hundreds of waves.  No atomics; the summation order depends
// only on G.
template <int G, class Epi>
__global__ __launch_bounds__(HQ_BLOCK) void k_csr(int nrows, const int* __restrict__ rowptr,
                                                  const int* __restrict__ col,
                                                  const double* __restrict__ val,
                                                  const double* __restrict__ xin, Epi epi,
                                                  const DevParams* __restrict__ prm, int j, RedOut red) {
  static_assert(G >= 1 && G <= HQ_BLOCK && (HQ_BLOCK % G) == 0, "lanes per row");
  constexpr int RPB = HQ_BLOCK / G;  // rows per block per pass
  constexpr int NR = Epi::NR;
  const int gl = threadIdx.x % G;
  const int gi = threadIdx.x / G;
  Epi e = epi;
  e.setup(prm, j);
  double acc[NR > 0 ? NR : 1];
#pragma unroll
  for (int s = 0; s < (NR > 0 ? NR : 1); ++s) acc[s] = 0.0;
  for (long long r0 = (long long)blockIdx.x * RPB; r0 < nrows; r0 += (long long)gridDim.x * RPB) {
    const long long row = r0 + gi;
    double sum = 0.0;
    if (row < nrows) {
      const int b = rowptr[row], en = rowptr[row + 1];
#pragma unroll 4
      for (int k = b + gl; k < en; k += G) sum += ld_stream(val + k) * xin[ld_stream(col + k)];
    }
    if constexpr (G > 64) {
      __shared__ double wpart[HQ_BLOCK / HQ_WAVE];
      sum = wave_sum(sum);
      if ((threadIdx.x & (HQ_WAVE - 1)) == 0) wpart[threadIdx.x / HQ_WAVE] = sum;
      __syncthreads();
      if (gl == 0) {
        const int w0 = (gi * G) / HQ_WAVE;
        sum = wpart[w0];
#pragma unroll
        for (int w = 1; w < G / HQ_WAVE; ++w) sum += wpart[w0 + w];
      }
      __syncthreads();   // wpart is rewritten by the next pass
    } else if constexpr (G > 1) {
      sum = group_sum<G>(sum);
    }
    if (row < nrows && gl == 0) e((int)row, sum, acc);
  }
  if (red.active) block_reduce_store<NR, Epi::MAXMASK>(acc, red);
}

// CSR-stream SpMV for short rows.  A block owns HQ_BLOCK consecutive rows; the
// nonzeros of those rows (a contiguous range of the CSR arrays) are streamed
// in chunks of HQ_STREAM_CHUNK with fully coalesced loads, each thread forming
// val[k] * x[col[k]] for k = c0 + tid, c0 + tid + HQ_BLOCK, ... into LDS; then
// thread t adds up row t's products in CSR order (a fixed summation order)
// and runs the epilogue for that row.  Loads of the matrix and of the
// gathered vector are independent of the row structure, which keeps many
// gathers in flight per wave.
//
// XLDS: the whole input vector (ncols entries) is first copied into LDS
// (dynamic shared memory) and gathered from there: for vectors that fit
// (up to HQ_XLDS_MAX entries) the gathers then cost no L2 requests.  The grid
// is persistent (a few blocks per CU), so the copy is made once per block.
// BS: threads (= rows) per block; the chunk is 2048 products (4096 for
// 1024-thread blocks, keeping 32 KB of LDS beside the vector's copy).
#define HQ_STREAM_CHUNK 2048
#define HQ_XLDS_MAX 14336
#define HQ_XLDS_BLOCK 1024
template <class Epi, bool XLDS = false, int BS = HQ_BLOCK>
__global__ __launch_bounds__(BS) void k_csr_stream(int nrows, const int* __restrict__ rowptr,
                                                   const int* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ xin, Epi epi,
                                                   const DevParams* __restrict__ prm, int j, RedOut red,
                                                   int ncols = 0) {
  constexpr int NR = Epi::NR;
  constexpr int CH = BS > HQ_BLOCK ? 2 * HQ_STREAM_CHUNK : HQ_STREAM_CHUNK;
  __shared__ double prod[CH];
  __shared__ int srp[BS + 1];
  extern __shared__ double xs[];
  Epi e = epi;
  e.setup(prm, j);
  double acc[NR > 0 ? NR : 1];
#pragma unroll
  for (int s = 0; s < (NR > 0 ? NR : 1); ++s) acc[s] = 0.0;
  const int t = threadIdx.x;
  if constexpr (XLDS) {
    for (int i = t; i < ncols; i += BS) xs[i] = xin[i];
    __syncthreads();
  }
  const double* xg = XLDS ? xs : xin;
  const int nblk = (nrows + BS - 1) / BS;
  for (int rb = blockIdx.x; rb < nblk; rb += gridDim.x) {
    const int r0 = rb * BS;
    const int nr = min(BS, nrows - r0);
    for (int i = t; i <= nr; i += BS) srp[i] = rowptr[r0 + i];   // nr + 1 row pointers
    __syncthreads();
    const int kb = srp[0], ke = srp[nr];
    const int myb = t < nr ? srp[t] : 0, mye = t < nr ? srp[t + 1] : 0;
    double sum = 0.0;
    for (int c0 = kb; c0 < ke; c0 += CH) {
      const int c1 = min(ke, c0 + CH);
#pragma unroll 4
      for (int k = c0 + t; k < c1; k += BS) prod[k - c0] = ld_stream(val + k) * xg[ld_stream(col + k)];
      __syncthreads();
      const int lo = max(myb, c0), hi = min(mye, c1);
      for (int k = lo; k < hi; ++k) sum += prod[k - c0];
      __syncthreads();
    }
    if (t < nr) e(r0 + t, sum, acc);
    __syncthreads();   // srp is rewritten by the next row block
  }
  if (red.active) block_reduce_store<NR, Epi::MAXMASK>(acc, red);
}

// Row-split kernel (as k_csr, G <= 64 lanes per row) gathering from an LDS
// copy of the input vector (at most HQ_XLDS_MAX entries): for rows of tens to
// hundreds of nonzeros over a small vector (the Lasso's Ahat^T, p columns),
// where the stream kernel would add each long row serially.  Persistent
// 1024-thread blocks copy the vector once, then take rows in grid-stride
// order; the summation order is that of k_csr<G>.
template <int G, class Epi>
__global__ __launch_bounds__(HQ_XLDS_BLOCK) void k_csr_xrow(int nrows, const int* __restrict__ rowptr,
                                                            const int* __restrict__ col,
                                                            const double* __restrict__ val,
                                                            const double* __restrict__ xin, Epi epi,
                                                            const DevParams* __restrict__ prm, int j, RedOut red,
                                                            int ncols) {
  static_assert(G >= 1 && G <= HQ_WAVE && (HQ_WAVE % G) == 0, "lanes per row");
  constexpr int BS = HQ_XLDS_BLOCK;
  constexpr int RPB = BS / G;
  constexpr int NR = Epi::NR;
  extern __shared__ double xs[];
  const int gl = threadIdx.x % G;
  const int gi = threadIdx.x / G;
  Epi e = epi;
  e.setup(prm, j);
  double acc[NR > 0 ? NR : 1];
#pragma unroll
  for (int s = 0; s < (NR > 0 ? NR : 1); ++s) acc[s] = 0.0;
  for (int i = threadIdx.x; i < ncols; i += BS) xs[i] = xin[i];
  __syncthreads();
  for (long long r0 = (long long)blockIdx.x * RPB; r0 < nrows; r0 += (long long)gridDim.x * RPB) {
    const long long row = r0 + gi;
    double sum = 0.0;
    if (row < nrows) {
      const int b = rowptr[row], en = rowptr[row + 1];
#pragma unroll 4
      for (int k = b + gl; k < en; k += G) sum += ld_stream(val + k) * xs[ld_stream(col + k)];
    }
    if constexpr (G > 1) sum = group_sum<G>(sum);
    if (row < nrows && gl == 0) e((int)row, sum, acc);
  }
  if (red.active) block_reduce_store<NR, Epi::MAXMASK>(acc, red);
}

// Elementwise driver: epi(i, q_i) with a precomputed / zero q.
template <class Epi>
__global__ __launch_bounds__(HQ_BLOCK) void k_elem(int n, const double* __restrict__ q, Epi epi,
                                                   const DevParams* __restrict__ prm, int j, RedOut red) {
  constexpr int NR = Epi::NR;
  Epi e = epi;
  e.setup(prm, j);
  double acc[NR > 0 ? NR : 1];
#pragma unroll
  for (int s = 0; s < (NR > 0 ? NR : 1); ++s) acc[s] = 0.0;
  for (long long i = (long long)blockIdx.x * HQ_BLOCK + threadIdx.x; i < n;
       i += (long long)gridDim.x * HQ_BLOCK)
    e((int)i, q ? q[i] : 0.0, acc);
  if (red.active) block_reduce_store<NR, Epi::MAXMASK>(acc, red);
}
