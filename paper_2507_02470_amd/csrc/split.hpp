// split.hpp -- column-split CSR products for matrices with few, long rows
// over a vector too large for LDS (the Lasso's Ahat: p rows of thousands of
// nonzeros, q >> p columns).
//
// A row-split kernel gathers every nonzero's x entry through the L2 at the
// rate of its random 8-byte requests.  Here the columns are cut into panels
// of pw columns and the matrix is stored panel by panel, each panel
// a CSR over all rows (rows in order, a row's entries in their CSR order,
// columns as 16-bit offsets into the panel).  A workgroup owns one panel and a
// block of rows: it copies the panel's slice of x into LDS once, gathers from
// there, and writes one partial sum per row and panel; a second kernel adds a
// row's partials in panel order (four fixed segments, combined in a fixed
// order) and runs the epilogue.  Deterministic: inside a panel a row's
// entries are added in CSR order, then the panels' sums as stated.
#pragma once
#include "common.hpp"

#define HQ_SPLIT_PW 2048        // columns per panel, denser matrices (16 KB of LDS)
#define HQ_SPLIT_PW_WIDE 16384  // columns per panel, sparser ones (128 KB of LDS)
#define HQ_SPLIT_RED_ROWS 64    // rows per workgroup of the reduction
#define HQ_SPLIT_ROWS 1024      // rows per pass of a workgroup

struct SplitMat {
  int rows = 0, cols = 0;
  int pw = HQ_SPLIT_PW;              // columns per panel
  int np = 0;                        // panels
  int rpb = 0, nrb = 0;              // rows per workgroup (a multiple of HQ_SPLIT_ROWS), row blocks per panel
  const int* off = nullptr;          // np * rows + 1 starts: panel p, row r at off[p * rows + r]
  const unsigned short* lci = nullptr;   // column - p * pw
  const double* v = nullptr;
  double* partial = nullptr;         // np * rows partial sums
};

// The layout is built by two per-row steps, run by one thread per row on the
// device and by the host layout test on the CPU.
//
// Step 1, row r: how many of its nonzeros fall in each panel,
// cnt[p * rows + r] (zeroed beforehand).  Consecutive entries of one panel
// are counted together.
__host__ __device__ inline void split_count_row(int r, int rows, int pw, const int* rp, const int* ci, int* cnt) {
  int p = -1, run = 0;
  for (int k = rp[r]; k < rp[r + 1]; ++k) {
    const int q = ci[k] / pw;
    if (q != p) {
      if (run) cnt[(size_t)p * rows + r] += run;
      p = q;
      run = 0;
    }
    ++run;
  }
  if (run) cnt[(size_t)p * rows + r] += run;
}

// Step 2, row r: its entries into their panels in CSR order; cur holds the
// next free position of every (panel, row), initialised to the starts off.
__host__ __device__ inline void split_scatter_row(int r, int rows, int pw, const int* rp, const int* ci,
                                                  const double* v, int* cur, unsigned short* lci, double* sv) {
  int p = -1, pos = 0;
  for (int k = rp[r]; k < rp[r + 1]; ++k) {
    const int q = ci[k] / pw;
    if (q != p) {
      if (p >= 0) cur[(size_t)p * rows + r] = pos;
      p = q;
      pos = cur[(size_t)p * rows + r];
    }
    lci[pos] = (unsigned short)(ci[k] - q * pw);
    sv[pos] = v[k];
    ++pos;
  }
  if (p >= 0) cur[(size_t)p * rows + r] = pos;
}

__global__ void k_split_count(int rows, int pw, const int* __restrict__ rp, const int* __restrict__ ci, int* cnt) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x)
    split_count_row(r, rows, pw, rp, ci, cnt);
}

__global__ void k_split_scatter(int rows, int pw, const int* __restrict__ rp, const int* __restrict__ ci,
                                const double* __restrict__ v, int* cur, unsigned short* lci, double* sv) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x)
    split_scatter_row(r, rows, pw, rp, ci, v, cur, lci, sv);
}

// Partial sums: workgroup b takes panel b % np and the rpb rows of row block
// b / np, HQ_SPLIT_ROWS at a time.  Inside a panel the rows are short (a few
// to tens of nonzeros), so each pass's entries -- one contiguous range of the
// layout -- are streamed as by the CSR-stream kernel: coalesced loads,
// products staged in LDS, then every thread adds up its rows' products in
// order.  The loads run one step ahead: a chunk's entries are fetched while the
// previous chunk is summed (the first chunk of the next pass during the last of
// this one), and the next pass's row starts during this pass.  BS = 256 for
// the narrow panels (several workgroups per CU), 1024 for the wide ones (one
// workgroup per CU, its 128 KB copy of x in LDS).
template <int BS>
__global__ __launch_bounds__(BS) void k_split_partial(SplitMat S, const double* __restrict__ x) {
  static_assert(HQ_SPLIT_ROWS % BS == 0, "rows per pass");
  constexpr int RPT = HQ_SPLIT_ROWS / BS;   // rows per thread and pass
  constexpr int CH = 2048;                  // products staged per step
  constexpr int E = CH / BS;                // entries per thread and step
  extern __shared__ double xs[];            // S.pw entries
  __shared__ double prod[CH];
  __shared__ int srp[HQ_SPLIT_ROWS + 1];
  const int t = threadIdx.x;
  const int p = blockIdx.x % S.np, rb = blockIdx.x / S.np;
  const int rbeg = rb * S.rpb, rend = min(S.rows, rbeg + S.rpb);
  if (rbeg >= rend) return;                 // (the whole workgroup)
  const int cx = p * S.pw, nc = min(S.pw, S.cols - cx);
  const int* __restrict__ offp = S.off + (size_t)p * S.rows;
  double* __restrict__ part = S.partial + (size_t)p * S.rows;
  // row starts of the pass from row r (rows r .. r + n - 1, and the end)
  int sr[RPT], sr_end;
  auto load_starts = [&](int r, int n) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) sr[q] = t + q * BS < n ? offp[r + t + q * BS] : 0;
    sr_end = offp[r + n];   // (the next row's start, or the next panel's first)
  };
  auto store_starts = [&](int n) {
#pragma unroll
    for (int q = 0; q < RPT; ++q)
      if (t + q * BS < n) srp[t + q * BS] = sr[q];
    if (t == 0) srp[n] = sr_end;
  };
  // the entries [a, b) of one step, E per thread
  int ci[E];
  double v[E];
  auto fetch = [&](int a, int b) {
#pragma unroll
    for (int u = 0; u < E; ++u) {
      const int k = a + t + u * BS;
      ci[u] = k < b ? (int)ld_stream(S.lci + k) : 0;
      v[u] = k < b ? ld_stream(S.v + k) : 0.0;
    }
  };
  int r0 = rbeg, nr = min(HQ_SPLIT_ROWS, rend - r0);
  load_starts(r0, nr);
  for (int i = t; i < nc; i += BS) xs[i] = x[cx + i];
  store_starts(nr);
  __syncthreads();
  int kb = srp[0], ke = srp[nr];
  fetch(kb, min(ke, kb + CH));
  for (;;) {   // passes; the same trip counts in every thread
    const int r1 = r0 + HQ_SPLIT_ROWS;
    const bool more = r1 < rend;
    const int nr1 = more ? min(HQ_SPLIT_ROWS, rend - r1) : 0;
    if (more) load_starts(r1, nr1);
    double sum[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) sum[q] = 0.0;
    for (int c0 = kb; c0 < ke; c0 += CH) {
      const int c1 = min(ke, c0 + CH);
      int cc[E];
      double cv[E];
#pragma unroll
      for (int u = 0; u < E; ++u) { cc[u] = ci[u]; cv[u] = v[u]; }
      if (c1 < ke) fetch(c1, min(ke, c1 + CH));
      else if (more) fetch(ke, min(sr_end, ke + CH));   // the next pass's first step
#pragma unroll
      for (int u = 0; u < E; ++u)
        if (c0 + t + u * BS < c1) prod[t + u * BS] = cv[u] * xs[cc[u]];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int i = t + q * BS;
        if (i < nr) {
          const int lo = max(srp[i], c0), hi = min(srp[i + 1], c1);
          for (int k = lo; k < hi; ++k) sum[q] += prod[k - c0];
        }
      }
      __syncthreads();   // prod is rewritten by the next step
    }
    if (kb == ke && more) fetch(ke, min(sr_end, ke + CH));   // a pass without entries fetched nothing
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int i = t + q * BS;
      if (i < nr) part[r0 + i] = sum[q];
    }
    if (!more) break;
    __syncthreads();     // every thread has read this pass's row starts
    store_starts(nr1);
    __syncthreads();
    r0 = r1; nr = nr1; kb = ke; ke = srp[nr];
  }
}

// Row sums from the partials (panel order: four segments of the panel range,
// each added in order, then combined as ((s0 + s1) + s2) + s3), and the
// epilogue.  Workgroups take groups of HQ_SPLIT_RED_ROWS rows in grid-stride
// order (the grid is capped, so a reduction's partials fit their slots).
template <class Epi>
__global__ __launch_bounds__(4 * HQ_SPLIT_RED_ROWS) void k_split_reduce(int rows, int np,
                                                                        const double* __restrict__ partial, Epi epi,
                                                                        const DevParams* __restrict__ prm, int j,
                                                                        RedOut red) {
  constexpr int NR = Epi::NR;
  __shared__ double seg_sum[4][HQ_SPLIT_RED_ROWS];
  const int lr = threadIdx.x % HQ_SPLIT_RED_ROWS, seg = threadIdx.x / HQ_SPLIT_RED_ROWS;
  const int p0 = (int)((long long)seg * np / 4), p1 = (int)((long long)(seg + 1) * np / 4);
  Epi e = epi;
  e.setup(prm, j);
  double acc[NR > 0 ? NR : 1];
#pragma unroll
  for (int q = 0; q < (NR > 0 ? NR : 1); ++q) acc[q] = 0.0;
  const int groups = (rows + HQ_SPLIT_RED_ROWS - 1) / HQ_SPLIT_RED_ROWS;
  for (int g = blockIdx.x; g < groups; g += gridDim.x) {   // same trip count in every thread
    const int row = g * HQ_SPLIT_RED_ROWS + lr;
    double s = 0.0;
    if (row < rows) {
#pragma unroll 4
      for (int p = p0; p < p1; ++p) s += partial[(size_t)p * rows + row];
    }
    seg_sum[seg][lr] = s;
    __syncthreads();
    if (seg == 0 && row < rows) {
      const double t = ((seg_sum[0][lr] + seg_sum[1][lr]) + seg_sum[2][lr]) + seg_sum[3][lr];
      e(row, t, acc);
    }
    __syncthreads();   // seg_sum is rewritten by the next group
  }
  if (red.active) block_reduce_store<NR, Epi::MAXMASK>(acc, red);
}
