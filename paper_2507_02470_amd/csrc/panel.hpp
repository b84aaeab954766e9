// panel.hpp -- panel-ordered CSR products for matrices whose columns are
// spread at random over a large input vector.
//
// When the gathered vector is larger than an XCD's L2, about half of the
// random 8-byte gathers of a CSR product miss and each brings a 128-byte
// line.  Here the columns are cut into P panels, and the nonzeros of every
// block of HQ_BLOCK rows are stored panel by panel (rows in order inside a
// panel, local row offsets as 16-bit counts).  A persistent grid walks the
// panels in the same order in every workgroup, each workgroup owning BPB row
// blocks and keeping their row sums in registers across the panels, so at any
// time the whole GPU gathers from about one panel's slice of the vector, which
// the L2s hold.  Each chunk (row block, panel) is streamed like the
// CSR-stream kernel: coalesced loads, products staged in LDS, row sums in CSR
// order (deterministic; the order of the additions differs from the plain
// kernel only in that a row's panels are added one after the other).
#pragma once
#include <type_traits>
#include "common.hpp"

#define HQ_PANELS 4

struct PanelMat {
  int rows = 0, cols = 0;
  const int* pp = nullptr;               // chunk starts, (row blocks * P + 1)
  const unsigned short* lrp = nullptr;   // per chunk: HQ_BLOCK + 1 local row offsets
  const int* ci = nullptr;               // columns, panel order
  const double* v = nullptr;             // values, panel order
};

__device__ __forceinline__ int hq_panel_of(int col, int cols) {
  return (int)(((long long)col * HQ_PANELS) / cols);
}

// per row: how many of its nonzeros fall in each panel -> cnt[row * P + p]
__global__ void k_panel_count(int rows, int cols, const int* __restrict__ rp, const int* __restrict__ ci,
                              int* __restrict__ cnt) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) {
    int c[HQ_PANELS];
#pragma unroll
    for (int p = 0; p < HQ_PANELS; ++p) c[p] = 0;
    for (int k = rp[r]; k < rp[r + 1]; ++k) {
      const int p = hq_panel_of(ci[k], cols);
#pragma unroll
      for (int q = 0; q < HQ_PANELS; ++q) c[q] += (q == p);
    }
#pragma unroll
    for (int p = 0; p < HQ_PANELS; ++p) cnt[(size_t)r * HQ_PANELS + p] = c[p];
  }
}

// per chunk (row block rb, panel p): local row offsets and the chunk size
__global__ void k_panel_offsets(int rows, const int* __restrict__ cnt, unsigned short* __restrict__ lrp,
                                int* __restrict__ size) {
  const int nblk = (rows + HQ_BLOCK - 1) / HQ_BLOCK;
  for (int ch = blockIdx.x * blockDim.x + threadIdx.x; ch < nblk * HQ_PANELS; ch += gridDim.x * blockDim.x) {
    const int rb = ch / HQ_PANELS, p = ch % HQ_PANELS;
    int s = 0;
    for (int r = 0; r < HQ_BLOCK; ++r) {
      lrp[(size_t)ch * (HQ_BLOCK + 1) + r] = (unsigned short)(s < 65535 ? s : 65535);
      const int row = rb * HQ_BLOCK + r;
      if (row < rows) s += cnt[(size_t)row * HQ_PANELS + p];
    }
    lrp[(size_t)ch * (HQ_BLOCK + 1) + HQ_BLOCK] = (unsigned short)(s < 65535 ? s : 65535);
    size[ch] = s;
  }
}

// scatter every nonzero to its chunk (pp: exclusive scan of the chunk sizes)
__global__ void k_panel_scatter(int rows, int cols, const int* __restrict__ rp, const int* __restrict__ ci,
                                const double* __restrict__ v, const int* __restrict__ pp,
                                const unsigned short* __restrict__ lrp, int* __restrict__ pci,
                                double* __restrict__ pv) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) {
    const int rb = r / HQ_BLOCK, lr = r % HQ_BLOCK;
    int p_prev = -1, dst = 0;
    for (int k = rp[r]; k < rp[r + 1]; ++k) {
      const int p = hq_panel_of(ci[k], cols);
      if (p != p_prev) {   // columns are sorted: each panel's entries of the row are contiguous
        const int ch = rb * HQ_PANELS + p;
        dst = pp[ch] + lrp[(size_t)ch * (HQ_BLOCK + 1) + lr];
        p_prev = p;
      }
      pci[dst] = ci[k];
      pv[dst] = v[k];
      ++dst;
    }
  }
}

// Optional prefetch: the next chunk's loads are issued before the current
// chunk's products and sums, so that their latency overlaps the gathers and
// the LDS phase.  Chosen per epilogue (an epilogue type that declares
// PANEL_PREFETCH = true): measured on a random QP with n = 1e6 and 5e6
// nonzeros per matrix, it takes the product with the Halpern epilogue from
// 62.5 to 59.6 us, but slows the plain products down (A v 46 -> 52 us, the
// power method's Q product 41 -> 43 us), whose resident workgroups already
// hide that latency and whose early loads then only compete with the gathers.
template <class E, class = void> struct panel_prefetch : std::false_type {};
template <class E>
struct panel_prefetch<E, std::void_t<decltype(E::PANEL_PREFETCH)>> : std::bool_constant<E::PANEL_PREFETCH> {};

#define HQ_PANEL_PF 4                               // prefetched elements per thread
#define HQ_PANEL_PASS (HQ_PANEL_PF * HQ_BLOCK)      // elements per LDS pass

struct PanelChunk {
  int kb = 0, ke = 0, myb = 0, mye = 0;
  int ci[HQ_PANEL_PF];
  double v[HQ_PANEL_PF];
};

__device__ __forceinline__ void panel_fetch(const PanelMat& M, int rb, int p, int t, PanelChunk& c) {
  const int ch = rb * HQ_PANELS + p;
  c.kb = M.pp[ch];
  c.ke = M.pp[ch + 1];
  const int nr = min(HQ_BLOCK, M.rows - rb * HQ_BLOCK);
  c.myb = t < nr ? c.kb + M.lrp[(size_t)ch * (HQ_BLOCK + 1) + t] : 0;
  c.mye = t < nr ? c.kb + M.lrp[(size_t)ch * (HQ_BLOCK + 1) + t + 1] : 0;
#pragma unroll
  for (int i = 0; i < HQ_PANEL_PF; ++i) {
    const int k = c.kb + t + i * HQ_BLOCK;
    c.ci[i] = 0;
    c.v[i] = 0.0;
    if (k < c.ke) {
      c.ci[i] = ld_stream(M.ci + k);
      c.v[i] = ld_stream(M.v + k);
    }
  }
}

// the product with a fused epilogue; each workgroup owns BPB consecutive row
// blocks, grid = ceil(row blocks / BPB) (chosen so that the whole grid is
// resident at once: a late workgroup would gather from a panel the others
// have left)
template <class Epi, int BPB>
__global__ __launch_bounds__(HQ_BLOCK) void k_csr_panel(PanelMat M, const double* __restrict__ xin, Epi epi,
                                                        const DevParams* __restrict__ prm, int j, RedOut red) {
  constexpr int NR = Epi::NR;
  constexpr bool PF = panel_prefetch<Epi>::value;
  __shared__ double prod[PF ? HQ_PANEL_PASS : HQ_STREAM_CHUNK];
  Epi e = epi;
  e.setup(prm, j);
  double acc[NR > 0 ? NR : 1];
#pragma unroll
  for (int s = 0; s < (NR > 0 ? NR : 1); ++s) acc[s] = 0.0;
  const int nblk = (M.rows + HQ_BLOCK - 1) / HQ_BLOCK;
  const int t = threadIdx.x;
  double sum[BPB];
#pragma unroll
  for (int q = 0; q < BPB; ++q) sum[q] = 0.0;
  const int rb0 = blockIdx.x * BPB;
  if constexpr (PF) {
    const int nq = min(BPB, nblk - rb0);   // >= 1: grid = ceil(nblk / BPB)
    // chunks in the order (panel, row block); cur holds the loads of the next one
    PanelChunk cur;
    panel_fetch(M, rb0, 0, t, cur);
    for (int p = 0; p < HQ_PANELS; ++p) {
#pragma unroll
      for (int q = 0; q < BPB; ++q) {
        if (q < nq) {
          double xv[HQ_PANEL_PF];
#pragma unroll
          for (int i = 0; i < HQ_PANEL_PF; ++i)
            xv[i] = cur.kb + t + i * HQ_BLOCK < cur.ke ? xin[cur.ci[i]] : 0.0;
          const int kb = cur.kb, ke = cur.ke, myb = cur.myb, mye = cur.mye;
          double pv[HQ_PANEL_PF];
#pragma unroll
          for (int i = 0; i < HQ_PANEL_PF; ++i) pv[i] = cur.v[i];
          const bool last_q = q + 1 == nq;
          if (!last_q || p + 1 < HQ_PANELS) panel_fetch(M, rb0 + (last_q ? 0 : q + 1), last_q ? p + 1 : p, t, cur);
#pragma unroll
          for (int i = 0; i < HQ_PANEL_PF; ++i)
            if (kb + t + i * HQ_BLOCK < ke) prod[t + i * HQ_BLOCK] = pv[i] * xv[i];
          __syncthreads();
          {
            const int hi = min(mye, kb + HQ_PANEL_PASS);
            for (int k = myb; k < hi; ++k) sum[q] += prod[k - kb];
          }
          __syncthreads();
          // chunks longer than one pass: the rest without prefetch
          for (int c0 = kb + HQ_PANEL_PASS; c0 < ke; c0 += HQ_PANEL_PASS) {
            const int c1 = min(ke, c0 + HQ_PANEL_PASS);
#pragma unroll 4
            for (int k = c0 + t; k < c1; k += HQ_BLOCK) prod[k - c0] = ld_stream(M.v + k) * xin[ld_stream(M.ci + k)];
            __syncthreads();
            const int lo = max(myb, c0), hi = min(mye, c1);
            for (int k = lo; k < hi; ++k) sum[q] += prod[k - c0];
            __syncthreads();
          }
        }
      }
    }
  } else {
    for (int p = 0; p < HQ_PANELS; ++p) {
#pragma unroll
      for (int q = 0; q < BPB; ++q) {
        const int rb = rb0 + q;
        if (rb < nblk) {
          const int ch = rb * HQ_PANELS + p;
          const int kb = M.pp[ch], ke = M.pp[ch + 1];
          const int nr = min(HQ_BLOCK, M.rows - rb * HQ_BLOCK);
          const int myb = t < nr ? kb + M.lrp[(size_t)ch * (HQ_BLOCK + 1) + t] : 0;
          const int mye = t < nr ? kb + M.lrp[(size_t)ch * (HQ_BLOCK + 1) + t + 1] : 0;
          for (int c0 = kb; c0 < ke; c0 += HQ_STREAM_CHUNK) {
            const int c1 = min(ke, c0 + HQ_STREAM_CHUNK);
#pragma unroll 4
            for (int k = c0 + t; k < c1; k += HQ_BLOCK) prod[k - c0] = ld_stream(M.v + k) * xin[ld_stream(M.ci + k)];
            __syncthreads();
            const int lo = max(myb, c0), hi = min(mye, c1);
            for (int k = lo; k < hi; ++k) sum[q] += prod[k - c0];
            __syncthreads();
          }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < BPB; ++q) {
    const int rb = rb0 + q;
    if (rb < nblk && t < min(HQ_BLOCK, M.rows - rb * HQ_BLOCK)) e(rb * HQ_BLOCK + t, sum[q], acc);
  }
  if (red.active) block_reduce_store<NR, Epi::MAXMASK>(acc, red);
}
