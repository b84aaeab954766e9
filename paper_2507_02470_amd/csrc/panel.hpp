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
#include "spmv.hpp"   // HQ_STREAM_CHUNK

#ifndef HQ_PANELS
#define HQ_PANELS 4
#endif

struct PanelMat {
  int rows = 0, cols = 0;
  const int* pp = nullptr;               // chunk starts, (row blocks * P + 1)
  const unsigned short* lrp = nullptr;   // per chunk: HQ_BLOCK + 1 local row offsets
  const int* ci = nullptr;               // columns, panel order
  const double* v = nullptr;             // values, panel order
};

__host__ __device__ inline int hq_panel_of(int col, int cols) {
  return (int)(((long long)col * HQ_PANELS) / cols);
}

// The layout is built by three steps, each a function of one row or one chunk
// so that the kernels below run them in grid-stride loops and a host program
// can run the very same code (the layout tests do).
//
// Step 1, per row r: how many of its nonzeros fall in each panel ->
// cnt[r * P + p].
__host__ __device__ inline void panel_count_row(int r, int cols, const int* rp, const int* ci, int* cnt) {
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

// Step 2, per chunk ch = (row block rb, panel p): the local row offsets and
// the chunk size.  Offsets saturate at 65535; the host rejects the layout
// when a chunk holds more than 65535 nonzeros, so a saturated offset is never
// used.
__host__ __device__ inline void panel_offsets_chunk(int ch, int rows, const int* cnt, unsigned short* lrp,
                                                    int* size) {
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

// Step 3, per row r: every nonzero to its chunk (pp: exclusive scan of the
// chunk sizes).  One cursor per panel, so the columns of a row may come in
// any order: a row's entries of one panel keep their order in the row.
__host__ __device__ inline void panel_scatter_row(int r, int cols, const int* rp, const int* ci, const double* v,
                                                  const int* pp, const unsigned short* lrp, int* pci, double* pv) {
  const int rb = r / HQ_BLOCK, lr = r % HQ_BLOCK;
  int dst[HQ_PANELS];
#pragma unroll
  for (int p = 0; p < HQ_PANELS; ++p) {
    const int ch = rb * HQ_PANELS + p;
    dst[p] = pp[ch] + lrp[(size_t)ch * (HQ_BLOCK + 1) + lr];
  }
  for (int k = rp[r]; k < rp[r + 1]; ++k) {
    const int p = hq_panel_of(ci[k], cols);
    int d = 0;
#pragma unroll
    for (int q = 0; q < HQ_PANELS; ++q) {
      d = q == p ? dst[q] : d;
      dst[q] += (q == p);
    }
    pci[d] = ci[k];
    pv[d] = v[k];
  }
}

__global__ void k_panel_count(int rows, int cols, const int* __restrict__ rp, const int* __restrict__ ci,
                              int* __restrict__ cnt) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x)
    panel_count_row(r, cols, rp, ci, cnt);
}

__global__ void k_panel_offsets(int rows, const int* __restrict__ cnt, unsigned short* __restrict__ lrp,
                                int* __restrict__ size) {
  const int nblk = (rows + HQ_BLOCK - 1) / HQ_BLOCK;
  for (int ch = blockIdx.x * blockDim.x + threadIdx.x; ch < nblk * HQ_PANELS; ch += gridDim.x * blockDim.x)
    panel_offsets_chunk(ch, rows, cnt, lrp, size);
}

__global__ void k_panel_scatter(int rows, int cols, const int* __restrict__ rp, const int* __restrict__ ci,
                                const double* __restrict__ v, const int* __restrict__ pp,
                                const unsigned short* __restrict__ lrp, int* __restrict__ pci,
                                double* __restrict__ pv) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x)
    panel_scatter_row(r, cols, rp, ci, v, pp, lrp, pci, pv);
}

// Launch shape of the product: BPB row blocks per group, one group per
// workgroup when the whole grid is resident at once (the first BPB in 1..4
// for which it is, by the resident workgroups per CU of each instantiation,
// per_cu[1..4]); larger matrices take BPB = 4 and a grid of as many
// workgroups as are resident, each walking its groups in grid-stride order
// (so the workgroups still move through the panels together, group by group).
// The grid never exceeds HQ_PCAP, the block partials one reduction slot holds.
// min_bpb starts the search higher: the product with the prefetching epilogue
// runs fastest with 4 row blocks per workgroup (random QP, n = 1e6: Q d +
// Halpern 58.6 us against 62.0 us with the resident 3; its longer chain of
// prefetched chunks per workgroup), the plain products with the fewest.
struct PanelShape { int bpb, grid; };
inline PanelShape panel_launch_shape(int rows, int ncu, const int per_cu[5], int min_bpb = 1) {
  const long long nblk = (rows + HQ_BLOCK - 1) / HQ_BLOCK;
  for (int b = min_bpb; b <= 4; ++b) {
    const long long g = (nblk + b - 1) / b;
    if (g <= (long long)ncu * per_cu[b] && g <= HQ_PCAP) return {b, (int)(g > 0 ? g : 1)};
  }
  const long long groups = (nblk + 3) / 4;
  long long g = (long long)ncu * per_cu[4];
  if (g > HQ_PCAP) g = HQ_PCAP;
  if (g > groups) g = groups;
  return {4, (int)(g > 0 ? g : 1)};
}

// Optional prefetch: the next chunk's loads are issued before the current
// chunk's products and sums, so that their latency overlaps the gathers and
// the LDS phase.  Chosen per epilogue (an epilogue type that declares
// PANEL_PREFETCH = true): measured on a random QP with n = 1e6 and 5e6
// nonzeros per matrix, it takes the product with the Halpern epilogue from
// 62.5 to 59.6 us, but slows the plain products down (A v 46 -> 52 us, the
// power method's Q product 41 -> 43 us), whose resident workgroups already
// hide that latency and whose early loads then only compete with the gathers.
// An epilogue that prefetches also gets four row blocks per workgroup
// (panel_launch_shape), with which the Q xhat product gains slightly
// (46.4 -> 45.9 us) and A v, A^T ybar still lose (47.3 -> 48.9, 48.5 us).
template <class E, class = void> struct panel_prefetch : std::false_type {};
template <class E>
struct panel_prefetch<E, std::void_t<decltype(E::PANEL_PREFETCH)>> : std::bool_constant<E::PANEL_PREFETCH> {};

// Optional preload of epilogue operands: an epilogue type with a Pre struct,
// preload(i) and operator()(i, q, acc, pre) has its row-wise loads issued at
// the start of the last panel, so that they arrive during that panel's
// gathers instead of after the row sums.
template <class E, class = void> struct panel_preload : std::false_type {};
template <class E>
struct panel_preload<E, std::void_t<typename E::Pre>> : std::true_type {};
struct PanelNoPre {};
template <class E, bool PL> struct panel_pre_t { using type = PanelNoPre; };
template <class E> struct panel_pre_t<E, true> { using type = typename E::Pre; };

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

// the product with a fused epilogue; each workgroup owns groups of BPB
// consecutive row blocks (group g = blockIdx.x, blockIdx.x + gridDim.x, ...;
// see panel_launch_shape: one group per workgroup whenever the whole grid is
// resident, since a late workgroup would gather from a panel the others have
// left)
template <class Epi, int BPB, bool GS = false>
__global__ __launch_bounds__(HQ_BLOCK) void k_csr_panel(PanelMat M, const double* __restrict__ xin, Epi epi,
                                                        const DevParams* __restrict__ prm, int j, RedOut red) {
  constexpr int NR = Epi::NR;
  constexpr bool PF = panel_prefetch<Epi>::value;
  constexpr bool PL = PF && panel_preload<Epi>::value;
  __shared__ double prod[PF ? HQ_PANEL_PASS : HQ_STREAM_CHUNK];
  Epi e = epi;
  e.setup(prm, j);
  double acc[NR > 0 ? NR : 1];
#pragma unroll
  for (int s = 0; s < (NR > 0 ? NR : 1); ++s) acc[s] = 0.0;
  const int nblk = (M.rows + HQ_BLOCK - 1) / HQ_BLOCK;
  const int t = threadIdx.x;
  // one group of row blocks [g BPB, g BPB + BPB) of this workgroup
  auto group = [&](const int g) {
    const int rb0 = g * BPB;
    double sum[BPB];
    [[maybe_unused]] typename panel_pre_t<Epi, PL>::type pre[BPB];
#pragma unroll
    for (int q = 0; q < BPB; ++q) sum[q] = 0.0;
    if constexpr (PF) {
      const int nq = min(BPB, nblk - rb0);   // >= 1 by the loop condition
      // chunks in the order (panel, row block); cur holds the loads of the next one
      PanelChunk cur;
      panel_fetch(M, rb0, 0, t, cur);
      for (int p = 0; p < HQ_PANELS; ++p) {
        if constexpr (PL) {
          if (p == HQ_PANELS - 1) {
#pragma unroll
            for (int q = 0; q < BPB; ++q) {
              const int rb = rb0 + q;
              if (rb < nblk && t < min(HQ_BLOCK, M.rows - rb * HQ_BLOCK)) pre[q] = e.preload(rb * HQ_BLOCK + t);
            }
          }
        }
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
      if (rb < nblk && t < min(HQ_BLOCK, M.rows - rb * HQ_BLOCK)) {
        if constexpr (PL) e(rb * HQ_BLOCK + t, sum[q], acc, pre[q]);
        else e(rb * HQ_BLOCK + t, sum[q], acc);
      }
    }
  };
  // GS: groups in grid-stride order (matrices too tall for one group per
  // resident workgroup); else the one group blockIdx.x
  if constexpr (GS) {
    for (int g = blockIdx.x; g * BPB < nblk; g += gridDim.x) group(g);
  } else {
    if ((int)blockIdx.x * BPB < nblk) group(blockIdx.x);
  }
  if (red.active) block_reduce_store<NR, Epi::MAXMASK>(acc, red);
}
