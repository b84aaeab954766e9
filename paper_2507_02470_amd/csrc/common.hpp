// common.hpp -- shared device helpers for the HPR-QP kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define HQ_WAVE 64
#define HQ_BLOCK 256          // threads per block for vector/SpMV kernels (4 waves)
#define HQ_PCAP 4096          // max partial results per reduction slot
#define HQ_GRID_CAP 4096      // grid cap of grid-stride kernels (<= HQ_PCAP)

// Iteration scalars kept in device memory so that one captured graph can be
// replayed for every check segment (sigma changes only at restarts, the
// inner counter t advances by the segment length).
struct DevParams {
  double sigma;     // sigma_r of the current epoch
  double lamA;      // lambda_A >= lambda_1(A A^T)
  double lamQ;      // lambda_Q >= lambda_1(Q)
  int64_t t0;       // inner counter t at the first iteration of the segment
};

// Scalars derived from DevParams at iteration j of a segment.
struct IterScalars {
  double sigma, sQ, kappa, sA, rho;
  __device__ void load(const DevParams* p, int j) {
    sigma = p->sigma;
    sQ = sigma * p->lamQ;             // sigma lambda_Q
    kappa = sigma / (1.0 + sQ);       // sigma / (1 + sigma lambda_Q)
    sA = sigma * p->lamA;             // sigma lambda_A
    rho = 1.0 / (double)(p->t0 + j + 2);   // Halpern weight 1/(t+2)
  }
};

// Where a kernel's per-block partial reductions go: acc index s -> global
// reduction slot slot[s] (-1: skip).  counts[slot] receives gridDim.x.
struct RedOut {
  double* partials;   // [slot][HQ_PCAP]
  int* counts;        // [slot]
  int8_t slot[16];
  int active;
};

// Value of lane l ^ OFF.  Within a quad (OFF = 1, 2) a DPP quad permutation,
// otherwise a cross-lane shuffle (which goes through the LDS unit).  Every
// lane of the quad must be active (the callers use it outside divergent code,
// or within groups of lanes that are active together).
template <int OFF>
__device__ __forceinline__ double lane_xor(double x) {
  if constexpr (OFF == 1 || OFF == 2) {
    constexpr int ctrl = OFF == 1 ? 0xb1 : 0x4e;   // quad_perm [1,0,3,2] / [2,3,0,1]
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), ctrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), ctrl, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  } else {
    return __shfl_xor(x, OFF);
  }
}

// Butterfly sum (or max) over groups of G lanes (offsets G/2, ..., 1); every
// lane of a group ends with the group's result.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (G > 32) v += lane_xor<32>(v);
  if constexpr (G > 16) v += lane_xor<16>(v);
  if constexpr (G > 8) v += lane_xor<8>(v);
  if constexpr (G > 4) v += lane_xor<4>(v);
  if constexpr (G > 2) v += lane_xor<2>(v);
  if constexpr (G > 1) v += lane_xor<1>(v);
  return v;
}
template <int G>
__device__ __forceinline__ double group_max(double v) {
  if constexpr (G > 32) v = fmax(v, lane_xor<32>(v));
  if constexpr (G > 16) v = fmax(v, lane_xor<16>(v));
  if constexpr (G > 8) v = fmax(v, lane_xor<8>(v));
  if constexpr (G > 4) v = fmax(v, lane_xor<4>(v));
  if constexpr (G > 2) v = fmax(v, lane_xor<2>(v));
  if constexpr (G > 1) v = fmax(v, lane_xor<1>(v));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) { return group_sum<64>(v); }
__device__ __forceinline__ double wave_max(double v) { return group_max<64>(v); }

// Fixed-order block reduction of NR accumulators (sum, or max where bit s of
// MAXMASK is set) and store of one partial per block.  Deterministic.
template <int NR, unsigned MAXMASK, bool LOCAL = false>
__device__ __forceinline__ void block_reduce_store(const double* acc, const RedOut& red) {
  if constexpr (NR > 0) {
    __shared__ double sh[16][NR > 0 ? NR : 1];   // up to 1024-thread blocks
    const int lane = threadIdx.x & (HQ_WAVE - 1), wv = threadIdx.x / HQ_WAVE;
#pragma unroll
    for (int s = 0; s < NR; ++s) {
      double v = ((MAXMASK >> s) & 1u) ? wave_max(acc[s]) : wave_sum(acc[s]);
      if (lane == 0) sh[wv][s] = v;
    }
    __syncthreads();
    if (threadIdx.x < NR) {
      const int s = threadIdx.x;
      double v = sh[0][s];
      const bool mx = (MAXMASK >> s) & 1u;
      for (int w = 1; w < (int)(blockDim.x / HQ_WAVE); ++w) v = mx ? fmax(v, sh[w][s]) : v + sh[w][s];
      // LOCAL: red is a local of the kernel (the one-workgroup segments); its
      // slot is then picked by compares, since indexing it with the thread
      // index would keep the struct in scratch.  A kernel argument is indexed
      // directly (the compares would cost the multi-block kernels SGPRs).
      int slot;
      if constexpr (LOCAL) {
        slot = -1;
#pragma unroll
        for (int q = 0; q < NR; ++q) slot = s == q ? red.slot[q] : slot;
      } else {
        slot = red.slot[s];
      }
      if (slot >= 0) {
        red.partials[(size_t)slot * HQ_PCAP + blockIdx.x] = v;
        if (blockIdx.x == 0) red.counts[slot] = gridDim.x;
      }
    }
  }
}

__device__ __forceinline__ double clampd(double v, double lo, double hi) {
  return fmin(fmax(v, lo), hi);
}

// Prox of sigma phi for phi(x) = lambda |x| + delta_[L,U](x), t = sigma lambda:
// soft threshold at t, then the clamp to [L, U] (t = 0: the projection).
__device__ __forceinline__ double prox_phi(double r, double t, double L, double U) {
  const double v = r > t ? r - t : (r < -t ? r + t : 0.0);
  return clampd(v, L, U);
}

// -phi^*(-z) for phi(x) = lambda |x| + delta_[L,U](x): phi^*(s) is the max of
// s x - lambda |x| over x in {L, U, 0 if L <= 0 <= U}; it is +inf when L = -inf
// and z > lambda or U = +inf and z < -lambda (then *inf is set).  With
// lambda > 0 an excess of at most 1e-12 max(1, lambda) counts as rounding.
__device__ __forceinline__ double neg_conj_phi(double z, double lam, double L, double U, bool* inf) {
  const double slack = lam > 0.0 ? 1e-12 * fmax(lam, 1.0) : 0.0;
  if ((isinf(L) && z > lam + slack) || (isinf(U) && z < -lam - slack)) { *inf = true; return 0.0; }
  double best = -INFINITY;
  if (!isinf(L)) best = fmax(best, -z * L - lam * fabs(L));
  if (!isinf(U)) best = fmax(best, -z * U - lam * fabs(U));
  if (L <= 0.0 && 0.0 <= U) best = fmax(best, 0.0);
  return -best;
}

// streaming loads/stores for data touched once per product (matrix entries,
// single-use vector streams): marked non-temporal so they do not evict the
// vector being gathered from L2
__device__ __forceinline__ double ld_stream(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ int ld_stream(const int* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ unsigned short ld_stream(const unsigned short* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_stream(double* p, double v) { __builtin_nontemporal_store(v, p); }

static inline int hq_grid(long long work, int per_block) {
  long long g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > HQ_GRID_CAP) g = HQ_GRID_CAP;
  return (int)g;
}
