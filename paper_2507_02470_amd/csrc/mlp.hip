// mlp.hip -- the warm-start surrogate: a 3-layer GELU MLP trained and run
// with hand-written BF16 MFMA GEMMs (FP32 accumulate) on gfx950.
//
// Every GEMM is C[M x N] = A[M x K] * B[K x N] with both operands stored so
// that K is the contiguous dimension (the library keeps transposed BF16
// copies of weights, activations and gradients, with every leading
// dimension padded to a multiple of 8 and zero-filled), which lets each
// lane fetch its 8 consecutive K values of a v_mfma_f32_32x32x16_bf16
// operand with one 16-byte load.
#include "hprqp_mlp.h"
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace hq {
extern thread_local std::string g_err;
}

typedef __bf16 hm_bf16x8 __attribute__((ext_vector_type(8)));
typedef float hm_f32x16 __attribute__((ext_vector_type(16)));
typedef uint16_t hm_u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  const __bf16 b = (__bf16)f;   // round to nearest even
  return __builtin_bit_cast(uint16_t, b);
}
__device__ __forceinline__ float bf2f(uint16_t u) { return __builtin_bit_cast(float, (uint32_t)u << 16); }

static inline int rup8(int v) { return (v + 7) & ~7; }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// Optional epilogue of a GEMM of the forward pass: Z = A B + bias (FP32,
// stored in C) and, with act, its activation as BF16 (GELU for the hidden
// layers): the same FP32 operations as a separate bias/activation pass.
struct GemmEpi {
  const float* bias = nullptr;
  uint16_t* act = nullptr;
  long long ld_act = 0;
  int gelu_on = 0;
};
__device__ __forceinline__ void gemm_store(float* C, long long ldc, int row, int col, float v, int accumulate,
                                           const GemmEpi& ep) {
  float* p = C + (long long)row * ldc + col;
  float z = accumulate ? *p + v : v;
  if (ep.bias) z += ep.bias[col];
  *p = z;
  if (ep.act) ep.act[(long long)row * ep.ld_act + col] = f2bf(ep.gelu_on ? gelu(z) : z);
}

// ---------------------------------------------------------------------------
// GEMM.  Block = 4 waves in a 2 x 2 arrangement, each wave a 32 x 32 tile of
// C (one 32x32x16 MFMA per K step of 16).  Operand layout of the MFMA
// (measured on gfx950): lane l holds A[l%32][8(l/32) + e] and
// B[8(l/32) + e][l%32], e = 0..7; accumulator register v of lane l holds
// C[8(v/4) + 4(l/32) + v%4][l%32].
// A(i, k) = A[i*a_rs + k*a_cs], B(k, j) = B[k*b_rs + j*b_cs]; when a_cs == 1
// (resp. b_rs == 1) and the row start is 16-byte aligned the 8 values come
// from one vector load.
// Split K: blockIdx.z takes the K range [z kper, (z + 1) kper) (kper a
// multiple of 16) and writes its partial tile to W[z] (M x N, dense); a
// second kernel adds the partials in the order z = 0, 1, ... (deterministic).
// Without a split (W == nullptr) the tile goes to C directly.
// ---------------------------------------------------------------------------
#define HM_KUNROLL 8
__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, int kper, const uint16_t* __restrict__ A,
                                                  long long a_rs, long long a_cs, const uint16_t* __restrict__ B,
                                                  long long b_rs, long long b_cs, float* __restrict__ C, long long ldc,
                                                  int accumulate, float* __restrict__ W, GemmEpi ep) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 31, lh = lane >> 5;
  const int i0 = blockIdx.x * 64 + (wv & 1) * 32;
  const int j0 = blockIdx.y * 64 + (wv >> 1) * 32;
  const int ia = i0 + li, jb = j0 + li;
  const int kbeg = blockIdx.z * kper, kend = min(K, kbeg + kper);
  const bool a_vec = (a_cs == 1) && ((a_rs & 7) == 0) && ((((uintptr_t)A) & 15) == 0);
  const bool b_vec = (b_rs == 1) && ((b_cs & 7) == 0) && ((((uintptr_t)B) & 15) == 0);
  hm_f32x16 acc = {};
  auto frag_a = [&](int kb) {
    hm_u16x8 au;
    if (a_vec && ia < M && kb + 8 <= kend) {
      au = *reinterpret_cast<const hm_u16x8*>(A + (long long)ia * a_rs + kb);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        au[e] = (ia < M && kb + e < kend) ? A[(long long)ia * a_rs + (long long)(kb + e) * a_cs] : 0;
    }
    return au;
  };
  auto frag_b = [&](int kb) {
    hm_u16x8 bu;
    if (b_vec && jb < N && kb + 8 <= kend) {
      bu = *reinterpret_cast<const hm_u16x8*>(B + (long long)jb * b_cs + kb);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        bu[e] = (jb < N && kb + e < kend) ? B[(long long)(kb + e) * b_rs + (long long)jb * b_cs] : 0;
    }
    return bu;
  };
  // software pipeline: the fragments of the next HM_KUNROLL k-steps are
  // loaded before the MFMAs of the current ones, so their latency overlaps
  // the matrix-core work instead of stalling it
  hm_u16x8 au[HM_KUNROLL], bu[HM_KUNROLL];
#pragma unroll
  for (int u = 0; u < HM_KUNROLL; ++u) {
    const int kb = kbeg + 16 * u + 8 * lh;
    au[u] = frag_a(kb);
    bu[u] = frag_b(kb);
  }
  for (int k0 = kbeg; k0 < kend; k0 += 16 * HM_KUNROLL) {
    const int k1 = k0 + 16 * HM_KUNROLL;
    hm_u16x8 an[HM_KUNROLL], bn[HM_KUNROLL];
    if (k1 < kend) {
#pragma unroll
      for (int u = 0; u < HM_KUNROLL; ++u) {
        const int kb = k1 + 16 * u + 8 * lh;
        an[u] = frag_a(kb);
        bn[u] = frag_b(kb);
      }
    }
#pragma unroll
    for (int u = 0; u < HM_KUNROLL; ++u)
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(hm_bf16x8, au[u]),
                                                    __builtin_bit_cast(hm_bf16x8, bu[u]), acc, 0, 0, 0);
    if (k1 < kend) {
#pragma unroll
      for (int u = 0; u < HM_KUNROLL; ++u) {
        au[u] = an[u];
        bu[u] = bn[u];
      }
    }
  }
  float* const Wz = W ? W + (size_t)blockIdx.z * M * N : nullptr;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int row = i0 + 8 * (v >> 2) + 4 * lh + (v & 3);
    const int col = j0 + li;
    if (row < M && col < N) {
      if (Wz) Wz[(size_t)row * N + col] = acc[v];
      else gemm_store(C, ldc, row, col, acc[v], accumulate, ep);
    }
  }
}

// C (+)= sum over z = 0..S-1 of W[z] (M x N each), in that order, then the epilogue
__global__ void k_splitk_reduce(int M, int N, int S, const float* __restrict__ W, float* __restrict__ C, long long ldc,
                                int accumulate, GemmEpi ep) {
  const long long total = (long long)M * N;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    float sum = W[t];
    for (int z = 1; z < S; ++z) sum += W[(size_t)z * total + t];
    gemm_store(C, ldc, (int)(t / N), (int)(t % N), sum, accumulate, ep);
  }
}

// ---------------------------------------------------------------------------
// elementwise pieces
// ---------------------------------------------------------------------------
// dst (rows x cols_p, BF16) <- (src - mean) * inv_std (rows x cols, FP32), zero padding
__global__ void k_to_bf16_pad(int rows, int cols, int cols_p, const float* __restrict__ src, const float* __restrict__ mean,
                              const float* __restrict__ inv_std, uint16_t* __restrict__ dst) {
  const long long total = (long long)rows * cols_p;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(t / cols_p), c = (int)(t % cols_p);
    dst[t] = c < cols ? f2bf((src[(long long)r * cols + c] - mean[c]) * inv_std[c]) : (uint16_t)0;
  }
}
// T (rows x cols) -> (T - mean) * inv_std
__global__ void k_standardize(int rows, int cols, const float* __restrict__ src, const float* __restrict__ mean,
                              const float* __restrict__ inv_std, float* __restrict__ dst) {
  const long long total = (long long)rows * cols;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(t % cols);
    dst[t] = (src[t] - mean[c]) * inv_std[c];
  }
}
// network output (standardized, ld) -> FP32 user units: mean + std * Y
__global__ void k_destandardize(int rows, int cols, const float* __restrict__ Y, long long ld, const float* __restrict__ mean,
                                const float* __restrict__ sd, float* __restrict__ out) {
  const long long total = (long long)rows * cols;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(t / cols), c = (int)(t % cols);
    out[t] = mean[c] + sd[c] * Y[(long long)r * ld + c];
  }
}
// prediction [y (m); z (n); w (n) (; ell)] per sample (row length no) -> FP64
// warm start of HPR-QP: y0 = y, w0 = w, x0 = Pi_C(w) (z is not read by the
// iteration).  bad[s] = 1 if a predicted value of y or w is not finite: that
// sample's start is then the origin (y0 = w0 = x0 = 0, the cold start of
// Algorithm 4).  score (if given): the predicted length ell of each solve.
__global__ void k_warm_start(int batch, int n, int m, int no, const float* __restrict__ P, const double* __restrict__ L,
                             const double* __restrict__ U, double* __restrict__ y0, double* __restrict__ w0,
                             double* __restrict__ x0, int* __restrict__ bad, float* __restrict__ score) {
  const int s = blockIdx.x;
  if (s >= batch) return;
  const float* p = P + (long long)s * no;
  int nf = 0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) nf |= !isfinite(p[i]);
  for (int j = threadIdx.x; j < n; j += blockDim.x) nf |= !isfinite(p[m + n + j]);
  __shared__ int sbad;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  if (nf) atomicOr(&sbad, 1);
  __syncthreads();
  const bool cold = sbad != 0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) y0[(long long)s * m + i] = cold ? 0.0 : (double)p[i];
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double wv = cold ? 0.0 : (double)p[m + n + j];
    w0[(long long)s * n + j] = wv;
    x0[(long long)s * n + j] = cold ? 0.0 : fmin(fmax(wv, L[j]), U[j]);
  }
  if (threadIdx.x == 0) {
    bad[s] = cold ? 1 : 0;
    if (score) score[s] = p[m + 2 * n];
  }
}

// out (rows x cols, FP32) <- a stage tensor with leading dimension ld, FP32
// or BF16 bits (exact widening)
__global__ void k_export(int rows, int cols, long long ld, const float* __restrict__ f32,
                         const uint16_t* __restrict__ b16, float* __restrict__ out) {
  const long long total = (long long)rows * cols;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    const long long r = t / cols, c = t % cols;
    out[t] = f32 ? f32[r * ld + c] : __uint_as_float((unsigned)b16[r * ld + c] << 16);
  }
}

// Column statistics of a (rows x cols) FP32 matrix for the standardization:
// per column, the sum (pass 0) or the sum of squared deviations from `mean`
// (pass 1) over a chunk of rows into part[chunk][col], FP64, rows in order.
#define HM_STAT_ROWS 1024
__global__ void k_col_stats(long long rows, int cols, const float* __restrict__ X, const double* __restrict__ mean,
                            double* __restrict__ part) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  const long long r0 = (long long)blockIdx.y * HM_STAT_ROWS, r1 = min(rows, r0 + HM_STAT_ROWS);
  double s = 0.0;
  for (long long r = r0; r < r1; ++r) {
    const double v = X[r * cols + j];
    s += mean ? (v - mean[j]) * (v - mean[j]) : v;
  }
  part[(long long)blockIdx.y * cols + j] = s;
}
// out[j] = sum of the chunks' partials in chunk order, divided by `div`
// (sqrt of it when `root`): the mean (div = rows) or the standard deviation
// (div = rows - 1)
__global__ void k_col_finish(int chunks, int cols, const double* __restrict__ part, double div, int root,
                             double* __restrict__ out64, float* __restrict__ out32) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += part[(long long)c * cols + j];
  s /= div;
  if (root) s = sqrt(s);
  out64[j] = s;
  out32[j] = (float)s;
}

// Network input of family members: X[s] = [c_s (n); u_s (m)] in FP32
__global__ void k_family_features(int batch, int n, int m, const double* __restrict__ c, const double* __restrict__ u,
                                  float* __restrict__ X) {
  const long long total = (long long)batch * (n + m);
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    const long long s = t / (n + m);
    const int k = (int)(t % (n + m));
    X[t] = (float)(k < n ? c[s * n + k] : u[s * m + (k - n)]);
  }
}
// Training targets of family members: T[s] = [y_s (m); z_s (n); w_s (n)] in
// FP32, and with iters given a last column log(max(iters_s, 1)) (the length of
// the solve that produced the member's solution)
__global__ void k_family_targets(int batch, int n, int m, const double* __restrict__ y, const double* __restrict__ z,
                                 const double* __restrict__ w, const long long* __restrict__ iters,
                                 float* __restrict__ T) {
  const int no = m + 2 * n + (iters ? 1 : 0);
  const long long total = (long long)batch * no;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    const long long s = t / no;
    const int k = (int)(t % no);
    T[t] = k < m ? (float)y[s * m + k]
         : k < m + n ? (float)z[s * n + (k - m)]
         : k < m + 2 * n ? (float)w[s * n + (k - m - n)]
         : (float)log((double)(iters[s] > 1 ? iters[s] : 1));
  }
}

// dst (cols_p x rows_p) = transpose of src (rows x cols_p), zero rows beyond `rows`
__global__ void k_transpose_bf16(int rows, int rows_p, int cols_p, const uint16_t* __restrict__ src,
                                 uint16_t* __restrict__ dst) {
  __shared__ uint16_t tile[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
  for (int y = ty; y < 32; y += 8) {
    const int r = r0 + y, c = c0 + tx;
    tile[y][tx] = (r < rows && c < cols_p) ? src[(long long)r * cols_p + c] : (uint16_t)0;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int c = c0 + y, r = r0 + tx;
    if (c < cols_p && r < rows_p) dst[(long long)c * rows_p + r] = tile[tx][y];
  }
}


// weighted MSE: dY = 2 w (Y - T)/(B N) (FP32 and BF16 copies), per-block loss partials
__global__ __launch_bounds__(256) void k_mse(int B, int N, const float* __restrict__ Y, long long ldy,
                                             const float* __restrict__ T, const float* __restrict__ w,
                                             float* __restrict__ dYf, uint16_t* __restrict__ dYb, long long ldd,
                                             double* __restrict__ partial) {
  const double scale = 1.0 / ((double)B * (double)N);
  double acc = 0.0;
  const long long total = (long long)B * N;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(t / N), j = (int)(t % N);
    const float wj = w ? w[j] : 1.0f;
    const float r = Y[(long long)b * ldy + j] - T[t];
    acc += (double)wj * (double)r * (double)r;
    const float g = (float)(2.0 * scale) * wj * r;
    dYf[(long long)b * ldd + j] = g;
    dYb[(long long)b * ldd + j] = f2bf(g);
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0] * scale;
}

// dZ = dA * GELU'(Z)
__global__ void k_gelu_bwd(int B, int N, const float* __restrict__ dA, long long lda, const float* __restrict__ Z,
                           long long ldz, float* __restrict__ dZf, uint16_t* __restrict__ dZb, long long ldo) {
  const long long total = (long long)B * N;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(t / N), j = (int)(t % N);
    const float g = dA[(long long)b * lda + j] * gelu_d(Z[(long long)b * ldz + j]);
    dZf[(long long)b * ldo + j] = g;
    dZb[(long long)b * ldo + j] = f2bf(g);
  }
}

// db[j] = sum_b dZ[b][j]: a block of 256 threads covers 32 columns, thread
// (g, c) summing rows g, g + 8, ... of its column in FP64, and the 8 partial
// sums of a column are added in the order g = 0..7 (deterministic; reading
// rows 8 at a time keeps 8 loads per column in flight)
#define HM_CS_COLS 32
#define HM_CS_GRP 8
__global__ __launch_bounds__(256) void k_colsum(int B, int N, const float* __restrict__ dZ, long long ld,
                                                float* __restrict__ db) {
  __shared__ double part[HM_CS_GRP][HM_CS_COLS];
  const int c = threadIdx.x % HM_CS_COLS, g = threadIdx.x / HM_CS_COLS;
  for (int j0 = blockIdx.x * HM_CS_COLS; j0 < N; j0 += gridDim.x * HM_CS_COLS) {
    const int j = j0 + c;
    double s = 0.0;
    if (j < N)
      for (int b = g; b < B; b += HM_CS_GRP) s += dZ[(long long)b * ld + j];
    part[g][c] = s;
    __syncthreads();
    if (g == 0 && j < N) {
      double t = part[0][c];
#pragma unroll
      for (int q = 1; q < HM_CS_GRP; ++q) t += part[q][c];
      db[j] = (float)t;
    }
    __syncthreads();
  }
}

__global__ void k_adam(long long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi; v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// W (rows x cols, FP32 master) -> Wb (rows_p x cols_p, BF16) and Wt (cols_p x rows_p, BF16)
__global__ void k_weights_bf16(int rows, int cols, int rows_p, int cols_p, const float* __restrict__ W,
                               uint16_t* __restrict__ Wb, uint16_t* __restrict__ Wt) {
  const long long total = (long long)rows_p * cols_p;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(t / cols_p), c = (int)(t % cols_p);
    const uint16_t u = (r < rows && c < cols) ? f2bf(W[(long long)r * cols + c]) : (uint16_t)0;
    Wb[t] = u;
    Wt[(long long)c * rows_p + r] = u;
  }
}

// ---------------------------------------------------------------------------
// network object
// ---------------------------------------------------------------------------
struct hprqp_mlp {
  int d[4];          // n_in, h1, h2, n_out
  int dp[4];         // padded to multiples of 8
  int maxb, maxbp;
  hipStream_t st = nullptr, own_st = nullptr;
  long long np = 0;
  long long off_W[3], off_b[3];
  float *P = nullptr, *G = nullptr, *Mm = nullptr, *Vv = nullptr;   // params, grad, Adam moments
  long long adam_t = 0;
  uint16_t *Wb[3] = {}, *Wt[3] = {};
  uint16_t *Xb = nullptr, *Xt = nullptr, *A1b = nullptr, *A1t = nullptr, *A2b = nullptr, *A2t = nullptr;
  float *Z1 = nullptr, *Z2 = nullptr, *Y = nullptr;
  float *dYf = nullptr, *dA2 = nullptr, *dZ2f = nullptr, *dA1 = nullptr, *dZ1f = nullptr;
  uint16_t *dYb = nullptr, *dYt = nullptr, *dZ2b = nullptr, *dZ2t = nullptr, *dZ1b = nullptr, *dZ1t = nullptr;
  double* part = nullptr;
  float* ws = nullptr;          // split-K partials of the GEMMs
  long long ws_floats = 0;
  int ncu = 0;
  // input / output standardization (set by hprqp_mlp_set_scaling; identity by default)
  float *in_mean = nullptr, *in_istd = nullptr, *out_mean = nullptr, *out_sd = nullptr, *out_istd = nullptr;
  float *Tstd = nullptr, *Yuser = nullptr;
  std::vector<void*> owned;
  hipEvent_t ev[16] = {};
  int nev = 0;
  double last_flop = 0.0;
  int last_batch = 0;   // batch of the last forward / loss_grad
  ~hprqp_mlp() {
    for (void* p : owned) hipFree(p);
    for (auto e : ev)
      if (e) hipEventDestroy(e);
    if (own_st) hipStreamDestroy(own_st);
  }
};

namespace {
struct MErr {
  hprqp_status st;
  std::string msg;
};
[[noreturn]] void mfail(hprqp_status st, const std::string& m) { throw MErr{st, m}; }
void mcheck(hipError_t e, const char* w) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) mfail(HPRQP_ERR_OOM, std::string(w) + ": out of device memory");
    mfail(HPRQP_ERR_HIP, std::string(w) + ": " + hipGetErrorString(e));
  }
}
#define HMC(x) mcheck((x), #x)

template <class T>
T* malloc_dev(hprqp_mlp& n, size_t count) {
  void* p = nullptr;
  HMC(hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)));
  HMC(hipMemsetAsync(p, 0, std::max<size_t>(count, 1) * sizeof(T), n.st));
  n.owned.push_back(p);
  return (T*)p;
}

int eg(long long work) {
  long long g = (work + 255) / 256;
  return (int)std::max(1LL, std::min(g, 4096LL));
}

int cs_grid(int cols) { return std::max(1, std::min((cols + HM_CS_COLS - 1) / HM_CS_COLS, 4096)); }

// K splits of a GEMM: doubled while the launch holds fewer than 4 waves per
// CU, each split keeps at least 4 k-steps of 16 and the partials fit the
// workspace (the network's GEMMs are small: a 512 x 512 output is 64 tiles,
// 256 waves, too few to hide the fragment loads on 256 CUs)
int gemm_splits(int M, int N, int K, int ncu, long long ws_floats) {
  const long long waves = 4LL * ((M + 63) / 64) * ((N + 63) / 64);
  const int ksteps = (K + 15) / 16;
  int S = 1;
  while (S < 8 && waves * S < 4LL * ncu && ksteps >= 8 * S && (long long)(2 * S) * M * N <= ws_floats) S *= 2;
  return S;
}

// C (+)= A B with S K-splits (S > 1: the partials go through ws, which holds
// at least S M N floats)
void gemm_split(hipStream_t st, int M, int N, int K, const uint16_t* A, long long a_rs, long long a_cs,
                const uint16_t* B, long long b_rs, long long b_cs, float* C, long long ldc, int acc, int S, float* ws,
                const GemmEpi& ep = GemmEpi{}) {
  const int ksteps = (K + 15) / 16;
  if (S < 1) S = 1;
  const int kper = 16 * ((ksteps + S - 1) / S);
  const int Se = kper > 0 ? (K + kper - 1) / kper : 1;
  if (Se <= 1) {
    dim3 grid((M + 63) / 64, (N + 63) / 64, 1);
    k_gemm_bf16<<<grid, 256, 0, st>>>(M, N, K, std::max(kper, 16), A, a_rs, a_cs, B, b_rs, b_cs, C, ldc, acc, nullptr,
                                      ep);
    return;
  }
  dim3 grid((M + 63) / 64, (N + 63) / 64, Se);
  k_gemm_bf16<<<grid, 256, 0, st>>>(M, N, K, kper, A, a_rs, a_cs, B, b_rs, b_cs, C, ldc, acc, ws, GemmEpi{});
  k_splitk_reduce<<<eg((long long)M * N), 256, 0, st>>>(M, N, Se, ws, C, ldc, acc, ep);
}

// a GEMM of the network: K split by gemm_splits, partials in the handle's workspace
void gemm(hprqp_mlp& n, int M, int N, int K, const uint16_t* A, long long a_rs, long long a_cs, const uint16_t* B,
          long long b_rs, long long b_cs, float* C, long long ldc, int acc, const GemmEpi& ep = GemmEpi{}) {
  gemm_split(n.st, M, N, K, A, a_rs, a_cs, B, b_rs, b_cs, C, ldc, acc, gemm_splits(M, N, K, n.ncu, n.ws_floats), n.ws,
             ep);
}

void refresh_weights(hprqp_mlp& n) {
  for (int l = 0; l < 3; ++l) {
    const int rows = n.d[l + 1], cols = n.d[l], rows_p = n.dp[l + 1], cols_p = n.dp[l];
    k_weights_bf16<<<eg((long long)rows_p * cols_p), 256, 0, n.st>>>(rows, cols, rows_p, cols_p, n.P + n.off_W[l],
                                                                    n.Wb[l], n.Wt[l]);
  }
}

void create_impl(const int32_t dims[4], int32_t max_batch, const float* params_host, hipStream_t st, hprqp_mlp** out) {
  if (!dims || !out || max_batch <= 0) mfail(HPRQP_ERR_ARG, "bad arguments");
  for (int i = 0; i < 4; ++i)
    if (dims[i] <= 0 || dims[i] > (1 << 16)) mfail(HPRQP_ERR_SHAPE, "layer sizes must be in [1, 65536]");
  auto* n = new hprqp_mlp();
  try {
    if (!st) {
      HMC(hipStreamCreateWithFlags(&n->own_st, hipStreamNonBlocking));
      HMC(hipDeviceSynchronize());
      st = n->own_st;
    }
    n->st = st;
    for (int i = 0; i < 4; ++i) { n->d[i] = dims[i]; n->dp[i] = rup8(dims[i]); }
    n->maxb = max_batch;
    n->maxbp = rup8(max_batch);
    long long o = 0;
    for (int l = 0; l < 3; ++l) {
      n->off_W[l] = o; o += (long long)n->d[l + 1] * n->d[l];
      n->off_b[l] = o; o += n->d[l + 1];
    }
    n->np = o;
    n->P = malloc_dev<float>(*n, o);
    n->G = malloc_dev<float>(*n, o);
    n->Mm = malloc_dev<float>(*n, o);
    n->Vv = malloc_dev<float>(*n, o);
    if (params_host) HMC(hipMemcpyAsync(n->P, params_host, o * sizeof(float), hipMemcpyHostToDevice, st));
    for (int l = 0; l < 3; ++l) {
      n->Wb[l] = malloc_dev<uint16_t>(*n, (size_t)n->dp[l + 1] * n->dp[l]);
      n->Wt[l] = malloc_dev<uint16_t>(*n, (size_t)n->dp[l + 1] * n->dp[l]);
    }
    const size_t B = n->maxbp;
    n->Xb = malloc_dev<uint16_t>(*n, B * n->dp[0]);
    n->Xt = malloc_dev<uint16_t>(*n, B * n->dp[0]);
    n->A1b = malloc_dev<uint16_t>(*n, B * n->dp[1]);
    n->A1t = malloc_dev<uint16_t>(*n, B * n->dp[1]);
    n->A2b = malloc_dev<uint16_t>(*n, B * n->dp[2]);
    n->A2t = malloc_dev<uint16_t>(*n, B * n->dp[2]);
    n->Z1 = malloc_dev<float>(*n, B * n->dp[1]);
    n->Z2 = malloc_dev<float>(*n, B * n->dp[2]);
    n->Y = malloc_dev<float>(*n, B * n->dp[3]);
    n->dYf = malloc_dev<float>(*n, B * n->dp[3]);
    n->dYb = malloc_dev<uint16_t>(*n, B * n->dp[3]);
    n->dYt = malloc_dev<uint16_t>(*n, B * n->dp[3]);
    n->dA2 = malloc_dev<float>(*n, B * n->dp[2]);
    n->dZ2f = malloc_dev<float>(*n, B * n->dp[2]);
    n->dZ2b = malloc_dev<uint16_t>(*n, B * n->dp[2]);
    n->dZ2t = malloc_dev<uint16_t>(*n, B * n->dp[2]);
    n->dA1 = malloc_dev<float>(*n, B * n->dp[1]);
    n->dZ1f = malloc_dev<float>(*n, B * n->dp[1]);
    n->dZ1b = malloc_dev<uint16_t>(*n, B * n->dp[1]);
    n->dZ1t = malloc_dev<uint16_t>(*n, B * n->dp[1]);
    n->part = malloc_dev<double>(*n, 4096);
    {
      int dev = 0;
      HMC(hipGetDevice(&dev));
      HMC(hipDeviceGetAttribute(&n->ncu, hipDeviceAttributeMultiprocessorCount, dev));
      // split-K partials: gemm_splits only splits launches of fewer than 4
      // waves per CU, whose partials stay well below this; beyond it, fewer splits
      n->ws_floats = 2LL * n->ncu * 4096 * 4;
      n->ws = malloc_dev<float>(*n, (size_t)n->ws_floats);
    }
    n->in_mean = malloc_dev<float>(*n, n->d[0]);
    n->in_istd = malloc_dev<float>(*n, n->d[0]);
    n->out_mean = malloc_dev<float>(*n, n->d[3]);
    n->out_sd = malloc_dev<float>(*n, n->d[3]);
    n->out_istd = malloc_dev<float>(*n, n->d[3]);
    n->Tstd = malloc_dev<float>(*n, (size_t)n->maxb * n->d[3]);
    n->Yuser = malloc_dev<float>(*n, (size_t)n->maxb * n->d[3]);
    {
      std::vector<float> ones(std::max(n->d[0], n->d[3]), 1.0f);
      HMC(hipMemcpyAsync(n->in_istd, ones.data(), n->d[0] * sizeof(float), hipMemcpyHostToDevice, st));
      HMC(hipMemcpyAsync(n->out_sd, ones.data(), n->d[3] * sizeof(float), hipMemcpyHostToDevice, st));
      HMC(hipMemcpyAsync(n->out_istd, ones.data(), n->d[3] * sizeof(float), hipMemcpyHostToDevice, st));
      HMC(hipStreamSynchronize(st));
    }
    for (auto& e : n->ev) HMC(hipEventCreate(&e));
    refresh_weights(*n);
    HMC(hipStreamSynchronize(st));
    *out = n;
  } catch (...) {
    delete n;
    throw;
  }
}

void mark(hprqp_mlp& n) { HMC(hipEventRecord(n.ev[n.nev++], n.st)); }

void forward_impl(hprqp_mlp& n, int B, const float* X) {
  if (B <= 0 || B > n.maxb || !X) mfail(HPRQP_ERR_ARG, "batch out of range or NULL input");
  n.last_batch = B;
  const int in = n.d[0], h1 = n.d[1], h2 = n.d[2], out = n.d[3];
  const int inp = n.dp[0], h1p = n.dp[1], h2p = n.dp[2], outp = n.dp[3];
  k_to_bf16_pad<<<eg((long long)B * inp), 256, 0, n.st>>>(B, in, inp, X, n.in_mean, n.in_istd, n.Xb);
  n.nev = 0;
  mark(n);
  // each layer: Z = W x + b, then the hidden layers' GELU to BF16, in the GEMM's epilogue
  gemm(n, B, h1, inp, n.Xb, inp, 1, n.Wb[0], 1, inp, n.Z1, h1p, 0, GemmEpi{n.P + n.off_b[0], n.A1b, h1p, 1});
  mark(n);
  mark(n);
  gemm(n, B, h2, h1p, n.A1b, h1p, 1, n.Wb[1], 1, h1p, n.Z2, h2p, 0, GemmEpi{n.P + n.off_b[1], n.A2b, h2p, 1});
  mark(n);
  mark(n);
  gemm(n, B, out, h2p, n.A2b, h2p, 1, n.Wb[2], 1, h2p, n.Y, outp, 0, GemmEpi{n.P + n.off_b[2], nullptr, 0, 0});
  mark(n);
  n.last_flop = 2.0 * B * ((double)inp * h1 + (double)h1p * h2 + (double)h2p * out);
}

void loss_grad_impl(hprqp_mlp& n, int B, const float* X, const float* T, const float* w, float* loss_host,
                    float* grad) {
  if (!T) mfail(HPRQP_ERR_ARG, "NULL targets");
  forward_impl(n, B, X);
  const int in = n.d[0], h1 = n.d[1], h2 = n.d[2], out = n.d[3];
  const int inp = n.dp[0], h1p = n.dp[1], h2p = n.dp[2], outp = n.dp[3];
  const int Bp = rup8(B);
  const double fwd_flop = n.last_flop;
  // loss and dY
  const int gl = eg((long long)B * out);
  k_standardize<<<gl, 256, 0, n.st>>>(B, out, T, n.out_mean, n.out_istd, n.Tstd);
  k_mse<<<gl, 256, 0, n.st>>>(B, out, n.Y, outp, n.Tstd, w, n.dYf, n.dYb, outp, n.part);
  // transposed copies (K = batch for the weight gradients)
  auto tr = [&](const uint16_t* src, uint16_t* dst, int cols_p) {
    dim3 g((cols_p + 31) / 32, (Bp + 31) / 32);
    k_transpose_bf16<<<g, 256, 0, n.st>>>(B, Bp, cols_p, src, dst);
  };
  tr(n.Xb, n.Xt, inp);
  tr(n.A1b, n.A1t, h1p);
  tr(n.A2b, n.A2t, h2p);
  tr(n.dYb, n.dYt, outp);
  float* G = n.G;
  mark(n);
  // layer 3
  gemm(n, out, h2, Bp, n.dYt, Bp, 1, n.A2t, 1, Bp, G + n.off_W[2], h2, 0);          // dW3 = dY^T A2
  k_colsum<<<cs_grid(out), 256, 0, n.st>>>(B, out, n.dYf, outp, G + n.off_b[2]);
  gemm(n, B, h2, outp, n.dYb, outp, 1, n.Wt[2], 1, outp, n.dA2, h2p, 0);             // dA2 = dY W3
  mark(n);
  k_gelu_bwd<<<eg((long long)B * h2), 256, 0, n.st>>>(B, h2, n.dA2, h2p, n.Z2, h2p, n.dZ2f, n.dZ2b, h2p);
  tr(n.dZ2b, n.dZ2t, h2p);
  mark(n);
  // layer 2
  gemm(n, h2, h1, Bp, n.dZ2t, Bp, 1, n.A1t, 1, Bp, G + n.off_W[1], h1, 0);          // dW2 = dZ2^T A1
  k_colsum<<<cs_grid(h2), 256, 0, n.st>>>(B, h2, n.dZ2f, h2p, G + n.off_b[1]);
  gemm(n, B, h1, h2p, n.dZ2b, h2p, 1, n.Wt[1], 1, h2p, n.dA1, h1p, 0);              // dA1 = dZ2 W2
  mark(n);
  k_gelu_bwd<<<eg((long long)B * h1), 256, 0, n.st>>>(B, h1, n.dA1, h1p, n.Z1, h1p, n.dZ1f, n.dZ1b, h1p);
  tr(n.dZ1b, n.dZ1t, h1p);
  mark(n);
  // layer 1
  gemm(n, h1, in, Bp, n.dZ1t, Bp, 1, n.Xt, 1, Bp, G + n.off_W[0], in, 0);           // dW1 = dZ1^T X
  k_colsum<<<cs_grid(h1), 256, 0, n.st>>>(B, h1, n.dZ1f, h1p, G + n.off_b[0]);
  mark(n);
  n.last_flop = fwd_flop + 2.0 * ((double)out * h2 * Bp + (double)B * h2 * outp + (double)h2 * h1 * Bp +
                                  (double)B * h1 * h2p + (double)h1 * in * Bp);
  if (grad) HMC(hipMemcpyAsync(grad, G, n.np * sizeof(float), hipMemcpyDeviceToDevice, n.st));
  std::vector<double> part(gl);
  HMC(hipMemcpyAsync(part.data(), n.part, gl * sizeof(double), hipMemcpyDeviceToHost, n.st));
  HMC(hipStreamSynchronize(n.st));
  double L = 0.0;
  for (double p : part) L += p;
  if (loss_host) *loss_host = (float)L;
}

}  // namespace

// mean and standard deviation (divisor rows - 1) of every column of X
// (rows x cols, device, FP32), FP64 on the device, into mean64/sd64 (device)
// and the host arrays mean_h/sd_h
void col_moments(hipStream_t st, long long rows, int cols, const float* X, float* mean_h, float* sd_h) {
  const int chunks = (int)((rows + HM_STAT_ROWS - 1) / HM_STAT_ROWS);
  double *part = nullptr, *mean = nullptr, *sd = nullptr;
  float* f32 = nullptr;
  const auto done = [&] {
    for (void* p : {(void*)part, (void*)mean, (void*)sd, (void*)f32})
      if (p) hipFree(p);
  };
  try {
    HMC(hipMalloc(&part, (size_t)chunks * cols * sizeof(double)));
    HMC(hipMalloc(&mean, cols * sizeof(double)));
    HMC(hipMalloc(&sd, cols * sizeof(double)));
    HMC(hipMalloc(&f32, cols * sizeof(float)));
    const dim3 g((cols + 255) / 256, chunks);
    k_col_stats<<<g, 256, 0, st>>>(rows, cols, X, nullptr, part);
    k_col_finish<<<(cols + 255) / 256, 256, 0, st>>>(chunks, cols, part, (double)rows, 0, mean, f32);
    HMC(hipMemcpyAsync(mean_h, f32, cols * sizeof(float), hipMemcpyDeviceToHost, st));
    k_col_stats<<<g, 256, 0, st>>>(rows, cols, X, mean, part);
    k_col_finish<<<(cols + 255) / 256, 256, 0, st>>>(chunks, cols, part, (double)std::max(1ll, rows - 1), 1, sd, f32);
    HMC(hipMemcpyAsync(sd_h, f32, cols * sizeof(float), hipMemcpyDeviceToHost, st));
    HMC(hipStreamSynchronize(st));
  } catch (...) {
    done();
    throw;
  }
  done();
}

#define HM_GUARD(...)                 \
  try {                               \
    hq::g_err.clear();                \
    __VA_ARGS__;                      \
    return HPRQP_OK;                  \
  } catch (const MErr& e) {           \
    hq::g_err = e.msg;                \
    return e.st;                      \
  } catch (const std::exception& e) { \
    hq::g_err = e.what();             \
    return HPRQP_ERR_HIP;             \
  }

extern "C" {

hprqp_status hprqp_mlp_create(const int32_t dims[4], int32_t max_batch, const float* params_host, hipStream_t stream,
                              hprqp_mlp** out) {
  HM_GUARD(create_impl(dims, max_batch, params_host, stream, out));
}

int64_t hprqp_mlp_num_params(const hprqp_mlp* n) { return n ? n->np : 0; }

hprqp_status hprqp_mlp_forward(hprqp_mlp* n, int32_t batch, const float* X, float* Y) {
  HM_GUARD(if (!n || !Y) mfail(HPRQP_ERR_ARG, "NULL argument"); forward_impl(*n, batch, X);
           k_destandardize<<<eg((long long)batch * n->d[3]), 256, 0, n->st>>>(batch, n->d[3], n->Y, n->dp[3],
                                                                             n->out_mean, n->out_sd, Y);
           HMC(hipStreamSynchronize(n->st)));
}

hprqp_status hprqp_mlp_set_scaling(hprqp_mlp* n, const float* in_mean, const float* in_std, const float* out_mean,
                                   const float* out_std) {
  HM_GUARD(
      if (!n || !in_mean || !in_std || !out_mean || !out_std) mfail(HPRQP_ERR_ARG, "NULL argument");
      std::vector<float> ii(n->d[0]), oi(n->d[3]);
      for (int i = 0; i < n->d[0]; ++i) ii[i] = in_std[i] > 1e-12f ? 1.0f / in_std[i] : 0.0f;
      for (int i = 0; i < n->d[3]; ++i) oi[i] = out_std[i] > 1e-12f ? 1.0f / out_std[i] : 0.0f;
      HMC(hipMemcpyAsync(n->in_mean, in_mean, n->d[0] * sizeof(float), hipMemcpyHostToDevice, n->st));
      HMC(hipMemcpyAsync(n->in_istd, ii.data(), n->d[0] * sizeof(float), hipMemcpyHostToDevice, n->st));
      HMC(hipMemcpyAsync(n->out_mean, out_mean, n->d[3] * sizeof(float), hipMemcpyHostToDevice, n->st));
      HMC(hipMemcpyAsync(n->out_sd, out_std, n->d[3] * sizeof(float), hipMemcpyHostToDevice, n->st));
      HMC(hipMemcpyAsync(n->out_istd, oi.data(), n->d[3] * sizeof(float), hipMemcpyHostToDevice, n->st));
      HMC(hipStreamSynchronize(n->st)));
}

hprqp_status hprqp_mlp_warm_start(hprqp_mlp* n, int32_t batch, const float* X, int32_t qn, int32_t qm, const double* L,
                                  const double* U, double* y0, double* w0, double* x0, int32_t* bad, float* score) {
  HM_GUARD(
      if (!n || !L || !U || !w0 || !x0 || !bad || (qm > 0 && !y0)) mfail(HPRQP_ERR_ARG, "NULL argument");
      if (qn <= 0 || qm < 0 || (qm + 2 * qn != n->d[3] && qm + 2 * qn + 1 != n->d[3]))
        mfail(HPRQP_ERR_SHAPE, "n_out must equal m + 2 n or m + 2 n + 1");
      if (score && qm + 2 * qn + 1 != n->d[3]) mfail(HPRQP_ERR_SHAPE, "score needs n_out = m + 2 n + 1");
      forward_impl(*n, batch, X);
      k_destandardize<<<eg((long long)batch * n->d[3]), 256, 0, n->st>>>(batch, n->d[3], n->Y, n->dp[3], n->out_mean,
                                                                        n->out_sd, n->Yuser);
      if (batch > 0)
        k_warm_start<<<batch, 256, 0, n->st>>>(batch, qn, qm, n->d[3], n->Yuser, L, U, y0, w0, x0, bad, score);
      HMC(hipGetLastError());
      HMC(hipStreamSynchronize(n->st)));
}

hprqp_status hprqp_mlp_fit_scaling(hprqp_mlp* n, int64_t rows, const float* X, const float* T, float* stats_host) {
  HM_GUARD(
      if (!n || !X || !T) mfail(HPRQP_ERR_ARG, "NULL argument");
      if (rows < 2) mfail(HPRQP_ERR_SHAPE, "at least two samples are needed");
      std::vector<float> xm(n->d[0]), xs(n->d[0]), tm(n->d[3]), ts(n->d[3]);
      col_moments(n->st, rows, n->d[0], X, xm.data(), xs.data());
      col_moments(n->st, rows, n->d[3], T, tm.data(), ts.data());
      if (stats_host) {
        float* o = stats_host;
        for (int i = 0; i < n->d[0]; ++i) { o[i] = xm[i]; o[n->d[0] + i] = xs[i]; }
        o += 2 * n->d[0];
        for (int i = 0; i < n->d[3]; ++i) { o[i] = tm[i]; o[n->d[3] + i] = ts[i]; }
      }
      const hprqp_status st = hprqp_mlp_set_scaling(n, xm.data(), xs.data(), tm.data(), ts.data());
      if (st != HPRQP_OK) mfail(st, hq::g_err));
}

hprqp_status hprqp_mlp_intermediate(hprqp_mlp* n, int32_t which, float* out, int32_t* rows_host, int32_t* cols_host) {
  HM_GUARD(
      if (!n) mfail(HPRQP_ERR_ARG, "NULL handle");
      const int B = n->last_batch;
      const int in = n->d[0], h1 = n->d[1], h2 = n->d[2], o = n->d[3];
      const int inp = n->dp[0], h1p = n->dp[1], h2p = n->dp[2], op = n->dp[3];
      struct Src { int cols; long long ld; const float* f; const uint16_t* b; };
      Src s{};
      switch (which) {
        case 0: s = {in, inp, nullptr, n->Xb}; break;
        case 1: s = {h1, h1p, n->Z1, nullptr}; break;
        case 2: s = {h1, h1p, nullptr, n->A1b}; break;
        case 3: s = {h2, h2p, n->Z2, nullptr}; break;
        case 4: s = {h2, h2p, nullptr, n->A2b}; break;
        case 5: s = {o, op, n->Y, nullptr}; break;
        case 6: s = {o, op, n->dYf, nullptr}; break;
        case 7: s = {o, op, nullptr, n->dYb}; break;
        case 8: s = {h2, h2p, n->dA2, nullptr}; break;
        case 9: s = {h2, h2p, n->dZ2f, nullptr}; break;
        case 10: s = {h2, h2p, nullptr, n->dZ2b}; break;
        case 11: s = {h1, h1p, n->dA1, nullptr}; break;
        case 12: s = {h1, h1p, n->dZ1f, nullptr}; break;
        case 13: s = {h1, h1p, nullptr, n->dZ1b}; break;
        case 14: s = {o, o, n->Tstd, nullptr}; break;
        default: mfail(HPRQP_ERR_ARG, "which must be in [0, 14]");
      }
      if (rows_host) *rows_host = B;
      if (cols_host) *cols_host = s.cols;
      if (out && B > 0) {
        k_export<<<eg((long long)B * s.cols), 256, 0, n->st>>>(B, s.cols, s.ld, s.f, s.b, out);
        HMC(hipGetLastError());
      }
      HMC(hipStreamSynchronize(n->st)));
}

hprqp_status hprqp_family_features(int32_t batch, int32_t n, int32_t m, const double* c, const double* u, float* X,
                                   hipStream_t stream) {
  HM_GUARD(if (batch < 0 || n <= 0 || m < 0 || !c || !X || (m > 0 && !u)) mfail(HPRQP_ERR_ARG, "bad arguments");
           if (batch > 0) k_family_features<<<eg((long long)batch * (n + m)), 256, 0, stream>>>(batch, n, m, c, u, X);
           HMC(hipGetLastError()); HMC(hipStreamSynchronize(stream)));
}

hprqp_status hprqp_family_targets(int32_t batch, int32_t n, int32_t m, const double* y, const double* z,
                                  const double* w, const int64_t* iters, float* T, hipStream_t stream) {
  HM_GUARD(if (batch < 0 || n <= 0 || m < 0 || !z || !w || !T || (m > 0 && !y)) mfail(HPRQP_ERR_ARG, "bad arguments");
           if (batch > 0)
             k_family_targets<<<eg((long long)batch * (m + 2 * n + 1)), 256, 0, stream>>>(
                 batch, n, m, y, z, w, reinterpret_cast<const long long*>(iters), T);
           HMC(hipGetLastError()); HMC(hipStreamSynchronize(stream)));
}

hprqp_status hprqp_mlp_loss_grad(hprqp_mlp* n, int32_t batch, const float* X, const float* T, const float* out_w,
                                 float* loss_host, float* grad) {
  HM_GUARD(if (!n) mfail(HPRQP_ERR_ARG, "NULL handle"); loss_grad_impl(*n, batch, X, T, out_w, loss_host, grad));
}

hprqp_status hprqp_mlp_adam(hprqp_mlp* n, float lr, float beta1, float beta2, float eps) {
  HM_GUARD(if (!n) mfail(HPRQP_ERR_ARG, "NULL handle"); n->adam_t += 1;
           const float c1 = 1.0f - std::pow(beta1, (float)n->adam_t);
           const float c2 = 1.0f - std::pow(beta2, (float)n->adam_t);
           k_adam<<<eg(n->np), 256, 0, n->st>>>(n->np, n->P, n->G, n->Mm, n->Vv, lr, beta1, beta2, eps, c1, c2);
           refresh_weights(*n));
}

hprqp_status hprqp_mlp_get_params(hprqp_mlp* n, float* params_host) {
  HM_GUARD(if (!n || !params_host) mfail(HPRQP_ERR_ARG, "NULL argument");
           HMC(hipMemcpyAsync(params_host, n->P, n->np * sizeof(float), hipMemcpyDeviceToHost, n->st));
           HMC(hipStreamSynchronize(n->st)));
}

hprqp_status hprqp_mlp_set_params(hprqp_mlp* n, const float* params_host) {
  HM_GUARD(if (!n || !params_host) mfail(HPRQP_ERR_ARG, "NULL argument");
           HMC(hipMemcpyAsync(n->P, params_host, n->np * sizeof(float), hipMemcpyHostToDevice, n->st));
           refresh_weights(*n); HMC(hipStreamSynchronize(n->st)));
}

hprqp_status hprqp_mlp_gemm_stats(hprqp_mlp* n, double* ms_host, double* flop_host) {
  HM_GUARD(if (!n) mfail(HPRQP_ERR_ARG, "NULL handle"); HMC(hipStreamSynchronize(n->st)); double ms = 0.0;
           // GEMM intervals: forward (ev0-1, ev2-3, ev4-5); backward (ev6-7 ... ev10-11) if present
           for (int i = 0; i + 1 < n->nev; i += 2) {
             float t = 0.f;
             HMC(hipEventElapsedTime(&t, n->ev[i], n->ev[i + 1]));
             ms += t;
           } if (ms_host) *ms_host = ms;
           if (flop_host) *flop_host = n->last_flop);
}

void hprqp_mlp_destroy(hprqp_mlp* n) { delete n; }

hprqp_status hprqp_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t* A, int64_t a_rs, int64_t a_cs,
                             const uint16_t* B, int64_t b_rs, int64_t b_cs, float* C, int64_t ldc, int32_t accumulate,
                             int32_t split_k, float* workspace, hipStream_t stream) {
  HM_GUARD(if (M < 0 || N < 0 || K < 0 || !A || !B || !C) mfail(HPRQP_ERR_ARG, "bad GEMM arguments");
           if (split_k < 1 || split_k > 64) mfail(HPRQP_ERR_ARG, "split_k must be in [1, 64]");
           if (split_k > 1 && !workspace) mfail(HPRQP_ERR_ARG, "split_k > 1 needs a workspace of split_k M N floats");
           if (M > 0 && N > 0)
             gemm_split(stream, M, N, K, A, a_rs, a_cs, B, b_rs, b_cs, C, ldc, accumulate, split_k, workspace);
           HMC(hipGetLastError()); HMC(hipStreamSynchronize(stream)));
}

}  // extern "C"
