// precond.hip -- diagonal preconditioning of Section 4.1 of arXiv 2507.02470
// ("Preconditioning"): Ruiz equilibration passes followed by one
// Pock-Chambolle pass with alpha = 1, for a QP whose Q is an explicit matrix.
//
// The scaling is symmetric on K = [[Q, A^T], [A, 0]]: D scales the variables,
// E the rows of A.  Every pass computes the row norms of the currently scaled
// K (inf-norm for Ruiz, 1-norm for Pock-Chambolle) and divides each scale by
// the square root of its row's norm (rows of norm 0 keep their scale).  The
// row of variable j holds row j of D Q D and column j of E A D (= row j of
// the stored A^T, entries ordered by row of A); the row of constraint i is
// row i of E A D.  One thread per row, fixed summation order: deterministic.
//
// Results: D, E and the scaled data Q~ = D Q D, A~ = E A D (and its A^T, by
// the transpose permutation), c~ = D c, [L, U]~ = [L, U] / D, [l, u]~ = E [l, u].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "precond.hpp"

namespace {

__global__ void k_ones(int k, double* __restrict__ v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) v[i] = 1.0;
}

// out[r] = norm over the row r of the scaled entries; P1: 1-norm, else
// inf-norm.  An entry is |rs[r] val cs[col]|, multiplied left to right in the
// order (row scale of A, value, column scale of A): TRANS marks the rows of
// A^T, whose row scale is A's column scale.
template <bool P1, bool TRANS>
__global__ void k_row_norms(int rows, const int* __restrict__ rp, const int* __restrict__ ci,
                            const double* __restrict__ val, const double* __restrict__ rs,
                            const double* __restrict__ cs, double* __restrict__ out) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) {
    double acc = 0.0;
    const double f = rs[r];
    for (int k = rp[r]; k < rp[r + 1]; ++k) {
      const double a = TRANS ? fabs(cs[ci[k]] * val[k] * f) : fabs(f * val[k] * cs[ci[k]]);
      acc = P1 ? acc + a : fmax(acc, a);
    }
    out[r] = acc;
  }
}

// Variable rows: combine the Q part and the A^T part, then scale.
template <bool P1>
__global__ void k_update_var_scale(int n, const double* __restrict__ nq, const double* __restrict__ na,
                                   double* __restrict__ D) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const double a = nq ? nq[j] : 0.0, b = na ? na[j] : 0.0;
    const double v = P1 ? a + b : fmax(a, b);
    if (v > 0.0) D[j] /= sqrt(v);
  }
}

__global__ void k_update_row_scale(int m, const double* __restrict__ nrm, double* __restrict__ E) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    if (nrm[i] > 0.0) E[i] /= sqrt(nrm[i]);
}

// out[k] = rs[r] * val[k] * cs[col[k]] over a CSR matrix
__global__ void k_scale_csr(int rows, const int* __restrict__ rp, const int* __restrict__ ci,
                            const double* __restrict__ val, const double* __restrict__ rs,
                            const double* __restrict__ cs, double* __restrict__ out) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) {
    const double f = rs[r];
    for (int k = rp[r]; k < rp[r + 1]; ++k) out[k] = f * val[k] * cs[ci[k]];
  }
}

__global__ void k_permute(int64_t nnz, const int* __restrict__ perm, const double* __restrict__ src,
                          double* __restrict__ dst) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x)
    dst[k] = src[perm[k]];
}

__global__ void k_scale_var_data(int n, const double* __restrict__ D, const double* __restrict__ c,
                                 const double* __restrict__ L, const double* __restrict__ U, double* __restrict__ cs,
                                 double* __restrict__ Ls, double* __restrict__ Us) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    cs[j] = D[j] * c[j];
    Ls[j] = L[j] / D[j];     // +-inf stays +-inf (D > 0)
    Us[j] = U[j] / D[j];
  }
}

__global__ void k_scale_row_data(int m, const double* __restrict__ E, const double* __restrict__ l,
                                 const double* __restrict__ u, double* __restrict__ ls, double* __restrict__ us) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    ls[i] = E[i] * l[i];
    us[i] = E[i] * u[i];
  }
}

int grid_of(long long work) {
  long long g = (work + 255) / 256;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  return (int)g;
}

// one pass: norms of the currently scaled K, then the scale update
template <bool P1>
void pass(const HqPrecondIn& in, const HqPrecondOut& out, hipStream_t st) {
  const int n = in.n, m = in.m;
  const int gn = grid_of(n), gm = grid_of(m);
  double* nq = in.q_rp ? out.work_n : nullptr;
  double* na = m > 0 ? out.work_n2 : nullptr;
  if (nq) k_row_norms<P1, false><<<gn, 256, 0, st>>>(n, in.q_rp, in.q_ci, in.q_v, out.D, out.D, nq);
  if (m > 0) {
    k_row_norms<P1, true><<<gn, 256, 0, st>>>(n, in.at_rp, in.at_ci, in.at_v, out.D, out.E, na);
    k_row_norms<P1, false><<<gm, 256, 0, st>>>(m, in.a_rp, in.a_ci, in.a_v, out.E, out.D, out.work_m);
  }
  // all norms of this pass are taken before any scale changes
  k_update_var_scale<P1><<<gn, 256, 0, st>>>(n, nq, na, out.D);
  if (m > 0) k_update_row_scale<<<gm, 256, 0, st>>>(m, out.work_m, out.E);
}

}  // namespace

hipError_t hq_precondition(const HqPrecondIn& in, const HqPrecondOut& out, hipStream_t st) {
  const int n = in.n, m = in.m;
  k_ones<<<grid_of(n), 256, 0, st>>>(n, out.D);
  if (m > 0) k_ones<<<grid_of(m), 256, 0, st>>>(m, out.E);
  for (int it = 0; it < in.ruiz_iters; ++it) pass<false>(in, out, st);
  pass<true>(in, out, st);
  if (in.q_rp) k_scale_csr<<<grid_of(n), 256, 0, st>>>(n, in.q_rp, in.q_ci, in.q_v, out.D, out.D, out.q_v);
  if (m > 0) {
    k_scale_csr<<<grid_of(m), 256, 0, st>>>(m, in.a_rp, in.a_ci, in.a_v, out.E, out.D, out.a_v);
    k_permute<<<grid_of(in.a_nnz), 256, 0, st>>>(in.a_nnz, in.at_perm, out.a_v, out.at_v);
    k_scale_row_data<<<grid_of(m), 256, 0, st>>>(m, out.E, in.l, in.u, out.l, out.u);
  }
  k_scale_var_data<<<grid_of(n), 256, 0, st>>>(n, out.D, in.c, in.L, in.U, out.c, out.L, out.U);
  return hipGetLastError();
}
