// transpose.hip -- explicit A^T (CSR of an m x n CSR matrix) built on the device.
//
// Entries of each row of A^T are ordered by the row index of A: a stable
// radix sort of the nonzeros by column (keys) carrying their position
// (values) gives exactly that order, so every later A^T product has a fixed
// summation order.  A one-time histogram + scan produces the row pointers.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <stdint.h>

namespace {

__global__ void k_row_ids(int m, const int* __restrict__ rowptr, int* __restrict__ rid) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) rid[k] = i;
}

__global__ void k_iota(int64_t nnz, int* __restrict__ v) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x)
    v[k] = (int)k;
}

__global__ void k_zero_int(int n, int* __restrict__ v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) v[i] = 0;
}

__global__ void k_hist(int64_t nnz, const int* __restrict__ col, int* __restrict__ cnt) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[col[k]], 1);
}

__global__ void k_gather_t(int64_t nnz, const int* __restrict__ perm, const int* __restrict__ rid,
                           const double* __restrict__ val, int* __restrict__ tcol, double* __restrict__ tval,
                           int* __restrict__ tperm) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x) {
    const int p = perm[k];
    tcol[k] = rid[p];
    tval[k] = val[p];
    if (tperm) tperm[k] = p;
  }
}

int grid_for(int64_t work) {
  int64_t g = (work + 255) / 256;
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (int)g;
}

}  // namespace

// t_rowptr: n+1 ints, t_col: nnz ints, t_val: nnz doubles (device);
// t_perm (nnz ints, may be NULL): position in A of each entry of A^T.
hipError_t hq_build_transpose(int m, int n, int64_t nnz, const int* rowptr, const int* col, const double* val,
                              int* t_rowptr, int* t_col, double* t_val, int* t_perm, hipStream_t st) {
  hipError_t err = hipSuccess;
  k_zero_int<<<grid_for(n + 1), 256, 0, st>>>(n + 1, t_rowptr);
  if (nnz == 0) return hipGetLastError();
  int *rid = nullptr, *keys_in = nullptr, *keys_out = nullptr, *vals_in = nullptr, *vals_out = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0, tmp2 = 0;
  int bits = 1;
  while (bits < 31 && (1 << bits) < n) ++bits;
#define HQ_TRY(x) do { err = (x); if (err != hipSuccess) goto done; } while (0)
  HQ_TRY(hipMalloc(&rid, nnz * sizeof(int)));
  HQ_TRY(hipMalloc(&keys_out, nnz * sizeof(int)));
  HQ_TRY(hipMalloc(&vals_in, nnz * sizeof(int)));
  HQ_TRY(hipMalloc(&vals_out, nnz * sizeof(int)));
  keys_in = const_cast<int*>(col);
  k_row_ids<<<grid_for(m), 256, 0, st>>>(m, rowptr, rid);
  k_iota<<<grid_for(nnz), 256, 0, st>>>(nnz, vals_in);
  HQ_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys_in, keys_out, vals_in, vals_out,
                                            (int)nnz, 0, bits, st));
  HQ_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp2, t_rowptr, t_rowptr, n + 1, st));
  if (tmp2 > tmp_bytes) tmp_bytes = tmp2;
  HQ_TRY(hipMalloc(&tmp, tmp_bytes));
  HQ_TRY(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys_in, keys_out, vals_in, vals_out,
                                            (int)nnz, 0, bits, st));
  k_gather_t<<<grid_for(nnz), 256, 0, st>>>(nnz, vals_out, rid, val, t_col, t_val, t_perm);
  k_hist<<<grid_for(nnz), 256, 0, st>>>(nnz, col, t_rowptr);
  {
    size_t b = tmp_bytes;
    HQ_TRY(hipcub::DeviceScan::ExclusiveSum(tmp, b, t_rowptr, t_rowptr, n + 1, st));
  }
  HQ_TRY(hipStreamSynchronize(st));
done:
#undef HQ_TRY
  if (rid) hipFree(rid);
  if (keys_out) hipFree(keys_out);
  if (vals_in) hipFree(vals_in);
  if (vals_out) hipFree(vals_out);
  if (tmp) hipFree(tmp);
  return err;
}
