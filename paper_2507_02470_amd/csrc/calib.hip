// calib.hip -- a plain streaming copy, outside the solver: the benchmark runs
// it to scale the HBM byte counters (FETCH_SIZE, WRITE_SIZE) by what they read
// for a known number of bytes, and to measure the HBM rate this part reaches
// with nothing but coalesced streaming.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdint>
#include <string>
#include "hprqp.h"

namespace hq {
extern thread_local std::string g_err;
}

namespace {

hprqp_status calib_fail(hprqp_status st, const char* msg) {
  hq::g_err = msg;
  return st;
}

#define HC_BS 256
#define HC_UNROLL 4

// 16-byte loads and stores; each thread moves HC_UNROLL vectors per step,
// HC_BS apart, so every load instruction of a wave covers 1 KiB contiguously
__global__ __launch_bounds__(HC_BS) void k_stream_copy2(long long n2, const double2* __restrict__ s,
                                                        double2* __restrict__ d) {
  const long long step = (long long)gridDim.x * HC_BS * HC_UNROLL;
  for (long long base = (long long)blockIdx.x * HC_BS * HC_UNROLL + threadIdx.x; base < n2; base += step) {
    double2 r[HC_UNROLL];
#pragma unroll
    for (int u = 0; u < HC_UNROLL; ++u) {
      const long long i = base + (long long)u * HC_BS;
      if (i < n2) r[u] = s[i];
    }
#pragma unroll
    for (int u = 0; u < HC_UNROLL; ++u) {
      const long long i = base + (long long)u * HC_BS;
      if (i < n2) d[i] = r[u];
    }
  }
}

__global__ void k_stream_copy1(long long n, const double* __restrict__ s, double* __restrict__ d) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    d[i] = s[i];
}

}  // namespace

extern "C" hprqp_status hprqp_stream_copy(const double* src, double* dst, int64_t n, hipStream_t stream,
                                          double* ms_host) {
  hq::g_err.clear();
  if (n < 0 || (n > 0 && (!src || !dst))) return calib_fail(HPRQP_ERR_ARG, "bad arguments");
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return calib_fail(HPRQP_ERR_HIP, "no device");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms_host && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
    if (e0) hipEventDestroy(e0);
    return calib_fail(HPRQP_ERR_HIP, "hipEventCreate failed");
  }
  if (e0) hipEventRecord(e0, stream);
  if (n > 0) {
    const bool vec = ((uintptr_t)src % 16 == 0) && ((uintptr_t)dst % 16 == 0);
    if (vec) {
      const long long n2 = n / 2;
      if (n2 > 0) {
        const long long blocks = (n2 + HC_BS * HC_UNROLL - 1) / (HC_BS * HC_UNROLL);
        const int grid = (int)std::min<long long>(blocks, (long long)ncu * 16);
        k_stream_copy2<<<grid, HC_BS, 0, stream>>>(n2, reinterpret_cast<const double2*>(src),
                                                   reinterpret_cast<double2*>(dst));
      }
      if (n % 2) k_stream_copy1<<<1, 64, 0, stream>>>(1, src + n - 1, dst + n - 1);
    } else {
      const long long blocks = (n + 255) / 256;
      k_stream_copy1<<<(int)std::min<long long>(blocks, (long long)ncu * 16), 256, 0, stream>>>(n, src, dst);
    }
  }
  hipError_t err = hipGetLastError();
  if (e1) {
    hipEventRecord(e1, stream);
    hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    *ms_host = ms;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
  }
  if (err != hipSuccess) return calib_fail(HPRQP_ERR_HIP, hipGetErrorString(err));
  return HPRQP_OK;
}
