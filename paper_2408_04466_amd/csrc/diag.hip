// Diagnostics over a call's outputs: how many queries were not finite and
// how many finite queries still came back with the invalid crossing count
// (a traversal that found the tree malformed).  Integer counts, so the
// atomic order does not matter and the result is deterministic.
#include <algorithm>

#include "bvh_build.hpp"
#include "kernels.hpp"

namespace wn {

namespace {

constexpr int kDThreads = 256;

__global__ __launch_bounds__(kDThreads) void k_diagnose(const float* __restrict__ qx, const float* __restrict__ qy,
                                                       const float* __restrict__ qz,
                                                       const int32_t* __restrict__ chi, int64_t n,
                                                       unsigned long long* __restrict__ counts) {
  __shared__ unsigned red[2][kDThreads / 64];
  unsigned nonfin = 0, failed = 0;
  for (int64_t i = (int64_t)blockIdx.x * kDThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kDThreads) {
    const bool fin = isfinite(qx[i]) && isfinite(qy[i]) && isfinite(qz[i]);
    nonfin += fin ? 0u : 1u;
    failed += (fin && chi[i] == WN_CHI_INVALID) ? 1u : 0u;
  }
  for (int o = 32; o > 0; o >>= 1) {
    nonfin += __shfl_xor(nonfin, o, 64);
    failed += __shfl_xor(failed, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = nonfin;
    red[1][threadIdx.x >> 6] = failed;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    unsigned long long s = 0;
    for (int w = 0; w < kDThreads / 64; ++w) s += red[threadIdx.x][w];
    if (s) atomicAdd(&counts[threadIdx.x], s);
  }
}

}  // namespace

hipError_t diagnose(const float* qx, const float* qy, const float* qz, const int32_t* chi, int64_t n,
                    int64_t* counts, hipStream_t s) {
  hipError_t e = fill_u32(reinterpret_cast<unsigned*>(counts), 4, 0u, s);
  if (e != hipSuccess || n == 0) return e;
  // at most 4096 x 256 lanes: a workgroup's 32-bit sum holds 256 lanes of
  // ceil(n / 2^20) each, so up to 2^44 queries
  const int64_t blocks = std::min<int64_t>((n + kDThreads - 1) / kDThreads, 4096);
  hipLaunchKernelGGL(k_diagnose, dim3((unsigned)blocks), dim3(kDThreads), 0, s, qx, qy, qz, chi, n,
                     reinterpret_cast<unsigned long long*>(counts));
  return hipGetLastError();
}

}  // namespace wn
