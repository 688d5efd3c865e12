// Kernel of the exact ray-patch crossing count (the walk is in patches.hpp).
#include "patches.hpp"

namespace wn {

namespace {

__global__ __launch_bounds__(kPThreads) void k_patches3d(Frame F, const float* __restrict__ nets, int32_t np,
                                                        const float* __restrict__ qx, const float* __restrict__ qy,
                                                        const float* __restrict__ qz, int64_t nq,
                                                        int32_t* __restrict__ chi_out) {
  __shared__ PatchRot sp[kPatchChunk];
  const int64_t qi = (int64_t)blockIdx.x * kPThreads + threadIdx.x;
  const bool ok = qi < nq;
  const int64_t q = ok ? qi : 0;
  const float px = qx[q], py = qy[q], pz = qz[q];
  const bool fin = isfinite(px) && isfinite(py) && isfinite(pz);
  double Xp, Yp, Zp;
  rotate(F, px, py, pz, Xp, Yp, Zp);
  int chi = 0;
  for (int c0 = 0; c0 < np; c0 += kPatchChunk) {
    const int cnt = min(kPatchChunk, np - c0);
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kPThreads) stage_patch(F, nets, c0 + j, &sp[j]);
    __syncthreads();
    if (ok && fin) chi += patches_chi(sp, cnt, Xp, Yp, Zp);
  }
  if (ok) chi_out[qi] = fin ? chi : WN_CHI_INVALID;
}

}  // namespace

hipError_t launch_patches3d(const Frame& F, const float* nets, int64_t np, const float* qx, const float* qy,
                            const float* qz, int64_t nq, int32_t* chi_out, hipStream_t s) {
  const int64_t blocks = (nq + kPThreads - 1) / kPThreads;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_patches3d, dim3((unsigned)blocks), dim3(kPThreads), 0, s, F, nets, (int32_t)np, qx, qy, qz,
                     nq, chi_out);
  return hipGetLastError();
}

}  // namespace wn
