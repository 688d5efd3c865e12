// Many parametric surfaces in one launch: every surface has its own bicubic
// patches, boundary curves, ray direction and query range; each workgroup
// takes 256 consecutive queries of one surface and computes chi_d with the
// patch walk of patches.hpp and, when w is wanted, Theta with the curve walk
// of curves.hpp, then w = chi_d + Theta / (2 pi) (Sec. 5.1, "Parametric Surfaces";
// Eq. of the one-shot winding number).  The arithmetic per query is that of
// the single-surface path, in the same order, so a batched result equals
// the single call's bit for bit.
#include <vector>

#include "curves.hpp"
#include "patches.hpp"

namespace wn {

namespace {

constexpr int kSThreads = 256;
static_assert(kSThreads == kPThreads && kSThreads == kCThreads, "one query per lane, as the single-surface kernels");

constexpr size_t kStageBytes = sizeof(PatchRot) * kPatchChunk > sizeof(CurveRot) * kCurveChunk
                                   ? sizeof(PatchRot) * kPatchChunk
                                   : sizeof(CurveRot) * kCurveChunk;

// The work of one workgroup: 256 consecutive queries of the surface D.
__device__ __forceinline__ void psurf_tile(const PSurf& D, int64_t blk, const float* __restrict__ nets,
                                           const float* __restrict__ curves, const float* __restrict__ qx,
                                           const float* __restrict__ qy, const float* __restrict__ qz,
                                           float* __restrict__ w_out, int32_t* __restrict__ chi_out) {
  // patches and curves are staged one after the other through the same LDS
  __shared__ double stage[kStageBytes / sizeof(double)];
  PatchRot* sp = reinterpret_cast<PatchRot*>(stage);
  CurveRot* sc = reinterpret_cast<CurveRot*>(stage);
  const Frame F = D.F;
  const int64_t li = (blk - D.blk0) * kSThreads + threadIdx.x;
  const bool ok = li < D.nq;
  const int64_t q = D.q0 + (ok ? li : 0);
  const float px = qx[q], py = qy[q], pz = qz[q];
  const bool fin = isfinite(px) && isfinite(py) && isfinite(pz);
  double Xp, Yp, Zp;
  rotate(F, px, py, pz, Xp, Yp, Zp);
  const float* nb = nets + 48 * D.patch0;
  int chi = 0;
  for (int c0 = 0; c0 < D.npatch; c0 += kPatchChunk) {
    const int cnt = min(kPatchChunk, D.npatch - c0);
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kSThreads) stage_patch(F, nb, c0 + j, &sp[j]);
    __syncthreads();
    if (ok && fin) chi += patches_chi(sp, cnt, Xp, Yp, Zp);
  }
  if (w_out) {
    const float* cb = curves + 12 * D.curve0;
    double theta = 0.0;
    for (int c0 = 0; c0 < D.ncurve; c0 += kCurveChunk) {
      const int cnt = min(kCurveChunk, D.ncurve - c0);
      __syncthreads();
      for (int j = threadIdx.x; j < cnt; j += kSThreads) stage_curve(F, cb, c0 + j, &sc[j]);
      __syncthreads();
      if (ok && fin) theta += curves_theta(sc, cnt, Xp, Yp, Zp);
    }
    if (ok) w_out[q] = fin ? __fadd_rn((float)chi, __fmul_rn((float)theta, kInv2Pi)) : __int_as_float(0x7fc00000);
  }
  if (ok && chi_out) chi_out[q] = fin ? chi : WN_CHI_INVALID;
}

__global__ __launch_bounds__(kSThreads) void k_psurf_batched(const PSurf* __restrict__ desc,
                                                            const int32_t* __restrict__ blk_surf,
                                                            const float* __restrict__ nets,
                                                            const float* __restrict__ curves,
                                                            const float* __restrict__ qx, const float* __restrict__ qy,
                                                            const float* __restrict__ qz, float* __restrict__ w_out,
                                                            int32_t* __restrict__ chi_out) {
  psurf_tile(desc[blk_surf[blockIdx.x]], blockIdx.x, nets, curves, qx, qy, qz, w_out, chi_out);
}

// One surface, its descriptor in the kernel arguments (the single-surface
// entry point).
__global__ __launch_bounds__(kSThreads) void k_psurf_one(PSurf one, const float* __restrict__ nets,
                                                        const float* __restrict__ curves,
                                                        const float* __restrict__ qx, const float* __restrict__ qy,
                                                        const float* __restrict__ qz, float* __restrict__ w_out,
                                                        int32_t* __restrict__ chi_out) {
  psurf_tile(one, blockIdx.x, nets, curves, qx, qy, qz, w_out, chi_out);
}

}  // namespace

PBatch::~PBatch() {
  if (ws) (void)hipFree(ws);
}

hipError_t pbatch_create(const PSurf* surfs, int32_t n, hipStream_t s, PBatch* b) {
  std::vector<PSurf> d(surfs, surfs + n);
  std::vector<int32_t> bs;
  int64_t p = 0, c = 0, q = 0, blocks = 0;
  for (int32_t k = 0; k < n; ++k) {
    d[k].patch0 = p;
    d[k].curve0 = c;
    d[k].q0 = q;
    d[k].blk0 = blocks;
    const int64_t nb = (d[k].nq + kSThreads - 1) / kSThreads;
    bs.insert(bs.end(), (size_t)nb, k);
    p += d[k].npatch;
    c += d[k].ncurve;
    q += d[k].nq;
    blocks += nb;
  }
  b->nsurf = n;
  b->npatch = p;
  b->ncurve = c;
  b->nq = q;
  b->nblocks = blocks;
  if (blocks == 0) return hipSuccess;
  const size_t b_desc = ((size_t)n * sizeof(PSurf) + 255) & ~(size_t)255;
  hipError_t e = hipMalloc((void**)&b->ws, b_desc + bs.size() * sizeof(int32_t));
  if (e != hipSuccess) {
    b->ws = nullptr;
    return e;
  }
  b->desc = reinterpret_cast<PSurf*>(b->ws);
  b->blk_surf = reinterpret_cast<int32_t*>(b->ws + b_desc);
  e = hipMemcpyAsync(b->desc, d.data(), (size_t)n * sizeof(PSurf), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->blk_surf, bs.data(), bs.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);   // the host tables go out of scope
}

hipError_t eval_pbatch(const PBatch& b, const float* nets, const float* curves, const float* qx, const float* qy,
                       const float* qz, float* w_out, int32_t* chi_out, hipStream_t s) {
  if (b.nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_psurf_batched, dim3((unsigned)b.nblocks), dim3(kSThreads), 0, s, b.desc, b.blk_surf, nets,
                     curves, qx, qy, qz, w_out, chi_out);
  return hipGetLastError();
}

hipError_t launch_psurf_single(const Frame& F, const float* nets, int64_t np, const float* curves, int64_t nc,
                               const float* qx, const float* qy, const float* qz, int64_t nq, float* w_out,
                               int32_t* chi_out, hipStream_t s) {
  const int64_t blocks = (nq + kSThreads - 1) / kSThreads;
  if (blocks == 0) return hipSuccess;
  PSurf one{};
  one.F = F;
  one.nq = nq;
  one.npatch = (int32_t)np;
  one.ncurve = (int32_t)nc;
  hipLaunchKernelGGL(k_psurf_one, dim3((unsigned)blocks), dim3(kSThreads), 0, s, one, nets, curves, qx, qy, qz, w_out,
                     chi_out);
  return hipGetLastError();
}

}  // namespace wn
