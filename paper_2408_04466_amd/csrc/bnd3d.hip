// Boundary line integral of the one-shot winding number (3D) and the final
// combine w = chi_d + S/(2 pi): one lane per query (QPL queries per lane),
// queries read as coalesced structure-of-arrays; the boundary walk itself is
// in bndloop.hpp.
#include <cstdlib>

#include "bndloop.hpp"
#include "bvh_build.hpp"
#include "traverse.hpp"

namespace wn {

namespace {

using namespace bnd;

// Eight waves per SIMD for one query per lane (57 registers, no spills).
template <int QPL>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(QPL == 1 ? 8 : 4))) void k_bnd3d(BndArgs a, LoopTable L) {
  __shared__ RPt sv[kChunk];

  Lane<QPL> s;
  int64_t qi[QPL];
  bool ok[QPL];
  const int64_t base = (int64_t)blockIdx.x * (kThreads * QPL) + threadIdx.x;
#pragma unroll
  for (int j = 0; j < QPL; ++j) {
    qi[j] = base + (int64_t)j * kThreads;
    ok[j] = qi[j] < a.nq;
    const int64_t q = ok[j] ? qi[j] : 0;
    double X, Y, Z;
    rotate(a.F, a.qx[q], a.qy[q], a.qz[q], X, Y, Z);
    s.p[j] = make_qp(X, Y, Z);
    turns_init(s.T[j]);
  }
  lane_range(s);

  int staged = -1, pend = 0;
  const KernargLoops KL{L};
  boundary_walk(s, StageRotate<KernargLoops>{a.F, a.bnd, KL}, a.nb, KL, sv, staged, pend);
  finish_turns(s, pend);

#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    if (!ok[k]) continue;
    const int64_t q = qi[k];
    const int chi = a.chi_in[q];
    float w;
    if (chi == WN_CHI_INVALID || !(isfinite(a.qx[q]) && isfinite(a.qy[q]) && isfinite(a.qz[q]))) {
      w = __int_as_float(0x7fc00000);
    } else {
      w = lane_w(s, k, chi);
    }
    a.w_out[q] = w;
  }
}

// Fused forward, one query per lane: the crossing count (BVH traversal),
// then the boundary walk, then w.  While some waves wait on node fetches,
// others keep the vector units busy with the boundary arithmetic.
// Seven waves per SIMD (measured: eight, with the node fetches of more
// concurrent traversals, and six are both slower).
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(7))) void k_fwd3d(CrossArgs c, BndArgs a, LoopTable L, int32_t* chi_out) {
  __shared__ RPt sv[kChunk];
  const int64_t qi = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool ok = qi < a.nq;
  const int64_t q = ok ? qi : 0;
  const float px = a.qx[q], py = a.qy[q], pz = a.qz[q];
  const bool fin = isfinite(px) && isfinite(py) && isfinite(pz);
  Lane<1> s;
  {
    double X, Y, Z;
    rotate(a.F, px, py, pz, X, Y, Z);
    s.p[0] = make_qp(X, Y, Z);
  }
  turns_init(s.T[0]);
  lane_range(s);
  // odd workgroups walk the boundary first (uniform per workgroup, so the
  // staging barriers still meet): node fetches and boundary arithmetic then
  // overlap on every SIMD from the start
  int staged = -1, pend = 0;
  const KernargLoops KL{L};
  if (blockIdx.x & 1) boundary_walk(s, StageRotate<KernargLoops>{a.F, a.bnd, KL}, a.nb, KL, sv, staged, pend);
  const int chi = (ok && fin) ? traverse<kShortStack>(c, s.p[0]) : WN_CHI_INVALID;
  if (!(blockIdx.x & 1)) boundary_walk(s, StageRotate<KernargLoops>{a.F, a.bnd, KL}, a.nb, KL, sv, staged, pend);
  finish_turns(s, pend);
  if (ok) {
    a.w_out[q] = chi != WN_CHI_INVALID ? lane_w(s, 0, chi) : __int_as_float(0x7fc00000);
    if (chi_out) chi_out[q] = chi;
  }
}

}  // namespace

hipError_t launch_fwd3d(const CrossArgs& c, const BndArgs& a, const LoopTable& L, int32_t* chi_out,
                        hipStream_t s) {
  const int64_t blocks = (a.nq + kThreads - 1) / kThreads;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fwd3d, dim3((unsigned)blocks), dim3(kThreads), 0, s, c, a, L, chi_out);
  return hipGetLastError();
}

// Queries per lane: 1 or 2 (1 by default: 2 doubles the registers and
// halves occupancy for no gain at the issue limit; WN_BND_QPL overrides).
static int bnd_qpl() {
  static int q = [] {
    const char* e = getenv("WN_BND_QPL");
    const int v = e ? atoi(e) : 1;
    return (v == 2) ? 2 : 1;
  }();
  return q;
}

hipError_t launch_bnd3d(const BndArgs& a, const LoopTable& L, hipStream_t s) {
  const int qpl = bnd_qpl();
  const int64_t per = (int64_t)kThreads * qpl;
  const int64_t blocks = (a.nq + per - 1) / per;
  if (blocks == 0) return hipSuccess;
  if (qpl == 1)
    hipLaunchKernelGGL(k_bnd3d<1>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a, L);
  else
    hipLaunchKernelGGL(k_bnd3d<2>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a, L);
  return hipGetLastError();
}

}  // namespace wn
