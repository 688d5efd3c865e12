// Grid mode in 3D: queries (gx[i], gy[j], gz[k]) for a BVH built for d = +z,
// one lane per query with z fastest.
//
// Sec. 5 ("Optimization") reuses one ray for all points on a line parallel
// to the ray direction.  Here every column (x_i, y_j) is such a line, and its
// points are consecutive lanes: the 64 lanes of a wavefront lie on one
// column and have bit-identical frame coordinates X, Y (d = +z leaves the
// rotation rows e1, e2 without a z component), so they take the same path
// through the tree and every node fetch serves the whole wavefront - the
// shared ray, without storing its crossings.  Each lane then applies the
// exact triangle test with its own height, so chi and w equal wn_eval_3d on
// the same float32 points bit for bit.  (Storing a per-column candidate list
// and testing every candidate per query was measured slower: it also tests
// the triangles below the query, which the traversal culls.)
#include "bndloop.hpp"
#include "bvh_build.hpp"
#include "traverse.hpp"

namespace wn {

namespace {

using namespace bnd;

// 32-bit index arithmetic (the host limits grids to fewer than 2^32
// points): 64-bit divisions would be long emulated sequences per query.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_grid3d_fwd(CrossArgs c, BndArgs a, LoopTable L,
                                                         const float* __restrict__ gx, const float* __restrict__ gy,
                                                         const float* __restrict__ gz, int64_t ny64, int64_t nz64,
                                                         int32_t* chi_out) {
  __shared__ RPt sv[kChunk];
  const int64_t qi = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool ok = qi < a.nq;
  const int64_t q = ok ? qi : 0;
  const uint32_t ny = (uint32_t)ny64, nz = (uint32_t)nz64, qq = (uint32_t)q;
  const uint32_t col = qq / nz;
  const float px = gx[col / ny], py = gy[col % ny], pz = gz[qq % nz];
  const bool fin = isfinite(px) && isfinite(py) && isfinite(pz);
  Lane<1> s;
  {
    double X, Y, Z;
    rotate(a.F, px, py, pz, X, Y, Z);
    s.p[0] = make_qp(X, Y, Z);
  }
  turns_init(s.T[0]);
  lane_range(s);
  const int chi = (ok && fin) ? traverse<kShortStack>(c, s.p[0]) : WN_CHI_INVALID;
  int staged = -1, pend = 0;
  const KernargLoops KL{L};
  boundary_walk(s, StageRotate<KernargLoops>{a.F, a.bnd, KL}, a.nb, KL, sv, staged, pend);
  finish_turns(s, pend);
  if (ok) {
    a.w_out[q] = chi != WN_CHI_INVALID ? lane_w(s, 0, chi) : __int_as_float(0x7fc00000);
    if (chi_out) chi_out[q] = chi;
  }
}

}  // namespace

hipError_t launch_grid3d_fwd(const CrossArgs& c, const BndArgs& a, const LoopTable& L, const float* gx,
                             const float* gy, const float* gz, int64_t ny, int64_t nz, int32_t* chi_out,
                             hipStream_t s) {
  const int64_t blocks = (a.nq + kThreads - 1) / kThreads;
  if (blocks == 0) return hipSuccess;
  if (a.nq > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_grid3d_fwd, dim3((unsigned)blocks), dim3(kThreads), 0, s, c, a, L, gx, gy, gz, ny, nz,
                     chi_out);
  return hipGetLastError();
}

}  // namespace wn
