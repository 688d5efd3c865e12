// Grid mode in 3D: queries (gx[i], gy[j], gz[k]) for a BVH built for d = +z,
// one lane per query with z fastest.
//
// Sec. 5 ("Optimization") reuses one ray for all points on a line parallel
// to the ray direction: once the line's crossings with the surface are known,
// a point on it counts those above it.  Here every column (x_i, y_j) is such
// a line.  d = +z leaves the rotation rows e1, e2 without a z component, so
// all points of a column have bit-identical frame coordinates X, Y, and the
// exact inside test of a triangle (its three edge values, from the vertices'
// X, Y offsets) gives one answer for the whole column.  A wavefront whose 64
// lanes lie on one column (z fastest, 64 | nz) therefore traverses the tree
// once, with uniform control flow and the height test at its lowest query,
// and keeps in LDS the triangles the line passes through above that point;
// each lane then sums the same exact crossing test as the per-query path
// over that short list (the inside test again, and its own height), so chi
// and w equal wn_eval_3d on the same float32 points bit for bit.  The list
// is not sorted by height: a line holds a few crossings, and at a near-tie
// the query's own float64 height test decides, as in the per-query path.  A
// wavefront spanning two columns, a line with more than kColHits crossings
// or a malformed tree fall back to the per-lane traversal.  The line is
// traversed per wavefront rather than once per column: a separate pass over
// the columns left its traversals' latency exposed (0.99 against 0.76 ms on
// the 128^3 grid), while here it hides behind the boundary arithmetic of the
// other wavefronts.
#include "bndloop.hpp"
#include "bvh_build.hpp"
#include "traverse.hpp"

namespace wn {

namespace {

using namespace bnd;

constexpr int kColHits = 16;   // crossings kept per line

// 32-bit index arithmetic (the host limits grids to fewer than 2^32
// points): 64-bit divisions would be long emulated sequences per query.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_grid3d_fwd(CrossArgs c, BndArgs a, LoopTable L,
                                                         const float* __restrict__ gx, const float* __restrict__ gy,
                                                         const float* __restrict__ gz, int64_t ny64, int64_t nz64,
                                                         int32_t* chi_out) {
  __shared__ RPt sv[kChunk];
  __shared__ int32_t s_hits[kThreads / 64][kColHits];
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
  // the wavefront's line: one traversal when all its lanes share the column
  const uint32_t col0 = __builtin_amdgcn_readfirstlane(col);
  const bool one_col = __all(col == col0 || !ok);
  int n = kColHits + 1;
  if (one_col && isfinite(px) && isfinite(py)) {
    QP pu;   // the column's X, Y (identical in every lane; made uniform)
    pu.xh = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s.p[0].xh)));
    pu.xl = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s.p[0].xl)));
    pu.yh = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s.p[0].yh)));
    pu.yl = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s.p[0].yl)));
    pu.zh = pu.zl = 0.0f;
    // crossings below every lane of the wavefront count for none of them:
    // cull at the lowest query (a weaker cut than each lane's own)
    float zmin = s.p[0].zh;
    for (int o = 32; o > 0; o >>= 1) zmin = fminf(zmin, __shfl_xor(zmin, o));
    zmin = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(zmin)));
    int32_t* hits = s_hits[threadIdx.x / 64];
    int m = 0;
    const int st = traverse_leaves<kShortStack>(c, pu.xh, pu.yh, zmin, [&](int t, uint32_t ties) {
      if (tri_on_line(c.tris, t, ties, pu)) {
        if (m < kColHits) hits[m] = t;
        ++m;
      }
    });
    n = st ? kColHits + 1 : m;
  }
  int chi = WN_CHI_INVALID;
  if (ok && fin) {
    if (n <= kColHits) {
      const int32_t* hits = s_hits[threadIdx.x / 64];
      chi = 0;
      for (int k = 0; k < n; ++k) chi += tri_crossing(c.tris, hits[k], s.p[0]);
    } else {
      chi = traverse<kShortStack>(c, s.p[0]);
    }
  }
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
                             const float* gy, const float* gz, int64_t nx, int64_t ny, int64_t nz, int32_t* chi_out,
                             hipStream_t s) {
  (void)nx;
  const int64_t blocks = (a.nq + kThreads - 1) / kThreads;
  if (blocks == 0) return hipSuccess;
  if (a.nq > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_grid3d_fwd, dim3((unsigned)blocks), dim3(kThreads), 0, s, c, a, L, gx, gy, gz, ny, nz,
                     chi_out);
  return hipGetLastError();
}

}  // namespace wn
