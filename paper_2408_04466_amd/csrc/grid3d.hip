// Grid mode in 3D: query points on lines parallel to d share one ray.
//
// Sec. 4 ("Optimization") observes that points on one line along the ray
// direction can reuse a single ray: the surface crossings along the line
// are found once and every point's count follows from which crossings lie
// above it.  For a grid x[nx] by y[ny] by z[nz] and d = +z every column
// (x_i, y_j) is such a line.  Here one traversal per column collects the
// candidate triangles (those whose padded projection box contains the
// column, at any height); each query of the column then runs the exact
// per-query triangle test on that short list instead of walking the tree.
// Because all queries of a column have bit-identical frame coordinates X, Y
// (d = +z makes the rotation rows e1, e2 free of z) and a triangle culled by
// the per-query traversal (entirely below the query) fails the same test,
// chi equals the per-query traversal's bit for bit.  A column with more
// candidates than fit in its list falls back to per-query traversal.
#include "bndloop.hpp"
#include "bvh_build.hpp"
#include "traverse.hpp"

namespace wn {

namespace {

using namespace bnd;

// One lane per column: candidate triangles (sorted-triangle indices).
__global__ __launch_bounds__(256) void k_grid3d_columns(CrossArgs c, const float* __restrict__ gx,
                                                        const float* __restrict__ gy, int64_t nx, int64_t ny,
                                                        int32_t* __restrict__ cnt, int32_t* __restrict__ cand) {
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= nx * ny) return;
  const float x = gx[col / ny], y = gy[col % ny];
  if (!(isfinite(x) && isfinite(y))) {
    cnt[col] = -1;   // the column's queries are invalid
    return;
  }
  double X, Y, Z;
  rotate(c.F, x, y, 0.0f, X, Y, Z);
  int32_t* list = cand + col * kGridCand;
  int n = 0;
  const int st = traverse_leaves<kShortStack>(c, (float)X, (float)Y, -INFINITY, [&](int t) {
    if (n < kGridCand) list[n] = t;
    ++n;
  });
  cnt[col] = st ? kGridCand + 1 : n;   // a malformed tree sends the column to the per-query path
}

// One lane per query, z fastest: chi from the column's candidates (or a
// full traversal when the list overflowed), then the boundary walk.
__global__ __launch_bounds__(kThreads) void k_grid3d_fwd(CrossArgs c, BndArgs a, LoopTable L,
                                                         const float* __restrict__ gx, const float* __restrict__ gy,
                                                         const float* __restrict__ gz, int64_t ny, int64_t nz,
                                                         const int32_t* __restrict__ cnt,
                                                         const int32_t* __restrict__ cand, int32_t* chi_out) {
  __shared__ double4 sv[kChunk];
  const int64_t qi = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool ok = qi < a.nq;
  const int64_t q = ok ? qi : 0;
  const int64_t col = q / nz;
  const float px = gx[col / ny], py = gy[col % ny], pz = gz[q % nz];
  const bool fin = isfinite(px) && isfinite(py) && isfinite(pz);
  Lane<1> s;
  rotate(a.F, px, py, pz, s.Xp[0], s.Yp[0], s.Zp[0]);
  turns_init(s.T[0]);
  int chi = WN_CHI_INVALID;
  if (ok && fin) {
    const int n = cnt[col];
    if (n <= kGridCand) {
      chi = 0;
      const int32_t* list = cand + col * kGridCand;
      for (int k = 0; k < n; ++k) chi += tri_crossing(c.tris[list[k]], c.Vr, s.Xp[0], s.Yp[0], s.Zp[0]);
    } else {
      chi = traverse<kShortStack>(c, s.Xp[0], s.Yp[0], s.Zp[0]);
    }
  }
  int staged = -1;
  const KernargLoops KL{L};
  boundary_walk(s, StageRotate<KernargLoops>{a.F, a.bnd, KL}, a.nb, KL, sv, staged);
  if (ok) {
    a.w_out[q] = chi != WN_CHI_INVALID ? turns_to_w(s.T[0], chi) : __int_as_float(0x7fc00000);
    if (chi_out) chi_out[q] = chi;
  }
}

}  // namespace

hipError_t launch_grid3d_columns(const CrossArgs& c, const float* gx, const float* gy, int64_t nx, int64_t ny,
                                 int32_t* cnt, int32_t* cand, hipStream_t s) {
  const int64_t ncol = nx * ny;
  if (ncol == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grid3d_columns, dim3((unsigned)((ncol + 255) / 256)), dim3(256), 0, s, c, gx, gy, nx, ny,
                     cnt, cand);
  return hipGetLastError();
}

hipError_t launch_grid3d_fwd(const CrossArgs& c, const BndArgs& a, const LoopTable& L, const float* gx,
                             const float* gy, const float* gz, int64_t ny, int64_t nz, const int32_t* cnt,
                             const int32_t* cand, int32_t* chi_out, hipStream_t s) {
  const int64_t blocks = (a.nq + kThreads - 1) / kThreads;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grid3d_fwd, dim3((unsigned)blocks), dim3(kThreads), 0, s, c, a, L, gx, gy, gz, ny, nz, cnt,
                     cand, chi_out);
  return hipGetLastError();
}

}  // namespace wn
