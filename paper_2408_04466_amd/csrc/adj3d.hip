// Adjoint of the 3D winding number with respect to the query points and the
// boundary vertices, for a loss L with dL/dw = g per query (one tile of
// queries per workgroup; the walk is in adjloop.hpp), and the fixed-order
// float64 reduction of the per-wavefront partials.
#include "adjloop.hpp"

namespace wn {

namespace {

using namespace adj;

// Four waves per SIMD: the register allocator then fits 128 registers,
// spilling one pointer outside the walk.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_adj3d(AdjArgs a,
                                                                                            LoopTable L) {
  __shared__ float4 sv[kChunk];
  __shared__ float4 rsw[kWaves * kRowFloats / 4];
  const int wave = threadIdx.x >> 6;
  const int64_t bw = (int64_t)blockIdx.x * kWaves + wave;     // partial row
  float* pv = a.partial ? a.partial + bw * (int64_t)a.nb * 3 : nullptr;
  float* pl = a.partial_loop ? a.partial_loop + bw * (int64_t)L.n * 3 : nullptr;
  QState S[kQPL];
  int64_t qi[kQPL];
  bool ok[kQPL];
  const int64_t q0 = (int64_t)blockIdx.x * kTile;
  load_tile(S, a.qx, a.qy, a.qz, a.gw, q0, min((int64_t)kTile, a.nq - q0), qi, ok);
  walk(S, a.bnd, a.nb, bnd::KernargLoops{L}, sv, reinterpret_cast<float*>(rsw), pv, pl);
  store_gq(S, qi, ok, a.gq);
}

constexpr int kRowsPerGroup = 32;

// Stage 1: g-th group of kRowsPerGroup partial rows, summed per column in
// float64 (for a loop's first vertex the per-loop closing shares as well).
__global__ void k_reduce_rows(const float* __restrict__ pv, const float* __restrict__ pl,
                              int64_t rows, int32_t nb, LoopTable L, double* __restrict__ tmp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)nb * 3;
  if (t >= n) return;
  const int v = (int)(t / 3), c = (int)(t % 3);
  int lf = -1;
  for (int l = 0; l < L.n; ++l)
    if (L.off[l] == v && L.off[l + 1] > v) lf = l;
  const int64_t r0 = (int64_t)blockIdx.y * kRowsPerGroup;
  const int64_t r1 = min(rows, r0 + kRowsPerGroup);
  double s = 0.0;
  if (lf < 0) {
    s = ordered_sum(pv + r0 * n + t, n, r1 - r0, 0.0);
  } else {
    for (int64_t r = r0; r < r1; ++r) {
      s += (double)pv[r * n + t];
      s += (double)pl[(r * L.n + lf) * 3 + c];
    }
  }
  tmp[(int64_t)blockIdx.y * n + t] = s;
}

// Stage 2: out = -(1/4pi) * sum over groups, in group order.
__global__ void k_reduce_groups(const double* __restrict__ tmp, int64_t groups, int64_t n,
                                float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double s = ordered_sum(tmp + t, n, groups, 0.0);
  out[t] = (float)(-s * 0.07957747154594767 + 0.0);
}

}  // namespace

int64_t adj3d_blocks(int64_t nq) {
  const int64_t per = (int64_t)kThreads * kQPL;
  return (nq + per - 1) / per;
}

int64_t adj3d_rows(int64_t nblocks) { return nblocks * kWaves; }

hipError_t launch_adj3d(const AdjArgs& a, const LoopTable& L, int64_t nblocks, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj3d, dim3((unsigned)nblocks), dim3(kThreads), 0, s, a, L);
  return hipGetLastError();
}

int64_t reduce_groups(int64_t rows) { return (rows + kRowsPerGroup - 1) / kRowsPerGroup; }

hipError_t launch_reduce_partials(const float* pv, const float* pl, int64_t rows, int32_t nb,
                                  const LoopTable& L, double* tmp, float* out, hipStream_t s) {
  const int64_t n = (int64_t)nb * 3;
  if (n == 0) return hipSuccess;
  const int64_t groups = reduce_groups(rows);
  const unsigned bx = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_reduce_rows, dim3(bx, (unsigned)groups), dim3(256), 0, s, pv, pl, rows, nb, L, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_groups, dim3(bx), dim3(256), 0, s, tmp, groups, n, out);
  return hipGetLastError();
}

}  // namespace wn
