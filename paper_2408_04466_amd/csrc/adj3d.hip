// Adjoint of the 3D winding number with respect to the query points and the
// boundary vertices, for a loss L with dL/dw = g per query (one tile of
// queries per workgroup; the walk is in adjloop.hpp), and the fixed-order
// float64 reduction of the per-wavefront partials.
#include "adjloop.hpp"

namespace wn {

namespace {

using namespace adj;

// QPL queries per lane.  With 4, four waves per SIMD: the register
// allocator then fits 128 registers, spilling one pointer outside the walk.
template <int QPL>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(QPL == 4 ? 4 : (QPL == 2 ? 6 : 8)))) void k_adj3d(
    AdjArgs a, LoopTable L) {
  __shared__ float4 sv[kChunk];
  __shared__ float4 rsw[kWaves * kRowFloats / 4];
  const int wave = threadIdx.x >> 6;
  const int64_t bw = (int64_t)blockIdx.x * kWaves + wave;     // partial row
  float* pv = a.partial ? a.partial + bw * (int64_t)a.nb * 3 : nullptr;
  float* pl = a.partial_loop ? a.partial_loop + bw * (int64_t)L.n * 3 : nullptr;
  QState S[QPL];
  int64_t qi[QPL];
  bool ok[QPL];
  const int64_t tile = (int64_t)kThreads * QPL;
  const int64_t q0 = (int64_t)blockIdx.x * tile;
  load_tile<QPL>(S, a.qx, a.qy, a.qz, a.gw, q0, min(tile, a.nq - q0), qi, ok);
  walk<QPL>(S, a.bnd, a.nb, bnd::KernargLoops{L}, sv, reinterpret_cast<float*>(rsw), pv, pl);
  store_gq<QPL>(S, qi, ok, a.gq);
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

// Queries per lane for nq queries (measured on a 256-CU MI355X): 4 (the
// cheapest per pair: the cross-lane sums are shared by four queries) once
// that leaves four wavefronts per SIMD (nq >= 2^20); 2 down to one wavefront
// per SIMD (nq >= 2^17; at 2^18 queries x 2048 edges 0.75 ms against 0.87
// ms with 4 and 0.94 ms with 1); 1 below.
int adj3d_qpl(int64_t nq) {
  const int64_t simds = 4 * 256;
  if (nq >= (int64_t)kThreads * 4 * simds) return 4;
  if (nq >= (int64_t)kThreads * 2 * simds / 4) return 2;
  return 1;
}

int64_t adj3d_blocks(int64_t nq, int qpl) {
  const int64_t per = (int64_t)kThreads * qpl;
  return (nq + per - 1) / per;
}

int64_t adj3d_rows(int64_t nblocks) { return nblocks * kWaves; }

hipError_t launch_adj3d(const AdjArgs& a, const LoopTable& L, int64_t nblocks, int qpl, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  if (qpl == 4)
    hipLaunchKernelGGL(k_adj3d<4>, dim3((unsigned)nblocks), dim3(kThreads), 0, s, a, L);
  else if (qpl == 2)
    hipLaunchKernelGGL(k_adj3d<2>, dim3((unsigned)nblocks), dim3(kThreads), 0, s, a, L);
  else
    hipLaunchKernelGGL(k_adj3d<1>, dim3((unsigned)nblocks), dim3(kThreads), 0, s, a, L);
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
