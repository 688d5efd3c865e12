// Adjoint of the 3D winding number with respect to the query points and the
// boundary vertices, for a loss L with dL/dw = g per query (one tile of
// queries per workgroup; the walk is in adjloop.hpp), and the fixed-order
// float64 reduction of the per-wavefront partials.
#include "adj3d.hpp"
#include "adjloop.hpp"

namespace wn {

namespace {

using namespace adj;

// QPL queries per lane.  With 4, four waves per SIMD (at most 128 registers).
template <int QPL>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(QPL == 4 ? 4 : (QPL == 2 ? 6 : 8)))) void k_adj3d(
    AdjArgs a, LoopTable L) {
  __shared__ AdjLds lds;
  const int64_t bw = blockIdx.x;     // partial row
  float* pv = a.partial ? a.partial + bw * (int64_t)a.nb * 3 : nullptr;
  float* pl = a.partial_loop ? a.partial_loop + bw * (int64_t)L.n * 3 : nullptr;
  QState S[QPL];
  const int64_t tile = (int64_t)kThreads * QPL;
  const int64_t q0 = (int64_t)blockIdx.x * tile;
  const int64_t cnt = min(tile, a.nq - q0);
  load_tile<QPL>(S, a.qx, a.qy, a.qz, a.gw, q0, cnt);
  walk<QPL>(S, a.bnd, a.nb, bnd::KernargLoops{L}, lds, pv, pl);
  store_gq<QPL>(S, q0, cnt, a.gq);
}

// The walk of adjloop.hpp restricted to the edges that start at vertices
// [cbeg, cend) (whole chunks; a loop's closing edge starts at its last
// vertex).  Each vertex of the range is parked to pv exactly once, as in the
// full walk.  A range that starts inside a loop also takes the edge
// (cbeg - 1 -> cbeg); that edge's share of vertex cbeg - 1 goes to pc, and
// the previous range parks the rest of that vertex at its end.  The loop's
// first vertex and vertex cbeg - 1 then come from global memory.
template <int QPL>
__device__ __forceinline__ void walk_range(QState* S, const float* __restrict__ bnd, int nb,
                                           const bnd::KernargLoops& L, int cbeg, int cend, AdjLds& lds,
                                           float* pv, float* pl, float* pc) {
  const int lane = threadIdx.x & 63;
  float4* sv = lds.sv;
  Parker P = make_parker(lds, pv);
  Rel A[QPL], B[QPL];
  float4 vF = make_float4(0.f, 0.f, 0.f, 0.f);   // the loop's first vertex (uniform)
  float accA[3], accB[3];
  float4 eA = make_float4(0.f, 0.f, 0.f, 0.f);
  zero3(accA);
  int l = bnd::loop_of(L, cbeg);
  bool carry_in = cbeg > L.off(l);
  if (carry_in) {
    const int ls = L.off(l), i = cbeg - 1;   // i + 1 = cbeg lies in the same loop
    vF = make_float4(bnd[3 * ls], bnd[3 * ls + 1], bnd[3 * ls + 2], 0.f);
    const float x = bnd[3 * i], y = bnd[3 * i + 1], z = bnd[3 * i + 2];
    const float ex = __fsub_rn(bnd[3 * cbeg], x), ey = __fsub_rn(bnd[3 * cbeg + 1], y),
                ez = __fsub_rn(bnd[3 * cbeg + 2], z);
    const float4 v = make_float4(x, y, z, 0.f);
#pragma unroll
    for (int k = 0; k < QPL; ++k) A[k] = rel(S[k], v);
    eA = make_float4(ex, ey, ez, __fmaf_rn(ex, ex, __fmaf_rn(ey, ey, __fmul_rn(ez, ez))));
  }
  for (int c0 = cbeg; c0 < cend; c0 += kChunk) {
    const int c1 = min(c0 + kChunk, cend);
    __syncthreads();
    for (int j = threadIdx.x; j < c1 - c0; j += kThreads) stage_adj(bnd, L, c0 + j, j, sv);
    __syncthreads();
    for (; l < L.n() && L.off(l) < c1; ++l) {
      const int ls = L.off(l), le = L.off(l + 1);
      int j = max(ls, c0);
      const int j1 = min(le, c1);
      if (j == ls) {
        const float4 v = sv[j - c0];
        // kept in scalar registers (every lane reads the same vertex) and
        // seen from the queries again at the closing edge
        vF = make_float4(__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v.x))),
                         __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v.y))),
                         __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v.z))), 0.f);
#pragma unroll
        for (int k = 0; k < QPL; ++k) A[k] = rel(S[k], v);
        eA = sv[kChunk + j - c0];
        zero3(accA);
        ++j;
      } else if (carry_in) {   // edge (cbeg - 1 -> cbeg)
        carry_in = false;
        const float4 v0 = sv[j - c0];
#pragma unroll
        for (int k = 0; k < QPL; ++k) B[k] = rel(S[k], v0);
        edges<QPL>(S, A, B, eA, accA, accB);
        if (pc) put3(pc, accA, lds.sh, lane);
#pragma unroll
        for (int k = 0; k < QPL; ++k) A[k] = B[k];
        accA[0] = accB[0]; accA[1] = accB[1]; accA[2] = accB[2];
        eA = sv[kChunk + j - c0];
        ++j;
      }
      for (; j + 2 <= j1; j += 2) {
        const float4 v0 = sv[j - c0];
        const float4 v1 = sv[j + 1 - c0];
        const float4 e0 = sv[kChunk + j - c0];
#pragma unroll
        for (int k = 0; k < QPL; ++k) B[k] = rel(S[k], v0);
        step<QPL>(S, A, B, eA, accA, accB, P, j - 1, nb, lane);
#pragma unroll
        for (int k = 0; k < QPL; ++k) A[k] = rel(S[k], v1);
        step<QPL>(S, B, A, e0, accB, accA, P, j, nb, lane);
        eA = sv[kChunk + j + 1 - c0];
      }
      if (j < j1) {
        const float4 v0 = sv[j - c0];
#pragma unroll
        for (int k = 0; k < QPL; ++k) B[k] = rel(S[k], v0);
        step<QPL>(S, A, B, eA, accA, accB, P, j - 1, nb, lane);
#pragma unroll
        for (int k = 0; k < QPL; ++k) A[k] = B[k];
        accA[0] = accB[0]; accA[1] = accB[1]; accA[2] = accB[2];
        eA = sv[kChunk + j - c0];
        ++j;
      }
      if (j1 < le) {
        // the loop goes on: into the next chunk, or past the range, whose
        // last vertex is then parked with the share this range holds
        if (c1 == cend && pv) park(P, c1 - 1, nb, accA, lane);
        break;
      }
      float accF[3];
#pragma unroll
      for (int k = 0; k < QPL; ++k) B[k] = rel(S[k], vF);
      step<QPL>(S, A, B, eA, accA, accF, P, le - 1, nb, lane);
      if (pl) put3(pl + 3 * (int64_t)l, accF, lds.sh, lane);
      zero3(accA);
    }
  }
  flush_last(P);
}

template <int QPL>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(QPL == 4 ? 4 : (QPL == 2 ? 6 : 8)))) void k_adj3d_split(
    AdjArgs a, LoopTable L, int32_t span, int32_t parts, float* carry, float* gq_part) {
  __shared__ AdjLds lds;
  const int64_t bw = blockIdx.x;     // partial row
  const int p = blockIdx.y;
  float* pv = a.partial ? a.partial + bw * (int64_t)a.nb * 3 : nullptr;
  float* pl = a.partial_loop ? a.partial_loop + bw * (int64_t)L.n * 3 : nullptr;
  float* pc = (a.partial && carry) ? carry + (bw * parts + p) * 3 : nullptr;
  QState S[QPL];
  const int64_t tile = (int64_t)kThreads * QPL;
  const int64_t q0 = (int64_t)blockIdx.x * tile;
  const int64_t cnt = min(tile, a.nq - q0);
  load_tile<QPL>(S, a.qx, a.qy, a.qz, a.gw, q0, cnt);
  const int cbeg = p * span;
  const int cend = min(a.nb, cbeg + span);
  walk_range<QPL>(S, a.bnd, a.nb, bnd::KernargLoops{L}, cbeg, cend, lds, pv, pl, pc);
  if (a.gq) store_gq<QPL>(S, q0, cnt, gq_part + (int64_t)p * a.nq * 3);
}

__global__ void k_sum_parts(const float* __restrict__ part, int32_t parts, int64_t n, float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  out[t] = (float)ordered_sum(part + t, n, parts, 0.0);
}

constexpr int kRowsPerGroup = 16;

// Stage 1: g-th group of kRowsPerGroup partial rows, summed per column in
// float64 (for a loop's first vertex the per-loop closing shares as well).
// With vertex ranges (pc non-null): the vertex before a range that starts
// inside a loop adds that range's carry slot as well.
__global__ void k_reduce_rows(const float* __restrict__ pv, const float* __restrict__ pl,
                              const float* __restrict__ pc, int32_t parts, int32_t span,
                              int64_t rows, int32_t nb, LoopTable L, double* __restrict__ tmp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)nb * 3;
  if (t >= n) return;
  const int v = (int)(t / 3), c = (int)(t % 3);
  int lf = -1;
  int cp = (pc && (v + 1) % span == 0 && v + 1 < nb) ? (v + 1) / span : -1;
  const bnd::KernargLoops KL{L};
  for (int l = 0; l < L.n; ++l) {
    const int o = KL.off(l);
    if (o == v && KL.off(l + 1) > v) lf = l;
    if (o == v + 1) cp = -1;   // the range starts a loop: no carry
  }
  const int64_t r0 = (int64_t)blockIdx.y * kRowsPerGroup;
  const int64_t r1 = min(rows, r0 + kRowsPerGroup);
  double s = 0.0;
  if (lf < 0 && cp < 0) {
    s = ordered_sum(pv + r0 * n + t, n, r1 - r0, 0.0);
  } else {
    for (int64_t r = r0; r < r1; ++r) {
      s += (double)pv[r * n + t];
      if (lf >= 0) s += (double)pl[(r * L.n + lf) * 3 + c];
      if (cp >= 0) s += (double)pc[(r * parts + cp) * 3 + c];
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

// Queries per lane for nq queries when the grid cannot be filled by
// boundary ranges (measured on a 256-CU MI355X, 2048 edges, no ranges): 4
// (the cheapest per pair: the cross-lane sums are shared by four queries)
// once that leaves four wavefronts per SIMD (nq >= 2^20); 2 down to one
// wavefront per SIMD (nq >= 2^17; at 2^18 queries 0.75 ms against 0.87 ms
// with 4 and 0.94 ms with 1); 1 below.
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

int64_t adj3d_rows(int64_t nblocks) { return nblocks; }

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
  hipLaunchKernelGGL(k_reduce_rows, dim3(bx, (unsigned)groups), dim3(256), 0, s, pv, pl, (const float*)nullptr,
                     0, 0, rows, nb, L, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_groups, dim3(bx), dim3(256), 0, s, tmp, groups, n, out);
  return hipGetLastError();
}

// Queries per lane when the boundary spans more than one chunk: then the
// ranges below keep the grid full, so four queries per lane (the cheapest
// per pair) from 2^16 queries on.  Measured over 2048 edges: 2^18 queries
// 0.60 ms, 2^19 1.06 ms, 2^20 1.98 ms (0.66, 1.23, 2.08 ms with adj3d_qpl and
// no ranges).
int adj3d_qpl_ranges(int64_t nq, int64_t nb) {
  if (nb > kChunk && nq >= (int64_t)kThreads * 256) return 4;
  return adj3d_qpl(nq);
}

// Vertex ranges for few query tiles: with fewer than 2048 workgroups and more
// than one chunk, split the chunks into equal ranges until the grid reaches
// 2048 workgroups (2^16 queries over 2048 edges: 0.26 ms, 0.45 ms unsplit).
int adj3d_parts(int64_t nblocks, int64_t nb) {
  const int64_t chunks = (nb + kChunk - 1) / kChunk;
  if (nblocks <= 0 || nblocks >= 2048 || chunks < 2) return 1;
  const int64_t want = min(chunks, (2048 + nblocks - 1) / nblocks);
  const int64_t cpp = (chunks + want - 1) / want;
  return (int)((chunks + cpp - 1) / cpp);
}

int32_t adj3d_span(int64_t nb, int parts) {
  const int64_t chunks = (nb + kChunk - 1) / kChunk;
  return (int32_t)(((chunks + parts - 1) / parts) * kChunk);
}

hipError_t launch_adj3d_split(const AdjArgs& a, const LoopTable& L, int64_t nblocks, int qpl, int parts,
                              int32_t span, float* carry, float* gq_part, hipStream_t s) {
  if (nblocks == 0 || parts < 1) return hipSuccess;
  if ((int64_t)(parts - 1) * span >= a.nb) return hipErrorInvalidValue;   // every range non-empty
  const dim3 grid((unsigned)nblocks, (unsigned)parts);
  if (qpl == 4)
    hipLaunchKernelGGL(k_adj3d_split<4>, grid, dim3(kThreads), 0, s, a, L, span, parts, carry, gq_part);
  else if (qpl == 2)
    hipLaunchKernelGGL(k_adj3d_split<2>, grid, dim3(kThreads), 0, s, a, L, span, parts, carry, gq_part);
  else
    hipLaunchKernelGGL(k_adj3d_split<1>, grid, dim3(kThreads), 0, s, a, L, span, parts, carry, gq_part);
  return hipGetLastError();
}

hipError_t launch_sum_parts(const float* gq_part, int parts, int64_t n, float* gq, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, gq_part, parts, n, gq);
  return hipGetLastError();
}

hipError_t launch_reduce_partials_split(const float* pv, const float* pl, const float* carry, int parts,
                                        int32_t span, int64_t rows, int32_t nb, const LoopTable& L, double* tmp,
                                        float* out, hipStream_t s) {
  const int64_t n = (int64_t)nb * 3;
  if (n == 0) return hipSuccess;
  const int64_t groups = reduce_groups(rows);
  const unsigned bx = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_reduce_rows, dim3(bx, (unsigned)groups), dim3(256), 0, s, pv, pl, carry, parts, span, rows,
                     nb, L, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_groups, dim3(bx), dim3(256), 0, s, tmp, groups, n, out);
  return hipGetLastError();
}

}  // namespace wn
