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
// other wavefronts.  The boundary walk of such a wavefront shares the
// column's part of the arithmetic as well (column_walk, below).
#include "bndloop.hpp"
#include "bvh_build.hpp"
#include "traverse.hpp"

namespace wn {

namespace {

using namespace bnd;

constexpr int kColHits = 16;   // crossings kept per line

// ---------------------------------------------------------------------------
// Boundary walk of a wavefront whose lanes share one column
// ---------------------------------------------------------------------------
// The frame X, Y offsets of a boundary vertex are the same for every point of
// a column, and so is all that the walk derives from them alone: rho^2 of a
// vertex, and of an edge its N (certified in float32 or exact, with the tie)
// and the X, Y part of D.  The wavefront computes these once per staged chunk
// into LDS; each lane then adds what depends on its height: Z, r, alpha, D
// and the product.  Each value is the same float operation on the same
// operands as in vertex_q, edge_d and turns_edge, and the product is rescaled
// and its turns decided after the same edges as in boundary_walk, so w is
// bit-identical to the per-query walk.

// One slot per column of the workgroup (CPW columns of 4 / CPW wavefronts).
template <int CPW>
struct ColLds {
  float rho2[CPW][kChunk];
  float2 ng[CPW][kChunk];   // edge (j - 1 -> j) of the staged order: N, fma(X_a, X_b, Y_a Y_b)
};

// The column's data for the staged chunk (cnt vertices), the X, Y offsets
// taken from pc (the column's split coordinates); prev: the previous chunk's
// last vertex (used when has_prev).  The edge into a loop's first vertex is
// computed too and never read.  Vertices t0, t0 + stride, ... of the chunk.
__device__ __forceinline__ void column_chunk(const RPt* sv, int cnt, bool has_prev, const RPt& prev, const QP& pc,
                                             float* rho2, float2* ng, int t0, int stride) {
  for (int j = t0; j < cnt; j += stride) {
    const RPt v = sv[j];
    VQ b;
    b.x = vertex_x(v, pc);
    b.y = vertex_y(v, pc);
    b.a = 0.0f;
    rho2[j] = __fmaf_rn(b.x, b.x, __fmul_rn(b.y, b.y));
    if (j > 0 || has_prev) {
      const RPt u = j > 0 ? sv[j - 1] : prev;
      VQ a;
      a.x = vertex_x(u, pc);
      a.y = vertex_y(u, pc);
      a.a = 0.0f;
      const WalkN w = edge_n_walk(a, b);
      const float N = w.sure ? w.n : edge_n_exact(a, b, rpt_tie(u));
      ng[j] = make_float2(N, __fmaf_rn(a.x, b.x, __fmul_rn(a.y, b.y)));
    }
  }
}

// turns_mul with the sign registers pinned after the edge, as turns_edge
// does (the compiler would otherwise defer a step's bit insertions)
__device__ __forceinline__ void column_mul(Turns& t, float D, float N) {
  turns_mul(t, D, N);
  asm volatile("" : "+v"(t.bacc), "+v"(t.cacc));
}

// alpha of a staged vertex for the lane's query (vertex_q's arithmetic, with
// the column's rho^2).
__device__ __forceinline__ float column_alpha(const RPt& v, const QP& p, float rho2) {
  const float Z = vertex_z(v, p);
  const float s = __fmaf_rn(Z, Z, rho2);
  const float r = __builtin_amdgcn_sqrtf(s);
  const float u = __fadd_rn(r, fabsf(Z));
  return __fmaf_rn(rho2, __builtin_amdgcn_rcpf(u), __fsub_rn(fabsf(Z), Z));
}

// main_steps with the column's data (the same edges, rescales and flushes).
template <bool FAR>
__device__ __forceinline__ int column_steps(Lane<1>& s, const RPt* sv, const float* rho2, const float2* ng, int c0,
                                            int j, int j1, float& aA, int& pend) {
  for (; j + kStep <= j1; j += kStep) {
    if (pend > kStep) {
      flush(s, pend);
      pend = 0;
    }
#pragma unroll
    for (int u = 0; u < kStep; u += 2) {
      const int i = j + u - c0;
      const float a0 = column_alpha(sv[i], s.p[0], rho2[i]);
      const float2 e0 = ng[i];
      column_mul(s.T[0], __fmaf_rn(aA, a0, e0.y), e0.x);
      if (FAR) rescale(s);
      const float a1 = column_alpha(sv[i + 1], s.p[0], rho2[i + 1]);
      const float2 e1 = ng[i + 1];
      column_mul(s.T[0], __fmaf_rn(a0, a1, e1.y), e1.x);
      aA = a1;
      rescale(s);
      __builtin_amdgcn_sched_barrier(0);
    }
    pend += kStep;
    if (pend == 2 * kStep) {
      flush(s, pend);
      pend = 0;
    }
  }
  return j;
}

// boundary_walk for the wavefronts of a workgroup that lie on CPW columns (pc:
// the split X, Y of the thread's column, the same in all its lanes).  Every
// thread of the workgroup calls this or every thread calls boundary_walk.
template <int CPW, class Stager, class Loops>
__device__ __forceinline__ void column_walk(Lane<1>& s, const Stager& stage, int nb, const Loops& L, RPt* sv,
                                            ColLds<CPW>& cl, const QP& pc, int& pend) {
  constexpr int kWpc = (kThreads / 64) / CPW;   // wavefronts per column
  const int slot = (threadIdx.x >> 6) / kWpc;
  float* rho2 = cl.rho2[slot];
  float2* ng = cl.ng[slot];
  const int t0 = threadIdx.x % (64 * kWpc);
  VQ first[1];
  first[0].x = first[0].y = first[0].a = 0.0f;
  float aA = 0.0f;                 // alpha of the last vertex visited
  RPt prev;
  prev.xy = prev.zt = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  int l = 0;
  for (int c0 = 0; c0 < nb; c0 += kChunk) {
    const int c1 = min(c0 + kChunk, nb);
    if (c0 > 0) prev = sv[kChunk - 1];   // the previous chunk was full
    __syncthreads();
    stage(c0, c1 - c0, sv);
    __syncthreads();
    column_chunk(sv, c1 - c0, c0 > 0, prev, pc, rho2, ng, t0, 64 * kWpc);
    if constexpr (kWpc == 1) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();   // the column's wavefronts wrote its data together
    }
    for (; l < L.n() && L.off(l) < c1; ++l) {
      const int ls = L.off(l), le = L.off(l + 1);
      int j = max(ls, c0);
      const int j1 = min(le, c1);
      if (j == ls) {
        first[0] = vertex_q(sv[j - c0], s.p[0]);
        aA = first[0].a;
        ++j;
      }
      if (s.far)
        j = column_steps<true>(s, sv, rho2, ng, c0, j, j1, aA, pend);
      else
        j = column_steps<false>(s, sv, rho2, ng, c0, j, j1, aA, pend);
      for (; j < j1; ++j) {
        const int i = j - c0;
        const float a = column_alpha(sv[i], s.p[0], rho2[i]);
        const float2 e = ng[i];
        column_mul(s.T[0], __fmaf_rn(aA, a, e.y), e.x);
        rescale(s);
        aA = a;
        if (++pend == 32) {
          flush(s, 32);
          pend = 0;
        }
      }
      if (j1 < le) break;            // the loop continues in the next chunk
      // closing edge last -> first, with the per-query edge arithmetic
      const RPt v = sv[le - 1 - c0];
      VQ A[1];
      A[0].x = vertex_x(v, s.p[0]);
      A[0].y = vertex_y(v, s.p[0]);
      A[0].a = aA;
      edge_step(s, A, first, rpt_tie(v));
      rescale(s);
      if (++pend == 32) {
        flush(s, 32);
        pend = 0;
      }
    }
  }
}

// 32-bit index arithmetic (the host limits grids to fewer than 2^32
// points): 64-bit divisions would be long emulated sequences per query.
// CPW > 0: the workgroup's 256 points lie on CPW columns (the host sets 4, 2
// or 1 when nz is a multiple of 64, 128 or 256), and their shared walk keeps
// 6 KB of column data per column in LDS (4: four waves per SIMD, 2: five,
// 1: seven).  CPW = 0: the per-lane walk at eight waves per SIMD.
template <int CPW>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(CPW == 4 ? 4 : CPW == 2 ? 5 : CPW == 1 ? 7 : 8))) void k_grid3d_fwd(CrossArgs c, BndArgs a, LoopTable L,
                                                         const float* __restrict__ gx, const float* __restrict__ gy,
                                                         const float* __restrict__ gz, int64_t ny64, int64_t nz64,
                                                         int32_t* chi_out) {
  // the staged boundary, and before it the lines' crossing lists (read
  // before the walk stages its first chunk)
  __shared__ union {
    RPt sv[kChunk];
    int32_t hits[kThreads / 64][kColHits];
  } su;
  RPt* sv = su.sv;
  auto& s_hits = su.hits;
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
  QP pu;   // the column's X, Y (identical in every lane; made uniform)
  pu.xh = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s.p[0].xh)));
  pu.xl = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s.p[0].xl)));
  pu.yh = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s.p[0].yh)));
  pu.yl = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s.p[0].yl)));
  pu.zh = pu.zl = 0.0f;
  // wavefront-uniform: lane 0 is a query of the wavefront's column unless
  // the wavefront holds none
  const bool line = one_col && isfinite(pu.xh) && isfinite(pu.yh);
  int n = kColHits + 1;
  if (line) {
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
  // both walks stage their first chunk after a barrier, which every
  // wavefront reaches with its crossing list read
  if constexpr (CPW > 0) {
    __shared__ ColLds<CPW> cl;
    // the thread's column: that of the first point of its slot (clamped to
    // the grid, so that trailing lanes past the last point agree with it)
    constexpr int kWpc = (kThreads / 64) / CPW;
    const int64_t qs0 = (int64_t)blockIdx.x * kThreads + (int64_t)((threadIdx.x >> 6) / kWpc) * 64 * kWpc;
    const uint32_t qs = (uint32_t)min(qs0, a.nq - 1), cs = qs / nz;
    QP pc;
    {
      double X, Y, Z;
      rotate(a.F, gx[cs / ny], gy[cs % ny], gz[qs % nz], X, Y, Z);
      const QP t = make_qp(X, Y, Z);
      pc.xh = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(t.xh)));
      pc.xl = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(t.xl)));
      pc.yh = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(t.yh)));
      pc.yl = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(t.yl)));
      pc.zh = pc.zl = 0.0f;
    }
    // the shared walk, or the per-lane walk for a column with a non-finite x
    // or y: per wavefront when each has its own column (both walks pass the
    // same barriers), else for the whole workgroup (the shared walk adds a
    // barrier after the column data)
    bool shared = isfinite(pc.xh) && isfinite(pc.yh);
    if constexpr (kWpc > 1) shared = __syncthreads_and(shared);
    if (shared)
      column_walk<CPW>(s, StageRotate<KernargLoops>{a.F, a.bnd, KL}, a.nb, KL, sv, cl, pc, pend);
    else
      boundary_walk(s, StageRotate<KernargLoops>{a.F, a.bnd, KL}, a.nb, KL, sv, staged, pend);
  } else {
    boundary_walk(s, StageRotate<KernargLoops>{a.F, a.bnd, KL}, a.nb, KL, sv, staged, pend);
  }
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
  const dim3 g((unsigned)blocks), b(kThreads);
  if (nz % 256 == 0)
    hipLaunchKernelGGL(k_grid3d_fwd<1>, g, b, 0, s, c, a, L, gx, gy, gz, ny, nz, chi_out);
  else if (nz % 128 == 0)
    hipLaunchKernelGGL(k_grid3d_fwd<2>, g, b, 0, s, c, a, L, gx, gy, gz, ny, nz, chi_out);
  else if (nz % 64 == 0)
    hipLaunchKernelGGL(k_grid3d_fwd<4>, g, b, 0, s, c, a, L, gx, gy, gz, ny, nz, chi_out);
  else
    hipLaunchKernelGGL(k_grid3d_fwd<0>, g, b, 0, s, c, a, L, gx, gy, gz, ny, nz, chi_out);
  return hipGetLastError();
}

}  // namespace wn
