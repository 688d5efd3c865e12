// Boundary line integral of the one-shot winding number: the per-lane walk
// over the boundary loops, shared by the plain boundary kernel and the
// batched persistent kernel.
//
// S(p) = sum over boundary edges a->b of theta_e, theta_e = atan2(N, D): half
// the signed solid angle of the spherical triangle (-d, a - p, b - p).  This
// is Eq. wn_discrete_sum with the region of d as the seed of Alg. 1: by
// Lemma 2 every other region differs from it by the number of boundary
// crossings in between, so the region areas collapse into one line integral
// over the boundary (the paper evaluates region areas from boundary
// integrals as well, Sec. 5.1 "Exact Computations").
//
// Layout: the workgroup stages the boundary loops into LDS (rotated
// coordinates as float32 pairs plus the tie offset of the edge leaving each
// vertex, 32 bytes) in chunks
// of kChunk vertices, and every lane walks the same vertex sequence, so the
// LDS reads are broadcasts.  Per (query, vertex) the frame quantities are
// formed once and reused by the two edges that share the vertex.  Instead of
// one atan2 per edge, the edge factors D + iN are multiplied into a running
// complex product whose half-plane changes count whole turns exactly
// (wn::Turns); one atan2 per query remains.
#pragma once

#include "kernels.hpp"

namespace wn {
namespace bnd {

constexpr int kThreads = 256;
constexpr int kChunk = 512;      // vertices per LDS stage: 512 * 32 B = 16 KB
constexpr int kStep = 16;        // vertices per main-loop step
// The float32 running product is rescaled every second edge: two factors,
// each at most 2^1.5 r_a r_b, stay below 2^127 when every boundary vertex is
// within 2^31 of the query (frame units): true for queries within 2^30 of
// the frame's centre, where the scene has size O(1).  Wavefronts holding a
// farther query rescale after every edge, which covers queries out to 2^56
// (r^2 and a factor stay below 2^115).  Beyond kHuge the boundary subtends
// less than 2^-50 rad, |w| <= area / (4 pi |p|^2) < 2^-100, and w is
// returned as 0 (lane_w).
constexpr float kNear = 1073741824.0f;          // 2^30
constexpr float kHuge = 72057594037927936.0f;   // 2^56

// Loop table accessors: loops in the kernel arguments (or, for a long table,
// in device memory named there), or in device memory.  Device tables are
// read-only for the whole launch and read through the constant address
// space, so a uniform index gives a scalar load and the loop bounds stay
// wave-uniform.
struct KernargLoops {
  const LoopTable& L;
  __device__ __forceinline__ int n() const { return L.n; }
  __device__ __forceinline__ int off(int l) const {
    return L.dev ? ((const __attribute__((address_space(4))) int32_t*)(L.dev))[l] : L.off[l];
  }
};
struct DeviceLoops {
  const int32_t* o;   // [n + 1], relative to the surface's first vertex
  int nl;
  __device__ __forceinline__ int n() const { return nl; }
  __device__ __forceinline__ int off(int l) const {
    return ((const __attribute__((address_space(4))) int32_t*)(o))[l];
  }
};

// Loop containing flat vertex index i (binary search over the loop table).
template <class Loops>
__device__ __forceinline__ int loop_of(const Loops& L, int i) {
  int lo = 0, hi = L.n() - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (L.off(mid) <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Boundary vertex i as staged: rotated coordinates (split) and the tie
// offset of the edge v_i -> v_next(i).
template <class Loops>
__device__ __forceinline__ RPt stage_vertex(const Frame& F, const float* __restrict__ bnd, const Loops& L, int i) {
  const int l = loop_of(L, i);
  const int nxt = (i + 1 < L.off(l + 1)) ? i + 1 : L.off(l);
  double X, Y, Z, Xn, Yn, Zn;
  rotate(F, bnd[3 * i], bnd[3 * i + 1], bnd[3 * i + 2], X, Y, Z);
  rotate(F, bnd[3 * nxt], bnd[3 * nxt + 1], bnd[3 * nxt + 2], Xn, Yn, Zn);
  const RPt a = make_rpt(X, Y, Z, 0.0), b = make_rpt(Xn, Yn, Zn, 0.0);
  return make_rpt(X, Y, Z, tie_offset(rpt_less(a, b)));
}

// Stage vertices [c0, c0 + cnt) into LDS.
template <class Loops>
__device__ __forceinline__ void stage_chunk(const Frame& F, const float* __restrict__ bnd, const Loops& L,
                                            int c0, int cnt, RPt* sv) {
  for (int j = threadIdx.x; j < cnt; j += kThreads) sv[j] = stage_vertex(F, bnd, L, c0 + j);
}

// Stagers: fill LDS with vertices [c0, c0 + cnt).  StageRotate rotates the
// float32 boundary on the fly; StageCopy copies a boundary that was rotated
// beforehand with the same arithmetic (the batched path rotates each
// surface's boundary once, when the batch is created).
template <class Loops>
struct StageRotate {
  const Frame& F;
  const float* __restrict__ bnd;
  const Loops& L;
  __device__ __forceinline__ void operator()(int c0, int cnt, RPt* sv) const {
    stage_chunk(F, bnd, L, c0, cnt, sv);
  }
};
struct StageCopy {
  const RPt* __restrict__ src;
  __device__ __forceinline__ void operator()(int c0, int cnt, RPt* sv) const {
    for (int j = threadIdx.x; j < cnt; j += kThreads) sv[j] = src[c0 + j];
  }
};

template <int QPL>
struct Lane {
  QP p[QPL];
  Turns T[QPL];
  bool far;   // uniform: some query of the wavefront lies beyond kNear
};

__device__ __forceinline__ float qp_extent(const QP& p) {
  return fmaxf(fabsf(p.xh), fmaxf(fabsf(p.yh), fabsf(p.zh)));
}

// Set once the lane's queries are in place (every lane of the wavefront).
template <int QPL>
__device__ __forceinline__ void lane_range(Lane<QPL>& s) {
  bool f = false;
#pragma unroll
  for (int k = 0; k < QPL; ++k) f |= !(qp_extent(s.p[k]) < kNear);
  s.far = __any(f);
}

template <int QPL>
__device__ __forceinline__ void vert_q(const Lane<QPL>& s, const RPt& v, VQ* out) {
#pragma unroll
  for (int k = 0; k < QPL; ++k) out[k] = vertex_q(v, s.p[k]);
}

template <int QPL>
__device__ __forceinline__ void edge_step(Lane<QPL>& s, const VQ* a, const VQ* b, double tie) {
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    turns_edge(s.T[k], a[k], b[k], tie);
  }
}

template <int QPL>
__device__ __forceinline__ void rescale(Lane<QPL>& s) {
#pragma unroll
  for (int k = 0; k < QPL; ++k) turns_norm(s.T[k]);
}

template <int QPL>
__device__ __forceinline__ void flush(Lane<QPL>& s, int n) {
#pragma unroll
  for (int k = 0; k < QPL; ++k) turns_flush(s.T[k], n);
}

// Decide every pending turn of the lane (before reading its result).
template <int QPL>
__device__ __forceinline__ void finish_turns(Lane<QPL>& s, int& pend) {
  if (pend > 0) flush(s, pend);
  pend = 0;
}

// w of query k of the lane (every turn decided) for crossing count chi.
template <int QPL>
__device__ __forceinline__ float lane_w(const Lane<QPL>& s, int k, int chi) {
  return qp_extent(s.p[k]) < kHuge ? turns_to_w(s.T[k], chi) : 0.0f;
}

// Edges j-1 -> j ... while kStep more vertices of the loop segment [j, j1)
// remain; returns the next vertex.  The product is rescaled after every
// second edge, and after every edge for FAR wavefronts.
template <int QPL, bool FAR>
__device__ __forceinline__ int main_steps(Lane<QPL>& s, const RPt* sv, int c0, int j, int j1, VQ* A, VQ* B,
                                          double& ptie, int& pend) {
  for (; j + kStep <= j1; j += kStep) {
    if (pend > kStep) {
      flush(s, pend);
      pend = 0;
    }
    // the step's vertices through one vector register holding their LDS
    // address, the reads taking immediate offsets (the compiler otherwise
    // copies the uniform address into a vector register for every vertex)
    int vo = (j - c0) * (int)sizeof(RPt);
    asm volatile("" : "+v"(vo));
    const RPt* sp = reinterpret_cast<const RPt*>(reinterpret_cast<const char*>(sv) + vo);
#pragma unroll
    for (int u = 0; u < kStep; u += 2) {
      const RPt v0 = sp[u];
      vert_q(s, v0, B);
      edge_step(s, A, B, ptie);
      if (FAR) rescale(s);
      const RPt v1 = sp[u + 1];
      vert_q(s, v1, A);
      edge_step(s, B, A, rpt_tie(v0));
      ptie = rpt_tie(v1);
      rescale(s);
      // keep the scheduler from hoisting the LDS reads of later vertex
      // pairs to the top of the step: that prefetch holds extra vector
      // registers and cuts occupancy
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

// Multiply every boundary edge factor of the loops into the lane's turn
// accumulators.  All threads of the workgroup must call this together.
// `staged` tracks which chunk is in LDS (-1: none) so that a caller walking
// the same boundary again (next tile of queries) skips restaging when the
// whole boundary fits in one chunk.  The turns of the last edges may still
// be pending on return: call finish_turns before turns_to_w.
template <int QPL, class Stager, class Loops>
__device__ __forceinline__ void boundary_walk(Lane<QPL>& s, const Stager& stage, int nb, const Loops& L,
                                              RPt* sv, int& staged, int& pend) {
  VQ first[QPL], A[QPL], B[QPL];   // A holds the previous vertex between steps
  double ptie = 0.0;               // uniform: tie offset of the edge leaving A
  int l = 0;
  for (int c0 = 0; c0 < nb; c0 += kChunk) {
    const int c1 = min(c0 + kChunk, nb);
    if (staged != c0) {
      __syncthreads();
      stage(c0, c1 - c0, sv);
      __syncthreads();
      staged = c0;
    }
    // the loops overlapping [c0, c1), each as a straight-line vertex range
    for (; l < L.n() && L.off(l) < c1; ++l) {
      const int ls = L.off(l), le = L.off(l + 1);
      int j = max(ls, c0);
      const int j1 = min(le, c1);
      if (j == ls) {
        const RPt v = sv[j - c0];
        vert_q(s, v, first);
#pragma unroll
        for (int k = 0; k < QPL; ++k) A[k] = first[k];
        ptie = rpt_tie(v);
        ++j;
      }
      // kStep vertices per step, the roles of A and B alternating; the
      // turns are decided every second step (32 edges)
      if (s.far)
        j = main_steps<QPL, true>(s, sv, c0, j, j1, A, B, ptie, pend);
      else
        j = main_steps<QPL, false>(s, sv, c0, j, j1, A, B, ptie, pend);
      // the rest one vertex at a time, rescaled after every edge
      for (; j < j1; ++j) {
        const RPt v = sv[j - c0];
        vert_q(s, v, B);
        edge_step(s, A, B, ptie);
        rescale(s);
#pragma unroll
        for (int k = 0; k < QPL; ++k) A[k] = B[k];
        ptie = rpt_tie(v);
        if (++pend == 32) {
          flush(s, 32);
          pend = 0;
        }
      }
      if (j1 < le) break;            // the loop continues in the next chunk
      edge_step(s, A, first, ptie);  // closing edge last -> first
      rescale(s);
      if (++pend == 32) {
        flush(s, 32);
        pend = 0;
      }
    }
  }
}

}  // namespace bnd
}  // namespace wn
