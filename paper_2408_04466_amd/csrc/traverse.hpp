// Ray/triangle crossing and BVH traversal for chi_d, shared by the plain
// crossing kernel and the batched persistent kernel.
#pragma once

#include "kernels.hpp"

namespace wn {

// ---------------------------------------------------------------------------
// Triangle test (shared predicates with the boundary kernel)
// ---------------------------------------------------------------------------

// A vertex index (below 2^31) with the lexicographic order of the edge that
// leaves it in bit 31, as the sorted triangle records store it.
__device__ __forceinline__ int32_t tri_index(int32_t v, bool a_less_b) {
  return a_less_b ? (int32_t)((uint32_t)v | 0x80000000u) : v;
}

// The three edge values of a triangle for a query, each with its tie offset
// (t holds the vertex indices with the edges' lexicographic order in bit 31,
// tri_index).
struct TriEdges {
  double n01, n12, n20;
};

template <bool STORED_TIES>
__device__ __forceinline__ TriEdges tri_edges(const int4 t, const RPt& A, const RPt& B, const RPt& C, const QP& p) {
  // the three tie bits in one register, so that the indices die at once
  const uint32_t tb = ((uint32_t)t.x >> 31) | (((uint32_t)t.y >> 30) & 2u) | (((uint32_t)t.z >> 29) & 4u);
  const float ax = vertex_x(A, p), ay = vertex_y(A, p);
  const float bx = vertex_x(B, p), by = vertex_y(B, p);
  const float cx = vertex_x(C, p), cy = vertex_y(C, p);
  // the stored bits, or the same comparisons redone (fewer live registers
  // where the register budget is tight)
  const bool l01 = STORED_TIES ? (tb & 1u) != 0 : rpt_less(A, B);
  const bool l12 = STORED_TIES ? (tb & 2u) != 0 : rpt_less(B, C);
  const bool l20 = STORED_TIES ? (tb & 4u) != 0 : rpt_less(C, A);
  TriEdges e;
  e.n01 = edge_tie(edge_n(ax, ay, bx, by), tie_offset(l01));
  e.n12 = edge_tie(edge_n(bx, by, cx, cy), tie_offset(l12));
  e.n20 = edge_tie(edge_n(cx, cy, ax, ay), tie_offset(l20));
  return e;
}

// The line of the ray (both directions) passes through the triangle's
// interior: the three edge values share a sign.  It depends on the query's
// X and Y only, so every point of a vertical line gets the same answer.
__device__ __forceinline__ bool tri_inside(const TriEdges& e) {
  const bool s01 = e.n01 < 0.0, s12 = e.n12 < 0.0, s20 = e.n20 < 0.0;
  return s01 == s12 && s12 == s20;
}

// +1 / -1 when the ray p + t d (t > 0) passes through the triangle's
// interior along / against its normal (v1-v0)x(v2-v0), 0 otherwise.
template <bool STORED_TIES>
__device__ __forceinline__ int tri_crossing(const int4 t, const RPt* __restrict__ Vr, const QP& p) {
  const RPt A = Vr[t.x & 0x7fffffff];
  const RPt B = Vr[t.y & 0x7fffffff];
  const RPt C = Vr[t.z & 0x7fffffff];
  const TriEdges e = tri_edges<STORED_TIES>(t, A, B, C, p);
  if (!tri_inside(e)) return 0;
  const bool s01 = e.n01 < 0.0;
  // Height of the crossing above p: the barycentric weights are the edge
  // values opposite each vertex, so the crossing is above p iff
  // sum(N_opp * Z) has the sign of the N's.
  const double za = (double)vertex_z(A, p), zb = (double)vertex_z(B, p), zc = (double)vertex_z(C, p);
  const double num = __fma_rn(e.n12, za, __fma_rn(e.n20, zb, __dmul_rn(e.n01, zc)));
  const bool hit = s01 ? (num < 0.0) : (num > 0.0);
  return hit ? (s01 ? 1 : -1) : 0;
}

// The line through p along d (both directions) passes through the
// triangle's interior.
template <bool STORED_TIES>
__device__ __forceinline__ bool tri_on_line(const int4 t, const RPt* __restrict__ Vr, const QP& p) {
  const RPt A = Vr[t.x & 0x7fffffff];
  const RPt B = Vr[t.y & 0x7fffffff];
  const RPt C = Vr[t.z & 0x7fffffff];
  return tri_inside(tri_edges<STORED_TIES>(t, A, B, C, p));
}

// ---------------------------------------------------------------------------
// Traversal with a short stack in registers
// ---------------------------------------------------------------------------

// Traversal stack: the top S entries live in registers (push and pop shift
// them, plain moves, no indexed addressing); deeper entries spill to a
// separate private array that only overflowing traversals touch.  The LBVH's
// depth is below 64 (its split keys are 64-bit), which bounds the number of
// pending siblings.
constexpr int kSpill = 64;

template <int S>
struct RegStack {
  int32_t e[S];   // e[0] = top
  int n;
  __device__ __forceinline__ void init() { n = 0; }
  __device__ __forceinline__ bool push(int32_t v, int32_t* spill) {
    if (n >= S) {
      if (n - S >= kSpill) return false;
      spill[n - S] = e[S - 1];
    }
#pragma unroll
    for (int i = S - 1; i > 0; --i) e[i] = e[i - 1];
    e[0] = v;
    ++n;
    return true;
  }
  __device__ __forceinline__ int32_t pop(const int32_t* spill) {
    const int32_t v = e[0];
#pragma unroll
    for (int i = 0; i < S - 1; ++i) e[i] = e[i + 1];
    --n;
    if (n >= S) e[S - 1] = spill[n - S];
    return v;
  }
};

__device__ __forceinline__ bool in_box(const float4 b, float bz, float x, float y, float z) {
  return (x >= b.x) & (x <= b.y) & (y >= b.z) & (y <= b.w) & (z <= bz);
}

// Walk the tree for the vertical half line above (x, y, z) in the frame of
// d and call leaf(t) for every sorted triangle t whose padded box contains
// (x, y) with zmax >= z.  z = -inf visits every triangle whose projection box
// contains (x, y), whatever its height (the column pass of the grid mode).
// Returns 0, or WN_CHI_INVALID if the tree is malformed.
template <int S, class Leaf>
__device__ __forceinline__ int traverse_leaves(const CrossArgs& a, float x, float y, float z, Leaf&& leaf) {
  if (a.nf == 0) return 0;
  if (a.nf == 1) {
    if (in_box(a.leafbox[0], a.leafz[0], x, y, z)) leaf(0);
    return 0;
  }
  RegStack<S> st;
  int32_t spill[kSpill];
  st.init();
  int32_t node = 0;
  const int32_t nint = a.nf - 1;
  // a valid tree visits each node at most once per query
  for (int32_t it = 0;; ++it) {
    if (it > nint || (uint32_t)node >= (uint32_t)nint) return WN_CHI_INVALID;
    const BvhNode nd = a.nodes[node];
    bool hl = in_box(nd.lbox, nd.lzmax, x, y, z);
    bool hr = in_box(nd.rbox, nd.rzmax, x, y, z);
    if (hl && nd.left < 0) {
      if (~nd.left >= a.nf) return WN_CHI_INVALID;
      leaf(~nd.left);
      hl = false;
    }
    if (hr && nd.right < 0) {
      if (~nd.right >= a.nf) return WN_CHI_INVALID;
      leaf(~nd.right);
      hr = false;
    }
    if (hl && hr) {
      if (!st.push(nd.right, spill)) return WN_CHI_INVALID;
      node = nd.left;
    } else if (hl) {
      node = nd.left;
    } else if (hr) {
      node = nd.right;
    } else {
      if (st.n == 0) break;
      node = st.pop(spill);
    }
  }
  return 0;
}

// chi for one query (WN_CHI_INVALID if the tree is malformed).
template <int S, bool STORED_TIES = false>
__device__ int traverse(const CrossArgs& a, const QP& p) {
  int chi = 0;
  const int st = traverse_leaves<S>(a, p.xh, p.yh, p.zh, [&](int t) {
    chi += tri_crossing<STORED_TIES>(a.tris[t], a.Vr, p);
  });
  return st ? st : chi;
}

}  // namespace wn
