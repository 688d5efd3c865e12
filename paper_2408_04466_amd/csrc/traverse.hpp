// Ray/triangle crossing and BVH traversal for chi_d, shared by the plain
// crossing kernel and the batched persistent kernel.
#pragma once

#include "kernels.hpp"

namespace wn {

// ---------------------------------------------------------------------------
// Triangle test (shared predicates with the boundary kernel)
// ---------------------------------------------------------------------------

// The three edge values of a triangle for a query, each with its tie offset.
struct TriEdges {
  double n01, n12, n20;
};

__device__ __forceinline__ TriEdges tri_edges(const TriRec* __restrict__ r, uint32_t tb, const QP& p) {
  const float4 A = r->xy[0], B = r->xy[1], C = r->xy[2];
  const float ax = rel32(A.x, A.y, p.xh, p.xl), ay = rel32(A.z, A.w, p.yh, p.yl);
  const float bx = rel32(B.x, B.y, p.xh, p.xl), by = rel32(B.z, B.w, p.yh, p.yl);
  const float cx = rel32(C.x, C.y, p.xh, p.xl), cy = rel32(C.z, C.w, p.yh, p.yl);
  TriEdges e;
  e.n01 = edge_tie(edge_n(ax, ay, bx, by), tie_offset((tb & 1u) != 0u));
  e.n12 = edge_tie(edge_n(bx, by, cx, cy), tie_offset((tb & 2u) != 0u));
  e.n20 = edge_tie(edge_n(cx, cy, ax, ay), tie_offset((tb & 4u) != 0u));
  return e;
}

// The line of the ray (both directions) passes through the triangle's
// interior: the three edge values share a sign.  It depends on the query's
// X and Y only, so every point of a vertical line gets the same answer.
__device__ __forceinline__ bool tri_inside(const TriEdges& e) {
  const bool s01 = e.n01 < 0.0, s12 = e.n12 < 0.0, s20 = e.n20 < 0.0;
  return s01 == s12 && s12 == s20;
}

// +1 / -1 when the ray p + t d (t > 0) passes through the interior of sorted
// triangle t along / against its normal (v1-v0)x(v2-v0), 0 otherwise (ties:
// the record's tie signs, as its tree node holds them).
__device__ __forceinline__ int tri_crossing(const TriRec* __restrict__ recs, int32_t t, uint32_t ties, const QP& p) {
  const TriRec* r = recs + t;
  const TriEdges e = tri_edges(r, ties, p);
  if (!tri_inside(e)) return 0;
  const bool s01 = e.n01 < 0.0;
  // Height of the crossing above p: the barycentric weights are the edge
  // values opposite each vertex, so the crossing is above p iff
  // sum(N_opp * Z) has the sign of the N's.
  const float4 zab = r->zab;
  const double za = (double)rel32(zab.x, zab.y, p.zh, p.zl);
  const double zb = (double)rel32(zab.z, zab.w, p.zh, p.zl);
  const double zc = (double)rel32(r->zch, r->zcl, p.zh, p.zl);
  const double num = __fma_rn(e.n12, za, __fma_rn(e.n20, zb, __dmul_rn(e.n01, zc)));
  const bool hit = s01 ? (num < 0.0) : (num > 0.0);
  return hit ? (s01 ? 1 : -1) : 0;
}

// The same with the tie signs read from the record.
__device__ __forceinline__ int tri_crossing(const TriRec* __restrict__ recs, int32_t t, const QP& p) {
  return tri_crossing(recs, t, recs[t].ties, p);
}

// The line through p along d (both directions) passes through the interior
// of sorted triangle t.
__device__ __forceinline__ bool tri_on_line(const TriRec* __restrict__ recs, int32_t t, uint32_t ties, const QP& p) {
  return tri_inside(tri_edges(recs + t, ties, p));
}

// ---------------------------------------------------------------------------
// Traversal with a short stack in registers
// ---------------------------------------------------------------------------

// Traversal stack: the top S entries live in registers (push and pop shift
// them, plain moves, no indexed addressing); deeper entries spill to a
// separate private array that only overflowing traversals touch.  A node
// leaves at most three siblings pending beside the child walked next, and
// the four-wide tree over a binary LBVH of depth <= 64 (its split keys are
// 64-bit) has at most 33 levels, which bounds the number of pending entries.
constexpr int kSpill = 3 * 33;

template <int S>
struct RegStack {
  int32_t e[S];   // e[0] = top
  int n;
  bool lost;
  __device__ __forceinline__ void init() {
    n = 0;
    lost = false;
  }
  // Never fails: an entry beyond the spill array (only a malformed tree
  // gets there) is dropped and recorded in `lost`, which the caller checks
  // before its next pop.
  __device__ __forceinline__ void push(int32_t v, int32_t* spill) {
    if (n >= S) {
      if (n - S < kSpill)
        spill[n - S] = e[S - 1];
      else
        lost = true;
    }
#pragma unroll
    for (int i = S - 1; i > 0; --i) e[i] = e[i - 1];
    e[0] = v;
    ++n;
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

// Cell of coordinate v on one axis of a four-wide node's grid: floor(fma(v,
// i, m)), kept as a float (an integer value; +-inf or NaN for such v).
// Monotone non-decreasing in v (i > 0): the build assigns the children's
// cells with this same function, and an 8-bit cell converted to float
// compares with it exactly.  A NaN coordinate passes no comparison.
__device__ __forceinline__ float grid_cell(float v, float i, float m) { return floorf(__fmaf_rn(v, i, m)); }

// Cell k of a word of four 8-bit cells, as a float.
__device__ __forceinline__ float cell_of(uint32_t cells, int k) { return (float)((cells >> (8 * k)) & 0xffu); }

__device__ __forceinline__ int32_t child_ref(const BvhNode4& nd, int k) {
  return k == 0 ? nd.child[0] : k == 1 ? nd.child[1] : k == 2 ? nd.child[2] : nd.child[3];
}

// Walk the tree for the vertical half line above (x, y, z) in the frame of
// d and call leaf(t, ties) for every sorted triangle t (with its edge tie
// signs) whose padded box, widened to
// its node's grid, contains (x, y) with zmax >= z.  z = -inf visits every
// triangle whose box contains (x, y), whatever its height (the column pass
// of the grid mode).  The widening only adds triangles whose exact test
// then finds no crossing.  Returns 0, or WN_CHI_INVALID if the tree is
// malformed.
template <int S, class Leaf>
__device__ __forceinline__ int traverse_leaves(const CrossArgs& a, float x, float y, float z, Leaf&& leaf) {
  if (a.nf == 0) return 0;
  if (a.nf == 1) {
    if (in_box(a.leafbox[0], a.leafz[0], x, y, z)) leaf(0, a.tris[0].ties);
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
    const BvhNode4 nd = a.nodes[node];
    const float cx = grid_cell(x, nd.ix, nd.mx), cy = grid_cell(y, nd.iy, nd.my), cz = grid_cell(z, nd.iz, nd.mz);
    uint32_t lm = 0, im;   // hit leaves, hit nodes (the hit slots first, split without branches)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool h = (cell_of(nd.xlo, k) <= cx) & (cx <= cell_of(nd.xhi, k)) & (cell_of(nd.ylo, k) <= cy) &
                     (cy <= cell_of(nd.yhi, k)) & (cz <= cell_of(nd.zhi, k));
      lm |= h ? (1u << k) : 0u;
    }
    {
      const uint32_t leaves = (nd.ties >> 12) & 0xfu;   // bit k: child k is a leaf
      im = lm & ~leaves;
      lm &= leaves;
    }
    while (lm) {
      const int k = __builtin_ctz(lm);
      const int32_t c = child_ref(nd, k);
      lm &= lm - 1u;
      if (~c >= a.nf) return WN_CHI_INVALID;
      leaf(~c, (nd.ties >> (3 * k)) & 7u);
    }
    if (im) {
      node = child_ref(nd, __builtin_ctz(im));
      im &= im - 1u;
      // at most three siblings wait (unrolled: a loop keeps copies of the
      // register stack alive across its iterations)
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        if (im) {
          st.push(child_ref(nd, __builtin_ctz(im)), spill);
          im &= im - 1u;
        }
      }
      if (st.lost) return WN_CHI_INVALID;
    } else {
      if (st.n == 0) break;
      node = st.pop(spill);
    }
  }
  return 0;
}

// chi for one query (WN_CHI_INVALID if the tree is malformed).
template <int S>
__device__ int traverse(const CrossArgs& a, const QP& p) {
  int chi = 0;
  const int st = traverse_leaves<S>(a, p.xh, p.yh, p.zh, [&](int t, uint32_t ties) {
    chi += tri_crossing(a.tris, t, ties, p);
  });
  return st ? st : chi;
}

}  // namespace wn
