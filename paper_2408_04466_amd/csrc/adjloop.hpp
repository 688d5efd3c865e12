// Adjoint of the 3D winding number: the per-tile walk over the boundary,
// shared by the plain adjoint kernel and the batched persistent kernel.
//
// chi_d is piecewise constant, so w varies only through the boundary line
// integral, whose derivatives are independent of d.  For an edge a->b with
// a' = a - p, b' = b - p:  K = 1/(|a'||b'| + a'.b'),  c = (a' x b') K,
//   dw/dp += c (1/|a'| + 1/|b'|) / 4pi          (Biot-Savart field of dM)
//   dw/da += -c / (|a'| 4pi),  dw/db += -c / (|b'| 4pi)
// (the same field integrated against each vertex's hat function along the
// straight edge).  These vanish in sum: sum_v dw/dv + dw/dp = 0.
//
// A lane holds QPL queries (a template parameter); the workgroup stages the
// boundary in LDS (each vertex with the edge leaving it) and
// every lane walks the same vertex sequence.  A vertex's gradient is complete
// one step after the vertex is visited (its two edges are then done); it is
// summed over the lane's queries in registers and over each quad of 4 lanes
// with DPP moves; the sixteen quad sums wait in LDS until kBlk consecutive
// vertices are complete, and their sums (one per wavefront and vertex) then
// go to an LDS window of kWin vertices.  When the walk leaves a window, the
// workgroup adds the wavefronts' sums in wavefront order and writes them
// with coalesced stores as float32 partials, one per (tile, vertex).  The
// closing edge's share of each loop's first vertex goes to a separate
// per-loop partial, summed over the workgroup the same way.  The partials
// are reduced in a fixed order in float64 by separate kernels, so grad_bnd
// is bitwise reproducible.
#pragma once

#include "bndloop.hpp"
#include "kernels.hpp"

namespace wn {
namespace adj {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kQPL = 4;              // queries per lane of the batched adjoint (plain: 1, 2 or 4)
constexpr int kChunk = 512;
constexpr int kTile = kThreads * kQPL;   // queries per batched tile
constexpr int kBlk = 16;              // vertices per LDS quad-sum block
constexpr int kRowFloats = kBlk * 48; // LDS quad sums per wavefront: [kBlk][3][16 quads]
constexpr int kWin = 128;             // vertices per workgroup window (a multiple of kBlk)
constexpr float kInv4Pi = 0.07957747154594767f;

// LDS of the adjoint walk: the staged chunk (vertices, then the edges leaving
// them), each wavefront's quad-sum block, the workgroup's window of per-
// wavefront vertex sums [kWaves][kWin][3], and a small exchange area.
struct AdjLds {
  float4 sv[2 * kChunk];
  float rsw[kWaves * kRowFloats];
  float ps[kWaves * kWin * 3];
  float sh[kWaves * 3];
};

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

// Sum over the 64 lanes of a wavefront, left in lane 63, with DPP moves
// (no LDS traffic): butterflies inside quads, rotations inside rows of 16,
// then the row broadcasts of lanes 15 and 31.
__device__ __forceinline__ float wave_sum_last(float v) {
  v += dpp<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v += dpp<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v += dpp<0x124, 0xF>(v);   // row_ror:4
  v += dpp<0x128, 0xF>(v);   // row_ror:8  -> every lane holds its row's sum
  v += dpp<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

// Sum over each quad of 4 lanes (every lane of the quad holds it).  The
// empty asm keeps the sum computed in every lane at this point: sunk into the
// branch of the lanes that store it, the second step would become a move, a
// DPP move and an add instead of one DPP add.
__device__ __forceinline__ float quad_sum(float v) {
  v += dpp<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v += dpp<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  asm volatile("" : "+v"(v));
  return v;
}

// Wavefront-scope ordering of the LDS quad-sum block between the lanes that
// write it and the lanes that read it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Where a walk's completed vertices go (all fields wavefront-uniform).
// Vertices complete in increasing order without gaps, so the window holds
// the run [lo, hi) of them, inside [f0, f0 + kWin).
struct Parker {
  float* rs;      // this wavefront's quad-sum block [kRowFloats] (LDS)
  float* ps;      // the workgroup's window [kWaves][kWin][3] (LDS)
  float* pv;      // the workgroup's partial row [nb][3], or null
  int f0, lo, hi;
};

__device__ __forceinline__ Parker make_parker(AdjLds& s, float* pv) {
  Parker P;
  P.rs = s.rsw + (threadIdx.x >> 6) * kRowFloats;
  P.ps = s.ps;
  P.pv = pv;
  P.f0 = -2 * kWin;   // no window yet
  P.lo = P.hi = 0;
  return P;
}

// Every thread of the workgroup: the window's vertices, summed over the
// wavefronts in wavefront order, to the partial row.
__device__ __forceinline__ void flush_window(Parker& P) {
  __syncthreads();
  const int n = 3 * (P.hi - P.lo);
  const float* x = P.ps + 3 * (P.lo - P.f0);
  float* d = P.pv + 3 * (int64_t)P.lo;
  int t0 = threadIdx.x;   // a fresh copy: no lane address kept live across the walk
  asm volatile("" : "+v"(t0));
  for (int t = t0; t < n; t += kThreads) {
    float s = x[t];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s = __fadd_rn(s, x[w * kWin * 3 + t]);
    d[t] = s;
  }
  __syncthreads();
  P.lo = P.hi;
}

// Every thread of the workgroup, at the end of a walk: the last window.
__device__ __forceinline__ void flush_last(Parker& P) {
  if (P.pv && P.hi > P.lo) flush_window(P);
}

// Vertex va's quad sums (r[c], every lane of a quad holds its quad's sum)
// into the wavefront's LDS block at [va % kBlk][c][quad]; once the block is
// full (or va is the last vertex), lane t < 3 n adds the sixteen quad sums of
// entry t in quad order into the workgroup's window, after flushing the
// window if the block lies beyond it.  Every wavefront of the workgroup parks the same
// vertices, so the flush's barriers are reached by all of them.
__device__ __forceinline__ void park_sums(Parker& P, int va, int nb, const float r[3], int lane) {
  const int slot = va % kBlk;
  if ((lane & 3) == 3) {
    float* d = P.rs + slot * 48 + (lane >> 2);
    d[0] = r[0];
    d[16] = r[1];
    d[32] = r[2];
  }
  if (slot == kBlk - 1 || va == nb - 1) {
    const int b0 = va - slot;
    if (b0 >= P.f0 + kWin) {
      if (P.hi > P.lo) flush_window(P);
      P.f0 = b0 - b0 % kWin;
      P.lo = P.hi = b0;
    }
    wave_sync();
    const int n = slot + 1;
    if (lane < 3 * n) {
      const float4* x = reinterpret_cast<const float4*>(P.rs) + 4 * lane;
      float s = 0.f;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float4 y = x[k];
        s = k == 0 ? y.x : __fadd_rn(s, y.x);
        s = __fadd_rn(__fadd_rn(__fadd_rn(s, y.y), y.z), y.w);
      }
      P.ps[(threadIdx.x >> 6) * kWin * 3 + 3 * (b0 - P.f0) + lane] = s;
    }
    P.hi = va + 1;
    wave_sync();
  }
}

// Vertex va's partial (three values per lane).
__device__ __forceinline__ void park(Parker& P, int va, int nb, const float acc[3], int lane) {
  const float r[3] = {quad_sum(acc[0]), quad_sum(acc[1]), quad_sum(acc[2])};
  park_sums(P, va, nb, r, lane);
}

// The partials of vertices va and va + 1: the six quad sums first (six
// independent chains of lane moves instead of two runs of three), then the
// two LDS entries in vertex order.
__device__ __forceinline__ void park2(Parker& P, int va, int nb, const float a[3], const float b[3], int lane) {
  const float ra[3] = {quad_sum(a[0]), quad_sum(a[1]), quad_sum(a[2])};
  const float rb[3] = {quad_sum(b[0]), quad_sum(b[1]), quad_sum(b[2])};
  park_sums(P, va, nb, ra, lane);
  park_sums(P, va + 1, nb, rb, lane);
}

struct QState {
  float px, py, pz, g;       // g: twice dL/dw (see edge_grad)
  float gx, gy, gz;          // sum_e g c_e (1/|a'| + 1/|b'|)
};

// A boundary vertex seen from one query: v - p, |v - p|, 1/|v - p|.
struct Rel {
  float x, y, z, r, i;
};

__device__ __forceinline__ Rel rel(const QState& s, const float4& v) {
  Rel q;
  q.x = __fsub_rn(v.x, s.px);
  q.y = __fsub_rn(v.y, s.py);
  q.z = __fsub_rn(v.z, s.pz);
  const float r2 = __fmaf_rn(q.x, q.x, __fmaf_rn(q.y, q.y, __fmul_rn(q.z, q.z)));
  q.i = __builtin_amdgcn_rsqf(r2);
  q.r = __fmul_rn(r2, q.i);
  return q;
}

// Edge a->b for one query, with e = (b - a, |b - a|^2) taken from the
// boundary itself: c = g K (a' x b') with a' x b' = a' x (b - a) (no
// cancellation between the two long relative vectors of a far query) and
// 1/K = |a'||b'| + a'.b' = ((|a'| + |b'|)^2 - |b - a|^2) / 2, since
// |b - a|^2 = |a'|^2 + |b'|^2 - 2 a'.b' (the factor 2 sits in s.g); adds
// c (1/|a'| + 1/|b'|) to the query gradient and c/|a'|, c/|b'| to the two
// vertex accumulators (FIRST: acc_b starts here, for the lane's first query).
template <bool FIRST>
__device__ __forceinline__ void edge_grad(QState& s, const Rel& a, const Rel& b, const float4& e, float* acc_a,
                                          float* acc_b) {
  const float crx = __fmaf_rn(a.y, e.z, -__fmul_rn(a.z, e.y));
  const float cry = __fmaf_rn(a.z, e.x, -__fmul_rn(a.x, e.z));
  const float crz = __fmaf_rn(a.x, e.y, -__fmul_rn(a.y, e.x));
  const float rs = __fadd_rn(a.r, b.r);
  const float den2 = __fmaf_rn(rs, rs, -e.w);
  const float gk = __fmul_rn(s.g, __builtin_amdgcn_rcpf(den2));
  // c / |a'| = cr (gk / |a'|), c / |b'| = cr (gk / |b'|), and the query's
  // c (1/|a'| + 1/|b'|) = cr (ta + tb)
  const float ta = __fmul_rn(gk, a.i);
  const float tb = __fmul_rn(gk, b.i);
  const float h = __fadd_rn(ta, tb);
  s.gx = __fmaf_rn(crx, h, s.gx);
  s.gy = __fmaf_rn(cry, h, s.gy);
  s.gz = __fmaf_rn(crz, h, s.gz);
  acc_a[0] = __fmaf_rn(crx, ta, acc_a[0]);
  acc_a[1] = __fmaf_rn(cry, ta, acc_a[1]);
  acc_a[2] = __fmaf_rn(crz, ta, acc_a[2]);
  acc_b[0] = FIRST ? __fmul_rn(crx, tb) : __fmaf_rn(crx, tb, acc_b[0]);
  acc_b[1] = FIRST ? __fmul_rn(cry, tb) : __fmaf_rn(cry, tb, acc_b[1]);
  acc_b[2] = FIRST ? __fmul_rn(crz, tb) : __fmaf_rn(crz, tb, acc_b[2]);
}

// Edge A->B for every query of the lane: the query gradients, vertex A's
// accumulator, and vertex B's started afresh.
template <int QPL>
__device__ __forceinline__ void edges(QState* S, const Rel* A, const Rel* B, const float4& e, float* accA,
                                      float* accB) {
  edge_grad<true>(S[0], A[0], B[0], e, accA, accB);
#pragma unroll
  for (int k = 1; k < QPL; ++k) edge_grad<false>(S[k], A[k], B[k], e, accA, accB);
}

// Stage boundary vertex i (flat index, loops L) for the adjoint walk: its
// coordinates at sv[j] and, at sv[kChunk + j], the edge leaving it, v_next -
// v_i, with its squared length in .w.
template <class Loops>
__device__ __forceinline__ void stage_adj(const float* __restrict__ bnd, const Loops& L, int i, int j,
                                          float4* sv) {
  const int lp = bnd::loop_of(L, i);
  const int nx = (i + 1 < L.off(lp + 1)) ? i + 1 : L.off(lp);
  const float x = bnd[3 * i], y = bnd[3 * i + 1], z = bnd[3 * i + 2];
  const float ex = __fsub_rn(bnd[3 * nx], x), ey = __fsub_rn(bnd[3 * nx + 1], y),
              ez = __fsub_rn(bnd[3 * nx + 2], z);
  sv[j] = make_float4(x, y, z, 0.f);
  sv[kChunk + j] = make_float4(ex, ey, ez, __fmaf_rn(ex, ex, __fmaf_rn(ey, ey, __fmul_rn(ez, ez))));
}

// Every thread of the workgroup: acc summed over each wavefront, then over
// the wavefronts in order, to dst[0..2] (sh: kWaves * 3 floats of LDS).
__device__ __forceinline__ void put3(float* dst, const float acc[3], float* sh, int lane) {
  const float r0 = wave_sum_last(acc[0]);
  const float r1 = wave_sum_last(acc[1]);
  const float r2 = wave_sum_last(acc[2]);
  if (lane == 63) {
    float* d = sh + 3 * (threadIdx.x >> 6);
    d[0] = r0;
    d[1] = r1;
    d[2] = r2;
  }
  __syncthreads();
  int t = threadIdx.x;   // a fresh copy: no address kept live across the walk
  asm volatile("" : "+v"(t));
  if (t < 3) {
    float s = sh[t];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s = __fadd_rn(s, sh[3 * w + t]);
    dst[t] = s;
  }
  __syncthreads();
}

// Load the tile's queries [q0, q0 + cnt) into the lane states (QPL per lane;
// lane query k is tile entry k * kThreads + threadIdx.x).
template <int QPL>
__device__ __forceinline__ void load_tile(QState* S, const float* qx, const float* qy, const float* qz,
                                          const float* gw, int64_t q0, int64_t cnt) {
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int64_t r = (int64_t)k * kThreads + threadIdx.x;
    const bool ok = r < cnt;
    const int64_t q = q0 + (ok ? r : 0);
    S[k].px = qx[q];
    S[k].py = qy[q];
    S[k].pz = qz[q];
    S[k].g = ok ? 2.0f * gw[q] : 0.0f;   // padding lanes contribute nothing
    S[k].gx = S[k].gy = S[k].gz = 0.0f;
  }
}

__device__ __forceinline__ void zero3(float* a) { a[0] = a[1] = a[2] = 0.f; }

// Edge A->B for every query of the lane; the partial of vertex A is then
// complete and goes out (summed over the wavefront) to row entry `va`.
template <int QPL>
__device__ __forceinline__ void step(QState* S, const Rel* A, const Rel* B, const float4& e, float* accA,
                                     float* accB, Parker& P, int va, int nb, int lane) {
  edges<QPL>(S, A, B, e, accA, accB);
  if (P.pv) park(P, va, nb, accA, lane);
}

// Walk the boundary for one tile (every thread of the workgroup).  pv: the
// workgroup's partial row [nb][3] (or null), pl: its per-loop row
// [nloops][3] (the closing edge's share of each loop's first vertex; null
// with pv).  Loops are taken as straight vertex ranges (like the forward
// walk), two vertices per step; vertices complete in increasing order 0 ..
// nb-1.
template <int QPL, class Loops>
__device__ __forceinline__ void walk(QState* S, const float* __restrict__ bnd, int nb, const Loops& L,
                                     AdjLds& lds, float* pv, float* pl) {
  const int lane = threadIdx.x & 63;
  float4* sv = lds.sv;
  Parker P = make_parker(lds, pv);
  Rel A[QPL], B[QPL];              // A = last vertex visited
  float4 vF = make_float4(0.f, 0.f, 0.f, 0.f);   // the loop's first vertex (uniform)
  float accA[3], accB[3];          // pending partial of vertex A (and scratch for B)
  float4 eA = make_float4(0.f, 0.f, 0.f, 0.f);   // the edge leaving vertex A
  zero3(accA);
  int l = 0;
  for (int c0 = 0; c0 < nb; c0 += kChunk) {
    const int c1 = min(c0 + kChunk, nb);
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
      }
      for (; j + 2 <= j1; j += 2) {
        const float4 v0 = sv[j - c0];
        const float4 v1 = sv[j + 1 - c0];
        const float4 e0 = sv[kChunk + j - c0];
        float accC[3];
#pragma unroll
        for (int k = 0; k < QPL; ++k) B[k] = rel(S[k], v0);
        edges<QPL>(S, A, B, eA, accA, accB);
#pragma unroll
        for (int k = 0; k < QPL; ++k) A[k] = rel(S[k], v1);
        edges<QPL>(S, B, A, e0, accB, accC);
        // vertices j - 1 and j are complete
        if (pv) park2(P, j - 1, nb, accA, accB, lane);
        accA[0] = accC[0]; accA[1] = accC[1]; accA[2] = accC[2];
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
      if (j1 < le) break;            // the loop continues in the next chunk
      // closing edge last -> first: completes the last vertex; the first
      // vertex's share goes to the per-loop row
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

// x[0] + x[stride] + ... + x[(cnt - 1) stride] in float64, added in index
// order, with the loads issued eight at a time (the partial reductions are
// latency-bound: one dependent load per addition otherwise).
template <class T>
__device__ __forceinline__ double ordered_sum(const T* __restrict__ x, int64_t stride, int64_t cnt, double s) {
  int64_t i = 0;
  for (; i + 8 <= cnt; i += 8) {
    T v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = x[(i + k) * stride];
#pragma unroll
    for (int k = 0; k < 8; ++k) s += (double)v[k];
  }
  for (; i < cnt; ++i) s += (double)x[i * stride];
  return s;
}

// The query gradients of the tile loaded by load_tile (the indices are
// recomputed rather than held through the walk).
template <int QPL>
__device__ __forceinline__ void store_gq(const QState* S, int64_t q0, int64_t cnt, float* gq) {
  // a fresh copy of the lane index, so that the compiler does not keep the
  // load's index arithmetic alive through the walk
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const int64_t r = (int64_t)k * kThreads + t;
    if (r >= cnt || !gq) continue;
    const int64_t q = q0 + r;
    gq[3 * q + 0] = S[k].gx * kInv4Pi;
    gq[3 * q + 1] = S[k].gy * kInv4Pi;
    gq[3 * q + 2] = S[k].gz * kInv4Pi;
  }
}

}  // namespace adj
}  // namespace wn
