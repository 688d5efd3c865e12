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
// A lane holds kQPL queries; the workgroup stages the boundary in LDS and
// every lane walks the same vertex sequence.  A vertex's gradient is complete
// one step after the vertex is visited (its two edges are then done); it is
// summed over the lane's queries in registers, over the wavefront with DPP
// moves, and written once per (tile, wavefront, vertex) as a float32 partial.
// The closing edge's share of each loop's first vertex goes to a separate
// per-loop partial.  The partials are reduced in a fixed order in float64 by
// separate kernels, so grad_bnd is bitwise reproducible.
#pragma once

#include "bndloop.hpp"
#include "kernels.hpp"

namespace wn {
namespace adj {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kQPL = 4;
constexpr int kChunk = 512;
constexpr int kTile = kThreads * 4;   // queries per tile (kQPL per lane)
constexpr float kInv4Pi = 0.07957747154594767f;

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

struct QState {
  float px, py, pz, g;
  float gx, gy, gz;          // sum_e g c_e (1/|a'| + 1/|b'|)
  float ax, ay, az, ra, ia;  // previous vertex relative to p, |.|, 1/|.|
  float fx, fy, fz, rf, iff; // first vertex of the current loop
};

// Edge a->b for one query: c = g K (a' x b'); adds c (1/|a'| + 1/|b'|) to
// the query gradient.
__device__ __forceinline__ void edge_grad(QState& s, float ax, float ay, float az, float ra,
                                          float ia, float bx, float by, float bz, float rb,
                                          float ib, float& cx, float& cy, float& cz) {
  const float crx = __fmaf_rn(ay, bz, -__fmul_rn(az, by));
  const float cry = __fmaf_rn(az, bx, -__fmul_rn(ax, bz));
  const float crz = __fmaf_rn(ax, by, -__fmul_rn(ay, bx));
  const float dot = __fmaf_rn(ax, bx, __fmaf_rn(ay, by, __fmul_rn(az, bz)));
  const float den = __fmaf_rn(ra, rb, dot);
  const float gk = __fmul_rn(s.g, __builtin_amdgcn_rcpf(den));
  cx = __fmul_rn(gk, crx);
  cy = __fmul_rn(gk, cry);
  cz = __fmul_rn(gk, crz);
  const float h = __fadd_rn(ia, ib);
  s.gx = __fmaf_rn(cx, h, s.gx);
  s.gy = __fmaf_rn(cy, h, s.gy);
  s.gz = __fmaf_rn(cz, h, s.gz);
}

__device__ __forceinline__ void put3(float* dst, const float acc[3], int lane) {
  const float r0 = wave_sum_last(acc[0]);
  const float r1 = wave_sum_last(acc[1]);
  const float r2 = wave_sum_last(acc[2]);
  if (lane == 63) {
    dst[0] = r0;
    dst[1] = r1;
    dst[2] = r2;
  }
}

// Load the tile's queries [q0, q0 + cnt) into the lane states.
__device__ __forceinline__ void load_tile(QState* S, const float* qx, const float* qy, const float* qz,
                                          const float* gw, int64_t q0, int64_t cnt, int64_t* qi, bool* ok) {
#pragma unroll
  for (int k = 0; k < kQPL; ++k) {
    const int64_t r = (int64_t)k * kThreads + threadIdx.x;
    ok[k] = r < cnt;
    qi[k] = q0 + (ok[k] ? r : 0);
    S[k].px = qx[qi[k]];
    S[k].py = qy[qi[k]];
    S[k].pz = qz[qi[k]];
    S[k].g = ok[k] ? gw[qi[k]] : 0.0f;      // padding lanes contribute nothing
    S[k].gx = S[k].gy = S[k].gz = 0.0f;
  }
}

// Walk the boundary for one tile.  pv: this wavefront's partial row
// [nb][3] (or null), pl: its per-loop row [nloops][3].
template <class Loops>
__device__ __forceinline__ void walk(QState* S, const float* __restrict__ bnd, int nb, const Loops& L,
                                     float4* sv, float* pv, float* pl) {
  const int lane = threadIdx.x & 63;
  float accp[3] = {0.f, 0.f, 0.f};   // previous vertex, summed over the lane's queries
  int loop = 0;
  for (int c0 = 0; c0 < nb; c0 += kChunk) {
    const int cnt = min(kChunk, nb - c0);
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kThreads) {
      const int i = c0 + j;
      sv[j] = make_float4(bnd[3 * i], bnd[3 * i + 1], bnd[3 * i + 2], 0.f);
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const int i = c0 + j;
      const float4 v = sv[j];
      while (L.off(loop + 1) <= i) ++loop;
      const bool starts = (i == L.off(loop));
      const bool ends = (i + 1 == L.off(loop + 1));
      float accc[3] = {0.f, 0.f, 0.f};   // this vertex
      float accf[3] = {0.f, 0.f, 0.f};   // closing-edge share of the loop's first vertex
#pragma unroll
      for (int k = 0; k < kQPL; ++k) {
        QState& s = S[k];
        const float bx = __fsub_rn(v.x, s.px), by = __fsub_rn(v.y, s.py), bz = __fsub_rn(v.z, s.pz);
        const float r2 = __fmaf_rn(bx, bx, __fmaf_rn(by, by, __fmul_rn(bz, bz)));
        const float ib = __builtin_amdgcn_rsqf(r2);
        const float rb = __fmul_rn(r2, ib);
        if (starts) {
          s.fx = bx; s.fy = by; s.fz = bz; s.rf = rb; s.iff = ib;
        } else {
          float cx, cy, cz;
          edge_grad(s, s.ax, s.ay, s.az, s.ra, s.ia, bx, by, bz, rb, ib, cx, cy, cz);
          accp[0] = __fmaf_rn(cx, s.ia, accp[0]);
          accp[1] = __fmaf_rn(cy, s.ia, accp[1]);
          accp[2] = __fmaf_rn(cz, s.ia, accp[2]);
          accc[0] = __fmaf_rn(cx, ib, accc[0]);
          accc[1] = __fmaf_rn(cy, ib, accc[1]);
          accc[2] = __fmaf_rn(cz, ib, accc[2]);
        }
        if (ends) {
          // closing edge last -> first
          float cx, cy, cz;
          edge_grad(s, bx, by, bz, rb, ib, s.fx, s.fy, s.fz, s.rf, s.iff, cx, cy, cz);
          accc[0] = __fmaf_rn(cx, ib, accc[0]);
          accc[1] = __fmaf_rn(cy, ib, accc[1]);
          accc[2] = __fmaf_rn(cz, ib, accc[2]);
          accf[0] = __fmaf_rn(cx, s.iff, accf[0]);
          accf[1] = __fmaf_rn(cy, s.iff, accf[1]);
          accf[2] = __fmaf_rn(cz, s.iff, accf[2]);
        }
        s.ax = bx; s.ay = by; s.az = bz; s.ra = rb; s.ia = ib;
      }
      if (pv) {
        if (!starts) put3(pv + 3 * (int64_t)(i - 1), accp, lane);   // vertex i-1 is complete
        if (ends) {
          put3(pv + 3 * (int64_t)i, accc, lane);
          put3(pl + 3 * (int64_t)loop, accf, lane);
        }
      }
      accp[0] = accc[0]; accp[1] = accc[1]; accp[2] = accc[2];
    }
  }
}

__device__ __forceinline__ void store_gq(const QState* S, const int64_t* qi, const bool* ok, float* gq) {
#pragma unroll
  for (int k = 0; k < kQPL; ++k) {
    if (!ok[k] || !gq) continue;
    const int64_t q = qi[k];
    gq[3 * q + 0] = S[k].gx * kInv4Pi;
    gq[3 * q + 1] = S[k].gy * kInv4Pi;
    gq[3 * q + 2] = S[k].gz * kInv4Pi;
  }
}

}  // namespace adj
}  // namespace wn
