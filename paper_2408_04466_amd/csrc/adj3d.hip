// Adjoint of the 3D winding number with respect to the query points and the
// boundary vertices, for a loss L with dL/dw = g per query.
//
// chi_d is piecewise constant, so w varies only through the boundary line
// integral, whose derivatives are independent of d.  For an edge a->b with
// a' = a - p, b' = b - p:  K = 1/(|a'||b'| + a'.b'),  c = (a' x b') K,
//   dw/dp += c (1/|a'| + 1/|b'|) / 4pi          (Biot-Savart field of dM)
//   dw/da += -c / (|a'| 4pi),  dw/db += -c / (|b'| 4pi)
// (the same field integrated against each vertex's hat function along the
// straight edge).  These vanish in sum: sum_v dw/dv + dw/dp = 0.
//
// Layout: one lane holds kQPL queries; the workgroup stages the boundary in
// LDS and every lane walks the same vertex sequence.  A vertex's gradient is
// complete one step after the vertex is visited (its two edges are then
// done); it is summed over the lane's queries in registers, over the
// wavefront with cross-lane adds, and written once per (workgroup,
// wavefront, vertex) as a float32 partial.  The closing edge's share of each
// loop's first vertex goes to a separate per-loop partial.  Two more kernels
// add all partials in a fixed order in float64 (groups of rows, then the
// groups), so grad_bnd is bitwise reproducible (no floating-point atomics).
#include "kernels.hpp"

namespace wn {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kQPL = 4;
constexpr int kChunk = 512;
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

__global__ __launch_bounds__(kThreads) void k_adj3d(AdjArgs a, LoopTable L) {
  __shared__ float4 sv[kChunk];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t bw = (int64_t)blockIdx.x * kWaves + wave;     // partial row
  float* pv = a.partial ? a.partial + bw * (int64_t)a.nb * 3 : nullptr;
  float* pl = a.partial_loop ? a.partial_loop + bw * (int64_t)L.n * 3 : nullptr;

  QState S[kQPL];
  int64_t qi[kQPL];
  bool ok[kQPL];
  const int64_t base = (int64_t)blockIdx.x * (kThreads * kQPL) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kQPL; ++k) {
    qi[k] = base + (int64_t)k * kThreads;
    ok[k] = qi[k] < a.nq;
    const int64_t q = ok[k] ? qi[k] : 0;
    S[k].px = a.qx[q];
    S[k].py = a.qy[q];
    S[k].pz = a.qz[q];
    S[k].g = ok[k] ? a.gw[q] : 0.0f;      // padding lanes contribute nothing
    S[k].gx = S[k].gy = S[k].gz = 0.0f;
  }

  float accp[3] = {0.f, 0.f, 0.f};   // previous vertex, summed over the lane's queries
  int loop = 0;

  for (int c0 = 0; c0 < a.nb; c0 += kChunk) {
    const int cnt = min(kChunk, a.nb - c0);
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kThreads) {
      const int i = c0 + j;
      sv[j] = make_float4(a.bnd[3 * i], a.bnd[3 * i + 1], a.bnd[3 * i + 2], 0.f);
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const int i = c0 + j;
      const float4 v = sv[j];
      while (L.off[loop + 1] <= i) ++loop;
      const bool starts = (i == L.off[loop]);
      const bool ends = (i + 1 == L.off[loop + 1]);
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

#pragma unroll
  for (int k = 0; k < kQPL; ++k) {
    if (!ok[k] || !a.gq) continue;
    const int64_t q = qi[k];
    a.gq[3 * q + 0] = S[k].gx * kInv4Pi;
    a.gq[3 * q + 1] = S[k].gy * kInv4Pi;
    a.gq[3 * q + 2] = S[k].gz * kInv4Pi;
  }
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
  for (int64_t r = r0; r < r1; ++r) {
    s += (double)pv[r * n + t];
    if (lf >= 0) s += (double)pl[(r * L.n + lf) * 3 + c];
  }
  tmp[(int64_t)blockIdx.y * n + t] = s;
}

// Stage 2: out = -(1/4pi) * sum over groups, in group order.
__global__ void k_reduce_groups(const double* __restrict__ tmp, int64_t groups, int64_t n,
                                float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double s = 0.0;
  for (int64_t g = 0; g < groups; ++g) s += tmp[g * n + t];
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
