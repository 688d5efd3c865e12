// Kernels of the curve boundary term: the forward evaluation (chi_d from the
// caller or the BVH, plus the panel walk of curves.hpp) and its adjoint.
#include "curves.hpp"

namespace wn {

namespace {

__global__ __launch_bounds__(kCThreads) void k_curves3d(CrossArgs ca, Frame F, const float* __restrict__ ctrl,
                                                       int32_t nc, const float* __restrict__ qx,
                                                       const float* __restrict__ qy, const float* __restrict__ qz,
                                                       int64_t nq, const int32_t* __restrict__ chi_in,
                                                       float* __restrict__ w_out, int32_t* __restrict__ chi_out) {
  __shared__ CurveRot sc[kCurveChunk];
  const int64_t qi = (int64_t)blockIdx.x * kCThreads + threadIdx.x;
  const bool ok = qi < nq;
  const int64_t q = ok ? qi : 0;
  const float px = qx[q], py = qy[q], pz = qz[q];
  const bool fin = isfinite(px) && isfinite(py) && isfinite(pz);
  double Xp, Yp, Zp;
  rotate(F, px, py, pz, Xp, Yp, Zp);
  int chi;
  if (chi_in) chi = chi_in[q];
  else chi = (ok && fin) ? traverse<kShortStack>(ca, make_qp(Xp, Yp, Zp)) : WN_CHI_INVALID;
  double theta = 0.0;
  for (int c0 = 0; c0 < nc; c0 += kCurveChunk) {
    const int cnt = min(kCurveChunk, nc - c0);
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kCThreads) stage_curve(F, ctrl, c0 + j, &sc[j]);
    __syncthreads();
    if (ok && fin) theta += curves_theta(sc, cnt, Xp, Yp, Zp);
  }
  if (ok) {
    const bool valid = fin && chi != WN_CHI_INVALID;
    w_out[qi] = valid ? __fadd_rn((float)chi, __fmul_rn((float)theta, kInv2Pi)) : __int_as_float(0x7fc00000);
    if (chi_out) chi_out[qi] = fin ? chi : WN_CHI_INVALID;
  }
}

// ---------------------------------------------------------------------------
// Adjoint.  Away from the surface chi_d is locally constant, so dw/dp and
// dw/dc_k come from the boundary term alone and do not depend on d:
//   dw/dp   = +(1/4pi) int (gamma - p) x gamma' / |gamma - p|^3 dt,
//   dw/dc_k = -(1/4pi) int B_k(t) (gamma - p) x gamma' / |gamma - p|^3 dt
// (the Biot-Savart field of the curves, and that field weighted by each
// control point's Bernstein function).  The integrand is smooth away from
// the curves, so the panels need only the distance test; they are integrated
// by the same 6-node rule in world coordinates.
// ---------------------------------------------------------------------------

// G = int f, Gk[k] = int B_k f for one staged curve and one query.
__device__ void curve_bs(const CurveRot& C, double px, double py, double pz, float (&G)[3], float (&Gk)[4][3]) {
  const double A0[3] = {C.c0[0] - px, C.c0[1] - py, C.c0[2] - pz};
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    G[m] = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) Gk[k][m] = 0.f;
  }
  int depth = 0;
  uint32_t idx = 0;
  for (;;) {
    const double h = __builtin_ldexp(1.0, -depth);
    const double t0 = (double)idx * h;
    F3 b[4], c[4];
    float bb[4][3], ee[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double a1 = C.a1[k], a2 = C.a2[k], a3 = C.a3[k];
      const double B0 = __fma_rn(t0, __fma_rn(t0, __fma_rn(t0, a3, a2), a1), A0[k]);
      const double B1 = h * __fma_rn(t0, __fma_rn(3.0 * t0, a3, 2.0 * a2), a1);
      const double B2 = (h * h) * __fma_rn(3.0 * t0, a3, a2);
      const double B3 = (h * h * h) * a3;
      bb[0][k] = (float)B0;
      bb[1][k] = (float)B1;
      bb[2][k] = (float)B2;
      bb[3][k] = (float)B3;
      ee[k] = (float)(B0 + B1 + B2 + B3);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) b[i] = {bb[i][0], bb[i][1], bb[i][2]};
    c[0] = b[0];
    c[1] = {b[0].x + b[1].x * (1.f / 3.f), b[0].y + b[1].y * (1.f / 3.f), b[0].z + b[1].z * (1.f / 3.f)};
    c[2] = {b[0].x + (2.f * b[1].x + b[2].x) * (1.f / 3.f), b[0].y + (2.f * b[1].y + b[2].y) * (1.f / 3.f),
            b[0].z + (2.f * b[1].z + b[2].z) * (1.f / 3.f)};
    c[3] = {ee[0], ee[1], ee[2]};
    const float len = norm3(sub3(c[1], c[0])) + norm3(sub3(c[2], c[1])) + norm3(sub3(c[3], c[2]));
    const float m2 = fminf(fminf(sq3(c[0]), sq3(c[1])), fminf(sq3(c[2]), sq3(c[3])));
    const float fl = kFar * len;
    if (m2 > fl * fl || depth >= kMaxDepth) {
      const F3 d2 = {2.f * b[2].x, 2.f * b[2].y, 2.f * b[2].z};
      const F3 d3 = {3.f * b[3].x, 3.f * b[3].y, 3.f * b[3].z};
#pragma unroll
      for (int k = 0; k < kGL; ++k) {
        const float s = kGLs[k];
        const float X = __fmaf_rn(s, __fmaf_rn(s, __fmaf_rn(s, b[3].x, b[2].x), b[1].x), b[0].x);
        const float Y = __fmaf_rn(s, __fmaf_rn(s, __fmaf_rn(s, b[3].y, b[2].y), b[1].y), b[0].y);
        const float Z = __fmaf_rn(s, __fmaf_rn(s, __fmaf_rn(s, b[3].z, b[2].z), b[1].z), b[0].z);
        const float dX = __fmaf_rn(s, __fmaf_rn(s, d3.x, d2.x), b[1].x);
        const float dY = __fmaf_rn(s, __fmaf_rn(s, d3.y, d2.y), b[1].y);
        const float dZ = __fmaf_rn(s, __fmaf_rn(s, d3.z, d2.z), b[1].z);
        const float ir = __builtin_amdgcn_rsqf(__fmaf_rn(X, X, __fmaf_rn(Y, Y, __fmul_rn(Z, Z))));
        const float wk = __fmul_rn(kGLw[k], __fmul_rn(ir, __fmul_rn(ir, ir)));
        const float f0 = __fmul_rn(wk, __fmaf_rn(Y, dZ, -__fmul_rn(Z, dY)));
        const float f1 = __fmul_rn(wk, __fmaf_rn(Z, dX, -__fmul_rn(X, dZ)));
        const float f2 = __fmul_rn(wk, __fmaf_rn(X, dY, -__fmul_rn(Y, dX)));
        G[0] += f0;
        G[1] += f1;
        G[2] += f2;
        const float t = (float)(t0 + h * (double)s), t1 = 1.f - t;
        const float bt[4] = {t1 * t1 * t1, 3.f * t * t1 * t1, 3.f * t * t * t1, t * t * t};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          Gk[j][0] = __fmaf_rn(bt[j], f0, Gk[j][0]);
          Gk[j][1] = __fmaf_rn(bt[j], f1, Gk[j][1]);
          Gk[j][2] = __fmaf_rn(bt[j], f2, Gk[j][2]);
        }
      }
    } else {
      ++depth;
      idx <<= 1;
      continue;
    }
    while (depth > 0 && (idx & 1u)) {
      idx >>= 1;
      --depth;
    }
    if (depth == 0) break;
    ++idx;
  }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// One query per lane.  grad_q = g/(4pi) sum_curves G; per (workgroup,
// curve) the 12 sums over the workgroup's queries of g Gk go to `part`
// (wavefront butterfly sums, then the four wavefronts in order).
__global__ __launch_bounds__(kCThreads) void k_curves_adj(const float* __restrict__ ctrl, int32_t nc,
                                                         const float* __restrict__ qx, const float* __restrict__ qy,
                                                         const float* __restrict__ qz, int64_t nq,
                                                         const float* __restrict__ gw, float* __restrict__ gq,
                                                         float* __restrict__ part) {
  __shared__ CurveRot sc[kCurveChunk];
  __shared__ float red[kCThreads / 64][12];
  Frame Fid;
#pragma unroll
  for (int k = 0; k < 9; ++k) Fid.r[k] = (k % 4 == 0) ? 1.0 : 0.0;
  Fid.c[0] = Fid.c[1] = Fid.c[2] = 0.0;
  const int64_t qi = (int64_t)blockIdx.x * kCThreads + threadIdx.x;
  const bool ok = qi < nq;
  const int64_t q = ok ? qi : 0;
  const float px = qx[q], py = qy[q], pz = qz[q];
  const bool fin = ok && isfinite(px) && isfinite(py) && isfinite(pz);
  const float g = fin ? gw[q] : 0.f;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float gx = 0.f, gy = 0.f, gz = 0.f;
  for (int c0 = 0; c0 < nc; c0 += kCurveChunk) {
    const int cnt = min(kCurveChunk, nc - c0);
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kCThreads) stage_curve(Fid, ctrl, c0 + j, &sc[j]);
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      float G[3], Gk[4][3];
      if (fin) {
        curve_bs(sc[j], (double)px, (double)py, (double)pz, G, Gk);
      } else {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          G[m] = 0.f;
#pragma unroll
          for (int k = 0; k < 4; ++k) Gk[k][m] = 0.f;
        }
      }
      gx += G[0];
      gy += G[1];
      gz += G[2];
      if (part) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int m = 0; m < 3; ++m) {
            const float v = wave_sum(g * Gk[k][m]);
            if (lane == 0) red[wv][3 * k + m] = v;
          }
        __syncthreads();
        if (threadIdx.x < 12) {
          float v = red[0][threadIdx.x];
#pragma unroll
          for (int w = 1; w < kCThreads / 64; ++w) v += red[w][threadIdx.x];
          part[((int64_t)blockIdx.x * nc + c0 + j) * 12 + threadIdx.x] = v;
        }
        __syncthreads();
      }
    }
  }
  if (ok && gq) {
    const float k4 = 0.07957747154594767f * g;   // g / 4pi
    gq[3 * qi + 0] = fin ? k4 * gx : __int_as_float(0x7fc00000);
    gq[3 * qi + 1] = fin ? k4 * gy : __int_as_float(0x7fc00000);
    gq[3 * qi + 2] = fin ? k4 * gz : __int_as_float(0x7fc00000);
  }
}

// One workgroup per (curve, control point, component): fixed-order float64
// sum over the query workgroups' partials, times -1/4pi.
__global__ __launch_bounds__(kCThreads) void k_curves_adj_sum(const float* __restrict__ part, int64_t nblocks,
                                                             int32_t nc, float* __restrict__ gc) {
  __shared__ double red[kCThreads];
  const int o = blockIdx.x;   // curve * 12 + (3 k + m)
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < nblocks; b += kCThreads) acc += (double)part[b * nc * 12 + o];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kCThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) gc[o] = (float)(-red[0] * 0.07957747154594767);
}

}  // namespace

hipError_t backward_curves(const float* ctrl, int64_t nc, const float* qx, const float* qy, const float* qz,
                           int64_t nq, const float* gw, float* gq, float* gc, hipStream_t s) {
  const int64_t blocks = (nq + kCThreads - 1) / kCThreads;
  if (blocks == 0 || nc == 0) {
    // no queries: the control-point gradient is zero; no curves: so is dw/dp
    if (gc && nc > 0) {
      const hipError_t e = fill_u32((unsigned*)gc, nc * 12, 0u, s);
      if (e != hipSuccess) return e;
    }
    if (gq && nq > 0) {
      hipLaunchKernelGGL(k_curves_adj, dim3((unsigned)blocks), dim3(kCThreads), 0, s, ctrl, 0, qx, qy, qz, nq, gw,
                         gq, nullptr);
      return hipGetLastError();
    }
    return hipSuccess;
  }
  float* part = nullptr;
  hipError_t e = hipSuccess;
  if (gc) {
    e = hipMallocAsync((void**)&part, (size_t)blocks * nc * 12 * sizeof(float), s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_curves_adj, dim3((unsigned)blocks), dim3(kCThreads), 0, s, ctrl, (int32_t)nc, qx, qy, qz, nq,
                     gw, gq, part);
  e = hipGetLastError();
  if (e == hipSuccess && gc) {
    hipLaunchKernelGGL(k_curves_adj_sum, dim3((unsigned)(nc * 12)), dim3(kCThreads), 0, s, part, blocks, (int32_t)nc,
                       gc);
    e = hipGetLastError();
  }
  if (part) {
    const hipError_t e2 = hipFreeAsync(part, s);
    if (e == hipSuccess) e = e2;
  }
  return e;
}

hipError_t launch_curves3d(const CrossArgs& c, const float* ctrl, int64_t nc, const int32_t* chi_in, float* w_out,
                           int32_t* chi_out, hipStream_t s) {
  const int64_t blocks = (c.nq + kCThreads - 1) / kCThreads;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_curves3d, dim3((unsigned)blocks), dim3(kCThreads), 0, s, c, c.F, ctrl, (int32_t)nc, c.qx,
                     c.qy, c.qz, c.nq, chi_in, w_out, chi_out);
  return hipGetLastError();
}

}  // namespace wn
