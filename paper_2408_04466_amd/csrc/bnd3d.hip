// Boundary line integral of the one-shot winding number (3D) and the final
// combine w = chi_d + S/(2 pi).
//
// S(p) = sum over boundary edges a->b of theta_e, theta_e = atan2(N, D): half
// the signed solid angle of the spherical triangle (-d, a - p, b - p).  This
// is Eq. wn_discrete_sum with the region of d as the seed of Alg. 1: by
// Lemma 2 every other region differs from it by the number of boundary
// crossings in between, so the region areas collapse into one line integral
// over the boundary (the paper evaluates region areas from boundary
// integrals as well, Sec. 4 "Exact Computations").
//
// Layout: one lane per query (QPL queries per lane), queries read as
// coalesced structure-of-arrays; the workgroup stages the boundary loops into
// LDS (rotated float64 coordinates plus the tie offset of the edge leaving
// each vertex) in chunks of kChunk vertices, and every lane walks the same
// vertex sequence, so the LDS reads are broadcasts.  Per (query, vertex) the
// frame quantities are formed once and reused by the two edges that share
// the vertex.  Instead of one atan2 per edge, the edge factors D + iN are
// multiplied into a running complex product whose half-plane changes count
// whole turns exactly (wn::Turns); one atan2 per query remains.
#include <cstdlib>

#include "kernels.hpp"

namespace wn {

namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 512;      // vertices per LDS stage: 512 * 32 B = 16 KB
constexpr int kUnroll = 8;       // vertices per main-loop step (one rescale per step)

// Loop containing flat vertex index i (binary search over the loop table).
__device__ __forceinline__ int loop_of(const LoopTable& L, int i) {
  int lo = 0, hi = L.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (L.off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Stage vertices [c0, c0 + cnt) into LDS: rotated coordinates and, in .w,
// the tie offset of the edge v_i -> v_next(i).
__device__ __forceinline__ void stage_chunk(const BndArgs& a, const LoopTable& L, int c0,
                                            int cnt, double4* sv) {
  for (int j = threadIdx.x; j < cnt; j += kThreads) {
    const int i = c0 + j;
    const int l = loop_of(L, i);
    const int nxt = (i + 1 < L.off[l + 1]) ? i + 1 : L.off[l];
    double X, Y, Z, Xn, Yn, Zn;
    rotate(a.F, a.bnd[3 * i], a.bnd[3 * i + 1], a.bnd[3 * i + 2], X, Y, Z);
    rotate(a.F, a.bnd[3 * nxt], a.bnd[3 * nxt + 1], a.bnd[3 * nxt + 2], Xn, Yn, Zn);
    sv[j] = make_double4(X, Y, Z, tie_offset(lex_less(X, Y, Z, Xn, Yn, Zn)));
  }
}

template <int QPL>
struct Lane {
  double Xp[QPL], Yp[QPL], Zp[QPL];
  Turns T[QPL];
};

template <int QPL>
__device__ __forceinline__ void vert_q(const Lane<QPL>& s, const double4& v, VQ* out) {
#pragma unroll
  for (int k = 0; k < QPL; ++k) out[k] = vertex_q(v.x, v.y, v.z, s.Xp[k], s.Yp[k], s.Zp[k]);
}

template <int QPL>
__device__ __forceinline__ void edge_step(Lane<QPL>& s, const VQ* a, const VQ* b, double tie) {
#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    const double N = edge_tie(edge_n(a[k], b[k]), tie);
    const double D = edge_d(a[k], b[k]);
    turns_mul(s.T[k], D, N);
  }
}

template <int QPL>
__device__ __forceinline__ void rescale(Lane<QPL>& s) {
#pragma unroll
  for (int k = 0; k < QPL; ++k) turns_norm(s.T[k]);
}

template <int QPL>
__global__ __launch_bounds__(kThreads) void k_bnd3d(BndArgs a, LoopTable L) {
  __shared__ double4 sv[kChunk];

  Lane<QPL> s;
  int64_t qi[QPL];
  bool ok[QPL];
  const int64_t base = (int64_t)blockIdx.x * (kThreads * QPL) + threadIdx.x;
#pragma unroll
  for (int j = 0; j < QPL; ++j) {
    qi[j] = base + (int64_t)j * kThreads;
    ok[j] = qi[j] < a.nq;
    const int64_t q = ok[j] ? qi[j] : 0;
    rotate(a.F, a.qx[q], a.qy[q], a.qz[q], s.Xp[j], s.Yp[j], s.Zp[j]);
    turns_init(s.T[j]);
  }

  VQ first[QPL], A[QPL], B[QPL];   // A holds the previous vertex between steps
  double ptie = 0.0;               // uniform: tie offset of the edge leaving A
  int l = 0;
  for (int c0 = 0; c0 < a.nb; c0 += kChunk) {
    const int c1 = min(c0 + kChunk, a.nb);
    __syncthreads();
    stage_chunk(a, L, c0, c1 - c0, sv);
    __syncthreads();
    // the loops overlapping [c0, c1), each as a straight-line vertex range
    for (; l < L.n && L.off[l] < c1; ++l) {
      const int ls = L.off[l], le = L.off[l + 1];
      int j = max(ls, c0);
      const int j1 = min(le, c1);
      if (j == ls) {
        const double4 v = sv[j - c0];
        vert_q(s, v, first);
#pragma unroll
        for (int k = 0; k < QPL; ++k) A[k] = first[k];
        ptie = v.w;
        ++j;
      }
      // kUnroll vertices per step, the roles of A and B alternating
      for (; j + kUnroll <= j1; j += kUnroll) {
#pragma unroll
        for (int u = 0; u < kUnroll; u += 2) {
          const double4 v0 = sv[j + u - c0];
          vert_q(s, v0, B);
          edge_step(s, A, B, ptie);
          const double4 v1 = sv[j + u + 1 - c0];
          vert_q(s, v1, A);
          edge_step(s, B, A, v0.w);
          ptie = v1.w;
        }
        rescale(s);
      }
      for (; j < j1; ++j) {
        const double4 v = sv[j - c0];
        vert_q(s, v, B);
        edge_step(s, A, B, ptie);
#pragma unroll
        for (int k = 0; k < QPL; ++k) A[k] = B[k];
        ptie = v.w;
      }
      rescale(s);
      if (j1 < le) break;            // the loop continues in the next chunk
      edge_step(s, A, first, ptie);  // closing edge last -> first
    }
  }

#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    if (!ok[k]) continue;
    const int64_t q = qi[k];
    const int chi = a.chi_in[q];
    float w;
    if (chi == WN_CHI_INVALID || !(isfinite(a.qx[q]) && isfinite(a.qy[q]) && isfinite(a.qz[q]))) {
      w = __int_as_float(0x7fc00000);
    } else {
      w = turns_to_w(s.T[k], chi);
    }
    a.w_out[q] = w;
  }
}

}  // namespace

// Queries per lane: 1 or 2 (1 by default: 2 doubles the registers and
// halves occupancy for no gain at the issue limit; WN_BND_QPL overrides).
static int bnd_qpl() {
  static int q = [] {
    const char* e = getenv("WN_BND_QPL");
    const int v = e ? atoi(e) : 1;
    return (v == 2) ? 2 : 1;
  }();
  return q;
}

hipError_t launch_bnd3d(const BndArgs& a, const LoopTable& L, hipStream_t s) {
  const int qpl = bnd_qpl();
  const int64_t per = (int64_t)kThreads * qpl;
  const int64_t blocks = (a.nq + per - 1) / per;
  if (blocks == 0) return hipSuccess;
  if (qpl == 1)
    hipLaunchKernelGGL(k_bnd3d<1>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a, L);
  else
    hipLaunchKernelGGL(k_bnd3d<2>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a, L);
  return hipGetLastError();
}

}  // namespace wn
