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
// coalesced structure-of-arrays; the workgroup stages the boundary loop into
// LDS (rotated float64 coordinates plus one tie bit per edge) in chunks of
// kChunk vertices and every lane walks the same vertex sequence, so the LDS
// reads are broadcasts.  Per (query, vertex) the frame quantities are formed
// once and reused by the two edges that share the vertex.  Instead of one
// atan2 per edge, the edge factors D + iN are multiplied into a running
// complex product whose half-plane changes count whole turns exactly
// (see wn::Turns); one atan2 per query remains.
#include "kernels.hpp"

namespace wn {

namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 512;   // vertices per LDS stage: 512 * 32 B = 16 KB

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
// the tie bit lex_less(v_i, v_next) of the edge leaving v_i.
__device__ __forceinline__ void stage_chunk(const BndArgs& a, const LoopTable& L, int c0,
                                            int cnt, double4* sv) {
  for (int j = threadIdx.x; j < cnt; j += kThreads) {
    const int i = c0 + j;
    const int l = loop_of(L, i);
    const int nxt = (i + 1 < L.off[l + 1]) ? i + 1 : L.off[l];
    double X, Y, Z, Xn, Yn, Zn;
    rotate(a.F, a.bnd[3 * i], a.bnd[3 * i + 1], a.bnd[3 * i + 2], X, Y, Z);
    rotate(a.F, a.bnd[3 * nxt], a.bnd[3 * nxt + 1], a.bnd[3 * nxt + 2], Xn, Yn, Zn);
    sv[j] = make_double4(X, Y, Z, lex_less(X, Y, Z, Xn, Yn, Zn) ? 1.0 : 0.0);
  }
}

template <int QPL>
__global__ __launch_bounds__(kThreads) void k_bnd3d(BndArgs a, LoopTable L) {
  __shared__ double4 sv[kChunk];

  double Xp[QPL], Yp[QPL], Zp[QPL];
  int64_t qi[QPL];
  bool ok[QPL];
  const int64_t base = (int64_t)blockIdx.x * (kThreads * QPL) + threadIdx.x;
#pragma unroll
  for (int j = 0; j < QPL; ++j) {
    qi[j] = base + (int64_t)j * kThreads;
    ok[j] = qi[j] < a.nq;
    const int64_t q = ok[j] ? qi[j] : 0;
    rotate(a.F, a.qx[q], a.qy[q], a.qz[q], Xp[j], Yp[j], Zp[j]);
  }

  Turns T[QPL];
  VQ first[QPL], prev[QPL];
  int ec = 0;                 // uniform: edges multiplied so far
  int loop = 0;               // uniform: loop of the current vertex
  bool prev_tie = false;      // uniform: tie bit of the edge leaving prev

  for (int c0 = 0; c0 < a.nb; c0 += kChunk) {
    const int cnt = min(kChunk, a.nb - c0);
    __syncthreads();
    stage_chunk(a, L, c0, cnt, sv);
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const int i = c0 + j;
      const double4 v = sv[j];
      while (L.off[loop + 1] <= i) ++loop;           // skip empty loops
      const bool starts = (i == L.off[loop]);
      const bool ends = (i + 1 == L.off[loop + 1]);
      const bool tie_close = v.w != 0.0;
#pragma unroll
      for (int k = 0; k < QPL; ++k) {
        const VQ cur = vertex_q(v.x, v.y, v.z, Xp[k], Yp[k], Zp[k]);
        if (starts) {
          first[k] = cur;
        } else {
          float N = edge_n(prev[k], cur);
          if (N == 0.0f) N = tie_zero(prev_tie);
          const float D = edge_d(prev[k], cur);
          if (ec == 0) turns_init(T[k], D, N); else turns_mul(T[k], D, N);
          if (ec & 1) turns_norm(T[k]);
        }
        if (ends) {
          // closing edge last -> first; its tie bit is stored with `last`
          float N = edge_n(cur, first[k]);
          if (N == 0.0f) N = tie_zero(tie_close);
          const float D = edge_d(cur, first[k]);
          turns_mul(T[k], D, N);
          if ((ec + 1) & 1) turns_norm(T[k]);
        }
        prev[k] = cur;
      }
      ec += (starts ? 0 : 1) + (ends ? 1 : 0);
      prev_tie = tie_close;
    }
  }
  const bool have_edge = ec > 0;

#pragma unroll
  for (int k = 0; k < QPL; ++k) {
    if (!ok[k]) continue;
    const int64_t q = qi[k];
    const int chi = a.chi_in[q];
    float w;
    if (chi == WN_CHI_INVALID || !(isfinite(a.qx[q]) && isfinite(a.qy[q]) && isfinite(a.qz[q]))) {
      w = __int_as_float(0x7fc00000);
    } else {
      w = have_edge ? turns_to_w(T[k], chi) : (float)chi;
    }
    a.w_out[q] = w;
  }
}

}  // namespace

hipError_t launch_bnd3d(const BndArgs& a, const LoopTable& L, hipStream_t s) {
  constexpr int QPL = 2;
  const int64_t per = (int64_t)kThreads * QPL;
  const int64_t blocks = (a.nq + per - 1) / per;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bnd3d<QPL>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a, L);
  return hipGetLastError();
}

}  // namespace wn
