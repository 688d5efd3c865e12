// Winding numbers of loops of cubic Bezier curves (2D), ray direction +x.
//
// Sec. 3 defines w_C(p) = (1/2pi) int_C dtheta(p).  With one ray direction
// d = +x for every query (the seed region of Alg. 1 is the one containing
// d), w = chi(p) + (1/2pi) sum over open loops [phi(end - p) - phi(start - p)]
// where chi is the signed number of crossings of the ray p + t (1, 0), t > 0,
// with the curves (Eq. chi) and phi measures the angle of a vector
// counter-clockwise from +x in [0, 2pi).  A point on the ray's line counts as
// lying above it (y >= p_y), on the same side that phi in [0, 2pi) puts it.
//
// Steps:
//  * k_pieces: split every cubic at the roots of y'(t) into at most three
//    y-monotone pieces (the subdivision the paper performs per ray).
//  * points mode: one lane per query walks the pieces (staged in LDS): a
//    piece is crossed iff its end ordinates lie on different sides; the
//    crossing counts if it lies right of p, decided by the piece's x bounds
//    or, when p_x falls inside them, by solving y(t) = p_y on the piece
//    (safeguarded Newton) and comparing x(t*).
//  * grid mode: the paper's one-shot reuse (Sec. 5 "Optimization"; Sec. 7,
//    2D results): one workgroup per (row, column tile) solves each piece that
//    crosses the row once, bins the crossing by the number of grid columns
//    left of it (an LDS histogram of integer counts), and a suffix scan gives
//    chi for every column of the row.
// Both modes decide "crossing right of p" as p_x < clamp(x*, xmin, xmax) with
// the same solver, so they agree bit for bit.
#include <algorithm>
#include <cmath>
#include <vector>

#include "geom.hpp"
#include "kernels.hpp"

namespace wn {

namespace {

template <class T>
struct Piece {
  T cx[4];        // x(t) = ((cx3 t + cx2) t + cx1) t + cx0   (segment power basis)
  T cy[4];        // y(t) likewise
  T t0, t1;       // parameter range of the monotone piece
  T y0, y1;       // y(t0), y(t1) (exact control values at segment ends)
  T xmin, xmax;   // x bounds of the segment's control polygon
};

struct Loops2D {
  int32_t n;
  int32_t off[WN_MAX_LOOPS + 1];
  uint8_t closed[WN_MAX_LOOPS];
};

template <class T> __device__ __forceinline__ T fma_t(T a, T b, T c);
template <> __device__ __forceinline__ float fma_t<float>(float a, float b, float c) { return __fmaf_rn(a, b, c); }
template <> __device__ __forceinline__ double fma_t<double>(double a, double b, double c) { return __fma_rn(a, b, c); }

template <class T>
__device__ __forceinline__ T horner(const T c[4], T t) {
  return fma_t(fma_t(fma_t(c[3], t, c[2]), t, c[1]), t, c[0]);
}
template <class T>
__device__ __forceinline__ T horner_d(const T c[4], T t) {
  return fma_t(fma_t((T)3 * c[3], t, (T)2 * c[2]), t, c[1]);
}

template <class T>
__device__ __forceinline__ void power_basis(T p0, T p1, T p2, T p3, T c[4]) {
  c[0] = p0;
  c[1] = (T)3 * (p1 - p0);
  c[2] = (T)3 * (p0 - (T)2 * p1 + p2);
  c[3] = (p3 - p0) + (T)3 * (p1 - p2);
}

template <class T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

// Split segment s into three pieces (empty pieces have t0 == t1, y0 == y1);
// yr gets the end ordinates of every piece for the straddle tests.
template <class T>
__device__ void split_segment(const T* __restrict__ P, Piece<T>* __restrict__ out,
                              typename Vec2<T>::type* __restrict__ yr) {
  T cx[4], cy[4];
  power_basis(P[0], P[2], P[4], P[6], cx);
  power_basis(P[1], P[3], P[5], P[7], cy);
  // roots of y'(t) = 3 c3 t^2 + 2 c2 t + c1 in (0, 1)
  const T a = (T)3 * cy[3], b = (T)2 * cy[2], c = cy[1];
  T r[2];
  int nr = 0;
  if (a != (T)0) {
    const T disc = b * b - (T)4 * a * c;
    if (disc > (T)0) {
      const T sq = sqrt(disc);
      // numerically stable pair
      const T q = (b >= (T)0) ? -(T)0.5 * (b + sq) : -(T)0.5 * (b - sq);
      T u = q / a, v = (q != (T)0) ? c / q : u;
      if (u > v) { const T w = u; u = v; v = w; }
      if (u > (T)0 && u < (T)1) r[nr++] = u;
      if (v > (T)0 && v < (T)1 && v != u) r[nr++] = v;
    }
  } else if (b != (T)0) {
    const T u = -c / b;
    if (u > (T)0 && u < (T)1) r[nr++] = u;
  }
  T ts[4];
  T ys[4];
  int m = 0;
  ts[m] = (T)0; ys[m++] = P[1];
  for (int k = 0; k < nr; ++k) { ts[m] = r[k]; ys[m++] = horner(cy, r[k]); }
  ts[m] = (T)1; ys[m++] = P[7];
  const T xmin = fmin(fmin(P[0], P[2]), fmin(P[4], P[6]));
  const T xmax = fmax(fmax(P[0], P[2]), fmax(P[4], P[6]));
  for (int k = 0; k < 3; ++k) {
    Piece<T> pc;
    for (int i = 0; i < 4; ++i) { pc.cx[i] = cx[i]; pc.cy[i] = cy[i]; }
    if (k + 1 < m) {
      pc.t0 = ts[k]; pc.t1 = ts[k + 1]; pc.y0 = ys[k]; pc.y1 = ys[k + 1];
    } else {
      pc.t0 = pc.t1 = (T)1; pc.y0 = pc.y1 = P[7];
    }
    pc.xmin = xmin;
    pc.xmax = xmax;
    out[k] = pc;
    yr[k] = {pc.y0, pc.y1};
  }
}

template <class T>
__global__ void k_pieces(const T* __restrict__ ctrl, int32_t nseg, Piece<T>* __restrict__ out,
                         typename Vec2<T>::type* __restrict__ yr) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  split_segment(ctrl + 8 * (int64_t)s, out + 3 * (int64_t)s, yr + 3 * (int64_t)s);
}

// x(t*) for the t* in [t0, t1] with y(t*) = yq on a monotone piece whose end
// ordinates straddle yq (y >= yq counts as above).  Safeguarded Newton: the
// bracket [lo, hi] keeps lo below and hi above; a Newton step that leaves it
// is replaced by bisection.
template <class T>
__device__ T solve_x(const Piece<T>& pc, T yq) {
  const bool up = pc.y1 >= yq;      // piece goes from below (at t0) to above (at t1)
  T lo = up ? pc.t0 : pc.t1;        // parameter where y is below yq
  T hi = up ? pc.t1 : pc.t0;        // parameter where y is above (or on) yq
  // regula falsi start between the end ordinates
  T t = pc.t0 + (pc.t1 - pc.t0) * ((yq - pc.y0) / (pc.y1 - pc.y0));
  if (!(t >= fmin(lo, hi) && t <= fmax(lo, hi))) t = (T)0.5 * (lo + hi);
  const int maxit = sizeof(T) == 4 ? 40 : 80;
  for (int it = 0; it < maxit; ++it) {
    const T f = horner(pc.cy, t) - yq;
    if (f >= (T)0) hi = t; else lo = t;
    const T fp = horner_d(pc.cy, t);
    // the step needs no correctly rounded quotient (the bracket guards it):
    // in float32 one reciprocal instead of a full division
    const T q = sizeof(T) == 4 ? (T)(f * __builtin_amdgcn_rcpf((float)fp)) : f / fp;
    T tn = (fp != (T)0) ? t - q : (T)0.5 * (lo + hi);
    const T a = fmin(lo, hi), b = fmax(lo, hi);
    const T tol = (T)4 * (sizeof(T) == 4 ? (T)1.2e-7 : (T)2.3e-16) * fmax((T)1, fabs(b));
    // converged: a step below the tolerance (also one that lands on the
    // bracket's end, as it does once f rounds to zero or changes sign
    // between neighbouring parameters; bisecting then would walk away from
    // the root)
    if (fabs(tn - t) <= tol) {
      if (tn >= a && tn <= b) t = tn;
      break;
    }
    if (!(tn > a && tn < b)) tn = (T)0.5 * (lo + hi);
    if (b - a <= tol) {
      t = tn;
      break;
    }
    t = tn;
  }
  return horner(pc.cx, t);
}

// The crossing of piece pc with the row yq lies right of px.
template <class T>
__device__ __forceinline__ bool right_of(const Piece<T>& pc, T yq, T px) {
  if (px < pc.xmin) return true;
  if (px >= pc.xmax) return false;
  return solve_x(pc, yq) > px;
}

// atan2(y, x) in float64, with the octant reduction of atan2_f32 (one
// division: t = a/b, or (a - b)/(a + b) with pi/4 added back, |t| <= tan(pi/8))
// and atan(t) = t P(t^2), P of degree 10 fitted in this project to atan(t)/t on
// [0, tan(pi/8)^2] (Chebyshev fit in 40-digit arithmetic, 3.5e-17 relative;
// about one ulp once evaluated in float64).  The sign of the result is the
// sign bit of y and a negative zero x counts as negative, as for atan2.
__device__ __forceinline__ double atan2_f64(double y, double x) {
  constexpr double kP[11] = {
    1.0,
    -0.3333333333332844,
    0.1999999999885511,
    -0.14285714180976467,
    0.11111106180455946,
    -0.09090773074808414,
    0.07689953496306857,
    -0.06640233930429408,
    0.056883492268090106,
    -0.04348052215716462,
    0.021135373157693246};
  const double ax = fabs(x), ay = fabs(y);
  const double a = fmin(ax, ay), b = fmax(ax, ay);
  const bool big = a > 0.41421356237309503 * b;
  const double num = big ? a - b : a;
  const double den = big ? a + b : b;
  const double t = den > 0.0 ? num / den : 0.0;
  const double s = t * t;
  double p = kP[10];
#pragma unroll
  for (int k = 9; k >= 0; --k) p = __fma_rn(p, s, kP[k]);
  double r = t * p;
  if (big) r += 0.78539816339744831;
  if (ay > ax) r = 1.5707963267948966 - r;
  if (signbit(x)) r = 3.1415926535897931 - r;   // x = -0 too, as atan2
  return copysign(r, y);
}

template <class T> __device__ __forceinline__ T atan2_t(T y, T x);
template <> __device__ __forceinline__ float atan2_t<float>(float y, float x) { return atan2_f32(y, x); }
template <> __device__ __forceinline__ double atan2_t<double>(double y, double x) { return atan2_f64(y, x); }

// phi(e) - phi(s) for the vectors s, e from p to an open loop's start and
// end, with one atan2: the signed angle theta from s to e lies in (-pi, pi],
// and phi (in [0, 2pi), cut along +x) differs from it by 2 pi exactly when
// the chord s -> e crosses the ray p + t(1, 0), t > 0: upward (s below,
// e on or above the ray's line) gives phi(e) - phi(s) = theta - 2 pi,
// downward theta + 2 pi.  The crossing lies right of p iff s x e has the
// direction's sign, the same sign theta takes, so the two decisions cannot
// disagree through rounding.  p on the chord between s and e (s x e = 0,
// s . e < 0) gives -pi when e is in [0, pi) (above, or on the +x side of
// the line), +pi otherwise.
// Written with selects only, so that several queries' evaluations can be
// interleaved without branches.
template <class T>
__device__ __forceinline__ T open_loop_angle(T sx, T sy, T ex, T ey) {
  const T cr = fma_t(sx, ey, -(sy * ex));
  const T dt = fma_t(sx, ex, sy * ey);
  const T th = atan2_t(cr, dt);
  const bool s_above = sy >= (T)0, e_above = ey >= (T)0;
  T r = (!s_above && e_above && cr > (T)0) ? th - (T)6.283185307179586 : th;
  r = (s_above && !e_above && cr < (T)0) ? th + (T)6.283185307179586 : r;
  const bool e_upper = ey > (T)0 || (ey == (T)0 && ex > (T)0);
  const T on_chord = e_upper ? -(T)3.141592653589793 : (T)3.141592653589793;
  return (cr == (T)0 && dt < (T)0) ? on_chord : r;
}

// Loop table in device memory (batched calls): same members as Loops2D.
struct DevLoops2D {
  int32_t n;
  const int32_t* off;
  const uint8_t* closed;
};

// w from the crossing count and the end-point angle sum (every kernel
// finishes with this one expression, so their results agree bit for bit).
template <class T>
__device__ __forceinline__ T finish_w(int c, T e) {
  return (T)c + e * (T)0.15915494309189535;
}

// sum over open loops of phi(end - p) - phi(start - p)
template <class T, class LoopsT>
__device__ T endpoint_term(const T* __restrict__ ctrl, const LoopsT& L, T px, T py) {
  T e = (T)0;
  for (int l = 0; l < L.n; ++l) {
    if (L.closed[l] || L.off[l + 1] <= L.off[l]) continue;
    const T* s = ctrl + 8 * (int64_t)L.off[l];
    const T* f = ctrl + 8 * (int64_t)(L.off[l + 1] - 1);
    e += open_loop_angle(s[0] - px, s[1] - py, f[6] - px, f[7] - py);
  }
  return e;
}

constexpr int kThreads = 256;
constexpr int kPieceChunk = 256;

template <class T, class LoopsT>
__global__ __launch_bounds__(kThreads) void k_points(const Piece<T>* __restrict__ pcs, int32_t npc,
                                                     const T* __restrict__ ctrl, LoopsT L,
                                                     const T* __restrict__ x, const T* __restrict__ y,
                                                     int64_t n, T* __restrict__ w, int32_t* __restrict__ chi) {
  __shared__ Piece<T> sp[kPieceChunk];
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool ok = q < n;
  const T px = ok ? x[q] : (T)0, py = ok ? y[q] : (T)0;
  int c = 0;
  for (int p0 = 0; p0 < npc; p0 += kPieceChunk) {
    const int cnt = min(kPieceChunk, npc - p0);
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kThreads) sp[j] = pcs[p0 + j];
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const T y0 = sp[j].y0, y1 = sp[j].y1;
      const bool s0 = y0 >= py, s1 = y1 >= py;
      if (s0 == s1) continue;
      if (right_of(sp[j], py, px)) c += s1 ? 1 : -1;
    }
  }
  if (!ok) return;
  if (!(isfinite(px) && isfinite(py))) {
    w[q] = (T)NAN;
    if (chi) chi[q] = WN_CHI_INVALID;
    return;
  }
  const T e = endpoint_term(ctrl, L, px, py);
  w[q] = finish_w(c, e);
  if (chi) chi[q] = c;
}

constexpr int kColTile = kGridColTile2D;
constexpr int kSolveChunk = 1024;   // pieces examined per pass (LDS list of those needing a solve)

constexpr int kMaxOpen = 64;   // open loops whose end points a grid tile stages in LDS

// Histogram slot c lives at word c + c / 32: threads that own consecutive
// blocks of 8 columns then read and write different banks.
__host__ __device__ constexpr int hist_at(int c) { return c + (c >> 5); }
__host__ __device__ constexpr int hist_words(int tile) { return hist_at(tile) + 1; }

template <class T>
struct alignas(sizeof(T) * 4) EndPts {
  T sx, sy, ex, ey;
};

// Number of tile columns with x_i < xe (x ascending, ncol >= 1): first the
// position xe would have on an evenly spaced axis, then steps of doubling
// length to a bracket of the answer, then bisection inside it.  On an evenly
// spaced axis the guess is the answer or next to it (two reads instead of
// the eleven of a bisection over 2048 columns); any ascending axis gets the
// exact count.
template <class T>
__device__ __forceinline__ int count_below(const T* sx, int ncol, T xe, T xlo, T xscale) {
  const T f = fmin(fmax((xe - xlo) * xscale, (T)-1), (T)ncol);
  const int g = min((int)f + 1, ncol);   // f >= -1: g in [0, ncol]
  int lo, hi;                            // the answer lies in [lo, hi]
  if (g < ncol && sx[g] < xe) {
    lo = g + 1;
    hi = lo;
    for (int step = 1; hi < ncol && sx[hi] < xe; step <<= 1) {
      lo = hi + 1;
      hi = min(ncol, hi + step);
    }
  } else {
    hi = g;
    lo = hi;
    for (int step = 1; lo > 0 && !(sx[lo - 1] < xe); step <<= 1) {
      hi = lo - 1;
      lo = max(0, lo - step);
    }
  }
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (sx[mid] < xe) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Inclusive suffix sum over the lanes of a wavefront (lane i gets the sum of
// lanes i..63).
__device__ __forceinline__ int wave_suffix_sum(int v) {
  const int lane = threadIdx.x & 63;
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_down(v, o);
    if (lane + o < 64) v += u;
  }
  return v;
}

// One workgroup per (row, column tile).  Histogram slot c (0..ncol) counts the
// crossings with exactly c tile columns left of them; columns at or beyond
// the tile end get every crossing right of the whole tile through `base`.
// Pieces are examined in chunks: a first pass settles the pieces that miss
// the row or lie beside the whole tile and lists the others in LDS, so that
// the Newton solves run on consecutive lanes without idle lanes in between.
// All counts are integer additions, so their order does not matter.
template <class T, class LoopsT>
__device__ void grid_tile(const Piece<T>* __restrict__ pcs, const typename Vec2<T>::type* __restrict__ yr,
                          int32_t npc, const T* __restrict__ ctrl, const LoopsT& L, const T* __restrict__ x,
                          int64_t nx, T yq, int64_t row, int64_t i0, int ncol, T* __restrict__ w,
                          int32_t* __restrict__ chi, T* sx, int* hist, int* sscan, int* list, int* nlist,
                          EndPts<T>* sep, int* snopen) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < ncol; i += kThreads) sx[i] = x[i0 + i];
  for (int i = threadIdx.x; i < hist_words(ncol); i += kThreads) hist[i] = 0;
  // the open loops' end points, compacted in loop order by the first
  // wavefront (the same for every query of the row; -1: more than kMaxOpen,
  // then each query walks the loop table itself)
  if (wv == 0) {
    int cnt = 0;
    for (int l0 = 0; l0 < L.n; l0 += 64) {
      const int l = l0 + lane;
      const bool open = l < L.n && !L.closed[l] && L.off[l + 1] > L.off[l];
      const uint64_t m = __ballot(open);
      if (open) {
        const int at = cnt + __popcll(m & ((1ull << lane) - 1ull));
        if (at < kMaxOpen) {
          const T* f0 = ctrl + 8 * (int64_t)L.off[l];
          const T* f1 = ctrl + 8 * (int64_t)(L.off[l + 1] - 1);
          sep[at] = EndPts<T>{f0[0], f0[1], f1[6], f1[7]};
        }
      }
      cnt += __popcll(m);
    }
    if (lane == 0) *snopen = cnt <= kMaxOpen ? cnt : -1;
  }
  __syncthreads();
  const T xlo = sx[0], xhi = sx[ncol - 1];
  // columns per unit of x on an evenly spaced axis (the search's first guess)
  const T xscale = (xhi > xlo && ncol > 1) ? (T)(ncol - 1) / (xhi - xlo) : (T)0;
  int base = 0;   // crossings right of every column of the tile
  for (int c0 = 0; c0 < npc; c0 += kSolveChunk) {
    const int c1 = min(c0 + kSolveChunk, npc);
    if (threadIdx.x == 0) *nlist = 0;
    __syncthreads();
    for (int j = c0 + threadIdx.x; j < c1; j += kThreads) {
      const typename Vec2<T>::type e = yr[j];
      const bool s0 = e.x >= yq, s1 = e.y >= yq;
      if (s0 == s1) continue;
      const int sg = s1 ? 1 : -1;
      const T pxmin = pcs[j].xmin, pxmax = pcs[j].xmax;
      if (xhi < pxmin) base += sg;                          // right of every column
      else if (xlo < pxmax) list[atomicAdd(nlist, 1)] = j;  // needs the solve
      // else: right of no column
    }
    __syncthreads();
    const int n = *nlist;
    for (int k = threadIdx.x; k < n; k += kThreads) {
      const int j = list[k];
      const Piece<T>& pc = pcs[j];
      const int sg = yr[j].y >= yq ? 1 : -1;
      const T xs = solve_x(pc, yq);
      const T xe = fmin(fmax(xs, pc.xmin), pc.xmax);
      const int a = count_below(sx, ncol, xe, xlo, xscale);
      if (a == ncol) base += sg;
      else if (a > 0) atomicAdd(&hist[hist_at(a)], sg);
    }
    __syncthreads();
  }
  // chi(col i) = btot + sum_{c > i} hist[c]: suffix sums over [1, ncol),
  // each thread owning a contiguous block of columns.  Integer sums, so
  // their order does not matter: wavefront shuffles, then one exchange of
  // the four wavefronts' totals (and of `base`) through LDS.
  const int per = (ncol + kThreads - 1) / kThreads;
  const int a0 = threadIdx.x * per;
  const int a1 = min(a0 + per, ncol);
  int part = 0;
  for (int c = a0 + 1; c <= a1 && c < ncol; ++c) part += hist[hist_at(c)];
  const int suf = wave_suffix_sum(part);              // parts of lanes >= this one in the wavefront
  const int bw = wave_suffix_sum(base);               // lane 0: the wavefront's base
  if (lane == 0) {
    sscan[wv] = suf;
    sscan[kThreads / 64 + wv] = bw;
  }
  __syncthreads();
  int btot = 0, later = 0;
#pragma unroll
  for (int k = 0; k < kThreads / 64; ++k) {
    btot += sscan[kThreads / 64 + k];
    if (k > wv) later += sscan[k];
  }
  int run = btot + (suf - part) + later;
  // walk this thread's columns from the right; chi(i) replaces hist[i + 1],
  // which no thread reads after this point (thread blocks are disjoint and
  // the slot is read just before it is overwritten)
  for (int i = a1 - 1; i >= a0; --i) {
    if (i + 1 < ncol) run += hist[hist_at(i + 1)];
    hist[hist_at(i + 1)] = run;
  }
  __syncthreads();
  // coalesced output: consecutive lanes write consecutive columns.  A thread
  // takes kOutQ of its columns at once, so that each end point is read from
  // LDS once for all of them and their angle chains interleave.
  const int nopen = *snopen;
  constexpr int kOutQ = 8;
  for (int ib = 0; ib < ncol; ib += kOutQ * kThreads) {
    T px[kOutQ], e[kOutQ];
#pragma unroll
    for (int k = 0; k < kOutQ; ++k) {
      const int i = ib + k * kThreads + threadIdx.x;
      px[k] = i < ncol ? sx[i] : (T)0;
      e[k] = (T)0;
    }
    if (nopen > 0) {
      // endpoint_term's terms in its order
      for (int t = 0; t < nopen; ++t) {
        const EndPts<T> q = sep[t];
        const T sy = q.sy - yq, ey = q.ey - yq;
#pragma unroll
        for (int k = 0; k < kOutQ; ++k) e[k] += open_loop_angle(q.sx - px[k], sy, q.ex - px[k], ey);
      }
    }
#pragma unroll
    for (int k = 0; k < kOutQ; ++k) {
      const int i = ib + k * kThreads + threadIdx.x;
      if (i >= ncol) continue;
      const int64_t o = row * nx + i0 + i;
      if (!(isfinite(px[k]) && isfinite(yq))) {
        w[o] = (T)NAN;
        if (chi) chi[o] = WN_CHI_INVALID;
        continue;
      }
      const int c = hist[hist_at(i + 1)];
      const T ek = nopen >= 0 ? e[k] : endpoint_term(ctrl, L, px[k], yq);
      w[o] = finish_w(c, ek);
      if (chi) chi[o] = c;
    }
  }
}

// One workgroup per (row, column tile).  Histogram slot c (0..ncol) counts the
// crossings with exactly c tile columns left of them; columns at or beyond
// the tile end get every crossing right of the whole tile through `base`.
// Pieces are examined in chunks: a first pass settles the pieces that miss
// the row or lie beside the whole tile and lists the others in LDS, so that
// the Newton solves run on consecutive lanes without idle lanes in between.
// All counts are integer additions, so their order does not matter.
template <class T, class LoopsT>
__global__ __launch_bounds__(kThreads) void k_grid(const Piece<T>* __restrict__ pcs,
                                                   const typename Vec2<T>::type* __restrict__ yr, int32_t npc,
                                                   const T* __restrict__ ctrl, LoopsT L,
                                                   const T* __restrict__ x, int64_t nx,
                                                   const T* __restrict__ y, int64_t ny,
                                                   T* __restrict__ w, int32_t* __restrict__ chi, int tile) {
  // dynamic LDS sized to the tile: sx [tile] T, hist [tile + 1] int
  extern __shared__ __align__(16) unsigned char dyn[];
  T* sx = reinterpret_cast<T*>(dyn);
  int* hist = reinterpret_cast<int*>(sx + tile);
  __shared__ int sscan[2 * (kThreads / 64)];
  __shared__ int list[kSolveChunk];
  __shared__ int nlist, nopen;
  __shared__ EndPts<T> sep[kMaxOpen];
  const int64_t row = blockIdx.y;
  const int64_t i0 = (int64_t)blockIdx.x * tile;
  const int ncol = (int)min((int64_t)tile, nx - i0);
  grid_tile(pcs, yr, npc, ctrl, L, x, nx, y[row], row, i0, ncol, w, chi, sx, hist, sscan, list, &nlist, sep,
            &nopen);
}

// ---------------------------------------------------------------------------
// Batched grid mode: many curve sets, each with its own grid, in one launch.
// ---------------------------------------------------------------------------

// One curve set of a batch; offsets index the batch's concatenated arrays.
struct Set2D {
  int64_t item_off;    // first (row, tile) workgroup of the set
  int64_t x_off, y_off, out_off;
  int32_t seg_off;     // first segment (pieces at 3 seg_off)
  int32_t nseg;
  int32_t off_base;    // first entry of the set's loop offsets in the batch table
  int32_t closed_base; // first entry of the set's closed flags
  int32_t nloops;
  int32_t nx, ny;
  int32_t ntiles, tile;
  int32_t rows;        // rows per item (wavefront kernel; 1 for the workgroup kernel)
};

// Set containing index v of a per-set prefix (binary search).
template <class F>
__device__ __forceinline__ int find_set(const Set2D* __restrict__ sets, int nsets, int64_t v, F start) {
  int lo = 0, hi = nsets - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start(sets[mid]) <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_grid_batched(const Set2D* __restrict__ sets, int32_t nsets,
                                                           const Piece<T>* __restrict__ pcs,
                                                           const typename Vec2<T>::type* __restrict__ yr,
                                                           const int32_t* __restrict__ loop_off,
                                                           const uint8_t* __restrict__ loop_closed,
                                                           const T* __restrict__ ctrl, const T* __restrict__ x,
                                                           const T* __restrict__ y, T* __restrict__ w,
                                                           int32_t* __restrict__ chi) {
  extern __shared__ __align__(16) unsigned char dyn[];
  __shared__ int sscan[2 * (kThreads / 64)];
  __shared__ int list[kSolveChunk];
  __shared__ int nlist, nopen;
  __shared__ EndPts<T> sep[kMaxOpen];
  const int64_t item = blockIdx.x;
  const int k = find_set(sets, nsets, item, [](const Set2D& d) { return d.item_off; });
  const Set2D d = sets[k];
  const int64_t local = item - d.item_off;
  const int64_t row = local / d.ntiles;
  const int64_t i0 = (local % d.ntiles) * d.tile;
  const int ncol = (int)min((int64_t)d.tile, (int64_t)d.nx - i0);
  T* sx = reinterpret_cast<T*>(dyn);
  int* hist = reinterpret_cast<int*>(sx + d.tile);
  const DevLoops2D L{d.nloops, loop_off + d.off_base, loop_closed + d.closed_base};
  grid_tile(pcs + 3 * (int64_t)d.seg_off, yr + 3 * (int64_t)d.seg_off, 3 * d.nseg, ctrl + 8 * (int64_t)d.seg_off,
            L, x + d.x_off, (int64_t)d.nx, y[d.y_off + row], row, i0, ncol, w + d.out_off,
            chi ? chi + d.out_off : nullptr, sx, hist, sscan, list, &nlist, sep, &nopen);
}

// Sets with at most 64 monotone pieces (21 segments): one wavefront per
// (set, group of rows, column tile), four per workgroup.  Lane r*npc + j
// takes piece j on row r of the group (rows = 64 / npc, at most
// kRowsPerWave): a piece that straddles the row gets its crossing abscissa
// xe, clamped to the piece's x range (pieces beside the whole tile take a
// bound instead of a solve), and each row's crossings are compacted into the
// wavefront's LDS list.  chi of a column is the signed count of its row's
// entries with x_i < xe, which is what k_grid's histogram and suffix scan
// count: a crossing lands in slot a = #{columns with x < xe} and adds to
// every column i < a.  Columns left of a piece's x range always count it and
// columns right of it never do, with or without the solve, so the two
// kernels agree bit for bit.  The open loops' end points (the same for every
// query of the set) are staged in LDS once, in loop order, and summed in the
// order and arithmetic of endpoint_term.
constexpr int kRowWaves = kThreads / 64;
constexpr int kRowPieces = kRowPieces2D;
constexpr int kRowLoops = kRowPieces2D / 3;   // a loop has at least one segment
constexpr int kRowColTile = kRowColTile2D;
constexpr int kRowsPerWave = kRowsPerWave2D;

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_rows_batched(const Set2D* __restrict__ sets, int32_t nsets,
                                                           const int32_t* __restrict__ blk_set, int64_t nitems,
                                                           const Piece<T>* __restrict__ pcs,
                                                           const typename Vec2<T>::type* __restrict__ yr,
                                                           const int32_t* __restrict__ loop_off,
                                                           const uint8_t* __restrict__ loop_closed,
                                                           const T* __restrict__ ctrl, const T* __restrict__ x,
                                                           const T* __restrict__ y, T* __restrict__ w,
                                                           int32_t* __restrict__ chi) {
  using V4 = T[4];
  __shared__ T sxe[kRowWaves][kRowPieces];
  __shared__ int ssg[kRowWaves][kRowPieces];
  __shared__ V4 sep[kRowWaves][kRowLoops];
  const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t item = (int64_t)blockIdx.x * kRowWaves + wv;
  if (item >= nitems) return;   // whole wavefronts leave; no workgroup barrier below
  // the set of the block's first item, then forward (sets may hold no items)
  int k = blk_set[blockIdx.x];
  while (k + 1 < nsets && sets[k + 1].item_off <= item) ++k;
  const Set2D d = sets[k];
  const int64_t local = item - d.item_off;
  const int64_t r0 = (local / d.ntiles) * d.rows;
  const int nr = (int)min((int64_t)d.rows, (int64_t)d.ny - r0);
  const int64_t i0 = (local % d.ntiles) * d.tile;
  const int ncol = (int)min((int64_t)d.tile, (int64_t)d.nx - i0);
  const T* xs = x + d.x_off + i0;
  const T* ys = y + d.y_off + r0;
  const T xlo = xs[0], xhi = xs[ncol - 1];
  const int npc = 3 * d.nseg;   // <= kRowPieces; rows * npc <= 64
  // crossings: lane r * npc + j <-> (row r, piece j)
  const int r = npc ? lane / npc : 0;
  const int j = lane - r * npc;
  int sg = 0;
  T xe = (T)0;
  if (npc && r < nr) {
    const T yq = ys[r];
    const int64_t pj = 3 * (int64_t)d.seg_off + j;
    const typename Vec2<T>::type e = yr[pj];
    const bool s0 = e.x >= yq, s1 = e.y >= yq;
    if (s0 != s1) {
      sg = s1 ? 1 : -1;
      const Piece<T>& pc = pcs[pj];
      if (xhi < pc.xmin) xe = pc.xmin;          // right of every column
      else if (xlo >= pc.xmax) xe = pc.xmax;    // right of no column
      else xe = fmin(fmax(solve_x(pc, yq), pc.xmin), pc.xmax);
    }
  }
  const uint64_t m = __ballot(sg != 0);
  const uint64_t rowbits = npc >= 64 ? ~0ull : ((1ull << npc) - 1);
  if (sg != 0) {
    const int at = __popcll(m & (rowbits << (r * npc)) & ((1ull << lane) - 1));
    sxe[wv][r * npc + at] = xe;
    ssg[wv][r * npc + at] = sg;
  }
  // open loops' end points, compacted in loop order
  bool open = false;
  T e4[4] = {(T)0, (T)0, (T)0, (T)0};
  if (lane < d.nloops) {
    const int o0 = loop_off[d.off_base + lane], o1 = loop_off[d.off_base + lane + 1];
    open = !loop_closed[d.closed_base + lane] && o1 > o0;
    if (open) {
      const T* sp = ctrl + 8 * ((int64_t)d.seg_off + o0);
      const T* fp = ctrl + 8 * ((int64_t)d.seg_off + o1 - 1);
      e4[0] = sp[0];
      e4[1] = sp[1];
      e4[2] = fp[6];
      e4[3] = fp[7];
    }
  }
  const uint64_t mo = __ballot(open);
  const int nopen = __popcll(mo);
  if (open) {
    const int at = __popcll(mo & ((1ull << lane) - 1));
    for (int t = 0; t < 4; ++t) sep[wv][at][t] = e4[t];
  }
  wave_fence();
  T* wr = w + d.out_off + r0 * d.nx + i0;
  int32_t* cr = chi ? chi + d.out_off + r0 * d.nx + i0 : nullptr;
  for (int rr = 0; rr < nr; ++rr, wr += d.nx, cr = cr ? cr + d.nx : nullptr) {
    const T yq = ys[rr];
    const int n = __popcll(m & (rowbits << (rr * npc)));
    const T* lx = &sxe[wv][rr * npc];
    const int* lg = &ssg[wv][rr * npc];
    for (int i = lane; i < ncol; i += 64) {
      const T px = xs[i];
      if (!(isfinite(px) && isfinite(yq))) {
        wr[i] = (T)NAN;
        if (cr) cr[i] = WN_CHI_INVALID;
        continue;
      }
      int c = 0;
      for (int t = 0; t < n; ++t) c += px < lx[t] ? lg[t] : 0;
      T e = (T)0;
      for (int t = 0; t < nopen; ++t)
        e += open_loop_angle(sep[wv][t][0] - px, sep[wv][t][1] - yq, sep[wv][t][2] - px, sep[wv][t][3] - yq);
      wr[i] = finish_w(c, e);
      if (cr) cr[i] = c;
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint.  Away from the curves chi is locally constant, so w moves only
// with the open loops' end-point angles; with A(v) = (-v_y, v_x)/|v|^2 (the
// gradient of the angle of v) and c = g/(2 pi) per query:
//   dL/dp += c (A(s - p) - A(e - p)),  dL/ds -= c A(s - p),  dL/de += c A(e - p).
// Interior control points and closed loops get zero.  Per wavefront the
// end-point sums are reduced by DPP moves in T (a fixed pattern), the
// workgroup adds its wavefronts in float64 in order after one barrier and stores its
// partials value-major (part[value][workgroup]); two more kernels add the
// workgroup partials in chunks and then the chunks, each in a fixed order,
// so grad_ctrl is bitwise reproducible.
// ---------------------------------------------------------------------------

// Sum over the 64 lanes of a wavefront, left in lane 63, by DPP moves (no
// LDS traffic): butterflies inside quads, rotations inside rows of 16, then
// the row broadcasts of lanes 15 and 31.  Doubles move as two halves.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_t(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_t(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <class T>
__device__ __forceinline__ T wave_sum_last(T v) {
  v += dpp_t<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v += dpp_t<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v += dpp_t<0x124, 0xF>(v);   // row_ror:4
  v += dpp_t<0x128, 0xF>(v);   // row_ror:8: every lane holds its row's sum
  v += dpp_t<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_t<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

template <class T>
__device__ __forceinline__ void angle_grad(T vx, T vy, T& ax, T& ay) {
  const T r2 = fma_t(vx, vx, vy * vy);
  const T inv = (T)1 / r2;
  ax = -vy * inv;
  ay = vx * inv;
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_back2d(const T* __restrict__ ctrl, Loops2D L, int32_t kind,
                                                     const T* __restrict__ x, const T* __restrict__ y, int64_t nx,
                                                     int64_t n, const T* __restrict__ gw, T* __restrict__ gq,
                                                     double* __restrict__ part, int64_t nslots) {
  // [4 open loops][kThreads / 64] wavefront partials (dynamic, sized by the host)
  extern __shared__ __align__(16) unsigned char dyn_b[];
  double* wpart = reinterpret_cast<double*>(dyn_b);
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool ok = q < n;
  T px = (T)0, py = (T)0, g = (T)0;
  if (ok) {
    int64_t row, col;
    if (kind == 0) {
      row = col = q;
    } else if (n <= (int64_t)UINT32_MAX) {   // 32-bit division where it suffices
      const uint32_t q32 = (uint32_t)q, nx32 = (uint32_t)nx;
      row = q32 / nx32;
      col = q32 - (uint32_t)row * nx32;
    } else {
      row = q / nx;
      col = q - row * nx;
    }
    px = x[col];
    py = y[row];
    g = gw[q];
  }
  const bool fin = ok && isfinite(px) && isfinite(py);
  const T c = fin ? g * (T)0.15915494309189535 : (T)0;
  T gpx = (T)0, gpy = (T)0;
  int k = 0;
  for (int l = 0; l < L.n; ++l) {
    if (L.closed[l] || L.off[l + 1] <= L.off[l]) continue;
    const T* sp = ctrl + 8 * (int64_t)L.off[l];
    const T* ep = ctrl + 8 * (int64_t)(L.off[l + 1] - 1);
    T asx = (T)0, asy = (T)0, aex = (T)0, aey = (T)0;
    if (fin) {
      angle_grad(sp[0] - px, sp[1] - py, asx, asy);
      angle_grad(ep[6] - px, ep[7] - py, aex, aey);
      gpx += asx - aex;
      gpy += asy - aey;
    }
    if (part) {   // uniform: end-point gradients requested
      // wavefront sums by DPP moves (a fixed pattern, in T), parked in LDS
      // per (open loop, wavefront)
      T v[4] = {-(c * asx), -(c * asy), c * aex, c * aey};
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = wave_sum_last(v[j]);
      if ((threadIdx.x & 63) == 63) {
#pragma unroll
        for (int j = 0; j < 4; ++j) wpart[(k * 4 + j) * (kThreads / 64) + (threadIdx.x >> 6)] = (double)v[j];
      }
    }
    ++k;
  }
  if (part) {
    // one barrier: the workgroup's partial of every end-point value is the
    // sum of its wavefronts' in order
    __syncthreads();
    for (int t = threadIdx.x; t < 4 * k; t += kThreads) {
      double a = wpart[t * (kThreads / 64)];
#pragma unroll
      for (int wv = 1; wv < kThreads / 64; ++wv) a += wpart[t * (kThreads / 64) + wv];
      part[(int64_t)t * nslots + blockIdx.x] = a;
    }
  }
  if (ok && gq) {
    if (fin) {
      gq[2 * q] = c * gpx;
      gq[2 * q + 1] = c * gpy;
    } else {
      gq[2 * q] = gq[2 * q + 1] = (T)NAN;
    }
  }
}

// Fixed-order sums of the end-point partials part[value][nslots]: first
// over chunks of kSumChunk workgroup partials (grid: chunks x values, into
// tmp[value][chunk]), then over the chunks (one workgroup per value), into
// the value's grad_ctrl entry.
constexpr int kSumChunk = 2048;

__global__ __launch_bounds__(kThreads) void k_back2d_chunks(const double* __restrict__ part, int64_t nslots,
                                                           int64_t nchunks, double* __restrict__ tmp) {
  __shared__ double red[kThreads];
  const int64_t v = blockIdx.y, c0 = (int64_t)blockIdx.x * kSumChunk;
  const double* p = part + v * nslots;
  double a = 0.0;
  for (int i = threadIdx.x; i < kSumChunk && c0 + i < nslots; i += kThreads) a += p[c0 + i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) tmp[v * nchunks + blockIdx.x] = red[0];
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_back2d_sum(const double* __restrict__ tmp, int64_t nchunks,
                                                         Loops2D L, T* __restrict__ gc) {
  __shared__ double red[kThreads];
  const double* p = tmp + (int64_t)blockIdx.x * nchunks;
  double sacc = 0.0;
  for (int64_t b = threadIdx.x; b < nchunks; b += kThreads) sacc += p[b];
  red[threadIdx.x] = sacc;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int k = blockIdx.x / 4, j = blockIdx.x % 4;
    int seen = -1, l = 0;
    for (; l < L.n; ++l) {
      if (L.closed[l] || L.off[l + 1] <= L.off[l]) continue;
      if (++seen == k) break;
    }
    const int64_t at = j < 2 ? 8 * (int64_t)L.off[l] + j : 8 * (int64_t)(L.off[l + 1] - 1) + 6 + (j - 2);
    gc[at] = (T)red[0];
  }
}

template <class T>
__global__ void k_zero(T* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (T)0;
}

template <class T>
hipError_t back2d(const T* ctrl, int64_t nseg, const Loops2D& L, int32_t kind, const T* x, const T* y,
                  int64_t nx, int64_t n, const T* gw, T* gq, T* gc, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (gc && nseg > 0) {
    hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)((8 * nseg + 255) / 256)), dim3(256), 0, s, gc, 8 * nseg);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (n == 0) return hipSuccess;
  int nopen = 0;
  for (int l = 0; l < L.n; ++l)
    if (!L.closed[l] && L.off[l + 1] > L.off[l]) ++nopen;
  const int64_t nblocks = (n + kThreads - 1) / kThreads;
  const int64_t nchunks = (nblocks + kSumChunk - 1) / kSumChunk;
  double* part = nullptr;   // [4 nopen][nblocks] workgroup partials, then [4 nopen][nchunks]
  if (gc && nopen > 0) {
    e = hipMallocAsync((void**)&part, (size_t)nopen * 4 * (nblocks + nchunks) * sizeof(double), s);
    if (e != hipSuccess) return e;
  }
  const size_t lds = part ? (size_t)nopen * 4 * (kThreads / 64) * sizeof(double) : 0;
  hipLaunchKernelGGL(k_back2d<T>, dim3((unsigned)nblocks), dim3(kThreads), lds, s, ctrl, L, kind, x, y, nx, n, gw,
                     gq, part, nblocks);
  e = hipGetLastError();
  if (e == hipSuccess && part) {
    double* tmp = part + (size_t)nopen * 4 * nblocks;
    hipLaunchKernelGGL(k_back2d_chunks, dim3((unsigned)nchunks, (unsigned)(4 * nopen)), dim3(kThreads), 0, s, part,
                       nblocks, nchunks, tmp);
    e = hipGetLastError();
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_back2d_sum<T>, dim3((unsigned)(4 * nopen)), dim3(kThreads), 0, s, tmp, nchunks, L, gc);
      e = hipGetLastError();
    }
  }
  if (part) hipFreeAsync(part, s);
  return e;
}

template <class T, class LoopsT>
hipError_t run2d(const T* ctrl, int64_t nseg, const LoopsT& L, int32_t kind, const T* x, const T* y,
                 int64_t nx, int64_t ny, T* w, int32_t* chi, hipStream_t s) {
  using V2 = typename Vec2<T>::type;
  const int64_t npc = 3 * nseg;
  Piece<T>* pcs = nullptr;
  V2* yr = nullptr;
  hipError_t e = hipSuccess;
  if (npc > 0) {
    e = hipMallocAsync((void**)&pcs, (size_t)npc * (sizeof(Piece<T>) + sizeof(V2)), s);
    if (e != hipSuccess) return e;
    yr = reinterpret_cast<V2*>(pcs + npc);
    hipLaunchKernelGGL(k_pieces<T>, dim3((unsigned)((nseg + 127) / 128)), dim3(128), 0, s, ctrl,
                       (int32_t)nseg, pcs, yr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    if (kind == 0) {
      hipLaunchKernelGGL((k_points<T, LoopsT>), dim3((unsigned)((nx + kThreads - 1) / kThreads)), dim3(kThreads),
                         0, s, pcs, (int32_t)npc, ctrl, L, x, y, nx, w, chi);
    } else {
      // tiles of at most kColTile columns, as even as possible; LDS sized to the tile
      const int64_t ntiles = (nx + kColTile - 1) / kColTile;
      const int tile = (int)((nx + ntiles - 1) / ntiles);
      const size_t lds = ((size_t)tile * sizeof(T) + (size_t)hist_words(tile) * sizeof(int) + 15) & ~(size_t)15;
      hipLaunchKernelGGL((k_grid<T, LoopsT>), dim3((unsigned)ntiles, (unsigned)ny), dim3(kThreads), lds, s, pcs,
                         yr, (int32_t)npc, ctrl, L, x, nx, y, ny, w, chi, tile);
    }
    e = hipGetLastError();
  }
  if (pcs) {
    const hipError_t e2 = hipFreeAsync(pcs, s);
    if (e == hipSuccess) e = e2;
  }
  return e;
}

}  // namespace

Batch2D::~Batch2D() {
  if (ws) (void)hipFree(ws);
}

hipError_t batch2d_create(int32_t dtype, const wn_curveset_2d* sets, int32_t nsets, hipStream_t s, Batch2D* b) {
  // sets with few pieces go to the wavefront-per-row kernel, the others to
  // the workgroup (histogram) kernel; each kernel numbers its own items
  std::vector<Set2D> dg, dw;
  std::vector<int32_t> offs;
  std::vector<uint8_t> cls;
  int64_t seg = 0, xo = 0, yo = 0, oo = 0, items_g = 0, items_w = 0;
  int max_tile = 1;
  for (int32_t k = 0; k < nsets; ++k) {
    const wn_curveset_2d& c = sets[k];
    const bool wave = 3 * c.nseg <= kRowPieces;
    Set2D e;
    e.x_off = xo;
    e.y_off = yo;
    e.out_off = oo;
    e.seg_off = (int32_t)seg;
    e.nseg = (int32_t)c.nseg;
    e.off_base = (int32_t)offs.size();
    e.closed_base = (int32_t)cls.size();
    e.nloops = c.nloops;
    for (int32_t l = 0; l <= c.nloops; ++l) offs.push_back(c.nloops ? (int32_t)c.loop_off[l] : 0);
    for (int32_t l = 0; l < c.nloops; ++l) cls.push_back(c.loop_closed[l] ? 1 : 0);
    e.nx = (int32_t)c.nx;
    e.ny = (int32_t)c.ny;
    // column tiles as even as possible (the workgroup kernel uses the
    // single-set call's tiling)
    const int64_t cap = wave ? kRowColTile : kColTile;
    e.ntiles = (int32_t)((c.nx + cap - 1) / cap);
    e.tile = e.ntiles ? (int32_t)((c.nx + e.ntiles - 1) / e.ntiles) : 1;
    e.rows = wave ? (int32_t)std::min<int64_t>(kRowsPerWave, kRowPieces / std::max<int64_t>(3 * c.nseg, 1)) : 1;
    int64_t& items = wave ? items_w : items_g;
    e.item_off = items;
    items += (int64_t)e.ntiles * ((c.ny + e.rows - 1) / e.rows);
    if (!wave) max_tile = std::max(max_tile, (int)e.tile);
    (wave ? dw : dg).push_back(e);
    seg += c.nseg;
    xo += c.nx;
    yo += c.ny;
    oo += c.nx * c.ny;
  }
  b->dtype = dtype;
  b->nsets_g = (int32_t)dg.size();
  b->nsets_w = (int32_t)dw.size();
  b->nseg = seg;
  b->nx = xo;
  b->ny = yo;
  b->nout = oo;
  b->items_g = items_g;
  b->items_w = items_w;
  const size_t tsz = dtype == WN_F64 ? sizeof(double) : sizeof(float);
  b->lds = ((size_t)max_tile * tsz + (size_t)hist_words(max_tile) * sizeof(int) + 15) & ~(size_t)15;
  // set of the first item of every wavefront-kernel workgroup
  std::vector<int32_t> bs((size_t)((items_w + kRowWaves - 1) / kRowWaves));
  for (size_t k = 0, blk = 0; blk < bs.size(); ++blk) {
    const int64_t it = (int64_t)blk * kRowWaves;
    while (k + 1 < dw.size() && dw[k + 1].item_off <= it) ++k;
    bs[blk] = (int32_t)k;
  }
  // one device allocation: descriptors (workgroup sets, then wavefront
  // sets) | loop offsets | closed flags | block -> set | pieces | y ranges
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t b_dg = up(dg.size() * sizeof(Set2D));
  const size_t b_dw = up(dw.size() * sizeof(Set2D));
  const size_t b_off = up(offs.size() * sizeof(int32_t));
  const size_t b_cls = up(cls.size() + 1);
  const size_t b_bs = up(bs.size() * sizeof(int32_t));
  const size_t piece = dtype == WN_F64 ? sizeof(Piece<double>) + sizeof(double2) : sizeof(Piece<float>) + sizeof(float2);
  const size_t bytes = b_dg + b_dw + b_off + b_cls + b_bs + (size_t)(3 * seg) * piece;
  hipError_t e = hipMalloc((void**)&b->ws, std::max(bytes, (size_t)256));
  if (e != hipSuccess) {
    b->ws = nullptr;
    return e;
  }
  b->desc_g = b->ws;
  b->desc_w = b->ws + b_dg;
  b->loop_off = b->ws + b_dg + b_dw;
  b->loop_closed = b->loop_off + b_off;
  b->blk_set = b->loop_closed + b_cls;
  b->pieces = b->blk_set + b_bs;
  auto put = [&](void* dst, const void* src, size_t n) {
    if (n && e == hipSuccess) e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s);
  };
  put(b->desc_g, dg.data(), dg.size() * sizeof(Set2D));
  put(b->desc_w, dw.data(), dw.size() * sizeof(Set2D));
  put(b->loop_off, offs.data(), offs.size() * sizeof(int32_t));
  put(b->loop_closed, cls.data(), cls.size());
  put(b->blk_set, bs.data(), bs.size() * sizeof(int32_t));
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);   // the host tables go out of scope
}

template <class T>
hipError_t run2d_batched(const Batch2D& b, const T* ctrl, const T* x, const T* y, T* w, int32_t* chi,
                         hipStream_t s) {
  using V2 = typename Vec2<T>::type;
  if (b.items_g + b.items_w == 0) return hipSuccess;
  const int32_t* doff = reinterpret_cast<const int32_t*>(b.loop_off);
  const uint8_t* dcl = b.loop_closed;
  Piece<T>* pcs = reinterpret_cast<Piece<T>*>(b.pieces);
  V2* yr = reinterpret_cast<V2*>(pcs + 3 * b.nseg);
  if (b.nseg > 0) {
    // the sets' segments are contiguous: split them all in one launch
    hipLaunchKernelGGL(k_pieces<T>, dim3((unsigned)((b.nseg + 127) / 128)), dim3(128), 0, s, ctrl, (int32_t)b.nseg,
                       pcs, yr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (b.items_w > 0) {
    const int64_t blocks = (b.items_w + kRowWaves - 1) / kRowWaves;
    hipLaunchKernelGGL(k_rows_batched<T>, dim3((unsigned)blocks), dim3(kThreads), 0, s,
                       reinterpret_cast<const Set2D*>(b.desc_w), b.nsets_w,
                       reinterpret_cast<const int32_t*>(b.blk_set), b.items_w, pcs, yr, doff, dcl, ctrl, x, y, w,
                       chi);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (b.items_g > 0) {
    hipLaunchKernelGGL(k_grid_batched<T>, dim3((unsigned)b.items_g), dim3(kThreads), b.lds, s,
                       reinterpret_cast<const Set2D*>(b.desc_g), b.nsets_g, pcs, yr, doff, dcl, ctrl, x, y, w, chi);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t eval_2d_batched(const Batch2D& b, const void* ctrl, const void* x, const void* y, void* w, int32_t* chi,
                           hipStream_t s) {
  if (b.dtype == WN_F64)
    return run2d_batched<double>(b, (const double*)ctrl, (const double*)x, (const double*)y, (double*)w, chi, s);
  return run2d_batched<float>(b, (const float*)ctrl, (const float*)x, (const float*)y, (float*)w, chi, s);
}

template <class LoopsT>
hipError_t run2d_typed(int32_t dtype, const void* ctrl, int64_t nseg, const LoopsT& L, int32_t kind, const void* x,
                       const void* y, int64_t nx, int64_t ny, void* w, int32_t* chi, hipStream_t s) {
  if (dtype == WN_F64)
    return run2d<double>((const double*)ctrl, nseg, L, kind, (const double*)x, (const double*)y, nx, ny,
                         (double*)w, chi, s);
  return run2d<float>((const float*)ctrl, nseg, L, kind, (const float*)x, (const float*)y, nx, ny, (float*)w,
                      chi, s);
}

hipError_t eval_2d(int32_t dtype, const void* ctrl, int64_t nseg, const int64_t* loop_off,
                   const uint8_t* closed, int32_t nloops, int32_t kind, const void* x, const void* y,
                   int64_t nx, int64_t ny, void* w, int32_t* chi, hipStream_t s) {
  if (nloops <= WN_MAX_LOOPS) {   // the table in the kernel arguments
    Loops2D L;
    L.n = nloops;
    for (int l = 0; l <= nloops; ++l) L.off[l] = (int32_t)loop_off[l];
    for (int l = 0; l < nloops; ++l) L.closed[l] = closed[l] ? 1 : 0;
    return run2d_typed(dtype, ctrl, nseg, L, kind, x, y, nx, ny, w, chi, s);
  }
  // a longer table: one device copy (offsets, then flags) for this call
  std::vector<int32_t> h((size_t)nloops + 1 + ((size_t)nloops + 3) / 4, 0);
  for (int l = 0; l <= nloops; ++l) h[l] = (int32_t)loop_off[l];
  uint8_t* hc = reinterpret_cast<uint8_t*>(h.data() + nloops + 1);
  for (int l = 0; l < nloops; ++l) hc[l] = closed[l] ? 1 : 0;
  int32_t* d = nullptr;
  hipError_t e = hipMallocAsync((void**)&d, h.size() * sizeof(int32_t), s);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(d, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // the host copy must outlive the transfer
  if (e == hipSuccess) {
    const DevLoops2D L{nloops, d, reinterpret_cast<const uint8_t*>(d + nloops + 1)};
    e = run2d_typed(dtype, ctrl, nseg, L, kind, x, y, nx, ny, w, chi, s);
  }
  const hipError_t e2 = hipFreeAsync(d, s);
  return e != hipSuccess ? e : e2;
}

hipError_t backward_2d(int32_t dtype, const void* ctrl, int64_t nseg, const int64_t* loop_off,
                       const uint8_t* closed, int32_t nloops, int32_t kind, const void* x, const void* y,
                       int64_t nx, int64_t ny, const void* gw, void* gq, void* gc, hipStream_t s) {
  Loops2D L;
  L.n = nloops;
  for (int l = 0; l <= nloops; ++l) L.off[l] = (int32_t)loop_off[l];
  for (int l = 0; l < nloops; ++l) L.closed[l] = closed[l] ? 1 : 0;
  const int64_t n = kind == 0 ? nx : nx * ny;
  if (dtype == WN_F64)
    return back2d<double>((const double*)ctrl, nseg, L, kind, (const double*)x, (const double*)y, nx, n,
                          (const double*)gw, (double*)gq, (double*)gc, s);
  return back2d<float>((const float*)ctrl, nseg, L, kind, (const float*)x, (const float*)y, nx, n,
                       (const float*)gw, (float*)gq, (float*)gc, s);
}

}  // namespace wn
