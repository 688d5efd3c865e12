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
//  * grid mode: the paper's one-shot reuse (Sec. 4 "Optimization"; Sec. 6,
//    2D results): one workgroup per (row, column tile) solves each piece that
//    crosses the row once, bins the crossing by the number of grid columns
//    left of it (an LDS histogram of integer counts), and a suffix scan gives
//    chi for every column of the row.
// Both modes decide "crossing right of p" as p_x < clamp(x*, xmin, xmax) with
// the same solver, so they agree bit for bit.
#include <cmath>

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
__global__ void k_pieces(const T* __restrict__ ctrl, int32_t nseg, Piece<T>* __restrict__ out,
                         typename Vec2<T>::type* __restrict__ yr) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  const T* P = ctrl + 8 * (int64_t)s;
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
    out[3 * (int64_t)s + k] = pc;
    yr[3 * (int64_t)s + k] = {pc.y0, pc.y1};
  }
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
    T tn = (fp != (T)0) ? t - f / fp : (T)0.5 * (lo + hi);
    const T a = fmin(lo, hi), b = fmax(lo, hi);
    if (!(tn > a && tn < b)) tn = (T)0.5 * (lo + hi);
    if (tn == t || b - a <= (T)4 * (sizeof(T) == 4 ? (T)1.2e-7 : (T)2.3e-16) * fmax((T)1, fabs(b))) {
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

template <class T> __device__ __forceinline__ T atan2_t(T y, T x);
template <> __device__ __forceinline__ float atan2_t<float>(float y, float x) { return atan2_f32(y, x); }
template <> __device__ __forceinline__ double atan2_t<double>(double y, double x) { return atan2(y, x); }

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
template <class T>
__device__ __forceinline__ T open_loop_angle(T sx, T sy, T ex, T ey) {
  const T cr = fma_t(sx, ey, -(sy * ex));
  const T dt = fma_t(sx, ex, sy * ey);
  if (cr == (T)0 && dt < (T)0) {
    const bool e_upper = ey > (T)0 || (ey == (T)0 && ex > (T)0);
    return e_upper ? -(T)3.141592653589793 : (T)3.141592653589793;
  }
  const T th = atan2_t(cr, dt);
  const bool s_above = sy >= (T)0, e_above = ey >= (T)0;
  if (!s_above && e_above && cr > (T)0) return th - (T)6.283185307179586;
  if (s_above && !e_above && cr < (T)0) return th + (T)6.283185307179586;
  return th;
}

// sum over open loops of phi(end - p) - phi(start - p)
template <class T>
__device__ T endpoint_term(const T* __restrict__ ctrl, const Loops2D& L, T px, T py) {
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

template <class T>
__global__ __launch_bounds__(kThreads) void k_points(const Piece<T>* __restrict__ pcs, int32_t npc,
                                                     const T* __restrict__ ctrl, Loops2D L,
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
  w[q] = (T)c + e * (T)0.15915494309189535;
  if (chi) chi[q] = c;
}

constexpr int kColTile = 4096;
constexpr int kSolveChunk = 1024;   // pieces examined per pass (LDS list of those needing a solve)

// One workgroup per (row, column tile).  Histogram slot c (0..ncol) counts the
// crossings with exactly c tile columns left of them; columns at or beyond
// the tile end get every crossing right of the whole tile through `base`.
// Pieces are examined in chunks: a first pass settles the pieces that miss
// the row or lie beside the whole tile and lists the others in LDS, so that
// the Newton solves run on consecutive lanes without idle lanes in between.
// All counts are integer additions, so their order does not matter.
template <class T>
__global__ __launch_bounds__(kThreads) void k_grid(const Piece<T>* __restrict__ pcs,
                                                   const typename Vec2<T>::type* __restrict__ yr, int32_t npc,
                                                   const T* __restrict__ ctrl, Loops2D L,
                                                   const T* __restrict__ x, int64_t nx,
                                                   const T* __restrict__ y, int64_t ny,
                                                   T* __restrict__ w, int32_t* __restrict__ chi, int tile) {
  // dynamic LDS sized to the tile: sx [tile] T, hist [tile + 1] int
  extern __shared__ __align__(16) unsigned char dyn[];
  T* sx = reinterpret_cast<T*>(dyn);
  int* hist = reinterpret_cast<int*>(sx + tile);
  __shared__ int sscan[kThreads];
  __shared__ int list[kSolveChunk];
  __shared__ int nlist;
  const int64_t row = blockIdx.y;
  const int64_t i0 = (int64_t)blockIdx.x * tile;
  const int ncol = (int)min((int64_t)tile, nx - i0);
  const T yq = y[row];
  for (int i = threadIdx.x; i < ncol; i += kThreads) sx[i] = x[i0 + i];
  for (int i = threadIdx.x; i <= ncol; i += kThreads) hist[i] = 0;
  __syncthreads();
  const T xlo = sx[0], xhi = sx[ncol - 1];
  int base = 0;   // crossings right of every column of the tile
  for (int c0 = 0; c0 < npc; c0 += kSolveChunk) {
    const int c1 = min(c0 + kSolveChunk, npc);
    if (threadIdx.x == 0) nlist = 0;
    __syncthreads();
    for (int j = c0 + threadIdx.x; j < c1; j += kThreads) {
      const typename Vec2<T>::type e = yr[j];
      const bool s0 = e.x >= yq, s1 = e.y >= yq;
      if (s0 == s1) continue;
      const int sg = s1 ? 1 : -1;
      const T pxmin = pcs[j].xmin, pxmax = pcs[j].xmax;
      if (xhi < pxmin) base += sg;                     // right of every column
      else if (xlo < pxmax) list[atomicAdd(&nlist, 1)] = j;   // needs the solve
      // else: right of no column
    }
    __syncthreads();
    const int n = nlist;
    for (int k = threadIdx.x; k < n; k += kThreads) {
      const int j = list[k];
      const Piece<T>& pc = pcs[j];
      const int sg = yr[j].y >= yq ? 1 : -1;
      const T xs = solve_x(pc, yq);
      const T xe = fmin(fmax(xs, pc.xmin), pc.xmax);
      // number of tile columns with x_i < xe (x ascending)
      int a = 0, b = ncol;
      while (a < b) {
        const int mid = (a + b) >> 1;
        if (sx[mid] < xe) a = mid + 1; else b = mid;
      }
      if (a == ncol) base += sg;
      else if (a > 0) atomicAdd(&hist[a], sg);
    }
    __syncthreads();
  }
  // block-wide sum of `base`
  sscan[threadIdx.x] = base;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sscan[threadIdx.x] += sscan[threadIdx.x + s];
    __syncthreads();
  }
  const int btot = sscan[0];
  __syncthreads();
  // chi(col i) = btot + sum_{c > i} hist[c]: suffix sums over [1, ncol),
  // each thread owning a contiguous block of columns
  const int per = (ncol + kThreads - 1) / kThreads;
  const int a0 = threadIdx.x * per;
  const int a1 = min(a0 + per, ncol);
  int part = 0;
  for (int c = a0 + 1; c <= a1 && c < ncol; ++c) part += hist[c];
  sscan[threadIdx.x] = part;
  __syncthreads();
  // exclusive suffix offsets: sum of parts of later threads
  for (int s = 1; s < kThreads; s <<= 1) {
    const int v = ((int)threadIdx.x + s < kThreads) ? sscan[threadIdx.x + s] : 0;
    __syncthreads();
    sscan[threadIdx.x] += v;
    __syncthreads();
  }
  int run = btot + (((int)threadIdx.x + 1 < kThreads) ? sscan[threadIdx.x + 1] : 0);
  // walk this thread's columns from the right; chi(i) replaces hist[i + 1],
  // which no thread reads after this point (thread blocks are disjoint and
  // the slot is read just before it is overwritten)
  for (int i = a1 - 1; i >= a0; --i) {
    if (i + 1 < ncol) run += hist[i + 1];
    hist[i + 1] = run;
  }
  __syncthreads();
  // coalesced output: consecutive lanes write consecutive columns
  for (int i = threadIdx.x; i < ncol; i += kThreads) {
    const int64_t o = row * nx + i0 + i;
    const T px = sx[i];
    if (!(isfinite(px) && isfinite(yq))) {
      w[o] = (T)NAN;
      if (chi) chi[o] = WN_CHI_INVALID;
      continue;
    }
    const int c = hist[i + 1];
    const T e = endpoint_term(ctrl, L, px, yq);
    w[o] = (T)c + e * (T)0.15915494309189535;
    if (chi) chi[o] = c;
  }
}

// ---------------------------------------------------------------------------
// Adjoint.  Away from the curves chi is locally constant, so w moves only
// with the open loops' end-point angles; with A(v) = (-v_y, v_x)/|v|^2 (the
// gradient of the angle of v) and c = g/(2 pi) per query:
//   dL/dp += c (A(s - p) - A(e - p)),  dL/ds -= c A(s - p),  dL/de += c A(e - p).
// Interior control points and closed loops get zero.  Per workgroup the
// end-point sums are reduced in LDS by a fixed-order tree in float64 and
// stored value-major (part[value][block]); a second kernel adds the blocks
// in a fixed order, so grad_ctrl is bitwise reproducible.
// ---------------------------------------------------------------------------

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
                                                     double* __restrict__ part, int64_t nblocks) {
  __shared__ double red[4][kThreads];
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool ok = q < n;
  T px = (T)0, py = (T)0, g = (T)0;
  if (ok) {
    px = kind == 0 ? x[q] : x[q % nx];
    py = kind == 0 ? y[q] : y[q / nx];
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
      red[0][threadIdx.x] = -(double)(c * asx);
      red[1][threadIdx.x] = -(double)(c * asy);
      red[2][threadIdx.x] = (double)(c * aex);
      red[3][threadIdx.x] = (double)(c * aey);
      __syncthreads();
      for (int h = kThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
          for (int j = 0; j < 4; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + h];
        __syncthreads();
      }
      if (threadIdx.x < 4) part[((int64_t)k * 4 + threadIdx.x) * nblocks + blockIdx.x] = red[threadIdx.x][0];
      __syncthreads();
    }
    ++k;
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

// One workgroup per end-point value v = 4 k + j (k-th open loop; j: start x,
// start y, end x, end y): fixed-order sum over the blocks, into its grad_ctrl
// entry.
template <class T>
__global__ __launch_bounds__(kThreads) void k_back2d_sum(const double* __restrict__ part, int64_t nblocks,
                                                         Loops2D L, T* __restrict__ gc) {
  __shared__ double red[kThreads];
  const double* p = part + (int64_t)blockIdx.x * nblocks;
  double sacc = 0.0;
  for (int64_t b = threadIdx.x; b < nblocks; b += kThreads) sacc += p[b];
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
  double* part = nullptr;   // [4 nopen][nblocks] float64 partial sums
  if (gc && nopen > 0) {
    e = hipMallocAsync((void**)&part, (size_t)nopen * 4 * nblocks * sizeof(double), s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_back2d<T>, dim3((unsigned)nblocks), dim3(kThreads), 0, s, ctrl, L, kind, x, y, nx, n, gw, gq,
                     part, nblocks);
  e = hipGetLastError();
  if (e == hipSuccess && part) {
    hipLaunchKernelGGL(k_back2d_sum<T>, dim3((unsigned)(4 * nopen)), dim3(kThreads), 0, s, part, nblocks, L, gc);
    e = hipGetLastError();
  }
  if (part) hipFreeAsync(part, s);
  return e;
}

template <class T>
hipError_t run2d(const T* ctrl, int64_t nseg, const Loops2D& L, int32_t kind, const T* x, const T* y,
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
      hipLaunchKernelGGL(k_points<T>, dim3((unsigned)((nx + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                         pcs, (int32_t)npc, ctrl, L, x, y, nx, w, chi);
    } else {
      // tiles of at most kColTile columns, as even as possible; LDS sized to the tile
      const int64_t ntiles = (nx + kColTile - 1) / kColTile;
      const int tile = (int)((nx + ntiles - 1) / ntiles);
      const size_t lds = ((size_t)tile * sizeof(T) + (size_t)(tile + 1) * sizeof(int) + 15) & ~(size_t)15;
      hipLaunchKernelGGL(k_grid<T>, dim3((unsigned)ntiles, (unsigned)ny), dim3(kThreads), lds, s, pcs, yr,
                         (int32_t)npc, ctrl, L, x, nx, y, ny, w, chi, tile);
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

hipError_t eval_2d(int32_t dtype, const void* ctrl, int64_t nseg, const int64_t* loop_off,
                   const uint8_t* closed, int32_t nloops, int32_t kind, const void* x, const void* y,
                   int64_t nx, int64_t ny, void* w, int32_t* chi, hipStream_t s) {
  Loops2D L;
  L.n = nloops;
  for (int l = 0; l <= nloops; ++l) L.off[l] = (int32_t)loop_off[l];
  for (int l = 0; l < nloops; ++l) L.closed[l] = closed[l] ? 1 : 0;
  if (dtype == WN_F64)
    return run2d<double>((const double*)ctrl, nseg, L, kind, (const double*)x, (const double*)y, nx, ny,
                         (double*)w, chi, s);
  return run2d<float>((const float*)ctrl, nseg, L, kind, (const float*)x, (const float*)y, nx, ny, (float*)w,
                      chi, s);
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
