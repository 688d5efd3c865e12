// Device geometry shared by the crossing-count and boundary-integral kernels.
//
// Both kernels evaluate the same predicates through these functions, so the
// ray/triangle decision of chi_d (Eq. chi) and the branch of the per-edge
// boundary angle (Lemma 2: crossing the projected boundary changes chi by
// one) flip at exactly the same floating-point inputs.  The library is built
// with -ffp-contract=off, and every multiply-add that matters is spelled out.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wn {

// Frame of one ray direction d: centre c (float32-representable, so v - c of
// a float32 v is exact in float64) and rotation R with rows (e1, e2, d)
// scaled by a power of two (exact), row-major.  R maps d to +Z, so every ray
// of a call is vertical in this frame and coordinates are O(1).
struct Frame {
  double r[9];
  double c[3];
};

// Rotated float64 coordinates R (v - c) of a float32 point (fixed order).
__device__ __forceinline__ void rotate(const Frame& F, float x, float y, float z,
                                       double& X, double& Y, double& Z) {
  const double dx = (double)x - F.c[0];
  const double dy = (double)y - F.c[1];
  const double dz = (double)z - F.c[2];
  X = __fma_rn(F.r[0], dx, __fma_rn(F.r[1], dy, __dmul_rn(F.r[2], dz)));
  Y = __fma_rn(F.r[3], dx, __fma_rn(F.r[4], dy, __dmul_rn(F.r[5], dz)));
  Z = __fma_rn(F.r[6], dx, __fma_rn(F.r[7], dy, __dmul_rn(F.r[8], dz)));
}

// Rotated points as pairs of float32 (hi, lo): v = hi + lo to 2^-48
// relative.  A vertex (of the mesh or of the boundary) is stored in 32 bytes:
// xy = (Xh, Xl, Yh, Yl) and zt = (Zh, Zl, and the two words of a float64 that
// holds the tie offset of the edge leaving a boundary vertex, else 0).
struct alignas(16) RPt {
  float4 xy;
  float4 zt;
};

// A query in the frame (the same split).
struct QP {
  float xh, xl, yh, yl, zh, zl;
};

__device__ __forceinline__ float split_lo(double v, float h) { return (float)__dsub_rn(v, (double)h); }

__device__ __forceinline__ RPt make_rpt(double X, double Y, double Z, double tie) {
  const float xh = (float)X, yh = (float)Y, zh = (float)Z;
  RPt p;
  p.xy = make_float4(xh, split_lo(X, xh), yh, split_lo(Y, yh));
  const long long t = __double_as_longlong(tie);
  p.zt = make_float4(zh, split_lo(Z, zh), __int_as_float((int)(t & 0xffffffff)), __int_as_float((int)(t >> 32)));
  return p;
}

__device__ __forceinline__ QP make_qp(double X, double Y, double Z) {
  QP q;
  q.xh = (float)X;
  q.xl = split_lo(X, q.xh);
  q.yh = (float)Y;
  q.yl = split_lo(Y, q.yh);
  q.zh = (float)Z;
  q.zl = split_lo(Z, q.zh);
  return q;
}

__device__ __forceinline__ double rpt_tie(const RPt& p) {
  return __hiloint2double(__float_as_int(p.zt.w), __float_as_int(p.zt.z));
}

// The float64 value of a (hi, lo) pair (exact).
__device__ __forceinline__ double hilo(float h, float l) { return __dadd_rn((double)h, (double)l); }

// Difference of two split coordinates, rounded to float32: (vh - ph) + (vl -
// pl).  Relative to the exact difference it errs by at most about 2^-23 of
// its size, also when v and p are close (no cancellation), and it depends on
// the two points alone: every kernel and every edge or triangle that uses
// the vertex for this query sees the same value.
__device__ __forceinline__ float rel32(float vh, float vl, float ph, float pl) {
  return __fadd_rn(__fsub_rn(vh, ph), __fsub_rn(vl, pl));
}

// A vertex seen from a query, in the frame:
//   (X, Y, Z) relative offsets (float32, rel32);
//   alpha = r - Z, with r = |v - p|: the stereographic denominator of the
//   vertex seen from d (the region term of Eq. wn_discrete_sum, per edge, is
//   the angle of alpha_a alpha_b + X_a X_b + Y_a Y_b + i N).  It is evaluated
//   without cancellation as rho^2 / u + (|Z| - Z) with u = r + |Z| (= rho^2 /
//   (r + Z) for Z > 0 and r + |Z| for Z <= 0).
struct VQ {
  float x, y, a;
};

__device__ __forceinline__ float vertex_x(const RPt& v, const QP& p) { return rel32(v.xy.x, v.xy.y, p.xh, p.xl); }
__device__ __forceinline__ float vertex_y(const RPt& v, const QP& p) { return rel32(v.xy.z, v.xy.w, p.yh, p.yl); }
__device__ __forceinline__ float vertex_z(const RPt& v, const QP& p) { return rel32(v.zt.x, v.zt.y, p.zh, p.zl); }

__device__ __forceinline__ VQ vertex_q(const RPt& v, const QP& p) {
  VQ q;
  q.x = vertex_x(v, p);
  q.y = vertex_y(v, p);
  const float Z = vertex_z(v, p);
  const float rho2 = __fmaf_rn(q.x, q.x, __fmul_rn(q.y, q.y));
  const float s = __fmaf_rn(Z, Z, rho2);
  const float r = __builtin_amdgcn_sqrtf(s);
  const float u = __fadd_rn(r, fabsf(Z));
  q.a = __fmaf_rn(rho2, __builtin_amdgcn_rcpf(u), __fsub_rn(fabsf(Z), Z));
  return q;
}

// Edge predicate N(a, b) = Y_a X_b - X_a Y_b of the projected edge a->b
// relative to the ray (proportional to d.(b' x a')), from the float32
// offsets of its end points.  Both products are exact in float64 and the
// fused multiply-add rounds the exact difference once: N is correctly
// rounded, N(b, a) = -N(a, b) bit for bit, and N == 0 exactly when the two
// projected vertices are collinear with the ray.  The crossing count is thus
// decided exactly on the vertices' float32 offsets, a perturbation of each
// vertex by about 2^-23 of its distance that every triangle and the boundary
// share.  Every triangle edge goes through this function followed by
// `edge_tie`; the boundary walk (edge_n_walk) takes the sign from here
// whenever a float32 evaluation cannot certify it, so the crossing count and
// the branch of the boundary term flip at the same inputs.
__device__ __forceinline__ double edge_n(float ax, float ay, float bx, float by) {
  return __fma_rn((double)ay, (double)bx, -__dmul_rn((double)ax, (double)by));
}

// Lexicographic order of two stored vertices (on their split coordinates);
// distinct vertices have distinct splits.
__device__ __forceinline__ bool rpt_less(const RPt& a, const RPt& b) {
  const float av[6] = {a.xy.x, a.xy.y, a.xy.z, a.xy.w, a.zt.x, a.zt.y};
  const float bv[6] = {b.xy.x, b.xy.y, b.xy.z, b.xy.w, b.zt.x, b.zt.y};
#pragma unroll
  for (int k = 0; k < 6; ++k)
    if (av[k] != bv[k]) return av[k] < bv[k];
  return false;
}

// Tie offset of the directed edge a->b: -2^-1022 if a precedes b
// lexicographically, +2^-1022 otherwise (antisymmetric in a, b).  A nonzero
// N is at least 2^-298 in magnitude (a difference of products of float32
// values), so adding the offset changes nothing but an exact zero, which
// becomes a value whose sign picks the side of the lexicographically smaller
// end point.  N(a,b) + tie(a,b) stays exactly antisymmetric, so of two
// triangles sharing an edge exactly one claims a ray through it, and the
// boundary term breaks the tie the same way.
constexpr double kTie = 2.2250738585072014e-308;   // 2^-1022
__device__ __forceinline__ double tie_offset(bool a_less_b) {
  return a_less_b ? -kTie : kTie;
}

__device__ __forceinline__ double edge_tie(double n, double tie) {
  return __dadd_rn(n, tie);
}

// Edge factor D + iN: the angle theta_e = atan2(N, D) is half the signed
// solid angle of the spherical triangle (-d, a - p, b - p), i.e. the
// per-edge boundary term (D = alpha_a alpha_b + X_a X_b + Y_a Y_b, in
// float32: only N's sign has to be exact).
__device__ __forceinline__ float edge_d(const VQ& a, const VQ& b) {
  return __fmaf_rn(a.a, b.a, __fmaf_rn(a.x, b.x, __fmul_rn(a.y, b.y)));
}

// N of a boundary edge for the walk in float32, with the sign of
// edge_tie(edge_n(a, b), tie) (the triangles' predicate).  n = fl(Y_a X_b -
// fl(X_a Y_b)) is within |fl(X_a Y_b) - X_a Y_b| <= 2^-24 |p| (+ half the
// least subnormal) of a quantity with N's sign, and rounding keeps signs, so
// |n| > 2^-23 |p| + 2^-126 certifies sign(n) = sign(N) with N != 0.  Other
// lanes (the query within about 2^-23 of the projected edge's line, rare)
// take the exact float64 value with the tie offset (edge_n_exact); rounded
// to float32 it keeps its sign bit, also where it becomes a signed zero.
struct WalkN {
  float n;
  bool sure;
};

__device__ __forceinline__ WalkN edge_n_walk(const VQ& a, const VQ& b) {
  const float p = __fmul_rn(a.x, b.y);
  WalkN r;
  r.n = __fmaf_rn(a.y, b.x, -p);
  r.sure = fabsf(r.n) > __fmaf_rn(fabsf(p), 0x1p-23f, 0x1p-126f);
  return r;
}

__device__ __forceinline__ float edge_n_exact(const VQ& a, const VQ& b, double tie) {
  return (float)edge_tie(edge_n(a.x, a.y, b.x, b.y), tie);
}

// Running product of the edge factors with an exact count of turns:
// sum_e theta_e = arg(zr + i zi) + 2 pi k.  The product is kept in
// float32 and rescaled by a power of two every two edges (every edge for far
// queries): a factor is at most 2^1.5 r_a r_b in size, and two of them stay
// inside float32's range unless a factor is below 2^-62, i.e. the query lies
// within about 1e-19 (frame units) of the boundary, where w has no float32
// value anyway.  Multiplying by a factor whose angle lies in (-pi, pi]
// carries the argument across the negative real axis exactly when the old
// product and the factor lie in the same closed half plane (by sign bit)
// and the new product in the other one; the sign bits make the count agree
// with atan2's branch.  A factor with N = +-0 (a tie, or an exact N below
// float32's range) moves a product with zi != 0 by +-pi as its sign bit
// says; the product starts from 1 + (+0)i, for which the rule holds as well.
//
// The three sign bits of an edge are not combined edge by edge: the sign of
// each factor's N and of each new product's imaginary part are shifted into
// two bit registers (bacc, cacc) as the edges go by, and every group of at
// most 32 edges is decided at once (turns_flush): with the old product's
// sign a_j = c_(j-1), a turn backward past -pi is a_j & b_j & ~c_j and one
// forward past pi is ~a_j & ~b_j & c_j, counted by population counts into k
// (forward turns minus backward turns), kept as 2 k beside the last decided
// sign bit in one register.
struct Turns {
  float zr, zi;
  uint32_t bacc, cacc;   // sign bits of the group's N and new zi (newest in bit 0)
  int kc;                // 2 k + (zi's sign bit when the last group was decided), where
                         // k = turns forward past pi minus turns backward past -pi
};

__device__ __forceinline__ void turns_init(Turns& t) {
  t.zr = 1.0f;
  t.zi = 0.0f;
  t.bacc = 0u;
  t.cacc = 0u;
  t.kc = 0;
}

__device__ __forceinline__ void turns_mul(Turns& t, float D, float N) {
  const float nr = __fmaf_rn(t.zr, D, -__fmul_rn(t.zi, N));
  const float ni = __fmaf_rn(t.zr, N, __fmul_rn(t.zi, D));
  t.bacc = __builtin_amdgcn_alignbit(t.bacc, __float_as_uint(N), 31);
  t.cacc = __builtin_amdgcn_alignbit(t.cacc, __float_as_uint(ni), 31);
  t.zr = nr;
  t.zi = ni;
}

// One boundary edge a->b into the product.  The factor is multiplied in
// with the float32 N first; the rare lanes whose N's sign that value cannot
// certify redo the multiplication from the old product with the exact N
// (after the product, so that the common path stays one straight block).
__device__ __forceinline__ void turns_edge(Turns& t, const VQ& a, const VQ& b, double tie) {
  const WalkN w = edge_n_walk(a, b);
  const float D = edge_d(a, b);
  const float zr = t.zr, zi = t.zi;
  float N = w.n;
  float nr = __fmaf_rn(zr, D, -__fmul_rn(zi, N));
  float ni = __fmaf_rn(zr, N, __fmul_rn(zi, D));
  if (__builtin_expect(!w.sure, 0)) {
    N = edge_n_exact(a, b, tie);
    nr = __fmaf_rn(zr, D, -__fmul_rn(zi, N));
    ni = __fmaf_rn(zr, N, __fmul_rn(zi, D));
  }
  t.bacc = __builtin_amdgcn_alignbit(t.bacc, __float_as_uint(N), 31);
  t.cacc = __builtin_amdgcn_alignbit(t.cacc, __float_as_uint(ni), 31);
  // an empty statement that takes the bit registers as operands: the
  // compiler would otherwise defer the insertions to the end of an unrolled
  // run of edges and keep every edge's N and zi alive until then
  asm volatile("" : "+v"(t.bacc), "+v"(t.cacc));
  t.zr = nr;
  t.zi = ni;
}

// Decide the last n (1..32, the same for every lane) edges' turns.  The
// old sign of edge j of the group is the new sign of edge j - 1, i.e. cacc
// shifted by one, with the sign from before the group (bit 0 of kc)
// entering at the top; bacc restarts, cacc keeps running and its newest
// bit becomes bit 0 of kc.
__device__ __forceinline__ void turns_flush(Turns& t, int n) {
  const uint32_t m = n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u);
  const uint32_t a = __builtin_amdgcn_alignbit((uint32_t)t.kc, t.cacc, 1);
  const uint32_t b = t.bacc;           // zero above bit n - 1
  const uint32_t c = t.cacc & m;
  const int dk = __popc(~a & ~b & c) - __popc(a & b & ~c);
  t.kc = (int)((((uint32_t)t.kc + 2u * (uint32_t)dk) & ~1u) | (t.cacc & 1u));
  t.bacc = 0u;
}

// Rescale by a power of two (exact; keeps signs and zeros): with m = |zr| +
// |zi| in [2^E, 2^(E+1)), the float with exponent field (254 - (E + 127) -
// borrow) is 2^(-E) or 2^(-E-1), which brings m into [0.5, 2).  A product
// that has sunk below the normal range is scaled by at most 2^127.
__device__ __forceinline__ void turns_norm(Turns& t) {
  const uint32_t m = __float_as_uint(__fadd_rn(fabsf(t.zr), fabsf(t.zi)));
  const float sc = __uint_as_float((0x7F000000u - m) & 0x7F800000u);
  t.zr = __fmul_rn(t.zr, sc);
  t.zi = __fmul_rn(t.zi, sc);
}

constexpr float kInv2Pi = 0.15915494309189535f;

// atan2(y, x) in float32, written out operation by operation so that every
// kernel including it produces the same bits (a library atan2f may lower its
// internal division differently from one kernel to the next).  Octant
// reduction to |t| <= tan(pi/8): t = a/b, or (a - b)/(a + b) with pi/4 added
// back, where a <= b are |x| and |y|; then atan(t) = t P(t^2) with P of
// degree 4 and P(0) = 1, the minimax fit of atan(t) by t P(t^2) on that
// range, rounded to float32 (derived by fit_atan.py; absolute error 4.5e-8
// evaluated in float32, almost all of it float32 rounding).  One hardware
// reciprocal replaces the division.  The sign of the result is the sign bit of y, so
// on the negative real axis y = +0 gives +pi and y = -0 gives -pi.
__device__ __forceinline__ float atan2_f32(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float a = fminf(ax, ay), b = fmaxf(ax, ay);
  const bool big = a > __fmul_rn(0.41421356f, b);
  const float num = big ? __fsub_rn(a, b) : a;
  const float den = big ? __fadd_rn(a, b) : b;
  const float t = den > 0.0f ? __fmul_rn(num, __builtin_amdgcn_rcpf(den)) : 0.0f;
  const float s = __fmul_rn(t, t);
  float p = 0.078978031873703f;
  p = __fmaf_rn(p, s, -0.13842841982841492f);
  p = __fmaf_rn(p, s, 0.1997738480567932f);
  p = __fmaf_rn(p, s, -0.333331435918808f);
  p = __fmaf_rn(p, s, 1.0f);
  float r = __fmul_rn(t, p);
  if (big) r = __fadd_rn(r, 0.7853981633974483f);
  if (ay > ax) r = __fsub_rn(1.5707963267948966f, r);
  if (x < 0.0f) r = __fsub_rn(3.141592653589793f, r);
  return copysignf(r, y);
}

// w = chi + k + atan2(zi, zr) / (2 pi) (every turn flushed).  The
// branch on the negative real axis (+pi for zi = +0, -pi for zi = -0) is the
// one the turn count assumed.
__device__ __forceinline__ float turns_to_w(Turns t, int chi) {
  turns_norm(t);
  const float ang = atan2_f32(t.zi, t.zr);
  return __fadd_rn((float)(chi + (t.kc >> 1)), __fmul_rn(ang, kInv2Pi));
}

}  // namespace wn
