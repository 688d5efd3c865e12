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

// Per (query, vertex) quantities in the frame, relative to the query.
//   (X, Y, Z) = R (v - p): float64 difference of rotated coordinates, rounded
//   once to float32 (no cancellation for nearby points).
//   rho^2 = X^2 + Y^2, r = |v - p|, u = r + |Z|.
//   alpha = r - Z is the stereographic denominator of the vertex seen from d;
//   it is evaluated without cancellation by scaling the vertex with
//   lam = u when Z > 0 (then lam*alpha = rho^2) and lam = 1 otherwise
//   (alpha = u).  The edge terms are homogeneous of degree one in each
//   vertex's (X, Y, alpha), so a positive per-vertex scale changes neither
//   the angle of an edge nor the sign of any predicate.
// The scaled values are float32 numbers held in float64 registers, so the
// products of two of them in the edge terms below are exact.
struct VQ {
  double x, y;  // lam * X, lam * Y
  double a;     // lam * alpha
};

__device__ __forceinline__ VQ vertex_q(double Xv, double Yv, double Zv,
                                       double Xp, double Yp, double Zp, float* lz = nullptr) {
  const float X = (float)(Xv - Xp);
  const float Y = (float)(Yv - Yp);
  const float Z = (float)(Zv - Zp);
  const float rho2 = __fmaf_rn(X, X, __fmul_rn(Y, Y));
  const float s = __fmaf_rn(Z, Z, rho2);
  const float r = __builtin_amdgcn_sqrtf(s);
  const float u = __fadd_rn(r, fabsf(Z));
  const bool front = Z > 0.0f;
  const float lam = front ? u : 1.0f;
  VQ q;
  q.x = (double)__fmul_rn(lam, X);
  q.y = (double)__fmul_rn(lam, Y);
  q.a = (double)(front ? rho2 : u);
  if (lz) *lz = __fmul_rn(lam, Z);
  return q;
}

// Edge predicate N(a, b) = Y_a X_b - X_a Y_b of the projected edge a->b
// relative to the ray (proportional to d.(b' x a')).  The inputs are float32
// values, so X_a*Y_b is exact in float64 and the fused multiply-add rounds
// the exact difference once: N is correctly rounded, N(b, a) = -N(a, b) bit
// for bit, and N == 0 exactly when the two projected vertices are collinear
// with the ray.  Every triangle edge and every boundary edge goes through
// this one function followed by `edge_tie`.
__device__ __forceinline__ double edge_n(const VQ& a, const VQ& b) {
  return __fma_rn(a.y, b.x, -__dmul_rn(a.x, b.y));
}

// Lexicographic order of two rotated vertices; distinct float32 vertices
// have distinct rotated float64 coordinates.
__device__ __forceinline__ bool lex_less(double ax, double ay, double az,
                                         double bx, double by, double bz) {
  return ax < bx || (ax == bx && (ay < by || (ay == by && az < bz)));
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

// Edge factor D + iN (up to the positive scale lam_a*lam_b): the angle
// theta_e = atan2(N, D) is half the signed solid angle of the spherical
// triangle (-d, a - p, b - p), i.e. the per-edge boundary term.
__device__ __forceinline__ double edge_d(const VQ& a, const VQ& b) {
  return __fma_rn(a.y, b.y, __fma_rn(a.x, b.x, __dmul_rn(a.a, b.a)));
}

// Running product of the edge factors with an exact count of turns:
// sum_e theta_e = arg(zr + i zi) + 2 pi k.  The product is kept in float64
// (its magnitude changes by the factors' magnitudes; float64 range allows
// rescaling only every few edges).  Multiplying by a factor whose angle lies
// in (-pi, pi] carries the argument across the negative real axis exactly
// when the old product and the factor lie in the same closed half plane (by
// sign bit) and the new product in the other one; the sign bits make the
// count agree with atan2's branch.  The tie offset keeps N nonzero, so the
// product starts from 1 without losing the sign of a zero.
struct Turns {
  double zr, zi;
  int k;
};

__device__ __forceinline__ void turns_init(Turns& t) {
  t.zr = 1.0;
  t.zi = 0.0;
  t.k = 0;
}

__device__ __forceinline__ int hi_word(double x) {
  return (int)(__double_as_longlong(x) >> 32);
}

__device__ __forceinline__ void turns_mul(Turns& t, double D, double N) {
  const double nr = __fma_rn(t.zr, D, -__dmul_rn(t.zi, N));
  const double ni = __fma_rn(t.zr, N, __dmul_rn(t.zi, D));
  const int A = hi_word(t.zi);
  const int B = hi_word(N);
  const int C = hi_word(ni);
  const int up = (~A & ~B & C) >> 31;   // -1: turned forward past pi
  const int dn = (A & B & ~C) >> 31;    // -1: turned backward past -pi
  t.k += dn - up;
  t.zr = nr;
  t.zi = ni;
}

// Rescale by a power of two (exact; keeps signs and zeros).
__device__ __forceinline__ void turns_norm(Turns& t) {
  const int e = max(__builtin_amdgcn_frexp_exp(t.zr), __builtin_amdgcn_frexp_exp(t.zi));
  t.zr = __builtin_amdgcn_ldexp(t.zr, -e);
  t.zi = __builtin_amdgcn_ldexp(t.zi, -e);
}

// Combine two partial products (edge chunks of one query).
__device__ __forceinline__ void turns_join(Turns& t, const Turns& o) {
  const double nr = __fma_rn(t.zr, o.zr, -__dmul_rn(t.zi, o.zi));
  const double ni = __fma_rn(t.zr, o.zi, __dmul_rn(t.zi, o.zr));
  const int A = hi_word(t.zi);
  const int B = hi_word(o.zi);
  const int C = hi_word(ni);
  const int up = (~A & ~B & C) >> 31;
  const int dn = (A & B & ~C) >> 31;
  t.k += o.k + dn - up;
  t.zr = nr;
  t.zi = ni;
}

constexpr float kInv2Pi = 0.15915494309189535f;

// atan2(y, x) in float32, written out operation by operation so that every
// kernel including it produces the same bits (a library atan2f may lower its
// internal division differently from one kernel to the next).  Octant
// reduction to |t| <= tan(pi/8): t = a/b, or (a - b)/(a + b) with pi/4 added
// back, where a <= b are |x| and |y|; then atan(t) = t P(t^2) with P of
// degree 4, fitted here to atan(t)/t on that range by weighted least squares
// (absolute error 4e-8 evaluated in float32).  One hardware reciprocal
// replaces the division.  The sign of the result is the sign bit of y, so
// on the negative real axis y = +0 gives +pi and y = -0 gives -pi.
__device__ __forceinline__ float atan2_f32(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float a = fminf(ax, ay), b = fmaxf(ax, ay);
  const bool big = a > __fmul_rn(0.41421356f, b);
  const float num = big ? __fsub_rn(a, b) : a;
  const float den = big ? __fadd_rn(a, b) : b;
  const float t = den > 0.0f ? __fmul_rn(num, __builtin_amdgcn_rcpf(den)) : 0.0f;
  const float s = __fmul_rn(t, t);
  float p = 0.07993615418672562f;
  p = __fmaf_rn(p, s, -0.1385444849729538f);
  p = __fmaf_rn(p, s, 0.199747234582901f);
  p = __fmaf_rn(p, s, -0.3333280682563782f);
  p = __fmaf_rn(p, s, 1.0f);
  float r = __fmul_rn(t, p);
  if (big) r = __fadd_rn(r, 0.7853981633974483f);
  if (ay > ax) r = __fsub_rn(1.5707963267948966f, r);
  if (x < 0.0f) r = __fsub_rn(3.141592653589793f, r);
  return copysignf(r, y);
}

// w = chi + k + atan2(zi, zr) / (2 pi).  After a power-of-two rescale the
// larger component lies in [0.5, 1), so both round to float32 without
// overflow; a component that underflows keeps its sign bit, so the branch
// (+pi or -pi on the negative real axis) is the one the turn count assumed.
// The float32 angle is off by about 1e-7 rad, below the float32 rounding of
// w itself.
__device__ __forceinline__ float turns_to_w(Turns t, int chi) {
  turns_norm(t);
  const float ang = atan2_f32((float)t.zi, (float)t.zr);
  return __fadd_rn((float)(chi + t.k), __fmul_rn(ang, kInv2Pi));
}

}  // namespace wn
