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
struct VQ {
  float x, y;   // lam * X, lam * Y
  float a;      // lam * alpha
  float lz;     // lam * Z   (used by the depth test of the crossing kernel)
};

__device__ __forceinline__ VQ vertex_q(double Xv, double Yv, double Zv,
                                       double Xp, double Yp, double Zp) {
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
  q.x = __fmul_rn(lam, X);
  q.y = __fmul_rn(lam, Y);
  q.a = front ? rho2 : u;
  q.lz = __fmul_rn(lam, Z);
  return q;
}

// Edge predicate N(a, b) = Y_a X_b - X_a Y_b of the projected edge a->b
// relative to the ray (proportional to d.(b' x a')).  Both products are
// rounded before the subtraction, so N(b, a) = -N(a, b) bit for bit (IEEE
// round-to-nearest is symmetric); an exact zero is then resolved by the
// caller with `tie_zero`, which is antisymmetric as well.  Every triangle
// edge and every boundary edge goes through this one function.
__device__ __forceinline__ float edge_n(const VQ& a, const VQ& b) {
  return __fsub_rn(__fmul_rn(a.y, b.x), __fmul_rn(a.x, b.y));
}

// Lexicographic order of two rotated vertices; distinct float32 vertices
// have distinct rotated float64 coordinates.
__device__ __forceinline__ bool lex_less(double ax, double ay, double az,
                                         double bx, double by, double bz) {
  return ax < bx || (ax == bx && (ay < by || (ay == by && az < bz)));
}

// Signed zero that an exact N(a, b) == 0 is replaced with: the ray counts as
// passing on the side of the edge that its lexicographically smaller end
// point picks, which is opposite for the two orientations of the edge.
__device__ __forceinline__ float tie_zero(bool a_less_b) {
  return a_less_b ? -0.0f : 0.0f;
}

// Edge factor D + iN (up to the positive scale lam_a*lam_b): the angle
// theta_e = atan2(N, D) is half the signed solid angle of the spherical
// triangle (-d, a - p, b - p), i.e. the per-edge boundary term.
__device__ __forceinline__ float edge_d(const VQ& a, const VQ& b) {
  return __fmaf_rn(a.y, b.y, __fmaf_rn(a.x, b.x, __fmul_rn(a.a, b.a)));
}

// Running product of the edge factors with an exact count of turns:
// sum_e theta_e = arg(zr + i zi) + 2 pi k.  Multiplying by a factor whose
// angle lies in (-pi, pi] can carry the argument across the negative real
// axis; that happens exactly when the old product and the factor lie in the
// same closed half plane (by sign bit) and the new product in the other one.
// Using sign bits makes a signed-zero N select its branch the same way
// atan2 does.
struct Turns {
  float zr, zi;
  int k;
};

__device__ __forceinline__ void turns_init(Turns& t, float D, float N) {
  t.zr = D;
  t.zi = N;
  t.k = 0;
}

__device__ __forceinline__ void turns_mul(Turns& t, float D, float N) {
  const float nr = __fmaf_rn(t.zr, D, -__fmul_rn(t.zi, N));
  const float ni = __fmaf_rn(t.zr, N, __fmul_rn(t.zi, D));
  const int A = __float_as_int(t.zi);
  const int B = __float_as_int(N);
  const int C = __float_as_int(ni);
  const int up = (~A & ~B & C) >> 31;   // -1: turned forward past pi
  const int dn = (A & B & ~C) >> 31;    // -1: turned backward past -pi
  t.k += dn - up;
  t.zr = nr;
  t.zi = ni;
}

// Rescale by a power of two (exact; keeps signs and zeros).
__device__ __forceinline__ void turns_norm(Turns& t) {
  const float m = fmaxf(fabsf(t.zr), fabsf(t.zi));
  const int e = __builtin_amdgcn_frexp_expf(m);
  t.zr = __builtin_amdgcn_ldexpf(t.zr, -e);
  t.zi = __builtin_amdgcn_ldexpf(t.zi, -e);
}

// Combine two partial products (edge chunks of one query).
__device__ __forceinline__ void turns_join(Turns& t, const Turns& o) {
  const float nr = __fmaf_rn(t.zr, o.zr, -__fmul_rn(t.zi, o.zi));
  const float ni = __fmaf_rn(t.zr, o.zi, __fmul_rn(t.zi, o.zr));
  const int A = __float_as_int(t.zi);
  const int B = __float_as_int(o.zi);
  const int C = __float_as_int(ni);
  const int up = (~A & ~B & C) >> 31;
  const int dn = (A & B & ~C) >> 31;
  t.k += o.k + dn - up;
  t.zr = nr;
  t.zi = ni;
}

constexpr float kInv2Pi = 0.15915494309189535f;

// w = chi + k + atan2(zi, zr) / (2 pi).
__device__ __forceinline__ float turns_to_w(const Turns& t, int chi) {
  return (float)(chi + t.k) + atan2f(t.zi, t.zr) * kInv2Pi;
}

}  // namespace wn
