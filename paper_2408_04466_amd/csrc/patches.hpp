#pragma once

// Signed crossings of the ray p + t d (t > 0) with bicubic Bezier patches:
// chi_d of a parametric surface without tessellating it.
//
// Sec. 5.1 ("Parametric Surfaces") intersects each ray with the patch by a
// generic nonlinear solver, started on subintervals of the ray's clip by the
// patch's bounding box.  For polynomial patches the roots can be isolated
// instead (the paper points to specialised techniques there), and that is
// what runs here.  In the frame of d, with (X, Y, Z) the patch relative to
// the query, a crossing is a zero of (X, Y)(u, v) with Z > 0, counted with the
// sign of X_u Y_v - X_v Y_u = d . (S_u x S_v).
//
// Per query a stackless depth-first walk over dyadic sub-squares of every
// patch (state: patch, level, iu, iv):
//   * the sub-patch's Bernstein net is formed relative to the query: its
//     constant term S(u0, v0) - p in float64, the rest of the power basis
//     shifted and scaled in float32, then converted to Bernstein form;
//   * by the convex hull property the sub-patch holds no crossing when all
//     control values of X (or of Y) share one sign, or all Z are negative;
//   * when all its Z are positive (the sub-patch lies wholly in front of p)
//     and the (X, Y) hull of each of its four boundary edges excludes the
//     origin, the zeros inside it, each with the sign of the Jacobian, add up
//     to the winding number around the origin of the image of its boundary
//     (the degree of the map (X, Y) on the sub-square).  Each edge's image
//     then turns by less than pi, so the winding is the sum of the principal
//     angles between consecutive corner images, divided by 2 pi.  A fold,
//     where two zeros of opposite sign meet, needs no special care;
//   * otherwise the sub-patch is split in four, down to level 16.
#include "kernels.hpp"

namespace wn {

namespace {

constexpr int kPThreads = 256;
constexpr int kPatchChunk = 32;   // patches per LDS stage: 32 * 576 B = 18 KB
constexpr int kMaxLevel = 16;

// Power basis of a staged patch, per frame coordinate: S_c(u, v) =
// sum a[c][k][l] u^k v^l (float64, rotated frame, not relative).
struct PatchRot {
  double a[3][4][4];
  float f[3][4][4];   // the same coefficients rounded to float32 (the walk's Taylor shift)
};

// Bernstein -> power basis of a cubic: a0 = p0, a1 = 3 (p1 - p0),
// a2 = 3 (p2 - 2 p1 + p0), a3 = p3 - 3 p2 + 3 p1 - p0.
__device__ __forceinline__ void to_power(double& p0, double& p1, double& p2, double& p3) {
  const double a1 = 3.0 * (p1 - p0);
  const double a2 = 3.0 * ((p2 - p1) - (p1 - p0));
  const double a3 = (p3 - p0) - 3.0 * (p2 - p1);
  p1 = a1;
  p2 = a2;
  p3 = a3;
}

__device__ void stage_patch(const Frame& F, const float* __restrict__ nets, int64_t k, PatchRot* out) {
  double P[3][4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      const float* c = nets + 48 * k + 12 * i + 3 * j;
      rotate(F, c[0], c[1], c[2], P[0][i][j], P[1][i][j], P[2][i][j]);
    }
  for (int c = 0; c < 3; ++c) {
    for (int j = 0; j < 4; ++j) to_power(P[c][0][j], P[c][1][j], P[c][2][j], P[c][3][j]);
    for (int i = 0; i < 4; ++i) to_power(P[c][i][0], P[c][i][1], P[c][i][2], P[c][i][3]);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        out->a[c][i][j] = P[c][i][j];
        out->f[c][i][j] = (float)P[c][i][j];
      }
  }
}

__device__ __forceinline__ double eval0(const double (&a)[4][4], double u, double v) {
  double f = 0.0;
#pragma unroll
  for (int k = 3; k >= 0; --k)
    f = __fma_rn(f, u, __fma_rn(__fma_rn(__fma_rn(a[k][3], v, a[k][2]), v, a[k][1]), v, a[k][0]));
  return f;
}

// Cubic power basis on [0, 1] -> Bernstein coefficients.
__device__ __forceinline__ void to_bern(float& a0, float& a1, float& a2, float& a3) {
  constexpr float t = 1.f / 3.f;
  const float b1 = __fmaf_rn(a1, t, a0);
  const float b2 = __fmaf_rn(__fmaf_rn(2.f, a1, a2), t, a0);
  const float b3 = a0 + a1 + a2 + a3;
  a1 = b1;
  a2 = b2;
  a3 = b3;
}

// Bernstein net o[i][j] (i along u) of one coordinate on the sub-square
// [u0, u0 + h] x [v0, v0 + h], relative to the query coordinate pc.
__device__ __forceinline__ void subnet(const double (&a)[4][4], const float (&af)[4][4], double pc, double u0,
                                       double v0, float h, float (&o)[4][4]) {
  const float uf = (float)u0, vf = (float)v0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int l = 0; l < 4; ++l) o[k][l] = af[k][l];
  // Taylor shift to (u0, v0)
#pragma unroll
  for (int l = 0; l < 4; ++l)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 2; j >= i; --j) o[j][l] = __fmaf_rn(uf, o[j + 1][l], o[j][l]);
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 2; j >= i; --j) o[k][j] = __fmaf_rn(vf, o[k][j + 1], o[k][j]);
  // scale to the sub-square
  const float hp[4] = {1.f, h, h * h, h * h * h};
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int l = 0; l < 4; ++l) o[k][l] *= hp[k] * hp[l];
  o[0][0] = (float)(eval0(a, u0, v0) - pc);   // the constant term, relative first
#pragma unroll
  for (int k = 0; k < 4; ++k) to_bern(o[k][0], o[k][1], o[k][2], o[k][3]);
#pragma unroll
  for (int l = 0; l < 4; ++l) to_bern(o[0][l], o[1][l], o[2][l], o[3][l]);
}

__device__ __forceinline__ void range16(const float (&o)[4][4], float& lo, float& hi) {
  lo = hi = o[0][0];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      lo = fminf(lo, o[k][l]);
      hi = fmaxf(hi, o[k][l]);
    }
}

// All values strictly of one sign (beyond a rounding allowance).
__device__ __forceinline__ bool one_sign(float lo, float hi) {
  const float tol = 1e-6f * fmaxf(fabsf(lo), fabsf(hi));
  return lo > tol || hi < -tol;
}

// Is the origin inside (or on) the convex hull of four points?  A point of
// the hull of four points lies in the triangle of three of them.
__device__ __forceinline__ bool hull4_has_origin(const float (&x)[4], const float (&y)[4]) {
  float cr[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = i + 1; j < 4; ++j) {
      cr[i][j] = __fmaf_rn(x[i], y[j], -__fmul_rn(x[j], y[i]));
      cr[j][i] = -cr[i][j];
    }
  auto tri = [&](int i, int j, int k) {
    const float a = cr[i][j], b = cr[j][k], e = cr[k][i];
    return (a >= 0.f && b >= 0.f && e >= 0.f) || (a <= 0.f && b <= 0.f && e <= 0.f);
  };
  return tri(0, 1, 2) || tri(0, 1, 3) || tri(0, 2, 3) || tri(1, 2, 3);
}

// Does the (X, Y) hull of any of the four boundary edges of the net contain
// the origin?  If none does, each edge's image turns by less than pi around
// the origin.
__device__ __forceinline__ bool edge_hull_has_axis(const float (&X)[4][4], const float (&Y)[4][4]) {
  float ex[4], ey[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int a = e == 0 ? i : (e == 1 ? 3 : (e == 2 ? i : 0));
      const int b = e == 0 ? 0 : (e == 1 ? i : (e == 2 ? 3 : i));
      ex[i] = X[a][b];
      ey[i] = Y[a][b];
    }
    if (hull4_has_origin(ex, ey)) return true;
  }
  return false;
}

__device__ __forceinline__ float turn(float ax, float ay, float bx, float by) {
  return atan2_f32(__fmaf_rn(ax, by, -__fmul_rn(ay, bx)), __fmaf_rn(ax, bx, __fmul_rn(ay, by)));
}

// Winding number around the origin of the image of the sub-square's boundary
// (u0, v0) -> (u1, v0) -> (u1, v1) -> (u0, v1) -> (u0, v0), each edge turning
// by the principal angle between its end points (edge_hull_has_axis false).
__device__ __forceinline__ int boundary_winding(const float (&X)[4][4], const float (&Y)[4][4]) {
  const float t = turn(X[0][0], Y[0][0], X[3][0], Y[3][0]) + turn(X[3][0], Y[3][0], X[3][3], Y[3][3]) +
                  turn(X[3][3], Y[3][3], X[0][3], Y[0][3]) + turn(X[0][3], Y[0][3], X[0][0], Y[0][0]);
  return (int)rintf(t * kInv2Pi);
}

// Signed crossings of the staged patches sc[0, cnt) for the query at rotated
// (Xp, Yp, Zp).
__device__ int patches_chi(const PatchRot* sc, int cnt, double Xp, double Yp, double Zp) {
  int chi = 0;
  int j = 0, L = 0;
  uint32_t iu = 0, iv = 0;
  while (j < cnt) {
    const PatchRot& S = sc[j];
    const double hd = __builtin_ldexp(1.0, -L);
    const float h = (float)hd;
    const double u0 = (double)iu * hd, v0 = (double)iv * hd;
    bool descend = false;
    float X[4][4], Y[4][4];
    float lo, hi;
    subnet(S.a[0], S.f[0], Xp, u0, v0, h, X);
    range16(X, lo, hi);
    if (!one_sign(lo, hi)) {
      subnet(S.a[1], S.f[1], Yp, u0, v0, h, Y);
      range16(Y, lo, hi);
      if (!one_sign(lo, hi)) {
        float Zn[4][4];
        subnet(S.a[2], S.f[2], Zp, u0, v0, h, Zn);
        range16(Zn, lo, hi);
        const float tz = 1e-6f * fmaxf(fabsf(lo), fabsf(hi));
        if (hi > -tz) {
          bool done = false;
          if (lo > tz && !edge_hull_has_axis(X, Y)) {
            // wholly in front of p: the zeros inside, with their Jacobian
            // signs, add up to the winding number of the boundary's image
            chi += boundary_winding(X, Y);
            done = true;
          }
          if (!done && L < kMaxLevel) descend = true;
        }
      }
    }
    if (descend) {
      ++L;
      iu <<= 1;
      iv <<= 1;
      continue;
    }
    // next sub-square: up past last children (1, 1), then the next sibling
    while (L > 0 && (iu & 1u) && (iv & 1u)) {
      iu >>= 1;
      iv >>= 1;
      --L;
    }
    if (L == 0) {
      ++j;
      iu = iv = 0;
    } else {
      const uint32_t k = (((iu & 1u) << 1) | (iv & 1u)) + 1u;
      iu = (iu & ~1u) | (k >> 1);
      iv = (iv & ~1u) | (k & 1u);
    }
  }
  return chi;
}

}  // namespace
}  // namespace wn
