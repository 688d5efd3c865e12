#pragma once

// Boundary term of w along cubic Bezier boundary curves (3D).
//
// For a surface bounded by loops of cubic Bezier curves, w = chi_d +
// Theta / (2 pi) with Theta the line integral over the curves of the form
// whose integral along a straight edge is the edge term atan2(N, D) of the
// polyline path (Sec. 5.1 "Exact Computations": region areas from boundary integrals, Gauss-Bonnet;
// Bezier boundaries need a numerical integral).  In the frame of d, with
// (X, Y, Z) the curve point relative to the query and r its distance,
//
//   omega = -(X dY - Y dX) / (2 r (r - Z))                      (form B)
//         = -dphi + (X dY - Y dX) / (2 r (r + Z))               (form A)
//
// (phi = atan2(Y, X); the two agree because rho^2 = (r - Z)(r + Z)).  Form B
// is singular only towards +d, form A only towards -d, and the -dphi of form
// A integrates exactly to the azimuth change between the panel's end points
// when the panel's projection stays in a half-plane around the d axis.
//
// Per query a depth-first walk over dyadic parameter panels of each curve in
// turn, with no stack (curve, panel index and depth are enough):
//   * the panel's power basis is formed in float64 from the query-relative
//     curve (a0 = c0 - p in float64, the other coefficients from the staged
//     rotated control points) and rounded once to float32, so every panel is
//     accurate relative to its own distance from p;
//   * a panel is integrated by 6-node Gauss-Legendre when its control points
//     lie farther from p than 1.5 times the control polygon's length: seen
//     from p the panel then lies within asin(2/3) < 42 degrees of its first
//     control point c0, so with form B when c0 is at or below p along d, else
//     with form A, the chosen form's singular direction stays more than 48
//     degrees away; form A also needs the control points' xy-hull to exclude
//     the d axis (the azimuth change is then the principal angle between the
//     end points);
//   * otherwise the panel is halved, down to 2^-24 of the curve, where the
//     chord's exact edge term stands in for the panel.
// chi_d comes from the caller or from the BVH traversal of the mesh whose
#include "bndloop.hpp"
#include "bvh_build.hpp"
#include "traverse.hpp"

namespace wn {

namespace {

constexpr int kCThreads = 256;
constexpr int kCurveChunk = 128;   // curves per LDS stage: 128 * 96 B = 12 KB
constexpr int kMaxDepth = 24;
constexpr float kFar = 1.5f;

// Gauss-Legendre, 6 nodes on [0, 1] (weights sum to 1).
constexpr int kGL = 6;
__constant__ float kGLs[kGL] = {0.033765242898423975f, 0.16939530676686776f, 0.38069040695840151f, 0.61930959304159849f, 0.83060469323313224f, 0.96623475710157603f};
__constant__ float kGLw[kGL] = {0.085662246189584873f, 0.18038078652406947f, 0.23395696728634569f, 0.23395696728634569f, 0.18038078652406947f, 0.085662246189584873f};

// A staged curve: rotated first control point and the power-basis
// coefficients of gamma(t) = c0 + a1 t + a2 t^2 + a3 t^3 (float64).
struct CurveRot {
  double c0[3];
  double a1[3], a2[3], a3[3];
};

__device__ __forceinline__ void stage_curve(const Frame& F, const float* __restrict__ ctrl, int64_t k,
                                            CurveRot* out) {
  double P[4][3];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float* c = ctrl + 12 * k + 3 * i;
    rotate(F, c[0], c[1], c[2], P[i][0], P[i][1], P[i][2]);
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    out->c0[j] = P[0][j];
    out->a1[j] = 3.0 * (P[1][j] - P[0][j]);
    out->a2[j] = 3.0 * ((P[2][j] - P[1][j]) - (P[1][j] - P[0][j]));
    out->a3[j] = (P[3][j] - P[0][j]) - 3.0 * (P[2][j] - P[1][j]);
  }
}

struct F3 {
  float x, y, z;
};

__device__ __forceinline__ float norm3(F3 a) {
  return __builtin_amdgcn_sqrtf(__fmaf_rn(a.x, a.x, __fmaf_rn(a.y, a.y, __fmul_rn(a.z, a.z))));
}
__device__ __forceinline__ F3 sub3(F3 a, F3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ float sq3(F3 a) { return __fmaf_rn(a.x, a.x, __fmaf_rn(a.y, a.y, __fmul_rn(a.z, a.z))); }

// Is the origin inside (or on) the convex hull of the xy-projections of c[4]?
// A point of the hull of four points lies in the triangle of three of them.
__device__ __forceinline__ bool hull_has_axis(const F3* c) {
  float cr[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = i + 1; j < 4; ++j) {
      cr[i][j] = __fmaf_rn(c[i].x, c[j].y, -__fmul_rn(c[j].x, c[i].y));
      cr[j][i] = -cr[i][j];
    }
  auto tri = [&](int i, int j, int k) {
    const float a = cr[i][j], b = cr[j][k], e = cr[k][i];
    return (a >= 0.f && b >= 0.f && e >= 0.f) || (a <= 0.f && b <= 0.f && e <= 0.f);
  };
  return tri(0, 1, 2) || tri(0, 1, 3) || tri(0, 2, 3) || tri(1, 2, 3);
}

// Exact edge term of the chord a -> b (query-relative, frame coordinates).
__device__ __forceinline__ float chord_term(F3 a, F3 b) {
  const float ra = norm3(a), rb = norm3(b);
  const float pa = __fmaf_rn(a.x, a.x, __fmul_rn(a.y, a.y)), pb = __fmaf_rn(b.x, b.x, __fmul_rn(b.y, b.y));
  const float aa = a.z > 0.f ? pa / (ra + a.z) : ra - a.z;
  const float ab = b.z > 0.f ? pb / (rb + b.z) : rb - b.z;
  const float N = __fmaf_rn(a.y, b.x, -__fmul_rn(a.x, b.y));
  const float D = __fmaf_rn(aa, ab, __fmaf_rn(a.x, b.x, __fmul_rn(a.y, b.y)));
  return atan2_f32(N, D);
}

// Gauss-Legendre of form A (sgn = +1, denominator r + Z) or form B (sgn = -1,
// denominator r - Z, integrand negated) over the panel with power basis b.
__device__ __forceinline__ float panel_gl(const F3* b, float sgn) {
  const F3 d2 = {2.f * b[2].x, 2.f * b[2].y, 2.f * b[2].z};
  const F3 d3 = {3.f * b[3].x, 3.f * b[3].y, 3.f * b[3].z};
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < kGL; ++k) {
    const float s = kGLs[k];
    const float X = __fmaf_rn(s, __fmaf_rn(s, __fmaf_rn(s, b[3].x, b[2].x), b[1].x), b[0].x);
    const float Y = __fmaf_rn(s, __fmaf_rn(s, __fmaf_rn(s, b[3].y, b[2].y), b[1].y), b[0].y);
    const float Z = __fmaf_rn(s, __fmaf_rn(s, __fmaf_rn(s, b[3].z, b[2].z), b[1].z), b[0].z);
    const float dX = __fmaf_rn(s, __fmaf_rn(s, d3.x, d2.x), b[1].x);
    const float dY = __fmaf_rn(s, __fmaf_rn(s, d3.y, d2.y), b[1].y);
    const float cr = __fmaf_rn(X, dY, -__fmul_rn(Y, dX));
    const float r = __builtin_amdgcn_sqrtf(__fmaf_rn(X, X, __fmaf_rn(Y, Y, __fmul_rn(Z, Z))));
    const float den = __fmul_rn(2.f * r, __fmaf_rn(sgn, Z, r));
    acc = __fmaf_rn(kGLw[k], __fmul_rn(cr, __builtin_amdgcn_rcpf(den)), acc);
  }
  return sgn * acc;
}

// Theta of the staged curves sc[0, cnt) for the query at rotated (Xp, Yp, Zp):
// one loop over (curve, panel) per lane, so that a lane that needs many
// panels on one curve and a lane that needs them on another do not wait for
// each other curve by curve.
__device__ double curves_theta(const CurveRot* sc, int cnt, double Xp, double Yp, double Zp) {
  double theta = 0.0;
  int j = 0, depth = 0;
  uint32_t idx = 0;
  double A0[3] = {sc[0].c0[0] - Xp, sc[0].c0[1] - Yp, sc[0].c0[2] - Zp};
  while (j < cnt) {
    const CurveRot& C = sc[j];
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
    bool done = false;
    if (m2 > fl * fl) {
      if (c[0].z <= 0.f) {
        theta += (double)panel_gl(b, -1.f);
        done = true;
      } else if (!hull_has_axis(c)) {
        const float dphi = atan2_f32(__fmaf_rn(c[0].x, c[3].y, -__fmul_rn(c[0].y, c[3].x)),
                                     __fmaf_rn(c[0].x, c[3].x, __fmul_rn(c[0].y, c[3].y)));
        theta += (double)(panel_gl(b, 1.f) - dphi);
        done = true;
      }
    }
    if (!done) {
      if (depth < kMaxDepth) {
        ++depth;
        idx <<= 1;
        continue;
      }
      theta += (double)chord_term(c[0], c[3]);
    }
    // next panel: up while this one is a right half, then to the right sibling
    while (depth > 0 && (idx & 1u)) {
      idx >>= 1;
      --depth;
    }
    if (depth > 0) {
      ++idx;
    } else if (++j < cnt) {   // curve finished: next curve
#pragma unroll
      for (int k = 0; k < 3; ++k) A0[k] = sc[j].c0[k] - (k == 0 ? Xp : (k == 1 ? Yp : Zp));
    }
  }
  return theta;
}

}  // namespace
}  // namespace wn
