"""Pins of the curved-boundary oracle (oracle.curves3d) against what the
mathematics fixes independently of it:

* a straight Bezier (collinear control points, any speed along the segment)
  integrates to half the Van Oosterom-Strackee solid angle of the spherical
  triangle (-d, a - p, b - p), the textbook closed form;
* a planar region bounded by a loop of Beziers has w = Omega / (4 pi), Omega
  its signed solid angle, computed here from a fine fan triangulation (sum
  of triangle solid angles, Richardson-extrapolated); the oracle gives
  chi_d + Theta / (2 pi) with chi_d from a point-in-polygon test, for
  several directions d;
* Theta is additive under a de Casteljau split and changes sign when the
  curve is reversed.
"""
import math

import numpy as np

import synth
from oracle import curves3d as OC


def vos(a, b, c):
    """Signed solid angle of the triangle (a, b, c) seen from the origin
    (Van Oosterom and Strackee, 1983)."""
    la, lb, lc = np.linalg.norm(a), np.linalg.norm(b), np.linalg.norm(c)
    num = float(np.dot(a, np.cross(b, c)))
    den = la * lb * lc + float(np.dot(a, b)) * lc + float(np.dot(a, c)) * lb + float(np.dot(b, c)) * la
    return 2.0 * math.atan2(num, den)


def split(c, t):
    """de Casteljau split of a cubic at t: (left, right) control points."""
    p01, p12, p23 = (1 - t) * c[0] + t * c[1], (1 - t) * c[1] + t * c[2], (1 - t) * c[2] + t * c[3]
    p012, p123 = (1 - t) * p01 + t * p12, (1 - t) * p12 + t * p23
    m = (1 - t) * p012 + t * p123
    return np.array([c[0], p01, p012, m]), np.array([m, p123, p23, c[3]])


def test_straight_bezier_is_the_spherical_triangle():
    g = synth.rng(41)
    for _ in range(25):
        a, b, p = g.normal(size=3), g.normal(size=3), g.normal(size=3)
        d = synth.random_direction(int(g.integers(1 << 30)))
        s1, s2 = g.uniform(-0.3, 1.3, 2)          # any speed, even running backwards
        c = np.array([a, a + s1 * (b - a), a + s2 * (b - a), b])
        ref = 0.5 * vos(-d, a - p, b - p)
        ang, dist = OC.curve_margins(c[None], p[None], d)
        if ang[0] < 1e-3 or dist[0] < 1e-3:
            continue                              # ray or point too close to the segment
        assert abs(OC.curve_integral(c, p, d) - ref) < 1e-11


def _star_loop(seed, n_seg=6, z=0.0):
    """Closed, star-shaped loop of n_seg cubics in the plane z, CCW around
    the origin (control points at increasing angles, radii U[0.6, 1])."""
    g = synth.rng(seed)
    m = 3 * n_seg
    ang = np.sort(g.uniform(0, 2 * math.pi, m))
    rad = g.uniform(0.6, 1.0, m)
    pts = np.stack([rad * np.cos(ang), rad * np.sin(ang), np.full(m, z)], 1)
    return np.array([[pts[3 * i], pts[3 * i + 1], pts[3 * i + 2], pts[(3 * i + 3) % m]] for i in range(n_seg)])


def _fan_solid_angle(ctrl, p, n):
    ts = np.linspace(0, 1, n + 1)
    o = np.zeros(3)
    tot = 0.0
    for c in ctrl:
        G = OC.bezier(c, ts)
        for k in range(n):
            tot += vos(o - p, G[k] - p, G[k + 1] - p)
    return tot


def _inside(ctrl, q):
    """2D winding number of the densely sampled loop around q (0 or 1)."""
    G = np.concatenate([OC.bezier(c, np.linspace(0, 1, 4001))[:-1] for c in ctrl])[:, :2] - q[:2]
    a = np.arctan2(G[:, 1], G[:, 0])
    da = np.diff(np.concatenate([a, a[:1]]))
    da = (da + math.pi) % (2 * math.pi) - math.pi
    return int(round(da.sum() / (2 * math.pi)))


def test_planar_region_matches_fan_triangulation():
    ctrl = _star_loop(42)
    g = synth.rng(43)
    checked = 0
    for _ in range(40):
        p = np.array([g.uniform(-1.2, 1.2), g.uniform(-1.2, 1.2), g.choice([-1, 1]) * g.uniform(0.05, 0.8)])
        d = synth.random_direction(int(g.integers(1 << 30)))
        ang, dist = OC.curve_margins(ctrl, p[None], d)
        if ang[0] < 1e-3 or dist[0] < 1e-3:
            continue
        # chi_d: the ray meets the plane z = 0 at t = -p_z / d_z
        chi = 0
        if d[2] != 0 and -p[2] / d[2] > 0:
            q = p - (p[2] / d[2]) * d
            chi = _inside(ctrl, q) * (1 if d[2] > 0 else -1)
        w = chi + OC.curve_term(ctrl, p[None], d)[0] / (2 * math.pi)
        o1, o2 = _fan_solid_angle(ctrl, p, 256), _fan_solid_angle(ctrl, p, 512)
        ref = (4 * o2 - o1) / 3 / (4 * math.pi)
        assert abs(w - ref) < 1e-8, (p, d, w, ref)
        checked += 1
    assert checked >= 25


def test_split_additivity_and_reversal():
    g = synth.rng(44)
    for _ in range(10):
        c = g.normal(size=(4, 3))
        p = g.normal(size=3) * 1.5
        d = synth.random_direction(int(g.integers(1 << 30)))
        ang, dist = OC.curve_margins(c[None], p[None], d)
        if ang[0] < 1e-3 or dist[0] < 1e-3:
            continue
        whole = OC.curve_integral(c, p, d)
        l, r = split(c, 0.37)
        assert abs(OC.curve_integral(l, p, d) + OC.curve_integral(r, p, d) - whole) < 1e-11
        assert abs(OC.curve_integral(c[::-1], p, d) + whole) < 1e-11
