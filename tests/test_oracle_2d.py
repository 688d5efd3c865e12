"""Pins for the 2D FP64 oracle (CPU only).

``oracle.wn2d`` is tied to: adaptive quadrature of dtheta along each cubic
(the definition of w_C, Sec. 3) to the paper's 1e-10 misclassification bar
(Sec. 7, 2D parametric geometry), a dense unwrapped angle sum, exact integers
for closed loops against a polygon crossing test, the closed form for a
straight segment, and invariance under a change of d.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import wn2d as W


def _bez(c, t):
    s = 1.0 - t
    return (s ** 3)[..., None] * c[0] + (3 * s * s * t)[..., None] * c[1] \
        + (3 * s * t * t)[..., None] * c[2] + (t ** 3)[..., None] * c[3]


def quad_w(ctrl, p):
    """(1/2pi) sum over segments of int_0^1 (v x B'(t)) / |v|^2 dt, v = B(t) - p."""
    tot = 0.0
    for c in ctrl:
        def f(t, c=c):
            s = 1.0 - t
            B = s ** 3 * c[0] + 3 * s * s * t * c[1] + 3 * s * t * t * c[2] + t ** 3 * c[3]
            dB = 3 * (s * s * (c[1] - c[0]) + 2 * s * t * (c[2] - c[1]) + t * t * (c[3] - c[2]))
            v = B - p
            return (v[0] * dB[1] - v[1] * dB[0]) / (v @ v)
        tot += integrate.quad(f, 0.0, 1.0, epsabs=1e-13, epsrel=1e-13, limit=400)[0]
    return tot / (2.0 * math.pi)


def dense_polyline(ctrl, n=4000):
    t = np.linspace(0.0, 1.0, n)
    return [_bez(np.asarray(c, np.float64), t) for c in ctrl]


def curve_distance(ctrl, P, n=4000):
    pts = np.concatenate(dense_polyline(ctrl, n), 0)
    return np.array([np.sqrt(((pts - p) ** 2).sum(1)).min() for p in P])


def dense_angle_w(ctrl, p, n=20000):
    tot = 0.0
    for pts in dense_polyline(ctrl, n):
        v = pts - p
        a, b = v[:-1], v[1:]
        tot += np.sum(np.arctan2(a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0], (a * b).sum(1)))
    return tot / (2.0 * math.pi)


def test_star_matches_quadrature_and_is_integer():
    C = synth.star2d()
    P = synth.rng(1).uniform(-1.5, 1.5, (200, 2))
    far = curve_distance(C.ctrl, P) > 1e-3
    r = W.wn2d(C.ctrl, C.loop_off, C.closed, P)
    q = np.array([quad_w(C.ctrl, p) for p in P[far]])
    assert np.abs(r["w"][far] - q).max() < 1e-10
    assert set(np.unique(r["w"])) <= {0.0, 1.0}


def test_random_loops_match_quadrature():
    L = synth.loops2d(2, n_loops=5, seg_per_loop=8, n_open=2, dtype=np.float64)
    P = synth.rng(2).uniform(-1.2, 1.2, (60, 2))
    far = curve_distance(L.ctrl, P, 1500) > 1e-3
    r = W.wn2d(L.ctrl, L.loop_off, L.closed, P[far])
    q = np.array([quad_w(L.ctrl, p) for p in P[far]])
    np.testing.assert_allclose(r["w"], q, atol=1e-10, rtol=0)


def test_paper_2d_setup_zero_misclassified():
    # Sec. 7 (2D parametric geometry): random cubics with control points in the
    # unit square, a regular grid in each curve's bounding box, 0 points off by
    # more than 1e-10.  Scaled down: 8 curves, 24 x 24 grid each; rows and
    # columns through the bounding-box extremes hit end points exactly.
    g = synth.rng(3)
    bad = 0
    for _ in range(8):
        c = g.uniform(0.0, 1.0, (1, 4, 2))
        lo, hi = c[0].min(0), c[0].max(0)
        xs = np.linspace(lo[0], hi[0], 24)
        ys = np.linspace(lo[1], hi[1], 24)
        P = np.stack(np.meshgrid(xs, ys), -1).reshape(-1, 2)
        keep = curve_distance(c, P, 3000) > 1e-3
        r = W.wn2d(c, [0, 1], [0], P[keep])
        q = np.array([quad_w(c, p) for p in P[keep]])
        bad += int(np.sum(np.abs(r["w"] - q) > 1e-10))
    assert bad == 0


def test_dense_angle_sum():
    L = synth.loops2d(5, n_loops=3, seg_per_loop=5, n_open=2, dtype=np.float64)
    P = synth.rng(4).uniform(-1.0, 1.0, (20, 2))
    far = curve_distance(L.ctrl, P) > 2e-2
    r = W.wn2d(L.ctrl, L.loop_off, L.closed, P[far])
    dn = np.array([dense_angle_w(L.ctrl, p) for p in P[far]])
    np.testing.assert_allclose(r["w"], dn, atol=1e-6)


def test_closed_loops_match_polygon_crossing_parity_count():
    L = synth.loops2d(6, n_loops=4, seg_per_loop=8, n_open=0, dtype=np.float64)
    P = synth.rng(5).uniform(-1.0, 1.0, (200, 2))
    far = curve_distance(L.ctrl, P) > 1e-3
    r = W.wn2d(L.ctrl, L.loop_off, L.closed, P[far])
    # winding of the dense polygons (one per loop, consecutive samples joined
    # within a loop only): signed upward/downward crossings of the +x ray
    A, B = [], []
    for l in range(len(L.closed)):
        poly = np.concatenate(dense_polyline(L.ctrl[L.loop_off[l]:L.loop_off[l + 1]], 3000), 0)
        A.append(poly[:-1])
        B.append(poly[1:])
    a, b = np.concatenate(A, 0), np.concatenate(B, 0)
    for w, p in zip(r["w"], P[far]):
        ya, yb = a[:, 1] - p[1], b[:, 1] - p[1]
        up = (ya < 0) & (yb >= 0)
        dn = (ya >= 0) & (yb < 0)
        with np.errstate(divide="ignore", invalid="ignore"):
            xc = a[:, 0] + (b[:, 0] - a[:, 0]) * (-ya) / (yb - ya)
        right = xc > p[0]
        wind = int(np.sum(up & right)) - int(np.sum(dn & right))
        assert w == wind


def test_straight_segment_closed_form():
    g = synth.rng(6)
    for _ in range(20):
        a, b = g.uniform(-1, 1, 2), g.uniform(-1, 1, 2)
        c = np.stack([a, a + (b - a) / 3.0, a + 2.0 * (b - a) / 3.0, b])[None]
        p = g.uniform(-1, 1, 2)
        u, v = a - p, b - p
        expect = math.atan2(u[0] * v[1] - u[1] * v[0], u @ v) / (2.0 * math.pi)
        r = W.wn2d(c, [0, 1], [0], p[None], d=synth.random_direction(int(g.integers(99)))[:2])
        if r.degenerate[0]:
            continue
        assert abs(r["w"][0] - expect) < 1e-12


@pytest.mark.parametrize("d", [(0.0, 1.0), (-1.0, 0.0), (0.6, -0.8), (-0.3, -0.2)])
def test_direction_invariance(d):
    L = synth.loops2d(dtype=np.float64)
    P = synth.rng(7).uniform(-1.2, 1.2, (300, 2))
    a = W.wn2d(L.ctrl, L.loop_off, L.closed, P)
    b = W.wn2d(L.ctrl, L.loop_off, L.closed, P, d=d)
    ok = ~a.degenerate & ~b.degenerate
    np.testing.assert_allclose(b["w"][ok], a["w"][ok], atol=1e-12)


def test_reversal_negates():
    L = synth.loops2d(8, n_loops=5, seg_per_loop=6, n_open=3, dtype=np.float64)
    rev = []
    for l in range(5):
        seg = L.ctrl[L.loop_off[l]:L.loop_off[l + 1]]
        rev.append(seg[::-1, ::-1])
    R = np.concatenate(rev, 0)
    P = synth.rng(8).uniform(-1.2, 1.2, (300, 2))
    a = W.wn2d(L.ctrl, L.loop_off, L.closed, P)
    b = W.wn2d(R, L.loop_off, L.closed, P)
    ok = ~a.degenerate & ~b.degenerate
    np.testing.assert_allclose(b["w"][ok], -a["w"][ok], atol=1e-12)
