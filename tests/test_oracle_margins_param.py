"""Pins for the degeneracy margins of the 2D, curve and patch oracles (CPU
only): the helpers that decide which queries the parity checks exempt.

As in tests/test_oracle_margins.py, each check is a function of the routine
it pins, so that the same check run on a planted mistake (a margin that is
not normalised, one that looks at the wrong side of the query, one that
counts exact ties) is shown to fail.  References: closed forms on straight
curves and flat or tilted patches, brute-force root finding and dense
sampling, and queries placed at known fractions of BAND.  The reading behind
the margins is Lemma 1 (Sec. 4) with the 2D example of its figure: chi
changes only where a crossing point, a joint or an open end point moves
across the ray, or where a crossing turns tangential.
"""
import math

import numpy as np
import pytest

import synth
from oracle import curves3d as CV
from oracle import patches3d as PT
from oracle import wn2d as W2


# ----------------------------------------------------------------------------
# 2D
# ----------------------------------------------------------------------------

def check_tangency(fn):
    # a straight piece at angle th to the ray's line, at any parametric speed
    for th in (0.3, 1.0, 1.5, 2.8, -0.7):
        for speed in (1.0, 3.0, 0.1):
            got = fn(np.array([speed * math.cos(th)]), np.array([speed * math.sin(th)]))[0]
            assert abs(got - abs(math.sin(th))) < 1e-15, (th, speed, got)


def check_crossing_margins(fn):
    # roots at x - p_x = -0.3 (left of p; the ray does not count it, and it is
    # nearly tangent) and 0.5 (right, counted)
    m_x, m_tan = fn(np.array([[-0.3, 0.5]]), np.array([1e-9, 0.7]))
    assert abs(m_x[0] - 0.3) < 1e-15 and m_tan[0] == 0.7
    # a root within BAND left of p still counts for the tangency
    m_x, m_tan = fn(np.array([[-0.5 * W2.BAND, 2.0]]), np.array([1e-9, 0.5]))
    assert m_x[0] == 0.5 * W2.BAND and m_tan[0] == 1e-9
    # no roots on the line
    m_x, m_tan = fn(np.zeros((3, 0)), np.zeros(0))
    assert np.all(np.isinf(m_x)) and np.all(np.isinf(m_tan))


def check_joint_margin(fn):
    ky = 0.3
    jx = np.array([0.5, -0.7, 2.0, 0.1, -0.5 * W2.BAND])
    jy = np.array([ky + 1e-7, ky + 1e-9, ky, ky, ky + 3e-8])
    # right of p: 1e-7 and two exact ties (decided by convention, not counted);
    # left of p: 1e-9 (not counted); within BAND left: 3e-8 (counted), but
    # 1.4 BAND left of the second query (not counted)
    got = fn(jx, jy, ky, np.array([0.0, 0.0 + 0.9 * W2.BAND]))
    assert got[0] == pytest.approx(3e-8, rel=1e-6)
    assert got[1] == pytest.approx(1e-7, rel=1e-6)
    got = fn(jx[:4], jy[:4], ky, np.array([0.0]))
    assert got[0] == pytest.approx(1e-7, rel=1e-6)
    assert np.isinf(fn(jx[2:4], jy[2:4], ky, np.array([0.0]))[0])


def test_2d_margin_helpers():
    check_tangency(W2.tangency)
    check_crossing_margins(W2.crossing_margins)
    check_joint_margin(W2.joint_margin)


def test_2d_margin_pins_catch_planted_mistakes():
    def unnormalised(xp, yp):
        return np.abs(yp)

    def nearest_right_only(dx, tang):
        m_x, m_tan = W2.crossing_margins(dx, tang)
        return np.where(dx > 0, dx, np.inf).min(1) if dx.shape[1] else m_x, m_tan

    def tangency_both_sides(dx, tang):
        m_x, _ = W2.crossing_margins(dx, tang)
        return m_x, (tang[None, :] + 0 * dx).min(1) if dx.shape[1] else m_x

    def joints_both_sides(jx, jy, ky, px):
        dj = np.abs(jy - ky)
        dj = np.where(dj == 0.0, np.inf, dj)
        return np.full(len(px), dj.min() if len(dj) else np.inf)

    def ties_count(jx, jy, ky, px):
        dj = np.abs(jy - ky)
        jd = np.where(jx[None, :] - px[:, None] > -W2.BAND, dj[None, :], np.inf)
        return jd.min(1)

    for check, bad in ((check_tangency, unnormalised), (check_crossing_margins, nearest_right_only),
                       (check_crossing_margins, tangency_both_sides), (check_joint_margin, joints_both_sides),
                       (check_joint_margin, ties_count)):
        with pytest.raises(AssertionError):
            check(bad)


def _bez(c, t):
    s = 1.0 - t
    return (s ** 3)[:, None] * c[0] + (3 * s * s * t)[:, None] * c[1] + (3 * s * t * t)[:, None] * c[2] + (t ** 3)[:, None] * c[3]


def _bez_d(c, t):
    s = 1.0 - t
    return (3 * s * s)[:, None] * (c[1] - c[0]) + (6 * s * t)[:, None] * (c[2] - c[1]) + (3 * t * t)[:, None] * (c[3] - c[2])


def brute_2d_margins(ctrl, loop_off, closed, P):
    """m_x, m_tan, m_joint for d = +x from sign changes of y(t) - p_y on 20001
    samples per segment, each refined by 60 bisection steps."""
    t = np.linspace(0.0, 1.0, 20001)
    m_x = np.full(len(P), np.inf)
    m_tan = np.full(len(P), np.inf)
    m_j = np.full(len(P), np.inf)
    joints = [c[0] for c in ctrl]
    for l in range(len(closed)):
        if not closed[l]:
            joints.append(ctrl[loop_off[l + 1] - 1][3])
    joints = np.array(joints)
    for i, p in enumerate(P):
        for c in ctrl:
            y = _bez(c, t)[:, 1] - p[1]
            for k in np.nonzero(np.sign(y[:-1]) * np.sign(y[1:]) < 0)[0]:
                lo, hi = t[k], t[k + 1]
                ylo = y[k]
                for _ in range(60):
                    mid = 0.5 * (lo + hi)
                    ym = _bez(c, np.array([mid]))[0, 1] - p[1]
                    if np.sign(ym) == np.sign(ylo):
                        lo, ylo = mid, ym
                    else:
                        hi = mid
                ts = np.array([0.5 * (lo + hi)])
                dx = _bez(c, ts)[0, 0] - p[0]
                m_x[i] = min(m_x[i], abs(dx))
                if dx > -W2.BAND:
                    v = _bez_d(c, ts)[0]
                    m_tan[i] = min(m_tan[i], abs(v[1]) / np.hypot(v[0], v[1]))
        dj = np.abs(joints[:, 1] - p[1])
        ok = (joints[:, 0] - p[0] > -W2.BAND) & (dj > 0)
        if ok.any():
            m_j[i] = dj[ok].min()
    return m_x, m_tan, m_j


def test_2d_margins_match_brute_force():
    C = synth.star2d(3)
    g = synth.rng(41)
    P = g.uniform(-1.2, 1.2, (40, 2))
    r = W2.wn2d(C.ctrl, C.loop_off, C.closed, P)
    bx, bt, bj = brute_2d_margins(C.ctrl, C.loop_off, C.closed, P)
    np.testing.assert_allclose(r["m_x"], bx, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(r["m_tan"], bt, rtol=1e-7, atol=1e-12)
    np.testing.assert_allclose(r["m_joint"], bj, rtol=0, atol=1e-15)
    # an open loop (end points count as joints)
    ctrl = np.array([[[0.0, -1.0], [0.3, -0.2], [0.8, 0.4], [1.0, 1.0]],
                     [[1.0, 1.0], [1.2, 1.3], [0.2, 1.5], [-0.4, 0.9]]])
    P = g.uniform(-1.0, 1.5, (30, 2))
    r = W2.wn2d(ctrl, np.array([0, 2]), np.array([0]), P)
    bx, bt, bj = brute_2d_margins(ctrl, np.array([0, 2]), np.array([0]), P)
    np.testing.assert_allclose(r["m_x"], bx, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(r["m_tan"], bt, rtol=1e-7, atol=1e-12)
    np.testing.assert_allclose(r["m_joint"], bj, rtol=0, atol=1e-15)


def test_2d_flagged_exactly_below_band():
    # one open straight piece from (1, -1) to (1, 1), d = +x
    ctrl = np.array([[[1.0, -1.0], [1.0, -1.0 / 3], [1.0, 1.0 / 3], [1.0, 1.0]]])
    lo, cl = np.array([0, 1]), np.array([0])
    B = W2.BAND
    # next to the crossing point
    r = W2.wn2d(ctrl, lo, cl, np.array([[1.0 - 0.5 * B, 0.2], [1.0 - 2.0 * B, 0.2], [1.0 + 0.5 * B, 0.2]]))
    assert list(r.degenerate) == [True, False, True]
    # a ray passing just below the upper end point (right of p)
    r = W2.wn2d(ctrl, lo, cl, np.array([[0.0, 1.0 - 0.5 * B], [0.0, 1.0 - 2.0 * B], [0.0, 1.0]]))
    assert list(r.degenerate) == [True, False, False]      # the exact tie is decided by convention
    # a nearly tangential crossing right of p
    ctrl_t = np.array([[[0.0, 0.0], [1.0, 0.5 * B], [2.0, B], [3.0, 1.5 * B]]])
    r = W2.wn2d(ctrl_t, np.array([0, 1]), np.array([0]), np.array([[-1.0, 0.75 * B]]))
    assert r["m_tan"][0] < B and r.degenerate[0]


# ----------------------------------------------------------------------------
# curves (boundary of curved surfaces and of patches)
# ----------------------------------------------------------------------------

def _straight(a, b, s1=0.1, s2=0.7):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.array([a, a + s1 * (b - a), a + s2 * (b - a), b])[None]


def check_curve_margins(fn):
    d = np.array([0.0, 0.0, 1.0])
    a, b = np.array([-1.0, 0.5, 2.0]), np.array([2.0, -0.5, 1.0])     # diag = |b - a|
    ctrl = _straight(a, b)
    diag = np.linalg.norm(b - a)
    g = synth.rng(42)
    P = g.uniform(-1.5, 1.5, (12, 3))
    ang, dist = fn(ctrl, P, d)
    from oracle import wn3d as W
    s = np.linspace(0.0, 1.0, 1000001)[:, None]
    pts = a + s * (b - a)
    for i, p in enumerate(P):
        want = W.segment_distance(p, a[None], b[None])[0] / diag
        assert abs(dist[i] - want) < 1e-10, (i, dist[i], want)
        v = pts - p
        z = v @ d
        front = z > 0
        ref = math.pi if not front.any() else float(np.arctan2(np.linalg.norm(v[front] - np.outer(z[front], d), axis=1), z[front]).min())
        assert abs(ang[i] - ref) < 1e-8, (i, ang[i], ref)
    # the whole curve behind the query: no angle margin
    ang, _ = fn(ctrl, np.array([[0.0, 0.0, 5.0]]), d)
    assert ang[0] == math.pi
    # queries whose ray passes beside the curve point above x = 0.5, offset by
    # 0.5e-5 and 4e-5 of the height (the angle to the tilted segment is a
    # little smaller than the offset): below and above the 1e-5 band
    hit = a + (0.5 - a[0]) / (b[0] - a[0]) * (b - a)
    for off, below in ((0.5e-5, True), (4e-5, False)):
        q = np.array([0.5, hit[1] + off * (hit[2] + 1.0), -1.0])
        ang, _ = fn(ctrl, q[None], d)
        assert 0.0 < ang[0] <= off and (ang[0] < 1e-5) == below, (off, ang[0])


def test_curve_margins():
    check_curve_margins(CV.curve_margins)


def test_curve_margin_pin_catches_planted_mistakes():
    def unnormalised(ctrl, P, d):
        ang, dist = CV.curve_margins(ctrl, P, d)
        pts = np.asarray(ctrl).reshape(-1, 3)
        return ang, dist * np.linalg.norm(pts.max(0) - pts.min(0))

    def with_points_behind(ctrl, P, d):
        # the angle over every curve point, also those behind the query
        ang, dist = CV.curve_margins(ctrl, P, d)
        ts = np.linspace(0, 1, 20001)
        out = ang.copy()
        for i, p in enumerate(np.asarray(P, float)):
            for c in np.asarray(ctrl, float):
                v = CV.bezier(c, ts) - p
                cosang = (v @ d) / np.linalg.norm(v, axis=1)
                out[i] = min(out[i], float(np.arccos(np.clip(cosang, -1, 1)).min()))
        return out, dist

    def full_length_angle(ctrl, P, d):
        # |v| where |v_perp| belongs: atan2(|v|, z)
        ang, dist = CV.curve_margins(ctrl, P, d)
        ts = np.linspace(0, 1, 20001)
        out = np.full(len(P), math.pi)
        for i, p in enumerate(np.asarray(P, float)):
            for c in np.asarray(ctrl, float):
                v = CV.bezier(c, ts) - p
                z = v @ d
                f = z > 0
                if f.any():
                    out[i] = min(out[i], float(np.arctan2(np.linalg.norm(v[f], axis=1), z[f]).min()))
        return out, dist

    for bad in (unnormalised, with_points_behind, full_length_angle):
        with pytest.raises(AssertionError):
            check_curve_margins(bad)


# ----------------------------------------------------------------------------
# patches
# ----------------------------------------------------------------------------

def _bilinear_net(S):
    """Bicubic net of the map (u, v) -> S(u, v) for an affine S."""
    k = np.arange(4) / 3.0
    U, V = np.meshgrid(k, k, indexing="ij")
    return np.stack([S(u, v) for u, v in zip(U.ravel(), V.ravel())]).reshape(4, 4, 3)


def check_patch_margin(fn):
    d = np.array([0.0, 0.0, 1.0])
    flat = _bilinear_net(lambda u, v: np.array([u, v, 0.0]))
    # the parameter distance of the hit to the square's boundary
    for u0, v0 in ((0.3, 0.6), (0.02, 0.5), (0.5, 0.97)):
        m = fn(flat[None], np.array([[u0, v0, -1.0]]), d).margin[0]
        assert abs(m - min(u0, 1 - u0, v0, 1 - v0)) < 1e-9, (u0, v0, m)
    # a tilted, stretched patch: |d . n| / |n| = |cos th| with n = S_u x S_v
    th = 1.2
    tilt = _bilinear_net(lambda u, v: np.array([2.0 * u, 2.0 * v * math.cos(th), 2.0 * v * math.sin(th)]))
    c = fn(tilt[None], np.array([[1.0, 1.0 * math.cos(th), -5.0]]), d)
    assert c.chi[0] != 0 and abs(c.margin[0] - abs(math.cos(th))) < 1e-9, c.margin[0]
    # the query next to the surface: |S - p| over the patch's size
    h = 3e-6
    big = _bilinear_net(lambda u, v: np.array([2.0 * u, 2.0 * v, 0.0]))
    p = np.array([[1.0, 1.0, -h]])
    size = np.linalg.norm((big.reshape(-1, 3) - p).max(0) - (big.reshape(-1, 3) - p).min(0))
    m = fn(big[None], p, d).margin[0]
    assert abs(m - h / size) < 1e-12, (m, h / size)
    assert fn(big[None], p, d).degenerate[0]
    # a ray that misses the patch has no crossing margin (the boundary curves'
    # margins cover near misses, below)
    assert np.isinf(fn(flat[None], np.array([[1.0 + 1e-3, 0.5, -1.0]]), d).margin[0])


def test_patch_margin():
    check_patch_margin(PT.patch_crossings)


def test_patch_margin_pin_catches_planted_mistakes(monkeypatch):
    def unnormalised_normal(u, v, S, n, size):
        return min(u, 1 - u, v, 1 - v, abs(n[2]), np.linalg.norm(S) / size)

    def absolute_distance(u, v, S, n, size):
        return min(u, 1 - u, v, 1 - v, abs(n[2]) / np.linalg.norm(n), np.linalg.norm(S))

    def no_boundary_term(u, v, S, n, size):
        return min(abs(n[2]) / np.linalg.norm(n), np.linalg.norm(S) / size)

    for bad in (unnormalised_normal, absolute_distance, no_boundary_term):
        with monkeypatch.context() as m:
            m.setattr(PT, "zero_margin", bad)
            with pytest.raises(AssertionError):
                check_patch_margin(PT.patch_crossings)


def test_ray_just_outside_a_patch_is_flagged_by_its_boundary_curves():
    # the parity tests combine the patch margin with curve_margins of the
    # patch's boundary curves: a ray passing 0.5 BAND (angle) outside the edge
    # u = 1 of a flat patch is flagged by the latter
    flat = _bilinear_net(lambda u, v: np.array([u, v, 0.0]))
    edge = flat[3][None]                               # the boundary curve u = 1
    d = np.array([0.0, 0.0, 1.0])
    for off, flagged in ((0.5e-5, True), (4e-5, False)):
        p = np.array([[1.0 + off, 0.5, -1.0]])
        assert not PT.patch_crossings(flat[None], p, d).degenerate[0]
        ang, dist = CV.curve_margins(edge, p, d)
        assert (ang[0] < 1e-5) == flagged, (off, ang[0])
