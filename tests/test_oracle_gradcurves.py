"""Pins of the curve-gradient oracle (oracle.gradcurves): central differences
of the curve-term oracle, closed polygons as straight Beziers against the
polyline gradient oracle, and translation invariance."""
import math

import numpy as np

import synth
from oracle import curves3d as OC
from oracle import grad3d as G3
from oracle import gradcurves as GC


def _w(curves, p, d):
    return OC.curve_term(curves, p[None], d)[0] / (2 * math.pi)


def test_central_differences():
    M = synth.coons_surface(61, 300, 16)
    curves = M.info["curves"]
    d = synth.random_direction(62)
    g = synth.rng(63)
    h = 1e-5
    checked = 0
    for _ in range(8):
        p = synth.box_queries(M.V, 1, int(g.integers(1 << 30)))[0].astype(np.float64)
        ang, dist = OC.curve_margins(curves, p[None], d)
        if ang[0] < 1e-2 or dist[0] < 5e-2:
            continue
        gp, gc = GC.grad_curves(curves, p[None])
        fd = np.array([(_w(curves, p + h * e, d) - _w(curves, p - h * e, d)) / (2 * h) for e in np.eye(3)])
        assert np.allclose(gp[0], fd, rtol=1e-5, atol=1e-7), (gp[0], fd)
        j, k = int(g.integers(4)), int(g.integers(4))
        fdc = []
        for e in np.eye(3):
            cp, cm = curves.copy(), curves.copy()
            cp[j, k] += h * e
            cm[j, k] -= h * e
            # keep the loop closed: a shared end point moves with its neighbour
            if k == 0:
                cp[(j - 1) % 4, 3] += h * e
                cm[(j - 1) % 4, 3] -= h * e
            if k == 3:
                cp[(j + 1) % 4, 0] += h * e
                cm[(j + 1) % 4, 0] -= h * e
            fdc.append((_w(cp, p, d) - _w(cm, p, d)) / (2 * h))
        want = gc[j, k].copy()
        if k == 0:
            want += gc[(j - 1) % 4, 3]
        if k == 3:
            want += gc[(j + 1) % 4, 0]
        assert np.allclose(want, fdc, rtol=1e-5, atol=1e-7), (want, fdc)
        checked += 1
    assert checked >= 5


def test_straight_beziers_match_the_polyline_gradient():
    g = synth.rng(64)
    loop = np.array([[0.0, 0.0, 0.1], [1.0, 0.2, 0.0], [1.2, 1.1, 0.3], [0.1, 0.9, -0.2], [-0.3, 0.5, 0.2]])
    n = len(loop)
    curves = np.array([[loop[i], (2 * loop[i] + loop[(i + 1) % n]) / 3, (loop[i] + 2 * loop[(i + 1) % n]) / 3,
                        loop[(i + 1) % n]] for i in range(n)])
    P = g.uniform(-0.5, 1.5, (6, 3))
    gp, gc = GC.grad_curves(curves, P)
    rp, rv = G3.grad3d([loop], P)
    assert np.allclose(gp, rp, rtol=1e-9, atol=1e-12)
    # vertex i: end of curve i-1 and start of curve i, plus the chain rule
    # through c1 = (2a + b)/3 and c2 = (a + 2b)/3
    gv = np.zeros((n, 3))
    for i in range(n):
        a, b = i, (i + 1) % n
        gv[a] += gc[i, 0] + (2 / 3) * gc[i, 1] + (1 / 3) * gc[i, 2]
        gv[b] += gc[i, 3] + (1 / 3) * gc[i, 1] + (2 / 3) * gc[i, 2]
    assert np.allclose(gv, rv[0], rtol=1e-9, atol=1e-12)


def test_translation_invariance():
    M = synth.coons_surface(65, 300, 16)
    curves = M.info["curves"]
    P = synth.box_queries(M.V, 5, 66).astype(np.float64)
    gq = synth.rng(67).normal(size=5)
    gp, gc = GC.grad_curves(curves, P, gq)
    assert np.allclose(gc.sum((0, 1)), -gp.sum(0), rtol=1e-9, atol=1e-11)
