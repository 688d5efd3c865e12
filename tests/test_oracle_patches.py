"""Pins of the patch-crossing oracle (oracle.patches3d) against what the
mathematics fixes independently of it:

* a planar bilinear patch (a non-parallelogram quadrilateral, degree-elevated
  to a bicubic net) is crossed iff the ray's hit on the plane lies inside
  the quadrilateral, with the sign of d . n;
* a fine tessellation of a curved Coons patch has the same crossing count
  (mesh oracle, brute force over triangles) for queries away from the surface;
* w = chi_d + Theta / 2pi, with Theta the curve oracle's integral along the
  patch's boundary curves, does not depend on d;
* a closed pillow of two patches with one boundary has chi in {0, 1} for
  every d, and the same value for all d.
"""
import math

import numpy as np

import synth
from oracle import curves3d as OC
from oracle import patches3d as OP
from oracle import wn3d as O


def _bilinear_net(c00, c10, c01, c11):
    e = np.array([1.0, 2.0 / 3.0, 1.0 / 3.0, 0.0])
    net = np.zeros((4, 4, 3))
    for i in range(4):
        for j in range(4):
            net[i, j] = (e[i] * e[j] * c00 + (1 - e[i]) * e[j] * c10 + e[i] * (1 - e[j]) * c01
                         + (1 - e[i]) * (1 - e[j]) * c11)
    return net


def _cross2(a, b):
    return a[0] * b[1] - a[1] * b[0]


def _in_convex_quad(q, quad):
    s = [_cross2(quad[(k + 1) % 4] - quad[k], q - quad[k]) for k in range(4)]
    return all(x > 0 for x in s) or all(x < 0 for x in s)


def test_planar_bilinear_patch():
    g = synth.rng(51)
    quad = np.array([[0.0, 0.0], [1.3, 0.1], [1.1, 0.9], [-0.2, 1.2]])   # convex, counter-clockwise
    c = np.concatenate([quad, np.zeros((4, 1))], 1)
    net = _bilinear_net(c[0], c[1], c[3], c[2])    # c00, c10, c01, c11
    checked = hits = 0
    for _ in range(120):
        p = np.array([g.uniform(-0.5, 1.6), g.uniform(-0.5, 1.5), g.choice([-1, 1]) * g.uniform(0.05, 1.0)])
        target = np.array([g.uniform(-0.4, 1.5), g.uniform(-0.1, 1.3), 0.0])
        d = (target - p) / np.linalg.norm(target - p) * g.choice([1, 1, 1, -1])   # mostly towards the plane
        r = OP.patch_crossings(net[None], p[None], d)
        t = -p[2] / d[2]
        q = (p + t * d)[:2]
        near = min(abs(_cross2(quad[(k + 1) % 4] - quad[k], q - quad[k])) /
                   np.linalg.norm(quad[(k + 1) % 4] - quad[k]) for k in range(4))
        if r.degenerate[0] or near < 1e-6:
            continue
        want = (1 if d[2] > 0 else -1) if (t > 0 and _in_convex_quad(q, quad)) else 0
        assert r.chi[0] == want, (p, d, r.chi[0], want)
        checked += 1
        hits += want != 0
    assert checked > 100 and hits >= 30


def _tessellate(net, n):
    t = np.linspace(0, 1, n + 1)
    U, V = np.meshgrid(t, t, indexing="ij")
    P = synth.bezier_patch(net, U.ravel(), V.ravel())
    idx = np.arange((n + 1) ** 2).reshape(n + 1, n + 1)
    a, b, c, e = idx[:-1, :-1].ravel(), idx[1:, :-1].ravel(), idx[1:, 1:].ravel(), idx[:-1, 1:].ravel()
    F = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, e], 1)])   # counter-clockwise in (u, v)
    return P, F


def test_fine_tessellation_agrees_away_from_the_surface():
    M = synth.coons_surface(21, 500, 32)
    net = M.info["net"]
    V, F = _tessellate(net, 160)
    d = synth.random_direction(52)
    P = synth.box_queries(M.V, 150, 53).astype(np.float64)
    r = OP.patch_crossings(net[None], P, d)
    m = O.crossings(V, F, P, d)
    # distance to the surface from the tessellation's vertices (dense)
    dist = np.array([np.min(np.linalg.norm(V - p, axis=1)) for p in P])
    ok = ~r.degenerate & (dist > 2e-2)
    assert ok.sum() > 60 and np.any(r.chi[ok] != 0)
    assert np.array_equal(r.chi[ok], np.asarray(m)[ok])


def test_w_does_not_depend_on_d():
    M = synth.coons_surface(22, 500, 32)
    net, curves = M.info["net"], M.info["curves"]
    g = synth.rng(54)
    P = synth.box_queries(M.V, 40, 55).astype(np.float64)
    dirs = [synth.random_direction(int(g.integers(1 << 30))) for _ in range(3)]
    W = []
    for d in dirs:
        r = OP.patch_crossings(net[None], P, d)
        ang, dist = OC.curve_margins(curves, P, d)
        th = OC.curve_term(curves, P, d)
        w = r.chi + th / (2 * math.pi)
        w[r.degenerate | (ang < 1e-5) | (dist < 1e-5)] = np.nan
        W.append(w)
    W = np.array(W)
    both = np.isfinite(W).all(0)
    assert both.sum() > 30
    assert np.abs(W[1:, both] - W[0, both]).max() < 1e-9
    assert np.any(np.abs(W[0, both]) > 0.05)


def test_closed_pillow():
    M = synth.coons_surface(23, 500, 32)
    net = M.info["net"]
    bump = net.copy()
    bump[1:3, 1:3] += np.array([0.0, 0.0, 0.8])     # same boundary, interior pushed up
    # the Coons patch faces up (+z): reversing it and keeping the raised copy
    # gives a closed surface with outward normals
    nets = np.stack([np.swapaxes(net, 0, 1), bump])
    g = synth.rng(56)
    P = synth.box_queries(M.V, 40, 57).astype(np.float64)
    P[:, 2] = g.uniform(-0.6, 1.2, len(P))
    vals = []
    for k in range(3):
        d = synth.random_direction(int(g.integers(1 << 30)))
        r = OP.patch_crossings(nets, P, d)
        c = r.chi.astype(float)
        c[r.degenerate] = np.nan
        vals.append(c)
    vals = np.array(vals)
    both = np.isfinite(vals).all(0)
    assert both.sum() > 30
    assert set(np.unique(vals[:, both])) <= {0.0, 1.0}
    assert np.all(vals[:, both] == vals[0, both]) and np.any(vals[0, both] == 1)
