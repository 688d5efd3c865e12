"""FP64 oracle: derivatives of w for a boundary of cubic Bezier curves.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Away from the surface chi_d is locally constant, so every derivative of
w = chi_d + Theta/(2 pi) is a derivative of the boundary term, which is the
solid angle of the boundary loops up to a locally constant multiple of 4 pi
and therefore independent of d.  For curves gamma(t) with Bernstein control
points c_k (gamma = sum_k B_k(t) c_k):

    grad_p w  = +(1/4pi) int (gamma - p) x gamma'(t) / |gamma - p|^3 dt
    dw/dc_k   = -(1/4pi) int B_k(t) (gamma - p) x gamma'(t) / |gamma - p|^3 dt

the continuous forms of ``oracle.grad3d``'s edge terms: a straight edge's
closed form (a' x b')(1/|a'| + 1/|b'|)/(|a'||b'| + a'.b') is the first
integral over the edge, and its hat-weighted vertex terms are the second
with the hat functions in place of B_k.  Tangential motions change nothing
((gamma - p) x gamma' is normal to gamma'), and translating every control
point moves w like moving p the other way (sum_k B_k = 1).

Quadrature: adaptive Gauss-Legendre (15 nodes) on each curve, a panel
accepted when it agrees with its two halves to 1e-12 relative to the
integrand's scale.

Pinned by (tests/test_oracle_gradcurves.py): central differences of
``oracle.curves3d`` with respect to the query and to single control
points; closed polygons written as straight Beziers against
``oracle.grad3d`` (through the chain rule for the interior control points);
translation invariance.
"""
from __future__ import annotations

import math

import numpy as np

from .curves3d import bezier, bezier_d

FOUR_PI = 4.0 * math.pi
_GX, _GW = np.polynomial.legendre.leggauss(15)


def _bern(t):
    t = np.asarray(t, np.float64)
    s = 1.0 - t
    return np.stack([s ** 3, 3 * t * s * s, 3 * t * t * s, t ** 3], 1)


def _panel(c, p, t0, t1):
    """(int f dt, int B_k f dt) over [t0, t1]: f = (gamma - p) x gamma' / |gamma - p|^3."""
    t = 0.5 * (t0 + t1) + 0.5 * (t1 - t0) * _GX
    v = bezier(c, t) - p
    dv = bezier_d(c, t)
    r = np.linalg.norm(v, axis=1)
    f = np.cross(v, dv) / (r ** 3)[:, None]
    w = 0.5 * (t1 - t0) * _GW
    B = _bern(t)
    return (w[:, None] * f).sum(0), np.einsum("n,nk,nc->kc", w, B, f)


def curve_grad(c, p, depth_max=40):
    """(G [3], Gk [4, 3]) = (int f, int B_k f) for one curve and query."""
    c = np.asarray(c, np.float64)
    p = np.asarray(p, np.float64)
    G = np.zeros(3)
    Gk = np.zeros((4, 3))
    g0, gk0 = _panel(c, p, 0.0, 1.0)
    stack = [(0.0, 1.0, g0, gk0, 0)]
    while stack:
        t0, t1, g, gk, depth = stack.pop()
        tm = 0.5 * (t0 + t1)
        ga, gka = _panel(c, p, t0, tm)
        gb, gkb = _panel(c, p, tm, t1)
        err = np.abs(ga + gb - g).max() + np.abs(gka + gkb - gk).max()
        scale = 1.0 + np.abs(ga + gb).max()
        if err <= 1e-12 * scale:
            G += ga + gb
            Gk += gka + gkb
        elif depth >= depth_max:
            return np.full(3, np.nan), np.full((4, 3), np.nan)
        else:
            stack.append((t0, tm, ga, gka, depth + 1))
            stack.append((tm, t1, gb, gkb, depth + 1))
    return G, Gk


def grad_curves(ctrl, P, g=None):
    """(grad_p [n, 3], grad_ctrl [nc, 4, 3]) of L = sum_q g_q w(p_q) for the
    boundary curves ctrl [nc, 4, 3] and queries P [n, 3] (g defaults to 1)."""
    ctrl = np.asarray(ctrl, np.float64).reshape(-1, 4, 3)
    P = np.asarray(P, np.float64).reshape(-1, 3)
    g = np.ones(len(P)) if g is None else np.asarray(g, np.float64)
    gp = np.zeros((len(P), 3))
    gc = np.zeros(ctrl.shape)
    for i, p in enumerate(P):
        for j, c in enumerate(ctrl):
            G, Gk = curve_grad(c, p)
            gp[i] += g[i] * G / FOUR_PI
            gc[j] -= g[i] * Gk / FOUR_PI
    return gp, gc
