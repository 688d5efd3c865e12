"""FP64 oracle: the boundary term of w along cubic Bezier boundary curves.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What is computed
----------------
A surface whose boundary is a set of closed loops of cubic Bezier curves has
w(p) = chi_d(p) + Theta(p) / (2 pi), where Theta is the line integral over the
boundary of the one-form whose integral along a straight edge a -> b is the
edge term of ``oracle.wn3d``: half the signed solid angle of the spherical
triangle (-d, a - p, b - p).  Sec. 5.1 ("Exact Computations") computes region
areas from boundary integrals (Gauss-Bonnet) and notes that along Bezier
boundaries they have to be integrated numerically; Theta is that integral for
the region decomposition seeded at d.

The form: shrink the edge to a point.  In the frame R (rows e1, e2, d) with
(X, Y, Z) = R (gamma - p) and r = |gamma - p|, the edge term's numerator
N = Y_a X_b - X_a Y_b tends to -(X dY - Y dX) and its denominator
D = alpha_a alpha_b + X_a X_b + Y_a Y_b (alpha = r - Z) tends to 2 r (r - Z),
so

    omega = -(X dY - Y dX) / (2 r (r - Z)).

It is singular where the curve meets the ray p + t d, t > 0 (there chi_d
jumps by one and Theta by 2 pi) and where the curve passes through p.

Quadrature: adaptive Gauss-Legendre with 15 nodes per panel.  A panel is
accepted when it agrees with the sum over its halves to 1e-13 (absolute, plus
1e-13 relative); otherwise both halves are refined, at most 48 levels deep
(a panel that has not converged by then makes the query's result NaN).
r - Z is evaluated as rho^2 / (r + Z) where Z > 0.

``curve_margins`` reports, per query, the smallest angle between d and the
direction of a curve point in front of p, and the smallest distance from p to
a curve relative to the curves' bounding-box diagonal (dense sampling refined
by golden-section search); queries with small margins are degenerate for
parity purposes.

Pinned by (tests/test_oracle_curves.py): straight Beziers of any speed against
the Van Oosterom-Strackee solid angle of (-d, a - p, b - p); planar regions
bounded by Bezier loops against fine fan triangulations (sum of triangle solid
angles, Richardson-extrapolated) with chi_d from a point-in-polygon test, for
several d; additivity under de Casteljau splits; reversal.  The margins
(tests/test_oracle_margins_param.py): straight Beziers of uneven speed against
the point-segment distance and a million-point angle search, curves behind
the query, rays offset at known fractions of the band, planted mistakes (an
unnormalised distance, points behind p counted, |v| for |v_perp|).
"""
from __future__ import annotations

import math

import numpy as np

from .wn3d import frame

_GX, _GW = np.polynomial.legendre.leggauss(15)
MAX_DEPTH = 48
TOL = 1e-13


def bezier(c, t):
    """Points of the cubic Bezier with control points c [4, 3] at t [n]."""
    t = np.asarray(t, np.float64)[:, None]
    s = 1.0 - t
    return s ** 3 * c[0] + 3 * s * s * t * c[1] + 3 * s * t * t * c[2] + t ** 3 * c[3]


def bezier_d(c, t):
    """Derivative d gamma / dt at t [n]."""
    t = np.asarray(t, np.float64)[:, None]
    s = 1.0 - t
    return 3 * (s * s * (c[1] - c[0]) + 2 * s * t * (c[2] - c[1]) + t * t * (c[3] - c[2]))


def _panel(c, p, R, t0, t1):
    t = 0.5 * (t0 + t1) + 0.5 * (t1 - t0) * _GX
    v = (bezier(c, t) - p) @ R.T
    dv = bezier_d(c, t) @ R.T
    X, Y, Z = v[:, 0], v[:, 1], v[:, 2]
    rho2 = X * X + Y * Y
    r = np.sqrt(rho2 + Z * Z)
    alpha = np.where(Z > 0, rho2 / (r + np.abs(Z)), r - Z)
    f = -(X * dv[:, 1] - Y * dv[:, 0]) / (2.0 * r * alpha)
    return 0.5 * (t1 - t0) * float(np.dot(_GW, f))


def curve_integral(c, p, d) -> float:
    """Theta of one curve c [4, 3] for one query p [3]."""
    c = np.asarray(c, np.float64)
    p = np.asarray(p, np.float64)
    R = frame(d)
    total = 0.0
    stack = [(0.0, 1.0, _panel(c, p, R, 0.0, 1.0), 0)]
    while stack:
        t0, t1, whole, depth = stack.pop()
        tm = 0.5 * (t0 + t1)
        a = _panel(c, p, R, t0, tm)
        b = _panel(c, p, R, tm, t1)
        if abs(a + b - whole) <= TOL * (1.0 + abs(a + b)):
            total += a + b
        elif depth >= MAX_DEPTH:
            return math.nan
        else:
            stack.append((t0, tm, a, depth + 1))
            stack.append((tm, t1, b, depth + 1))
    return total


def curve_term(ctrl, P, d) -> np.ndarray:
    """Theta(p) summed over every curve of ctrl [nc, 4, 3], for P [nq, 3]."""
    ctrl = np.asarray(ctrl, np.float64).reshape(-1, 4, 3)
    P = np.asarray(P, np.float64).reshape(-1, 3)
    out = np.zeros(len(P))
    for i, p in enumerate(P):
        out[i] = sum(curve_integral(c, p, d) for c in ctrl)
    return out


def _golden_min(f, a, b, iters=60):
    g = (math.sqrt(5.0) - 1.0) / 2.0
    x1, x2 = b - g * (b - a), a + g * (b - a)
    f1, f2 = f(x1), f(x2)
    for _ in range(iters):
        if f1 < f2:
            b, x2, f2 = x2, x1, f1
            x1 = b - g * (b - a)
            f1 = f(x1)
        else:
            a, x1, f1 = x1, x2, f2
            x2 = a + g * (b - a)
            f2 = f(x2)
    return min(f1, f2)


def curve_margins(ctrl, P, d, samples: int = 2049):
    """(angle, distance) margins per query: the smallest angle between d and
    (gamma(t) - p) over curve points with (gamma - p).d > 0 (pi if none), and
    the smallest |gamma(t) - p| divided by the diagonal of the curves'
    control-point box."""
    ctrl = np.asarray(ctrl, np.float64).reshape(-1, 4, 3)
    P = np.asarray(P, np.float64).reshape(-1, 3)
    d = np.asarray(d, np.float64)
    d = d / np.linalg.norm(d)
    pts = ctrl.reshape(-1, 3)
    diag = float(np.linalg.norm(pts.max(0) - pts.min(0)))
    ts = np.linspace(0.0, 1.0, samples)
    ang = np.full(len(P), math.pi)
    dist = np.full(len(P), np.inf)
    for c in ctrl:
        G = bezier(c, ts)
        for i, p in enumerate(P):
            v = G - p
            n = np.linalg.norm(v, axis=1)
            k = int(np.argmin(n))
            lo, hi = ts[max(k - 1, 0)], ts[min(k + 1, samples - 1)]
            dist[i] = min(dist[i], _golden_min(lambda t: float(np.linalg.norm(bezier(c, [t])[0] - p)), lo, hi))
            cosang = (v @ d) / np.maximum(n, 1e-300)
            a = np.where(v @ d > 0, np.arccos(np.clip(cosang, -1.0, 1.0)), math.pi)
            k = int(np.argmin(a))
            if a[k] < math.pi:
                lo, hi = ts[max(k - 1, 0)], ts[min(k + 1, samples - 1)]

                def angle_at(t, c=c, p=p):
                    w = bezier(c, [t])[0] - p
                    z = float(w @ d)
                    return math.atan2(float(np.linalg.norm(w - z * d)), z)
                ang[i] = min(ang[i], _golden_min(angle_at, lo, hi))
    return ang, dist / max(diag, 1e-300)
