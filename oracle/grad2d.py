"""FP64 oracle: derivatives of the 2D one-shot winding number.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Away from the curves the signed crossing count chi_d (Eq. chi) is locally
constant: a small move of the query or of any control point changes no
crossing unless a curve passes the query.  In the one-shot form

    w(p) = chi_d(p) + (1/2pi) sum_{open loops} [phi(e - p) - phi(s - p)]

(s, e the first and last control points of an open loop, phi the angle of a
vector from d) w therefore varies only through the end-point angles.  The
gradient of the angle of v is (-v_y, v_x) / |v|^2 (independent of d), so for
a loss L = sum_q g_q w(p_q):

    dL/dp_q  = (g_q / 2pi) sum_open [ A(s - p_q) - A(e - p_q) ],
    dL/de    = sum_q (g_q / 2pi) A(e - p_q),
    dL/ds    = -sum_q (g_q / 2pi) A(s - p_q),        A(v) = (-v_y, v_x) / |v|^2,

and every other control point (interior points, closed loops) has zero
gradient.  The end points are the entries ctrl[first segment, 0] and
ctrl[last segment, 3] of each open loop.

Pinned by tests/test_oracle_grad2d.py: central finite differences of
``oracle.wn2d`` itself with respect to the query and to both end points of
every open loop, zero finite-difference change under moves of interior
control points and of a closed loop, and the translation identity (moving
the query and every control point together leaves w unchanged).
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def _a(v):
    r2 = np.sum(v * v, axis=-1, keepdims=True)
    return np.stack([-v[..., 1], v[..., 0]], axis=-1) / r2


def grad2d(ctrl, loop_off, closed, P, g=None):
    """(dL/dP [nq, 2], dL/dctrl [nseg, 4, 2]) for L = sum_q g_q w(P_q)."""
    ctrl = np.asarray(ctrl, np.float64)
    P = np.atleast_2d(np.asarray(P, np.float64))
    loop_off = np.asarray(loop_off, np.int64)
    g = np.ones(len(P)) if g is None else np.asarray(g, np.float64)
    gq = np.zeros_like(P)
    gc = np.zeros_like(ctrl)
    for l in range(len(closed)):
        a, b = int(loop_off[l]), int(loop_off[l + 1])
        if closed[l] or b <= a:
            continue
        As = _a(ctrl[a, 0][None, :] - P)          # [nq, 2]
        Ae = _a(ctrl[b - 1, 3][None, :] - P)
        w = (g / TWO_PI)[:, None]
        gq += w * (As - Ae)
        gc[b - 1, 3] += np.sum(w * Ae, axis=0)
        gc[a, 0] -= np.sum(w * As, axis=0)
    return gq, gc
