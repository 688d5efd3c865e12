"""FP64 oracle: derivatives of the 3D winding number from the boundary alone.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

w(p) = chi_d(p) + S_d(p)/(2 pi) (see ``oracle.wn3d``).  chi_d is piecewise
constant in p and in the vertex positions, so almost everywhere every
derivative of w is a derivative of the boundary integral.  That integral is
the solid angle of the boundary loop up to a locally constant multiple of 4 pi,
so its derivatives do not depend on d.  For a straight edge a->b with
a' = a - p, b' = b - p:

    K_e = 1 / (|a'||b'| + a'.b'),   c_e = (a' x b') K_e
    grad_p w  = +(1/4pi) sum_e c_e (1/|a'| + 1/|b'|)
    dw/da    += -(1/4pi) c_e / |a'|      (a = start of e)
    dw/db    += -(1/4pi) c_e / |b'|      (b = end of e)

grad_p is the Biot-Savart field of the loop; the vertex terms are the same
field integrated against the piecewise-linear hat function of each vertex
(along a straight edge the integrand of that line integral points along
a' x b', and the hat-weighted integrals of 1/|x - p|^3 are K_e/|a'| and
K_e/|b'|).  Translation invariance sum_v dw/dv + grad_p w = 0 holds edge by
edge.  The overall sign follows the orientation conventions of oracle.wn3d.

Pinned by (tests/test_oracle_grad.py): central finite differences of
``oracle.wn3d`` (h = 1e-4 and 1e-6), Gauss-Legendre quadrature of the
hat-weighted Biot-Savart integrals, and the translation, scaling and rotation
identities.
"""
from __future__ import annotations

import math

import numpy as np

FOUR_PI = 4.0 * math.pi


def grad3d(loops_xyz, P, g=None):
    """Return (grad_p [q,3], [grad_v per loop [n_i,3]]) of L = sum_q g_q w(p_q).

    ``g`` defaults to ones (then grad_p is dw/dp per query and grad_v the sum
    over queries of dw/dv).
    """
    P = np.atleast_2d(np.asarray(P, np.float64))
    nq = len(P)
    g = np.ones(nq) if g is None else np.asarray(g, np.float64)
    gp = np.zeros((nq, 3))
    gv = []
    for L in loops_xyz:
        L = np.asarray(L, np.float64)
        n = len(L)
        acc = np.zeros((n, 3))
        if n == 0:
            gv.append(acc)
            continue
        a = L[None, :, :] - P[:, None, :]                 # [q, n, 3]
        b = np.roll(a, -1, axis=1)
        ra = np.linalg.norm(a, axis=2)
        rb = np.linalg.norm(b, axis=2)
        cr = np.cross(a, b)
        K = 1.0 / (ra * rb + np.einsum("qnk,qnk->qn", a, b))
        c = cr * K[..., None]
        gp += np.einsum("qnk,qn->qk", c, (1.0 / ra + 1.0 / rb)) / FOUR_PI * g[:, None]
        ga = np.einsum("qnk,qn->nk", c, g[:, None] / ra) / FOUR_PI
        gb = np.einsum("qnk,qn->nk", c, g[:, None] / rb) / FOUR_PI
        acc -= ga
        acc -= np.roll(gb, 1, axis=0)
        gv.append(acc)
    return gp, gv
