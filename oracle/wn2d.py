"""FP64 oracle: one-shot winding number of 2D cubic Bezier loops.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Definition (Sec. 3): w_C(p) = (1/2pi) int_C dtheta(p).  In 2D the "boundary"
of a curve is its pair of end points (Sec. 4 and its 2D figure), and the one
region split of the unit circle around p is cut by the directions of those end
points.  Taking one fixed direction d for every query (its region as the BFS
seed of Alg. 1):

    w(p) = chi_d(p) + (1/2pi) sum_{open loops} [phi(end - p) - phi(start - p)]

with phi(v) = atan2(d x v, d . v) reduced to [0, 2pi) (the angle of v measured
counter-clockwise from d) and chi_d(p) the signed number of crossings of the
ray p + t d, t > 0, with the curves (Eq. chi in 2D): a crossing counts
sign(d x B'(t*)), i.e. +1 where the curve passes the ray counter-clockwise
about p.  Closed loops have no end points and contribute only through chi.
A counter-clockwise loop around p therefore has w = +1.

Crossings: y(t) = d x (B(t) - p) is a cubic in t; its real roots on [0, 1]
are the eigenvalues of the companion matrix (numpy.linalg.eigvals, batched),
polished by a few Newton steps in float64; a root counts if
x(t*) = d . (B(t*) - p) > 0.  Reading for exact ties (a ray through a joint
or an end point; grid rows through a bounding-box extreme hit these exactly):
a point on the ray's line counts as lying on the side y >= 0, the same side
that phi in [0, 2pi) gives it, so chi and the end-point term jump together.
Queries whose y is constant along a ray line (grid rows for d = +x) share
their roots, as in the paper's one-shot reuse of one ray per row (Sec. 5
"Optimization"; Sec. 7, 2D results).

A query is *degenerate* (margins below BAND) if the ray passes within BAND of
a curve point it crosses (|x(t*)| small: p on or next to the curve), crosses
tangentially (|y'(t*)| small), or passes within BAND of (but not exactly
through) a segment joint or an open end point.  Exact ties at joints and end
points are not degenerate: the convention above decides them.

Pinned by (tests/test_oracle_2d.py): adaptive quadrature of dtheta/dt
(scipy.integrate.quad) per segment to 1e-10, a dense unwrapped angle sum,
exact integers for closed loops against a polygon crossing test, the closed
form for a straight segment, d-invariance, reversal negation.  The margins
(tests/test_oracle_margins_param.py): tangency on straight pieces of any
speed, brute-force root finding (sign changes refined by bisection) for m_x,
m_tan and m_joint, queries at known fractions of BAND from a crossing, an end
point and a nearly tangential crossing, and planted mistakes in each helper.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi
BAND = 2.0 ** -16


def _power_coeffs(y):
    """Power-basis coefficients (c3, c2, c1, c0) of the cubic Bezier with
    ordinates y[..., 0:4]."""
    y0, y1, y2, y3 = y[..., 0], y[..., 1], y[..., 2], y[..., 3]
    c0 = y0
    c1 = 3.0 * (y1 - y0)
    c2 = 3.0 * (y0 - 2.0 * y1 + y2)
    c3 = -y0 + 3.0 * y1 - 3.0 * y2 + y3
    return c3, c2, c1, c0


def _bez(c, t):
    s = 1.0 - t
    return s * s * s * c[..., 0] + 3 * s * s * t * c[..., 1] + 3 * s * t * t * c[..., 2] + t * t * t * c[..., 3]


def _bez_d(c, t):
    s = 1.0 - t
    return 3 * (s * s * (c[..., 1] - c[..., 0]) + 2 * s * t * (c[..., 2] - c[..., 1]) + t * t * (c[..., 3] - c[..., 2]))


def cubic_roots01(c3, c2, c1, c0):
    """Real roots in [0, 1] of c3 t^3 + c2 t^2 + c1 t + c0 for a batch of
    cubics.  Returns (index_of_cubic, t) arrays."""
    c3, c2, c1, c0 = (np.asarray(a, np.float64).ravel() for a in (c3, c2, c1, c0))
    scale = np.maximum(np.maximum(np.abs(c3), np.abs(c2)), np.maximum(np.abs(c1), np.abs(c0)))
    cub = np.abs(c3) > 1e-12 * scale
    idx_all, t_all = [], []
    if np.any(cub):
        ii = np.nonzero(cub)[0]
        M = np.zeros((ii.size, 3, 3))
        M[:, 0, 0] = -c2[ii] / c3[ii]
        M[:, 0, 1] = -c1[ii] / c3[ii]
        M[:, 0, 2] = -c0[ii] / c3[ii]
        M[:, 1, 0] = 1.0
        M[:, 2, 1] = 1.0
        ev = np.linalg.eigvals(M)                    # [k, 3] complex
        real = np.abs(ev.imag) <= 1e-9 * (1.0 + np.abs(ev.real))
        k, j = np.nonzero(real)
        idx_all.append(ii[k])
        t_all.append(ev.real[k, j])
    for i in np.nonzero(~cub & (scale > 0))[0]:
        r = np.roots([c2[i], c1[i], c0[i]]) if abs(c2[i]) > 1e-12 * scale[i] else (
            np.array([-c0[i] / c1[i]]) if c1[i] != 0 else np.array([]))
        r = r[np.abs(np.imag(r)) <= 1e-9 * (1.0 + np.abs(np.real(r)))].real
        idx_all.append(np.full(r.size, i))
        t_all.append(r)
    if not idx_all:
        return np.zeros(0, np.int64), np.zeros(0)
    idx = np.concatenate(idx_all).astype(np.int64)
    t = np.concatenate(t_all)
    # Newton polish on the polynomial itself
    for _ in range(4):
        f = ((c3[idx] * t + c2[idx]) * t + c1[idx]) * t + c0[idx]
        fp = (3.0 * c3[idx] * t + 2.0 * c2[idx]) * t + c1[idx]
        step = np.where(fp != 0, f / np.where(fp != 0, fp, 1.0), 0.0)
        t = t - step
    keep = (t >= 0.0) & (t <= 1.0)
    return idx[keep], t[keep]


def _first_nonzero_sign(*vals):
    """Sign of the first nonzero value (elementwise over arrays)."""
    out = np.zeros(np.shape(vals[0]))
    done = np.zeros(np.shape(vals[0]), bool)
    for v in vals:
        nz = (~done) & (v != 0)
        out = np.where(nz, np.sign(v), out)
        done |= nz
    return out


def segment_crossings(ys):
    """Crossings of one horizontal line with cubics whose ordinates relative
    to that line are ys[..., 0:4] (a batch of shape [k, nseg, 4]).

    The line itself counts as *above* (y >= 0 is above), which matches
    phi in [0, 2pi) for the end-point term.  A crossing is a change of side
    along the curve: +1 from below to above, -1 from above to below.
    Interior roots count sign(y'(t*)) (a double root counts 0).  An exact
    zero at t = 0 counts -1 when the curve leaves it downwards; an exact zero
    at t = 1 counts +1 when the curve arrives from below.

    Returns (flat_index, t, sign) arrays; flat_index indexes ys[..., 0].
    """
    c3, c2, c1, c0 = _power_coeffs(ys)
    idx, t = cubic_roots01(c3, c2, c1, c0)
    y0 = ys[..., 0].ravel()
    y3 = ys[..., 3].ravel()
    tie0 = (y0 == 0.0)[idx]
    tie1 = (y3 == 0.0)[idx]
    interior = ~((tie0 & (t < 1e-9)) | (tie1 & (t > 1.0 - 1e-9))) & (t > 0.0) & (t < 1.0)
    ii, ti = idx[interior], t[interior]
    yd = _bez_d(ys.reshape(-1, 4)[ii], ti)
    si = np.sign(yd)
    # exact end-point ties
    flat = ys.reshape(-1, 4)
    e0 = np.nonzero(y0 == 0.0)[0]
    after0 = _first_nonzero_sign(flat[e0, 1], flat[e0, 2], flat[e0, 3])
    k0 = after0 < 0
    e1 = np.nonzero(y3 == 0.0)[0]
    before1 = _first_nonzero_sign(flat[e1, 2], flat[e1, 1], flat[e1, 0])
    k1 = before1 < 0
    fi = np.concatenate([ii, e0[k0], e1[k1]])
    ft = np.concatenate([ti, np.zeros(int(k0.sum())), np.ones(int(k1.sum()))])
    fs = np.concatenate([si, -np.ones(int(k0.sum())), np.ones(int(k1.sum()))])
    return fi, ft, fs


def tangency(xp, yp):
    """|sin| of the angle between the curve and the ray's line at a crossing,
    from the curve's derivative (xp, yp) in the frame of d: |y'| / |B'|."""
    return np.abs(yp) / np.maximum(np.hypot(xp, yp), 1e-300)


def crossing_margins(dx, tang):
    """(m_x, m_tan) per query from dx [q, roots] = x(t*) - p_x of every root
    on the query's ray line and the roots' tangency: the distance along the
    line to the nearest crossing (either side: p next to the curve), and the
    smallest tangency among the crossings the ray counts (at or right of p,
    within BAND)."""
    if dx.shape[1] == 0:
        return np.full(dx.shape[0], np.inf), np.full(dx.shape[0], np.inf)
    m_x = np.abs(dx).min(1)
    m_tan = np.where(dx > -BAND, tang[None, :], np.inf).min(1)
    return m_x, m_tan


def joint_margin(jx, jy, ky, px):
    """Per query (abscissae px, all on the ray line of ordinate ky): the
    smallest distance from the line of the joints and open end points
    (jx, jy) at or right of p (within BAND).  Exact ties (jy == ky) are
    decided by the y >= 0 convention, so they do not count."""
    dj = np.abs(jy - ky)
    dj = np.where(dj == 0.0, np.inf, dj)
    jd = np.where(jx[None, :] - px[:, None] > -BAND, dj[None, :], np.inf)
    return jd.min(1) if jd.shape[1] else np.full(len(px), np.inf)


class Result2D(dict):
    @property
    def degenerate(self):
        return ((self["m_x"] < BAND) | (self["m_tan"] < BAND)
                | (self["m_joint"] < BAND))


def _phi(y, x):
    a = np.arctan2(y, x)
    return np.where(a < 0.0, a + TWO_PI, a)


def wn2d(ctrl, loop_off, closed, P, d=(1.0, 0.0), margins: bool = True) -> Result2D:
    """w, chi and margins for every query point.

    ctrl [nseg, 4, 2]; loop_off [nloops + 1] (segment offsets); closed
    [nloops] (nonzero = closed); P [nq, 2]; d the ray direction.
    """
    ctrl = np.asarray(ctrl, np.float64)
    P = np.atleast_2d(np.asarray(P, np.float64))
    loop_off = np.asarray(loop_off, np.int64)
    closed = np.asarray(closed)
    d = np.asarray(d, np.float64)
    d = d / np.linalg.norm(d)
    nq = len(P)
    # d-frame coordinates of the control points (absolute; rows of queries
    # share the ordinate offset d x p)
    cx = ctrl[..., 0] * d[0] + ctrl[..., 1] * d[1]          # d . c
    cy = d[0] * ctrl[..., 1] - d[1] * ctrl[..., 0]          # d x c
    px = P[:, 0] * d[0] + P[:, 1] * d[1]
    py = d[0] * P[:, 1] - d[1] * P[:, 0]
    keys, inv = np.unique(py, return_inverse=True)
    chi = np.zeros(nq, np.int64)
    m_x = np.full(nq, np.inf)
    m_tan = np.full(nq, np.inf)
    m_joint = np.full(nq, np.inf)
    nseg = ctrl.shape[0]
    # joints: start of every segment plus the end of open loops
    jx = [cx[:, 0]]
    jy = [cy[:, 0]]
    for l in range(len(closed)):
        if not closed[l] and loop_off[l + 1] > loop_off[l]:
            s = loop_off[l + 1] - 1
            jx.append(cx[s:s + 1, 3])
            jy.append(cy[s:s + 1, 3])
    jx = np.concatenate(jx)
    jy = np.concatenate(jy)
    CHUNK = max(1, 200000 // max(nseg, 1))
    for k0 in range(0, len(keys), CHUNK):
        kk = keys[k0:k0 + CHUNK]
        ys = cy[None, :, :] - kk[:, None, None]              # [k, nseg, 4]
        idx, t, sgn = segment_crossings(ys)
        row = idx // nseg
        seg = idx % nseg
        xr = _bez(cx[seg], t)                                 # absolute d . B(t*)
        yp = _bez_d(cy[seg], t)                               # d x B'(t*)
        xp = _bez_d(cx[seg], t)
        sgn = sgn.astype(np.int64)
        endpt = (t == 0.0) | (t == 1.0)
        tang = np.where(endpt, np.inf, tangency(xp, yp))
        for r in range(len(kk)):
            qs = np.nonzero(inv == k0 + r)[0]
            sel = row == r
            xr_r, s_r, tg_r = xr[sel], sgn[sel], tang[sel]
            dx = xr_r[None, :] - px[qs][:, None]               # [q, roots]
            chi[qs] = np.sum(np.where(dx > 0, s_r[None, :], 0), axis=1)
            if margins:
                m_x[qs], m_tan[qs] = crossing_margins(dx, tg_r)
                # exact ties are resolved by the convention; near ties are not
                m_joint[qs] = joint_margin(jx, jy, kk[r], px[qs])
    # end-point terms of open loops
    E = np.zeros(nq)
    for l in range(len(closed)):
        a, b = int(loop_off[l]), int(loop_off[l + 1])
        if closed[l] or b <= a:
            continue
        s0 = ctrl[a, 0]
        s1 = ctrl[b - 1, 3]
        vs = s0[None, :] - P
        ve = s1[None, :] - P
        ps = _phi(d[0] * vs[:, 1] - d[1] * vs[:, 0], vs @ d)
        pe = _phi(d[0] * ve[:, 1] - d[1] * ve[:, 0], ve @ d)
        E += pe - ps
    w = chi + E / TWO_PI
    return Result2D(w=w, chi=chi, E=E, m_x=m_x, m_tan=m_tan, m_joint=m_joint)
