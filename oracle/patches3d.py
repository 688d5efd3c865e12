"""FP64 oracle: signed crossings of the ray p + t d (t > 0) with bicubic
Bezier patches.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What is computed
----------------
chi_d (Eq. chi) for a parametric surface S(u, v), (u, v) in [0, 1]^2: the
points where the ray p + t d, t > 0, meets S, each counted with
sign(d . (S_u x S_v)).  Sec. 5.1 ("Parametric Surfaces") finds all roots of
f(xi) + (q - p) t = 0 with a generic nonlinear solver started on
subintervals of the ray; for polynomial patches it points to specialised
techniques.  This oracle isolates the roots by subdivision: in the frame R of
d with (X, Y, Z) = R (S - p), a crossing is a zero of the map (X, Y)(u, v)
with Z > 0, and d . (S_u x S_v) = X_u Y_v - X_v Y_u (R is a rotation with
third row d).  By the convex hull property a sub-patch whose control points
all have X > 0 (or all < 0, or the same for Y), or all Z <= 0, holds no
crossing.  Sub-patches are split in four by de Casteljau's algorithm at
their parameter midpoints until they are smaller than 2^-LEAF; from the
centre and the four corners of such a leaf Newton's method on the whole
patch looks for a zero, which is kept when it lies inside the leaf (closed,
tolerance 1e-12).  Zeros closer than 1e-9 in (u, v) are merged.

Margins (``Crossings``): per query the smallest, over the zeros found, of
the distance to the parameter-square boundary (the ray passes near a
boundary curve: chi jumps there), of |d . n| / |n| with n = S_u x S_v (the
ray nearly tangent: two zeros of opposite sign may merge), and of |S - p|
relative to the patch size (the query on the surface); zeros with Z <= 0 but
|Z| small count too.  Queries below BAND are degenerate for parity.

Pinned by (tests/test_oracle_patches.py): planar bilinear patches against a
point-in-quadrilateral test; fine tessellations of curved patches against
the mesh oracle's brute-force crossing count (oracle.wn3d.crossings) away
from the surface; w = chi_d + Theta / 2pi (Theta from oracle.curves3d along
the patch's boundary curves) independent of d; and closed two-patch pillows
(chi in {0, 1} for every d).  The margin (tests/test_oracle_margins_param.py):
flat, tilted and stretched bilinear patches against the parameter distance,
|cos| of the tilt and |S - p| / size in closed form, planted mistakes in
zero_margin; a ray passing just outside a patch has no crossing margin and is
flagged by curve_margins of the patch's boundary curves, which the parity
tests combine with it.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .wn3d import frame

LEAF = 7
BAND = 1e-5


def _split_u(N, t=0.5):
    """de Casteljau split of a net [4, 4, k] along its first index."""
    a = N
    rows_l, rows_r = [a[0]], [a[3]]
    for _ in range(3):
        a = (1 - t) * a[:-1] + t * a[1:]
        rows_l.append(a[0])
        rows_r.append(a[-1])
    return np.stack(rows_l), np.stack(rows_r[::-1])


def _split(N):
    L, R = _split_u(N)
    LL, LR = (np.swapaxes(x, 0, 1) for x in _split_u(np.swapaxes(L, 0, 1)))
    RL, RR = (np.swapaxes(x, 0, 1) for x in _split_u(np.swapaxes(R, 0, 1)))
    # (u-half, v-half): (0,0), (0,1), (1,0), (1,1)
    return LL, LR, RL, RR


def _bern(t):
    s = 1.0 - t
    return np.array([s ** 3, 3 * t * s * s, 3 * t * t * s, t ** 3])


def _bern_d(t):
    s = 1.0 - t
    return 3.0 * np.array([-s * s, s * s - 2 * t * s, 2 * t * s - t * t, t * t])


def patch_eval(net, u, v):
    """S, S_u, S_v of the patch net [4, 4, 3] at one (u, v)."""
    bu, bv, du, dv = _bern(u), _bern(v), _bern_d(u), _bern_d(v)
    S = np.einsum("i,j,ijk->k", bu, bv, net)
    Su = np.einsum("i,j,ijk->k", du, bv, net)
    Sv = np.einsum("i,j,ijk->k", bu, dv, net)
    return S, Su, Sv


def _newton(Q, u, v, iters=40):
    """Zero of (X, Y) of the frame-relative net Q from (u, v), or None."""
    for _ in range(iters):
        S, Su, Sv = patch_eval(Q, u, v)
        det = Su[0] * Sv[1] - Sv[0] * Su[1]
        if det == 0.0 or not np.isfinite(det):
            return None
        du = (S[0] * Sv[1] - Sv[0] * S[1]) / det
        dv = (Su[0] * S[1] - S[0] * Su[1]) / det
        u, v = u - du, v - dv
        if not (np.isfinite(u) and np.isfinite(v)) or abs(u) > 10 or abs(v) > 10:
            return None
        if abs(du) < 1e-15 and abs(dv) < 1e-15:
            break
    S, _, _ = patch_eval(Q, u, v)
    scale = np.abs(Q).max()
    if np.hypot(S[0], S[1]) > 1e-12 * scale:
        return None
    return u, v


@dataclass
class Crossings:
    chi: np.ndarray
    margin: np.ndarray

    @property
    def degenerate(self):
        return self.margin < BAND


def zero_margin(u, v, S, n, size):
    """Margin of one zero (u, v) of the projected map, in the frame where d
    is +z: its parameter distance to the square's boundary (the ray near a
    boundary curve), |d . n| / |n| with n = S_u x S_v (the ray nearly
    tangent) and |S - p| over the patch's size (p on the surface)."""
    return min(u, 1 - u, v, 1 - v, abs(n[2]) / max(np.linalg.norm(n), 1e-300),
               np.linalg.norm(S) / max(size, 1e-300))


def patch_crossings_one(net, p, d):
    """(chi, margin) of one patch net [4, 4, 3] for one query p."""
    R = frame(d)
    Q = (np.asarray(net, np.float64) - np.asarray(p, np.float64)) @ R.T
    size = float(np.linalg.norm(Q.reshape(-1, 3).max(0) - Q.reshape(-1, 3).min(0)))
    zeros = []
    stack = [(Q, 0.0, 0.0, 1.0)]
    while stack:
        N, u0, v0, h = stack.pop()
        X, Y, Z = N[..., 0], N[..., 1], N[..., 2]
        if X.min() > 0 or X.max() < 0 or Y.min() > 0 or Y.max() < 0:
            continue
        if Z.max() <= -BAND * size:
            continue
        if h > 2.0 ** -LEAF:
            h2 = 0.5 * h
            LL, LR, RL, RR = _split(N)
            stack += [(LL, u0, v0, h2), (LR, u0, v0 + h2, h2), (RL, u0 + h2, v0, h2), (RR, u0 + h2, v0 + h2, h2)]
            continue
        for su, sv in ((0.5, 0.5), (0, 0), (1, 0), (0, 1), (1, 1)):
            z = _newton(Q, u0 + su * h, v0 + sv * h)
            if z is None:
                continue
            u, v = z
            if u0 - 1e-12 <= u <= u0 + h + 1e-12 and v0 - 1e-12 <= v <= v0 + h + 1e-12:
                if not any(abs(u - a) < 1e-9 and abs(v - b) < 1e-9 for a, b in zeros):
                    zeros.append((u, v))
                break
    chi = 0
    margin = np.inf
    for u, v in zeros:
        if not (0.0 <= u <= 1.0 and 0.0 <= v <= 1.0):
            margin = min(margin, min(abs(u), abs(1 - u), abs(v), abs(1 - v)))
            continue
        S, Su, Sv = patch_eval(Q, u, v)
        n = np.cross(Su, Sv)
        margin = min(margin, zero_margin(u, v, S, n, size))
        if S[2] > 0:
            chi += 1 if n[2] > 0 else -1
    return chi, margin


def patch_crossings(nets, P, d) -> Crossings:
    """chi_d summed over the patches nets [np, 4, 4, 3] for queries P [n, 3]."""
    nets = np.asarray(nets, np.float64).reshape(-1, 4, 4, 3)
    P = np.asarray(P, np.float64).reshape(-1, 3)
    chi = np.zeros(len(P), np.int64)
    margin = np.full(len(P), np.inf)
    for i, p in enumerate(P):
        for net in nets:
            c, m = patch_crossings_one(net, p, d)
            chi[i] += c
            margin[i] = min(margin[i], m)
    return Crossings(chi, margin)
