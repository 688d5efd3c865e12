"""FP64 oracle: one-shot generalized winding number of an oriented triangle mesh.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What is computed
----------------
The winding number of a surface M at p (Sec. 3) equals the area-weighted mean
of the signed ray-crossing count chi over all directions (Eq. wn_chi).  By
Lemma 1 chi is constant on each region A_i cut out of the unit sphere around p
by the projected boundary, so w = (1/4pi) sum_i Area(A_i) chi_i
(Eq. wn_discrete_sum).  By Lemma 2 neighbouring regions differ by exactly one,
the in-sphere normal n x tau pointing to the larger value (Sec. 4).

Fix one unit direction d for all queries and take d's region as the seed of
Alg. 1 (the paper picks the largest region only as a heuristic; any seed gives
the same sum).  Then chi_j = chi_d + delta_j with delta_j the signed number of
boundary crossings between d and region j, and since the areas sum to 4pi,

    w(p) = chi_d(p) + (1/4pi) sum_j Area(A_j) delta_j .

The second term is a line integral over the boundary (the paper computes region
areas from boundary integrals, Sec. 4 "Exact Computations", Gauss-Bonnet).  For
a straight boundary edge a->b it is half the signed area of the spherical
triangle (-d, a-p, b-p), which in the rotated frame R (rows e1, e2, d; det +1)
with (X, Y, Z) = R (v - p), rho^2 = X^2 + Y^2, r = |v - p| and
alpha = r - Z (evaluated as rho^2 / (r + Z) when Z > 0) is

    theta_e = atan2(N, D),  N = Y_a X_b - X_a Y_b,
                            D = alpha_a alpha_b + X_a X_b + Y_a Y_b,

and w = chi_d + (1/2pi) sum_e theta_e.  theta_e jumps by 2pi exactly where the
ray p + t d (t > 0) passes through edge e, which is where chi_d changes by one.

chi_d (Eq. chi): the ray p + t d, t > 0, against every triangle, brute force.
A triangle (v0, v1, v2) has normal n = (v1 - v0) x (v2 - v0); a hit counts
sign(d . n) (+1 when the ray runs along the normal, i.e. enters from the back).

Readings of the paper taken here: strict t > 0 (the paper writes t >= 0 in
Alg. 1 and t > 0 in Eq. ray_bezier_int; w is undefined on M anyway); a ray
through an edge or vertex, or a query on M, is *degenerate* and reported
through the margins below instead of being resolved.

Pinned by (tests/test_oracle_3d.py): the per-triangle solid-angle sum (the
plain definition of w_M), quadrature of Eq. wn_chi over a spherical Fibonacci
set, the flat-disk closed form, exact {0, 1} for closed meshes, invariance
under a change of d, orientation flip, union additivity, Lemma 2 on random
direction pairs straddling one projected boundary edge, and an independent
Moller-Trumbore crossing count.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi
# Relative margin below which a query is degenerate.  Margins are normalised
# edge values d.(a x b)/(|a_perp||b_perp|), vertex offsets |a_perp|/|a| and
# depths |t|/max(|a|,|b|,|c|); a float32 evaluation of the same predicates
# relative to p (coordinates rounded once, two rounded products and one
# difference) errs by at most about 2^-22 in these units, so a band of 2^-20
# leaves a factor of four.
BAND = 2.0 ** -20


# ----------------------------------------------------------------------------
# topology
# ----------------------------------------------------------------------------

def boundary_loops(F) -> list:
    """Boundary of an oriented triangle mesh as closed vertex loops.

    A boundary half-edge a->b is an edge {a, b} used by exactly one face, kept
    in that face's orientation (Sec. 5 preprocessing: boundaries are segments
    adjacent to only one loop).  Half-edges are chained head to tail; each loop
    is returned as the vertex sequence v0, v1, ..., v_{n-1} (edges v_i -> v_{i+1}
    and v_{n-1} -> v0).  Raises on a vertex with two outgoing boundary edges.
    """
    F = np.asarray(F, np.int64)
    if F.size == 0:
        return []
    he = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], 0)
    lo = np.minimum(he[:, 0], he[:, 1])
    hi = np.maximum(he[:, 0], he[:, 1])
    n = int(F.max()) + 1
    key = lo * n + hi
    _, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
    bmask = cnt[inv] == 1
    bhe = he[bmask]
    nxt = {}
    for a, b in bhe:
        a, b = int(a), int(b)
        if a in nxt:
            raise ValueError(f"vertex {a} has two outgoing boundary edges")
        nxt[a] = b
    loops = []
    seen = set()
    for start in sorted(nxt):
        if start in seen:
            continue
        loop = [start]
        seen.add(start)
        v = nxt[start]
        while v != start:
            if v in seen or v not in nxt:
                raise ValueError("boundary half-edges do not close into loops")
            loop.append(v)
            seen.add(v)
            v = nxt[v]
        loops.append(np.array(loop, np.int64))
    return loops


# ----------------------------------------------------------------------------
# frame
# ----------------------------------------------------------------------------

def frame(d) -> np.ndarray:
    """Rotation R with rows (e1, e2, d/|d|), orthonormal and det R = +1, so
    that R d = |d| e_z."""
    d = np.asarray(d, np.float64)
    nd = np.linalg.norm(d)
    if not np.isfinite(nd) or nd == 0.0:
        raise ValueError("direction must be finite and nonzero")
    d = d / nd
    axis = np.zeros(3)
    axis[int(np.argmin(np.abs(d)))] = 1.0
    e1 = np.cross(d, axis)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(d, e1)
    return np.stack([e1, e2, d], 0)


# ----------------------------------------------------------------------------
# crossing count (Eq. chi)
# ----------------------------------------------------------------------------

def crossings(V, F, P, d, margins: bool = False):
    """Signed number of crossings of the ray p + t d (t > 0) with the mesh.

    Brute force over every triangle: the ray meets the triangle's interior iff
    the three triple products d.(a x b), d.(b x c), d.(c x a) of the vertices
    relative to p share one strict sign (that sign is then sign(d . n)); it
    meets it in front of p iff t = (n . a)/(d . n) > 0.

    With ``margins`` also returns, per query, over the triangles that the ray
    hits or misses by less than BAND: the smallest normalised edge value
    |d.(a x b)| / (|a_perp||b_perp|) (the sine of the angle at the ray between
    the projected vertices; a_perp is a's component perpendicular to d) or
    vertex offset |a_perp| / |a|, whichever is smaller, and the smallest
    |t| / max(|a|,|b|,|c|).
    """
    V = np.asarray(V, np.float64)
    F = np.asarray(F, np.int64)
    P = np.atleast_2d(np.asarray(P, np.float64))
    d = np.asarray(d, np.float64)
    d = d / np.linalg.norm(d)
    A, B, C = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    n = np.cross(B - A, C - A)
    dn = n @ d
    chi = np.zeros(len(P), np.int64)
    m_edge = np.full(len(P), np.inf)
    m_t = np.full(len(P), np.inf)
    for i, p in enumerate(P):
        a, b, c = A - p, B - p, C - p
        e_ab = np.cross(a, b) @ d
        e_bc = np.cross(b, c) @ d
        e_ca = np.cross(c, a) @ d
        pos = (e_ab > 0) & (e_bc > 0) & (e_ca > 0)
        neg = (e_ab < 0) & (e_bc < 0) & (e_ca < 0)
        inside = pos | neg
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.einsum("ij,ij->i", n, a) / dn
        hit = inside & (t > 0)
        chi[i] = int(np.sum(np.sign(dn[hit])))
        if margins:
            la = np.linalg.norm(a, axis=1)
            lb = np.linalg.norm(b, axis=1)
            lc = np.linalg.norm(c, axis=1)
            # distances of the vertices from the ray's line (projections
            # perpendicular to d)
            pa = np.linalg.norm(a - np.outer(a @ d, d), axis=1)
            pb = np.linalg.norm(b - np.outer(b @ d, d), axis=1)
            pc = np.linalg.norm(c - np.outer(c @ d, d), axis=1)
            with np.errstate(divide="ignore", invalid="ignore"):
                ab = e_ab / (pa * pb)
                bc = e_bc / (pb * pc)
                ca = e_ca / (pc * pa)
            near = (((ab > -BAND) & (bc > -BAND) & (ca > -BAND))
                    | ((ab < BAND) & (bc < BAND) & (ca < BAND)))
            near &= np.isfinite(t) & (t > -BAND * np.maximum(np.maximum(la, lb), lc))
            if np.any(near):
                em = np.minimum(np.minimum(np.abs(ab[near]), np.abs(bc[near])), np.abs(ca[near]))
                vm = np.minimum(np.minimum(pa[near] / la[near], pb[near] / lb[near]), pc[near] / lc[near])
                m_edge[i] = float(min(np.nan_to_num(em, nan=0.0).min(), vm.min()))
                sc = np.maximum(np.maximum(la[near], lb[near]), lc[near])
                m_t[i] = float((np.abs(t[near]) / sc).min())
    if margins:
        return chi, m_edge, m_t
    return chi


# ----------------------------------------------------------------------------
# boundary line integral
# ----------------------------------------------------------------------------

def boundary_term(loops_xyz, P, d) -> np.ndarray:
    """S(p) = sum over boundary edges of theta_e = atan2(N, D) in the frame of
    ``d`` (see the module docstring); w = chi_d + S / (2 pi).

    ``loops_xyz`` is a list of [n_i, 3] arrays, each a closed loop in order.
    Coordinates are taken relative to p first and rotated afterwards.
    """
    P = np.atleast_2d(np.asarray(P, np.float64))
    R = frame(d)
    S = np.zeros(len(P))
    for L in loops_xyz:
        L = np.asarray(L, np.float64)
        if len(L) == 0:
            continue
        rel = L[None, :, :] - P[:, None, :]              # [q, n, 3]
        Q = rel @ R.T
        X, Y, Z = Q[..., 0], Q[..., 1], Q[..., 2]
        rho2 = X * X + Y * Y
        r = np.sqrt(rho2 + Z * Z)
        with np.errstate(divide="ignore", invalid="ignore"):
            alpha = np.where(Z > 0, rho2 / (r + Z), r - Z)
        Xb, Yb, ab = np.roll(X, -1, 1), np.roll(Y, -1, 1), np.roll(alpha, -1, 1)
        N = Y * Xb - X * Yb
        D = alpha * ab + X * Xb + Y * Yb
        S += np.sum(np.arctan2(N, D), axis=1)
    return S


def boundary_distance(loops_xyz, P) -> np.ndarray:
    """Distance from each query to the boundary polyline."""
    P = np.atleast_2d(np.asarray(P, np.float64))
    best = np.full(len(P), np.inf)
    for L in loops_xyz:
        L = np.asarray(L, np.float64)
        A = L
        B = np.roll(L, -1, 0)
        E = B - A
        ee = np.einsum("ij,ij->i", E, E)
        for i, p in enumerate(P):
            with np.errstate(divide="ignore", invalid="ignore"):
                s = np.clip(np.einsum("ij,ij->i", p - A, E) / ee, 0.0, 1.0)
            s = np.where(ee > 0, s, 0.0)
            q = A + s[:, None] * E
            best[i] = min(best[i], float(np.sqrt(((q - p) ** 2).sum(1)).min()))
    return best


# ----------------------------------------------------------------------------
# full evaluation
# ----------------------------------------------------------------------------

class Result(dict):
    """w, chi, S and the margins m_edge, m_t, m_bnd (all per query)."""

    @property
    def degenerate(self):
        return (self["m_edge"] < BAND) | (self["m_t"] < BAND)


def loops_coords(V, loops):
    V = np.asarray(V, np.float64)
    return [V[L] for L in loops]


def wn3d(V, F, P, d, margins: bool = True, loops=None) -> Result:
    """w(p) = chi_d(p) + S(p)/(2 pi) for every query (float64)."""
    if loops is None:
        loops = boundary_loops(F)
    Lx = loops_coords(V, loops)
    if margins:
        chi, m_edge, m_t = crossings(V, F, P, d, margins=True)
        m_bnd = boundary_distance(Lx, P) if Lx else np.full(len(np.atleast_2d(P)), np.inf)
    else:
        chi = crossings(V, F, P, d)
        m_edge = m_t = m_bnd = None
    S = boundary_term(Lx, P, d) if Lx else np.zeros(len(chi))
    w = chi + S / TWO_PI
    return Result(w=w, chi=chi, S=S, m_edge=m_edge, m_t=m_t, m_bnd=m_bnd)
