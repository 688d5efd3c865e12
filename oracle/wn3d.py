"""FP64 oracle: one-shot generalized winding number of an oriented triangle mesh.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What is computed
----------------
The winding number of a surface M at p (Sec. 3) equals the area-weighted mean
of the signed ray-crossing count chi over all directions (Eq. wn_chi).  By
Lemma 1 chi is constant on each region A_i cut out of the unit sphere around p
by the projected boundary, so w = (1/4pi) sum_i Area(A_i) chi_i
(Eq. wn_discrete_sum).  By Lemma 2 neighbouring regions differ by exactly one,
the in-sphere normal n x tau pointing to the larger value (Lemma 2, Sec. 5).

Fix one unit direction d for all queries and take d's region as the seed of
Alg. 1 (the paper picks the largest region only as a heuristic; any seed gives
the same sum).  Then chi_j = chi_d + delta_j with delta_j the signed number of
boundary crossings between d and region j, and since the areas sum to 4pi,

    w(p) = chi_d(p) + (1/4pi) sum_j Area(A_j) delta_j .

The second term is a line integral over the boundary (the paper computes region
areas from boundary integrals, Sec. 5.1 "Exact Computations", Gauss-Bonnet).  For
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
Alg. 1 and t > 0 in Eq. ray_bezier_int; w is undefined on M anyway).  A query
is *degenerate* (its chi_d is not compared bit for bit) when the line of its
ray passes within BAND of the projected boundary, when p lies within BAND of
the surface, or when a triangle the ray nearly hits has an edge value too
small for the oracle's own float64 predicates (see BAND).  By Lemma 1 a ray
close to an interior edge or vertex is not degenerate: any consistent
evaluation (the two triangles of a shared edge decide it oppositely) gives
the same chi_d there.

Pinned by (tests/test_oracle_3d.py): the per-triangle solid-angle sum (the
plain definition of w_M), quadrature of Eq. wn_chi over a spherical Fibonacci
set, the flat-disk closed form, exact {0, 1} for closed meshes, invariance
under a change of d, orientation flip, union additivity, Lemma 2 on random
direction pairs straddling one projected boundary edge, and an independent
Moller-Trumbore crossing count.  The distance helpers and the margins
(tests/test_oracle_margins.py): analytic distances, brute-force sampling of
segments, triangles and loops, and queries placed at known fractions of
BAND from a boundary edge, a triangle, and an interior edge.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi
# Degeneracy bands.  A float32/float64 evaluation relative to p decides every
# ray/triangle predicate exactly on a *perturbed* copy of the mesh: each vertex
# moved in the plane perpendicular to d by at most 2^-23 |v - p| (its offset
# from p rounded to float32) plus 2^-47 of the scene size (the frame and the
# split float32 coordinates it is stored in).  The signed crossing count of that copy equals the exact one unless
# the perturbation carries the projected boundary across the ray or the
# surface across p (Lemma 1: chi is constant on the regions cut out by the
# projected boundary; it also changes where p crosses M).  BAND is the
# relative distance (ray to projected boundary, p to a triangle) below which
# a query is degenerate; a factor of eight above the perturbation.
BAND = 2.0 ** -20
# The oracle's own float64 predicates are exact for edge values above
# 2^-40 |a||b| (their rounding error is below 2^-50 |a||b|); a triangle the
# ray nearly hits with a smaller edge value makes the query degenerate too.
BAND_SELF = 2.0 ** -40
# Scene-size term added to every relative scale (covers the float64 frame).
ABS_REL = 2.0 ** -26


# ----------------------------------------------------------------------------
# topology
# ----------------------------------------------------------------------------

def boundary_loops(F) -> list:
    """Boundary of an oriented triangle mesh as closed vertex loops.

    A boundary half-edge a->b is an edge {a, b} used by exactly one face, kept
    in that face's orientation (Sec. 6.1 "Preprocessing": boundaries are segments
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

def point_triangle_distance(p, A, B, C) -> np.ndarray:
    """Euclidean distance from the point p to each triangle (A[i], B[i], C[i])
    (closest point in the plane when its projection falls inside, else on the
    nearest edge; degenerate triangles use their edges only)."""
    p = np.asarray(p, np.float64)
    A, B, C = (np.atleast_2d(np.asarray(x, np.float64)) for x in (A, B, C))
    n = np.cross(B - A, C - A)
    nn = np.einsum("ij,ij->i", n, n)
    out = np.minimum(np.minimum(segment_distance(p, A, B), segment_distance(p, B, C)),
                     segment_distance(p, C, A))
    ok = nn > 0
    if np.any(ok):
        a, b, c, m = A[ok] - p, B[ok] - p, C[ok] - p, n[ok]
        # the projection of p lies inside iff p sees every edge on the side of n
        s_ab = np.einsum("ij,ij->i", np.cross(a, b), m)
        s_bc = np.einsum("ij,ij->i", np.cross(b, c), m)
        s_ca = np.einsum("ij,ij->i", np.cross(c, a), m)
        inside = (s_ab >= 0) & (s_bc >= 0) & (s_ca >= 0)
        dplane = np.abs(np.einsum("ij,ij->i", a, m)) / np.sqrt(nn[ok])
        sub = out[ok]
        sub[inside] = dplane[inside]
        out[ok] = sub
    return out


def segment_distance(p, A, B) -> np.ndarray:
    """Distance from p to each segment [A[i], B[i]] (clamped projection)."""
    p = np.asarray(p, np.float64)
    A = np.atleast_2d(np.asarray(A, np.float64))
    B = np.atleast_2d(np.asarray(B, np.float64))
    E = B - A
    ee = np.einsum("ij,ij->i", E, E)
    with np.errstate(divide="ignore", invalid="ignore"):
        s = np.einsum("ij,ij->i", p - A, E) / ee
    s = np.where(ee > 0, np.clip(s, 0.0, 1.0), 0.0)
    q = A + s[:, None] * E
    return np.sqrt(np.einsum("ij,ij->i", q - p, q - p))


def ray_boundary_margin(loops_xyz, p, d, scene) -> float:
    """Smallest relative distance between the line p + t d and the boundary:
    per boundary edge a->b, the distance from the origin to the segment
    [a_perp, b_perp] of the edge's projection along d (relative to p),
    divided by max(|a - p|, |b - p|) + ABS_REL * scene.  (Conservative: an
    edge passing behind p counts as well.)"""
    best = np.inf
    for L in loops_xyz:
        L = np.asarray(L, np.float64)
        if len(L) == 0:
            continue
        a = L - p
        b = np.roll(a, -1, 0)
        ap = a - np.outer(a @ d, d)
        bp = b - np.outer(b @ d, d)
        dist = segment_distance(np.zeros(3), ap, bp)
        sc = np.maximum(np.linalg.norm(a, axis=1), np.linalg.norm(b, axis=1)) + ABS_REL * scene
        best = min(best, float((dist / sc).min()))
    return best


def crossings(V, F, P, d, margins: bool = False, loops=None):
    """Signed number of crossings of the ray p + t d (t > 0) with the mesh.

    Brute force over every triangle: the ray meets the triangle's interior iff
    the three triple products d.(a x b), d.(b x c), d.(c x a) of the vertices
    relative to p share one strict sign (that sign is then sign(d . n)); it
    meets it in front of p iff t = (n . a)/(d . n) > 0.

    With ``margins`` also returns a dict of per-query margins (see BAND):
      m_ray   distance from the ray's line to the projected boundary
              (ray_boundary_margin);
      m_surf  min over triangles of dist(p, T) / (max_k |v_k - p| + ABS_REL
              * scene): how close p is to the surface;
      m_self  min |edge value| / (|a||b|) over the triangles the ray hits or
              misses by less than BAND_SELF (the oracle's own exactness).
    ``loops`` (boundary vertex loops, default: from F) are needed for m_ray.
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
    if margins:
        if loops is None:
            loops = boundary_loops(F)
        Lx = loops_coords(V, loops)
        m = {k: np.full(len(P), np.inf) for k in ("m_ray", "m_surf", "m_self")}
        # bounding spheres of the triangles, to find the few that can be near p
        cen = (A + B + C) / 3.0
        rad = np.sqrt(np.max(np.stack([np.einsum("ij,ij->i", X - cen, X - cen) for X in (A, B, C)], 1), 1))
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
            scene = float(np.sqrt(np.einsum("ij,ij->i", V - p, V - p).max())) if len(V) else 0.0
            m["m_ray"][i] = ray_boundary_margin(Lx, p, d, scene)
            # p near a triangle: candidates from the bounding spheres
            dc = np.linalg.norm(cen - p, axis=1)
            cand = np.nonzero(dc - rad <= 4.0 * BAND * (dc + rad) + 4.0 * ABS_REL * scene)[0]
            if cand.size:
                dist = point_triangle_distance(p, A[cand], B[cand], C[cand])
                far = np.maximum(np.maximum(np.linalg.norm(a[cand], axis=1), np.linalg.norm(b[cand], axis=1)),
                                 np.linalg.norm(c[cand], axis=1))
                m["m_surf"][i] = float((dist / (far + ABS_REL * scene)).min())
            # the oracle's own float64 decisions: edge values normalised by
            # the product of the vertex distances, near-hit triangles only
            # (|a||b| <= scene^2 bounds the normalisation, which finds them)
            tol = BAND_SELF * scene * scene
            cand = np.nonzero(((e_ab > -tol) & (e_bc > -tol) & (e_ca > -tol))
                              | ((e_ab < tol) & (e_bc < tol) & (e_ca < tol)))[0]
            if cand.size:
                la = np.linalg.norm(a[cand], axis=1)
                lb = np.linalg.norm(b[cand], axis=1)
                lc = np.linalg.norm(c[cand], axis=1)
                with np.errstate(divide="ignore", invalid="ignore"):
                    ab = e_ab[cand] / (la * lb)
                    bc = e_bc[cand] / (lb * lc)
                    ca = e_ca[cand] / (lc * la)
                near = (((ab > -BAND_SELF) & (bc > -BAND_SELF) & (ca > -BAND_SELF))
                        | ((ab < BAND_SELF) & (bc < BAND_SELF) & (ca < BAND_SELF)))
                if np.any(near):
                    em = np.minimum(np.minimum(np.abs(ab[near]), np.abs(bc[near])), np.abs(ca[near]))
                    m["m_self"][i] = float(np.nan_to_num(em, nan=0.0).min())
    if margins:
        return chi, m
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
    """Distance from each query to the boundary polyline (every edge of every
    loop, the closing edge last -> first included)."""
    P = np.atleast_2d(np.asarray(P, np.float64))
    best = np.full(len(P), np.inf)
    for L in loops_xyz:
        L = np.asarray(L, np.float64)
        if len(L) == 0:
            continue
        A = L
        B = np.roll(L, -1, 0)
        for i, p in enumerate(P):
            best[i] = min(best[i], float(segment_distance(p, A, B).min()))
    return best


# ----------------------------------------------------------------------------
# full evaluation
# ----------------------------------------------------------------------------

class Result(dict):
    """w, chi, S and the margins m_ray, m_surf, m_self, m_bnd (per query)."""

    @property
    def degenerate(self):
        return (self["m_ray"] < BAND) | (self["m_surf"] < BAND) | (self["m_self"] < BAND_SELF)


def loops_coords(V, loops):
    V = np.asarray(V, np.float64)
    return [V[L] for L in loops]


def wn3d(V, F, P, d, margins: bool = True, loops=None) -> Result:
    """w(p) = chi_d(p) + S(p)/(2 pi) for every query (float64)."""
    if loops is None:
        loops = boundary_loops(F)
    Lx = loops_coords(V, loops)
    out = {}
    if margins:
        chi, m = crossings(V, F, P, d, margins=True, loops=loops)
        out.update(m)
        out["m_bnd"] = boundary_distance(Lx, P) if Lx else np.full(len(np.atleast_2d(P)), np.inf)
    else:
        chi = crossings(V, F, P, d)
    S = boundary_term(Lx, P, d) if Lx else np.zeros(len(chi))
    w = chi + S / TWO_PI
    return Result(w=w, chi=chi, S=S, **out)
