"""Pins for the helpers that decide which queries the parity checks exempt:
the distance functions of the 3D oracle and its degeneracy margins (CPU only).

Each check is written as a function of the routine it pins, so that the same
check can be run on a planted mistake (an unclamped projection, an
unprojected distance, a dropped closing edge, a plane distance that is not
normalised) and shown to fail.  References: analytic distances, brute-force
sampling, and queries placed at known fractions of BAND from a boundary edge
(Lemma 1: chi changes only where the projected boundary crosses the ray, or
where p crosses the surface), from a triangle, and next to an interior edge.
"""
import numpy as np
import pytest

import synth
from oracle import wn3d as W


# ----------------------------------------------------------------------------
# distance helpers
# ----------------------------------------------------------------------------

def check_segment_distance(fn):
    A = np.array([[0.0, 0.0, 0.0]])
    B = np.array([[1.0, 0.0, 0.0]])
    for p, want in (((0.5, 2.0, 0.0), 2.0),          # foot inside the segment
                    ((-3.0, 4.0, 0.0), 5.0),         # beyond A
                    ((4.0, 0.0, 4.0), 5.0),          # beyond B
                    ((0.25, 0.0, 0.0), 0.0)):        # on the segment
        assert abs(fn(np.array(p), A, B)[0] - want) < 1e-12, (p, want)
    # a segment of zero length is its point
    assert abs(fn(np.array([1.0, 2.0, 2.0]), A, A)[0] - 3.0) < 1e-12
    # brute force: dense samples of random segments
    g = synth.rng(31)
    for _ in range(20):
        a, b, p = g.normal(size=(3, 3))
        s = np.linspace(0.0, 1.0, 20001)[:, None]
        ref = np.linalg.norm(a + s * (b - a) - p, axis=1).min()
        got = fn(p, a[None], b[None])[0]
        assert got <= ref + 1e-12 and got >= ref - np.linalg.norm(b - a) / 20000, (got, ref)


def check_point_triangle_distance(fn):
    A, B, C = np.array([[0.0, 0, 0]]), np.array([[1.0, 0, 0]]), np.array([[0.0, 1, 0]])
    for p, want in (((0.2, 0.2, 3.0), 3.0),                 # above the interior
                    ((0.2, 0.2, -0.5), 0.5),                # below it
                    ((2.0, -1.0, 0.0), np.sqrt(2.0)),       # nearest a vertex
                    ((0.5, -2.0, 1.0), np.sqrt(5.0)),       # nearest an edge
                    ((1.0, 1.0, 0.0), 1.0 / np.sqrt(2.0))): # nearest the long edge
        assert abs(fn(np.array(p), A, B, C)[0] - want) < 1e-12, (p, want)
    # collinear triangle: the distance to its segments
    got = fn(np.array([0.5, 1.0, 0.0]), A, B, np.array([[2.0, 0, 0]]))[0]
    assert abs(got - 1.0) < 1e-12
    # brute force: barycentric samples of random triangles, scaled ones too
    g = synth.rng(32)
    k = np.arange(301)
    u, v = np.meshgrid(k, k, indexing="ij")
    keep = u + v <= 300
    u, v = u[keep] / 300.0, v[keep] / 300.0
    for scale in (1.0, 1e-3, 50.0):
        for _ in range(10):
            a, b, c, p = g.normal(size=(4, 3)) * scale
            pts = a + u[:, None] * (b - a) + v[:, None] * (c - a)
            ref = np.linalg.norm(pts - p, axis=1).min()
            got = fn(p, a[None], b[None], c[None])[0]
            h = max(np.linalg.norm(b - a), np.linalg.norm(c - a), np.linalg.norm(c - b)) / 300.0
            assert got <= ref + 1e-12 * scale and got >= ref - h, (got, ref, scale)


def check_boundary_distance(fn):
    # unit square loop; the query is nearest the closing edge (last -> first)
    L = [np.array([[0.0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]])]
    P = np.array([[-0.5, 0.5, 0.0], [0.5, 0.5, 2.0], [2.0, 2.0, 0.0]])
    want = np.array([0.5, np.sqrt(0.25 + 4.0), np.sqrt(2.0)])
    np.testing.assert_allclose(fn(L, P), want, atol=1e-12)
    # brute force over a random closed polyline
    g = synth.rng(33)
    Lr = g.normal(size=(7, 3))
    pts = []
    for i in range(7):
        a, b = Lr[i], Lr[(i + 1) % 7]
        s = np.linspace(0, 1, 4001)[:, None]
        pts.append(a + s * (b - a))
    pts = np.concatenate(pts)
    Q = g.normal(size=(25, 3)) * 2
    ref = np.array([np.linalg.norm(pts - q, axis=1).min() for q in Q])
    got = fn([Lr], Q)
    assert np.all(got <= ref + 1e-12) and np.all(got >= ref - 1e-3)


def test_segment_distance():
    check_segment_distance(W.segment_distance)


def test_point_triangle_distance():
    check_point_triangle_distance(W.point_triangle_distance)


def test_boundary_distance():
    check_boundary_distance(W.boundary_distance)


def test_distance_pins_catch_planted_mistakes():
    def unclamped(p, A, B):
        A, B = np.atleast_2d(A), np.atleast_2d(B)
        E = B - A
        s = np.einsum("ij,ij->i", p - A, E) / np.maximum(np.einsum("ij,ij->i", E, E), 1e-300)
        return np.linalg.norm(A + s[:, None] * E - p, axis=1)

    def plane_not_normalised(p, A, B, C):
        d = W.point_triangle_distance(p, A, B, C)
        n = np.cross(B - A, C - A)
        return d * np.linalg.norm(n, axis=1)

    def no_closing_edge(loops, P):
        return np.array([min(W.segment_distance(p, L[:-1], L[1:]).min() for L in loops) for p in P])

    for check, bad in ((check_segment_distance, unclamped),
                       (check_point_triangle_distance, plane_not_normalised),
                       (check_boundary_distance, no_closing_edge)):
        with pytest.raises(AssertionError):
            check(bad)


# ----------------------------------------------------------------------------
# degeneracy margins of the crossing count
# ----------------------------------------------------------------------------

def _frame_perp(d, e):
    """A unit vector perpendicular to d and to the edge direction e."""
    u = np.cross(d, e)
    return u / np.linalg.norm(u)


def ray_margin_of(margin_fn, M, p, d):
    L = W.loops_coords(M.V, W.boundary_loops(M.F))
    scene = float(np.linalg.norm(M.V.astype(np.float64) - p, axis=1).max())
    return margin_fn(L, p, d, scene), scene


def check_ray_boundary_margin(margin_fn):
    """Queries whose ray line passes a boundary edge (its interior) at a known
    perpendicular offset in the plane across d, from well below the edge's
    height: the margin is offset / (max(|a-p|,|b-p|) + ABS_REL scene)."""
    M = synth.bumpy_cap()
    V = M.V.astype(np.float64)
    L = W.boundary_loops(M.F)[0]
    d = synth.random_direction(41)
    for i in (0, 5, 11):
        a, b = V[L[i]], V[L[(i + 1) % len(L)]]
        m = 0.5 * (a + b)
        u = _frame_perp(d, b - a)
        base = m - 0.9 * d
        for frac in (0.5, 4.0):
            # offset delta solves delta = frac*BAND*(max(|a-p|,|b-p|) + ABS_REL*scene); the
            # scale hardly moves with delta, so two fixed-point steps settle it
            delta = 0.0
            for _ in range(3):
                p = base + delta * u
                scale = max(np.linalg.norm(a - p), np.linalg.norm(b - p))
                scene = float(np.linalg.norm(V - p, axis=1).max())
                delta = frac * W.BAND * (scale + W.ABS_REL * scene)
            p = base + delta * u
            got, _ = ray_margin_of(margin_fn, M, p, d)
            assert abs(got - frac * W.BAND) <= 1e-3 * frac * W.BAND, (got, frac)


def test_ray_boundary_margin_at_known_offsets():
    check_ray_boundary_margin(W.ray_boundary_margin)


def test_ray_margin_pin_catches_unprojected_distance():
    def unprojected(loops, p, d, scene):
        best = np.inf
        for L in loops:
            a = L - p
            b = np.roll(a, -1, 0)
            dist = W.segment_distance(np.zeros(3), a, b)   # 3D distance: the projection dropped
            sc = np.maximum(np.linalg.norm(a, axis=1), np.linalg.norm(b, axis=1)) + W.ABS_REL * scene
            best = min(best, float((dist / sc).min()))
        return best

    with pytest.raises(AssertionError):
        check_ray_boundary_margin(unprojected)


def test_queries_near_the_boundary_ray_are_flagged_exactly_below_band():
    M = synth.bumpy_cap()
    V = M.V.astype(np.float64)
    L = W.boundary_loops(M.F)[0]
    d = synth.random_direction(42)
    a, b = V[L[3]], V[L[4]]
    u = _frame_perp(d, b - a)
    base = 0.5 * (a + b) - 0.9 * d
    scale = max(np.linalg.norm(a - base), np.linalg.norm(b - base))
    P = np.stack([base + f * W.BAND * scale * u for f in (0.5, 0.9, 1.2, 4.0)])
    r = W.wn3d(M.V, M.F, P, d)
    np.testing.assert_array_equal(r.degenerate, [True, True, False, False])
    # the exemption is the ray's: the same points with a direction along the
    # edge's normal plane far from the boundary are regular
    r2 = W.wn3d(M.V, M.F, P, synth.random_direction(43))
    assert not r2.degenerate.any()


def test_surface_margin_at_known_heights():
    M = synth.bumpy_cap()
    V = M.V.astype(np.float64)
    f = M.F[len(M.F) // 2]
    A, B, C = V[f[0]], V[f[1]], V[f[2]]
    n = np.cross(B - A, C - A)
    n /= np.linalg.norm(n)
    c = (A + B + C) / 3.0
    far = max(np.linalg.norm(A - c), np.linalg.norm(B - c), np.linalg.norm(C - c))
    scene = float(np.linalg.norm(V - c, axis=1).max())
    # d along the surface's tangent plane (the ray does not meet this triangle)
    d = np.cross(n, B - A)
    d /= np.linalg.norm(d)
    got = []
    for frac in (0.5, 0.9, 1.2, 4.0):
        h = frac * W.BAND * (far + W.ABS_REL * scene)
        p = c + h * n
        _, m = W.crossings(M.V, M.F, p[None], d, margins=True)
        got.append(m["m_surf"][0])
    got = np.array(got)
    # the nearest triangle is this one (its centroid is far from its edges)
    np.testing.assert_allclose(got, np.array([0.5, 0.9, 1.2, 4.0]) * W.BAND, rtol=1e-3)


def test_rays_next_to_an_interior_edge_are_regular_and_exact():
    """By Lemma 1 chi does not change across an interior edge: a ray passing
    an interior edge at 1e-9 (relative; far above BAND_SELF) is not
    degenerate, and its chi equals that of rays 1e-4 to either side."""
    M = synth.bumpy_cap()
    V = M.V.astype(np.float64)
    he = {}
    for fi, f in enumerate(M.F):
        for k in range(3):
            he[(int(f[k]), int(f[(k + 1) % 3]))] = fi
    interior = [(a, b) for (a, b) in he if (b, a) in he and a < b]
    d = synth.random_direction(44)
    g = synth.rng(45)
    for j in g.choice(len(interior), 12, replace=False):
        a, b = (V[i] for i in interior[j])
        u = _frame_perp(d, b - a)
        base = 0.5 * (a + b) - 0.7 * d
        sc = max(np.linalg.norm(a - base), np.linalg.norm(b - base))
        P = np.stack([base + s * sc * u for s in (1e-9, -1e-9, 1e-4, -1e-4)])
        r = W.wn3d(M.V, M.F, P, d)
        if r["m_ray"].min() < 1e-3 or r["m_surf"].min() < 1e-3:
            continue    # too close to the boundary or the surface for this check
        assert not r.degenerate.any()
        assert len(set(r["chi"].tolist())) == 1, r["chi"]


def test_oracle_flags_its_own_exact_ties():
    """A ray exactly through an interior edge's midpoint or a vertex gives an
    exact (or below 2^-40) zero edge value in the oracle's float64
    predicates: flagged through m_self."""
    M = synth.bumpy_cap()
    V = M.V.astype(np.float64)
    d = np.array([0.0, 0.0, 1.0])
    f = M.F[10]
    for p in (V[f[0]] - 0.8 * d, 0.5 * (V[f[0]] + V[f[1]]) - 0.8 * d):
        _, m = W.crossings(M.V, M.F, p[None], d, margins=True)
        assert m["m_self"][0] < W.BAND_SELF
