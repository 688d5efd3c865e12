"""Seeded synthetic inputs for the winding-number path.

This module only *generates geometry and query points*: Bezier control points,
triangle meshes (a noise-displaced sphere with a polar cap removed, tessellated
bilinear Coons patches, small test meshes), query sets, ray directions and
training targets.  It holds none of the method's arithmetic (no boundary
extraction, no crossing count, no solid angle), so both the FP64 oracle and the
HIP path can consume the same arrays without sharing any computation.

Every generator draws from ``numpy.random.Generator(PCG64(seed))``, works in
float64 and rounds once to the requested dtype at the end.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "rng", "star2d", "loops2d", "grid_axis", "noise_field", "open_sphere",
    "box_queries", "random_direction", "coons_surface", "coons_batch",
    "icosphere", "disk_fan", "bumpy_cap", "random_open_mesh", "targets01",
    "Curves2D", "Mesh", "CoonsBatch",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# 2D cubic Bezier loops
# ----------------------------------------------------------------------------

@dataclass
class Curves2D:
    ctrl: np.ndarray          # [nseg, 4, 2]
    loop_off: np.ndarray      # int64 [nloops + 1]
    closed: np.ndarray        # uint8 [nloops]


def star2d(seed: int = 1, n_seg: int = 16, dtype=np.float64) -> Curves2D:
    """One closed CCW loop of ``n_seg`` C0-joined cubic Beziers whose 3*n_seg
    control points sit at angles 2*pi*k/(3*n_seg) with radii U[0.5, 1]."""
    g = rng(seed)
    n = 3 * n_seg
    ang = 2.0 * np.pi * np.arange(n) / n
    rad = g.uniform(0.5, 1.0, n)
    pts = np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=1)
    idx = (3 * np.arange(n_seg)[:, None] + np.arange(4)[None, :]) % n
    ctrl = pts[idx]
    return Curves2D(ctrl.astype(dtype), np.array([0, n_seg], np.int64),
                    np.array([1], np.uint8))


def loops2d(seed: int = 2, n_loops: int = 16, seg_per_loop: int = 64,
            n_open: int = 4, dtype=np.float32) -> Curves2D:
    """``n_loops`` loops of ``seg_per_loop`` cubics with joints and interior
    control points uniform in [-1, 1]^2.  The first ``n_loops - n_open`` loops
    are closed; the others end at ``start + g*u`` with a gap g ~ U[0.01, 0.05]
    along a random unit vector u."""
    g = rng(seed)
    segs = []
    closed = []
    for l in range(n_loops):
        joints = g.uniform(-1.0, 1.0, (seg_per_loop + 1, 2))
        inner = g.uniform(-1.0, 1.0, (seg_per_loop, 2, 2))
        is_closed = l < n_loops - n_open
        if is_closed:
            joints[-1] = joints[0]
        else:
            gap = g.uniform(0.01, 0.05)
            t = g.uniform(0.0, 2.0 * np.pi)
            joints[-1] = joints[0] + gap * np.array([np.cos(t), np.sin(t)])
        c = np.empty((seg_per_loop, 4, 2))
        c[:, 0] = joints[:-1]
        c[:, 1] = inner[:, 0]
        c[:, 2] = inner[:, 1]
        c[:, 3] = joints[1:]
        segs.append(c)
        closed.append(1 if is_closed else 0)
    ctrl = np.concatenate(segs, axis=0)
    off = np.arange(n_loops + 1, dtype=np.int64) * seg_per_loop
    # Rounding to the kernel dtype happens once; joints stay bit-identical
    # between consecutive segments because they are copies of one value.
    return Curves2D(ctrl.astype(dtype), off, np.array(closed, np.uint8))


def random_cubics(seed: int = 5, n: int = 1000, res: int = 250, dtype=np.float64):
    """The 2D experiment's input shape: ``n`` independent cubic Beziers with
    control points uniform in the unit square, each an open loop of one
    segment, each with a ``res`` x ``res`` grid spanning the bounding box of
    its control points (which contains the curve).  Returns a list of
    ``(Curves2D, xs, ys)``."""
    g = rng(seed)
    out = []
    for _ in range(n):
        c = g.uniform(0.0, 1.0, (1, 4, 2)).astype(dtype)
        lo, hi = c[0].min(0).astype(np.float64), c[0].max(0).astype(np.float64)
        xs = grid_axis(lo[0], hi[0], res, dtype)
        ys = grid_axis(lo[1], hi[1], res, dtype)
        out.append((Curves2D(c, np.array([0, 1], np.int64), np.array([0], np.uint8)), xs, ys))
    return out


def grid_axis(lo: float, hi: float, n: int, dtype=np.float64) -> np.ndarray:
    """``numpy.linspace(lo, hi, n)`` (endpoints included) rounded once."""
    return np.linspace(lo, hi, n).astype(dtype)


# ----------------------------------------------------------------------------
# 3D meshes
# ----------------------------------------------------------------------------

@dataclass
class Mesh:
    V: np.ndarray   # float32 [nv, 3]
    F: np.ndarray   # int32   [nf, 3]
    info: dict = field(default_factory=dict)


def noise_field(seed: int, n_waves: int = 16):
    """Smooth scalar field on the unit sphere: a normalised sum of ``n_waves``
    random plane sinusoids with wave-vector norms in [1, 6].  |n| <= 1."""
    g = rng(seed)
    k = g.normal(size=(n_waves, 3))
    k /= np.linalg.norm(k, axis=1, keepdims=True)
    k *= g.uniform(1.0, 6.0, (n_waves, 1))
    amp = g.uniform(0.5, 1.0, n_waves)
    ph = g.uniform(0.0, 2.0 * np.pi, n_waves)
    amp = amp / amp.sum()

    def f(x):
        return np.sin(x @ k.T + ph) @ amp
    return f


def open_sphere(seed: int = 3, n_lon: int = 512, n_rings: int = 1024,
                cap_deg: float = 30.0, amp: float = 0.05,
                top_refine: int = 1) -> Mesh:
    """Noise-displaced unit sphere with the polar cap ``theta < cap_deg``
    removed.  Rings of ``n_lon`` vertices at polar angles
    ``cap + j*(pi-cap)/n_rings`` (j = 0..n_rings-1) plus a south-pole vertex.
    Faces are oriented with outward normals, (v1-v0)x(v2-v0) pointing out.

    ``top_refine = r`` puts ``r*n_lon`` vertices on the top (boundary) ring and
    joins it to the next ring with a strip where every quad becomes a fan of
    r + 1 triangles, so the single boundary loop has ``r*n_lon`` edges.
    """
    f = noise_field(seed)
    cap = math.radians(cap_deg)
    dth = (math.pi - cap) / n_rings
    n_top = n_lon * top_refine
    # ring 0 (boundary ring)
    verts = []
    phi0 = 2.0 * np.pi * np.arange(n_top) / n_top
    th0 = np.full(n_top, cap)
    verts.append(np.stack([np.sin(th0) * np.cos(phi0), np.sin(th0) * np.sin(phi0), np.cos(th0)], 1))
    phi = 2.0 * np.pi * np.arange(n_lon) / n_lon
    for j in range(1, n_rings):
        th = cap + j * dth
        verts.append(np.stack([np.full(n_lon, math.sin(th)) * np.cos(phi),
                               np.full(n_lon, math.sin(th)) * np.sin(phi),
                               np.full(n_lon, math.cos(th))], 1))
    verts.append(np.array([[0.0, 0.0, -1.0]]))
    U = np.concatenate(verts, 0)
    R = 1.0 + amp * f(U)
    V = U * R[:, None]

    def ring(j, k):
        # vertex id of ring j >= 1, longitude k (mod n_lon)
        return n_top + (j - 1) * n_lon + (k % n_lon)

    faces = []
    k = np.arange(n_lon)
    # strip between ring 0 and ring 1
    if top_refine == 1:
        t0 = k
        t1 = (k + 1) % n_top
        b0 = ring(1, k)
        b1 = ring(1, k + 1)
        faces.append(np.stack([t0, b0, b1], 1))
        faces.append(np.stack([t0, b1, t1], 1))
    else:
        r = top_refine
        h = r // 2
        b0 = ring(1, k)
        b1 = ring(1, k + 1)
        for i in range(h):
            faces.append(np.stack([r * k + i, b0, (r * k + i + 1) % n_top], 1))
        faces.append(np.stack([(r * k + h) % n_top, b0, b1], 1))
        for i in range(h, r):
            faces.append(np.stack([(r * k + i) % n_top, b1, (r * k + i + 1) % n_top], 1))
    # bands between ring j and j+1
    for j in range(1, n_rings - 1):
        a0 = ring(j, k)
        a1 = ring(j, k + 1)
        c0 = ring(j + 1, k)
        c1 = ring(j + 1, k + 1)
        faces.append(np.stack([a0, c0, c1], 1))
        faces.append(np.stack([a0, c1, a1], 1))
    pole = V.shape[0] - 1
    last = n_rings - 1
    faces.append(np.stack([ring(last, k), np.full(n_lon, pole), ring(last, k + 1)], 1))
    F = np.concatenate(faces, 0).astype(np.int32)
    return Mesh(V.astype(np.float32), F,
                {"n_lon": n_lon, "n_rings": n_rings, "cap_deg": cap_deg,
                 "amp": amp, "top_edges": n_top, "seed": seed})


def box_queries(V: np.ndarray, n: int, seed: int, scale: float = 1.2,
                dtype=np.float32) -> np.ndarray:
    """``n`` points uniform in the axis-aligned bounding box of ``V`` scaled
    per axis by ``scale`` about its centre."""
    g = rng(seed)
    Vd = np.asarray(V, np.float64)
    lo, hi = Vd.min(0), Vd.max(0)
    c, h = 0.5 * (lo + hi), 0.5 * (hi - lo) * scale
    return (c + h * g.uniform(-1.0, 1.0, (n, 3))).astype(dtype)


def random_direction(seed: int) -> np.ndarray:
    """A unit vector from a seeded isotropic normal draw (float64)."""
    v = rng(seed).normal(size=3)
    return v / np.linalg.norm(v)


def targets01(n: int, seed: int, dtype=np.float32) -> np.ndarray:
    return rng(seed).integers(0, 2, n).astype(dtype)


# ----------------------------------------------------------------------------
# Bilinear Coons patches
# ----------------------------------------------------------------------------

def _bez3(P, t):
    t = np.asarray(t)[..., None]
    s = 1.0 - t
    return s**3 * P[0] + 3 * s * s * t * P[1] + 3 * s * t * t * P[2] + t**3 * P[3]


def _coons_eval(corners, sides, u, v):
    """Bilinearly blended Coons patch.  corners: dict c00,c10,c01,c11;
    sides: bottom c0(u), top c1(u), left d0(v), right d1(v) as 4x3 Beziers."""
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    c0 = _bez3(sides["bottom"], u)
    c1 = _bez3(sides["top"], u)
    d0 = _bez3(sides["left"], v)
    d1 = _bez3(sides["right"], v)
    uu = u[..., None]
    vv = v[..., None]
    bil = ((1 - uu) * (1 - vv) * corners["c00"] + uu * (1 - vv) * corners["c10"]
           + (1 - uu) * vv * corners["c01"] + uu * vv * corners["c11"])
    return (1 - vv) * c0 + vv * c1 + (1 - uu) * d0 + uu * d1 - bil


def _coons_net(corners, sides):
    """The 4x4 Bernstein net (index [i][j]: i along u, j along v) of the
    bilinearly blended Coons patch: its two ruled parts are cubic in one
    parameter and linear (degree-elevated to cubic) in the other, and the
    bilinear correction is degree-elevated in both."""
    e = np.array([1.0, 2.0 / 3.0, 1.0 / 3.0, 0.0])          # (1 - t) in the cubic Bernstein basis
    net = np.zeros((4, 4, 3))
    for i in range(4):
        for j in range(4):
            net[i, j] = (e[j] * sides["bottom"][i] + (1 - e[j]) * sides["top"][i]
                         + e[i] * sides["left"][j] + (1 - e[i]) * sides["right"][j]
                         - (e[i] * e[j] * corners["c00"] + (1 - e[i]) * e[j] * corners["c10"]
                            + e[i] * (1 - e[j]) * corners["c01"] + (1 - e[i]) * (1 - e[j]) * corners["c11"]))
    return net


def bezier_patch(net, u, v):
    """Points of the bicubic Bezier patch ``net`` [4, 4, 3] at (u, v)."""
    u = np.asarray(u, np.float64)[..., None]
    v = np.asarray(v, np.float64)[..., None]
    bu = [(1 - u) ** 3, 3 * u * (1 - u) ** 2, 3 * u * u * (1 - u), u ** 3]
    bv = [(1 - v) ** 3, 3 * v * (1 - v) ** 2, 3 * v * v * (1 - v), v ** 3]
    return sum(bu[i] * bv[j] * net[i, j] for i in range(4) for j in range(4))


def _perim(u, v, eps):
    """Perimeter parameter in [0, 4) of a point on the square [eps, 1-eps]^2
    boundary, counter-clockwise from (eps, eps)."""
    w = 1.0 - 2.0 * eps
    if abs(v - eps) < 1e-12 and u < 1.0 - eps - 1e-12:
        return (u - eps) / w
    if abs(u - (1.0 - eps)) < 1e-12 and v < 1.0 - eps - 1e-12:
        return 1.0 + (v - eps) / w
    if abs(v - (1.0 - eps)) < 1e-12 and u > eps + 1e-12:
        return 2.0 + (1.0 - eps - u) / w
    return 3.0 + (1.0 - eps - v) / w


def _square_ring(n_side, eps):
    """``4*n_side`` points CCW on the boundary of [eps, 1-eps]^2, corners
    included, starting at (eps, eps)."""
    t = eps + (1.0 - 2.0 * eps) * np.arange(n_side) / n_side
    lo, hi = eps, 1.0 - eps
    pts = ([(x, lo) for x in t] + [(hi, y) for y in t]
           + [(hi - (x - lo), hi) for x in t] + [(lo, hi - (y - lo)) for y in t])
    return np.array(pts)


def coons_surface(seed: int, n_tri: int, n_bnd: int) -> Mesh:
    """A bilinear Coons patch over [0,1]^2 with cubic Bezier sides, tessellated
    into about ``n_tri`` triangles with a boundary loop of ``n_bnd`` edges
    (rounded to a multiple of 4, at least 8).

    Layout: an m x m grid over [eps, 1-eps]^2 with 2(m-1)^2 ~ n_tri triangles,
    an outer ring of n_bnd vertices on the parameter-square boundary, and a
    zipper strip that joins the two rings in order of perimeter parameter.
    All triangles are counter-clockwise in parameter space."""
    g = rng(seed)
    n_bnd = max(8, 4 * int(round(n_bnd / 4)))
    base = {"c00": np.array([0.0, 0.0]), "c10": np.array([1.0, 0.0]),
            "c01": np.array([0.0, 1.0]), "c11": np.array([1.0, 1.0])}
    corners = {}
    for key, xy in base.items():
        corners[key] = np.array([xy[0] + g.uniform(-0.1, 0.1),
                                 xy[1] + g.uniform(-0.1, 0.1),
                                 g.uniform(-0.5, 0.5)])

    def side(a, b):
        P = np.empty((4, 3))
        P[0], P[3] = a, b
        P[1] = a + (b - a) / 3.0 + g.uniform(-0.3, 0.3, 3)
        P[2] = a + 2.0 * (b - a) / 3.0 + g.uniform(-0.3, 0.3, 3)
        return P
    sides = {"bottom": side(corners["c00"], corners["c10"]),
             "top": side(corners["c01"], corners["c11"]),
             "left": side(corners["c00"], corners["c01"]),
             "right": side(corners["c10"], corners["c11"])}

    m = max(3, int(round(math.sqrt(max(n_tri - n_bnd, 8) / 2.0))) + 1)
    eps = 0.25 / (m - 1)
    # inner grid
    gu = eps + (1.0 - 2.0 * eps) * np.arange(m) / (m - 1)
    UU, VV = np.meshgrid(gu, gu, indexing="xy")      # [m(v), m(u)]
    inner_uv = np.stack([UU.ravel(), VV.ravel()], 1)  # id = iv*m + iu
    faces = []
    iu, iv = np.meshgrid(np.arange(m - 1), np.arange(m - 1), indexing="xy")
    iu, iv = iu.ravel(), iv.ravel()
    a = iv * m + iu
    b = iv * m + iu + 1
    c = (iv + 1) * m + iu + 1
    d = (iv + 1) * m + iu
    faces.append(np.stack([a, b, c], 1))
    faces.append(np.stack([a, c, d], 1))
    # inner ring ids CCW from (eps, eps)
    ns = m - 1
    ring_in = ([0 * m + i for i in range(ns)] + [j * m + (m - 1) for j in range(ns)]
               + [(m - 1) * m + (m - 1 - i) for i in range(ns)]
               + [(m - 1 - j) * m + 0 for j in range(ns)])
    ring_in = np.array(ring_in)
    # outer ring
    outer_uv = _square_ring(n_bnd // 4, 0.0)
    n_in = inner_uv.shape[0]
    ring_out = n_in + np.arange(n_bnd)
    s_out = np.array([_perim(u, v, 0.0) for u, v in outer_uv])
    s_in = np.array([_perim(u, v, eps) for u, v in inner_uv[ring_in]])
    no, ni = len(ring_out), len(ring_in)
    i = j = 0
    strip = []
    while i < no or j < ni:
        so = s_out[i + 1] if i + 1 < no else 4.0
        si = s_in[j + 1] if j + 1 < ni else 4.0
        if i < no and (so <= si or j >= ni):
            strip.append((ring_out[i], ring_out[(i + 1) % no], ring_in[j % ni]))
            i += 1
        else:
            strip.append((ring_out[i % no], ring_in[(j + 1) % ni], ring_in[j]))
            j += 1
    faces.append(np.array(strip))
    uv = np.concatenate([inner_uv, outer_uv], 0)
    V = _coons_eval(corners, sides, uv[:, 0], uv[:, 1])
    F = np.concatenate(faces, 0).astype(np.int32)
    # boundary curves in the orientation the (counter-clockwise) faces induce:
    # bottom, right, then top and left reversed
    curves = np.stack([sides["bottom"], sides["right"], sides["top"][::-1], sides["left"][::-1]])
    return Mesh(V.astype(np.float32), F, {"n_bnd": n_bnd, "m": m, "seed": seed, "curves": curves,
                                          "net": _coons_net(corners, sides)})


@dataclass
class CoonsBatch:
    meshes: list
    queries: list
    direction: np.ndarray


def _log_uniform_int(g, lo, hi):
    return int(round(math.exp(g.uniform(math.log(lo), math.log(hi)))))


def coons_batch(seed: int = 4, n_surf: int = 256, f_range=(1000, 200000),
                b_range=(32, 4096), q_range=(4096, 262144), scale: float = 1.0) -> CoonsBatch:
    """``n_surf`` Coons patches of uneven size, each with its own uniform
    queries in 1.2x its bounding box, and one shared direction.  ``scale``
    shrinks every size range (used for small test batches)."""
    g = rng(seed)
    meshes, queries = [], []
    for s in range(n_surf):
        nf = max(64, int(_log_uniform_int(g, *f_range) * scale))
        nb = max(8, int(_log_uniform_int(g, *b_range) * scale))
        nq = max(16, int(_log_uniform_int(g, *q_range) * scale))
        sub = int(g.integers(0, 2**31 - 1))
        M = coons_surface(sub, nf, nb)
        meshes.append(M)
        queries.append(box_queries(M.V, nq, sub + 1))
    return CoonsBatch(meshes, queries, random_direction(seed + 1000))


# ----------------------------------------------------------------------------
# Small meshes for definition checks
# ----------------------------------------------------------------------------

def icosphere(subdiv: int = 1, radius: float = 1.0, center=(0.0, 0.0, 0.0)) -> Mesh:
    """Closed icosphere with outward-facing triangles."""
    t = (1.0 + 5 ** 0.5) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
         (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
         (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
         (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    V = [np.array(v, float) / np.linalg.norm(v) for v in V]
    for _ in range(subdiv):
        cache = {}
        newF = []

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = V[i] + V[j]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            newF += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = newF
    V = np.array(V) * radius + np.asarray(center)
    return Mesh(V.astype(np.float32), np.array(F, np.int32))


def disk_fan(n: int = 64, radius: float = 1.0, z: float = 0.0) -> Mesh:
    """Flat disk in the plane z = ``z``: a fan of ``n`` triangles around the
    centre, counter-clockwise seen from +z (normal +z)."""
    ang = 2.0 * np.pi * np.arange(n) / n
    rim = np.stack([radius * np.cos(ang), radius * np.sin(ang), np.full(n, z)], 1)
    V = np.concatenate([[[0.0, 0.0, z]], rim], 0)
    k = np.arange(n)
    F = np.stack([np.zeros(n, int), 1 + k, 1 + (k + 1) % n], 1)
    return Mesh(V.astype(np.float32), F.astype(np.int32))


def bumpy_cap(seed: int = 7, n_lon: int = 12, n_rings: int = 6, cap_deg: float = 50.0,
              amp: float = 0.15) -> Mesh:
    """Small open sphere (noise-displaced, cap removed) for brute-force pins."""
    return open_sphere(seed, n_lon=n_lon, n_rings=n_rings, cap_deg=cap_deg, amp=amp)


def random_open_mesh(seed: int, n: int = 5) -> Mesh:
    """A small bent, twisted (n x n)-vertex grid sheet: an open surface whose
    boundary projects with self-intersections from many viewpoints."""
    g = rng(seed)
    u = np.linspace(0.0, 1.0, n)
    UU, VV = np.meshgrid(u, u, indexing="xy")
    x = UU + 0.15 * g.normal(size=UU.shape)
    y = VV + 0.15 * g.normal(size=UU.shape)
    z = 0.8 * np.sin(3.0 * UU + 1.0) * np.cos(2.0 * VV) + 0.2 * g.normal(size=UU.shape)
    V = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
    iu, iv = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="xy")
    iu, iv = iu.ravel(), iv.ravel()
    a, b = iv * n + iu, iv * n + iu + 1
    c, d = (iv + 1) * n + iu + 1, (iv + 1) * n + iu
    F = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], 0)
    return Mesh(V.astype(np.float32), F.astype(np.int32))
