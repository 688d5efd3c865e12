"""Pins for the 3D FP64 oracle (CPU only).

Each check ties ``oracle.wn3d`` to something other than itself: the plain
per-triangle solid-angle sum (the definition of w_M, Sec. 3), quadrature of
Eq. wn_chi over directions with an independent Moller-Trumbore crossing
count, the flat-disk closed form, closed surfaces (Sec. 3: inside/outside),
Lemma 2 (Sec. 5), and invariances (change of d, orientation flip, union as a
sum of winding numbers as in Sec. 7, Fig. bool).
"""
import math

import numpy as np
import pytest

import synth
from oracle import wn3d as W


def vos_solid_angle_w(V, F, P):
    """w = (1/4pi) sum over triangles of the signed solid angle, each from the
    Van Oosterom-Strackee formula tan(Omega/2) = a.(b x c) / (|a||b||c| +
    (a.b)|c| + (a.c)|b| + (b.c)|a|)."""
    V = np.asarray(V, np.float64)
    out = []
    for p in np.atleast_2d(P):
        a = V[F[:, 0]] - p
        b = V[F[:, 1]] - p
        c = V[F[:, 2]] - p
        la, lb, lc = (np.linalg.norm(x, axis=1) for x in (a, b, c))
        num = np.einsum("ij,ij->i", a, np.cross(b, c))
        den = (la * lb * lc + np.einsum("ij,ij->i", a, b) * lc
               + np.einsum("ij,ij->i", a, c) * lb + np.einsum("ij,ij->i", b, c) * la)
        out.append(np.sum(2.0 * np.arctan2(num, den)) / (4.0 * math.pi))
    return np.array(out)


def moller_trumbore_chi(V, F, p, dirs):
    """Signed crossing count for many directions from one point, by the
    Moller-Trumbore ray/triangle test (an independent formulation)."""
    V = np.asarray(V, np.float64)
    v0, v1, v2 = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    e1, e2 = v1 - v0, v2 - v0
    n = np.cross(e1, e2)
    chi = np.zeros(len(dirs), np.int64)
    s = p - v0                                            # [f, 3]
    for k in range(0, len(dirs), 4096):
        D = dirs[k:k + 4096]                              # [m, 3]
        h = np.cross(D[:, None, :], e2[None, :, :])       # [m, f, 3]
        det = np.einsum("fk,mfk->mf", e1, h)
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / det
            u = np.einsum("fk,mfk->mf", s, h) * inv
            q = np.cross(s, e1)                           # [f, 3]
            v = np.einsum("mk,fk->mf", D, q) * inv
            t = np.einsum("fk,fk->f", e2, q)[None, :] * inv
        hit = (u > 0) & (v > 0) & (u + v < 1) & (t > 0)
        sg = np.sign(D @ n.T)
        chi[k:k + 4096] = np.sum(np.where(hit, sg, 0), axis=1).astype(np.int64)
    return chi


def fibonacci_sphere(n):
    i = np.arange(n) + 0.5
    z = 1.0 - 2.0 * i / n
    r = np.sqrt(1.0 - z * z)
    ph = math.pi * (3.0 - math.sqrt(5.0)) * i
    return np.stack([r * np.cos(ph), r * np.sin(ph), z], 1)


MESHES = {
    "bumpy_cap": lambda: synth.bumpy_cap(),
    "twisted_sheet": lambda: synth.random_open_mesh(3, n=5),
    "coons": lambda: synth.coons_surface(11, 300, 40),
}


@pytest.mark.parametrize("name", list(MESHES))
def test_boundary_loops_follow_faces(name):
    M = MESHES[name]()
    loops = W.boundary_loops(M.F)
    assert len(loops) == 1
    directed = {(int(a), int(b)) for f in M.F for a, b in ((f[0], f[1]), (f[1], f[2]), (f[2], f[0]))}
    for L in loops:
        for i in range(len(L)):
            e = (int(L[i]), int(L[(i + 1) % len(L)]))
            assert e in directed                       # oriented as in its face
            assert (e[1], e[0]) not in directed        # used by one face only


def test_boundary_loops_sphere_counts():
    M = synth.open_sphere(5, n_lon=24, n_rings=8, top_refine=3)
    loops = W.boundary_loops(M.F)
    assert [len(L) for L in loops] == [72]
    assert W.boundary_loops(synth.icosphere(1).F) == []


@pytest.mark.parametrize("name", list(MESHES))
def test_matches_per_triangle_solid_angle(name):
    M = MESHES[name]()
    P = synth.rng(1).uniform(-1.5, 1.5, (150, 3))
    ref = vos_solid_angle_w(M.V, M.F, P)
    for seed in (5, 6, 7):
        r = W.wn3d(M.V, M.F, P, synth.random_direction(seed), margins=True)
        ok = ~r.degenerate
        assert ok.sum() > 140
        np.testing.assert_allclose(r["w"][ok], ref[ok], atol=1e-12, rtol=0)


def test_direction_quadrature_of_eq_wn_chi():
    M = synth.random_open_mesh(4, n=3)                # 8 triangles
    dirs = fibonacci_sphere(2 ** 17)
    P = synth.rng(2).uniform(-0.3, 1.3, (4, 3))
    for p in P:
        wq = moller_trumbore_chi(M.V, M.F, p, dirs).mean()
        w = W.wn3d(M.V, M.F, p[None], synth.random_direction(3), margins=False)["w"][0]
        assert abs(w - wq) < 2e-3, (w, wq)


def test_crossings_match_moller_trumbore():
    M = synth.bumpy_cap()
    g = synth.rng(3)
    for _ in range(30):
        p = g.uniform(-1.3, 1.3, 3)
        d = synth.random_direction(int(g.integers(1 << 30)))
        chi, m = W.crossings(M.V, M.F, p[None], d, margins=True)
        if m["m_ray"][0] < W.BAND or m["m_surf"][0] < W.BAND or m["m_self"][0] < W.BAND_SELF:
            continue
        assert chi[0] == moller_trumbore_chi(M.V, M.F, p, d[None])[0]


def test_flat_disk_closed_form():
    R = 1.0
    M = synth.disk_fan(4096, R)
    zs = np.array([-2.0, -0.5, -0.1, 0.1, 0.5, 2.0])
    P = np.stack([np.zeros_like(zs), np.zeros_like(zs), zs], 1)
    r = W.wn3d(M.V, M.F, P, synth.random_direction(8))
    expect = -np.sign(zs) * 0.5 * (1.0 - np.abs(zs) / np.sqrt(zs * zs + R * R))
    # inscribed 4096-gon: relative area defect ~ (2 pi / n)^2 / 6
    np.testing.assert_allclose(r["w"], expect, atol=2e-6)


def test_closed_mesh_is_inside_outside():
    M = synth.icosphere(2, radius=1.0)
    P = synth.rng(4).uniform(-1.6, 1.6, (400, 3))
    rad = np.linalg.norm(P, axis=1)
    keep = np.abs(rad - 1.0) > 0.06                   # away from the faceted surface
    r = W.wn3d(M.V, M.F, P[keep], synth.random_direction(9))
    assert np.array_equal(r["w"], (rad[keep] < 1.0).astype(float))
    assert np.all(r["S"] == 0.0)


def test_open_sphere_from_centre():
    # undisplaced sphere with a 30 degree cap removed, seen from its centre:
    # w = 1 - (solid angle of the hole)/4pi, the hole being a regular n-gon cone
    n = 256
    M = synth.open_sphere(1, n_lon=n, n_rings=32, cap_deg=30.0, amp=0.0)
    w = W.wn3d(M.V, M.F, np.zeros((1, 3)), synth.random_direction(10))["w"][0]
    cap = 1.0 - math.cos(math.radians(30.0))
    assert abs(w - (1.0 - cap / 2.0)) < 2e-4


@pytest.mark.parametrize("name", list(MESHES))
def test_direction_invariance(name):
    M = MESHES[name]()
    P = synth.rng(5).uniform(-1.5, 1.5, (100, 3))
    rs = [W.wn3d(M.V, M.F, P, synth.random_direction(s)) for s in (11, 12, 13, 14)]
    ok = np.logical_and.reduce([~r.degenerate for r in rs])
    for r in rs[1:]:
        np.testing.assert_allclose(r["w"][ok], rs[0]["w"][ok], atol=1e-12, rtol=0)


def test_orientation_flip_negates():
    M = synth.bumpy_cap()
    Ff = M.F[:, ::-1].copy()
    P = synth.rng(6).uniform(-1.5, 1.5, (100, 3))
    d = synth.random_direction(15)
    a = W.wn3d(M.V, M.F, P, d)
    b = W.wn3d(M.V, Ff, P, d)
    ok = ~a.degenerate & ~b.degenerate
    np.testing.assert_allclose(b["w"][ok], -a["w"][ok], atol=1e-12)


def test_union_is_sum():
    A = synth.bumpy_cap()
    B = synth.random_open_mesh(5, n=4)
    VB = B.V + np.float32(2.0)
    V = np.concatenate([A.V, VB], 0)
    F = np.concatenate([A.F, B.F + len(A.V)], 0)
    P = synth.rng(7).uniform(-1.5, 3.5, (120, 3))
    d = synth.random_direction(16)
    u = W.wn3d(V, F, P, d)
    a = W.wn3d(A.V, A.F, P, d)
    b = W.wn3d(VB, B.F, P, d)
    ok = ~u.degenerate & ~a.degenerate & ~b.degenerate
    np.testing.assert_allclose(u["w"][ok], a["w"][ok] + b["w"][ok], atol=1e-12)


def test_lemma2_chi_steps_by_one_across_a_boundary_edge():
    M = synth.random_open_mesh(3, n=4)
    V = M.V.astype(np.float64)
    L = W.boundary_loops(M.F)[0]
    g = synth.rng(8)
    for _ in range(40):
        p = g.uniform(-0.5, 1.5, 3)
        i = int(g.integers(len(L)))
        a = V[L[i]] - p
        b = V[L[(i + 1) % len(L)]] - p
        m = (a + b) / np.linalg.norm(a + b)
        tau = (b - a) - ((b - a) @ m) * m
        tau /= np.linalg.norm(tau)
        nrm = np.cross(m, tau)                      # in-sphere normal n x tau
        up = W.crossings(M.V, M.F, p[None], m + 1e-6 * nrm)[0]
        dn = W.crossings(M.V, M.F, p[None], m - 1e-6 * nrm)[0]
        assert up - dn == 1


def test_w_is_continuous_where_chi_jumps():
    # moving p across the ray/boundary crossing changes chi by one and the
    # boundary term by the opposite amount
    M = synth.bumpy_cap()
    V = M.V.astype(np.float64)
    L = W.boundary_loops(M.F)[0]
    d = synth.random_direction(17)
    a, b = V[L[0]], V[L[1]]
    mid = 0.5 * (a + b)
    side = np.cross(d, b - a)
    side /= np.linalg.norm(side)
    base = mid - 0.7 * d                             # ray from base passes through mid
    P = np.stack([base + 1e-7 * side, base - 1e-7 * side])
    r = W.wn3d(M.V, M.F, P, d)
    assert abs(r["chi"][0] - r["chi"][1]) == 1
    assert abs(r["w"][0] - r["w"][1]) < 1e-5


def test_translation_and_scale_invariance():
    M = synth.random_open_mesh(6, n=4)
    P = synth.rng(9).uniform(-0.5, 1.5, (60, 3))
    d = synth.random_direction(18)
    a = W.wn3d(M.V, M.F, P, d)
    s, t = 2.5, np.array([0.25, -0.5, 1.0])
    b = W.wn3d(M.V.astype(np.float64) * s + t, M.F, P * s + t, d)
    ok = ~a.degenerate & ~b.degenerate
    np.testing.assert_allclose(b["w"][ok], a["w"][ok], atol=1e-12)


def test_margins_flag_a_ray_through_a_vertex():
    M = synth.bumpy_cap()
    V = M.V.astype(np.float64)
    d = synth.random_direction(19)
    v = V[40]
    p = v - 0.8 * d                                  # ray passes exactly through vertex 40
    r = W.wn3d(M.V, M.F, p[None], d)
    assert r.degenerate[0]
