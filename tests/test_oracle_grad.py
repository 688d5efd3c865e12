"""Pins for the FP64 gradient oracle (CPU only).

``oracle.grad3d`` is tied to central finite differences of ``oracle.wn3d``,
to Gauss-Legendre quadrature of the hat-weighted Biot-Savart line integrals
that its closed form evaluates, and to the translation / scaling / rotation
identities that any derivative of a solid angle must satisfy.
"""
import math

import numpy as np

import synth
from oracle import grad3d as G
from oracle import wn3d as W


def _setup():
    M = synth.bumpy_cap()
    loops = W.boundary_loops(M.F)
    Lx = W.loops_coords(M.V, loops)
    g = synth.rng(1)
    P = g.uniform(-1.5, 1.5, (400, 3))
    # keep queries well away from every vertex (hence from the surface)
    V = M.V.astype(np.float64)
    dist = np.array([np.sqrt(((V - p) ** 2).sum(1)).min() for p in P])
    P = P[dist > 0.3][:40]
    return M, loops, Lx, P


def test_grad_p_matches_central_differences():
    M, loops, Lx, P = _setup()
    d = synth.random_direction(3)
    gp, _ = G.grad3d(Lx, P)
    for h, tol in ((1e-4, 1e-6), (1e-6, 1e-8)):
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            fd = (W.wn3d(M.V, M.F, P + e, d, margins=False)["w"]
                  - W.wn3d(M.V, M.F, P - e, d, margins=False)["w"]) / (2 * h)
            assert np.abs(fd - gp[:, k]).max() < tol * max(1.0, np.abs(gp).max())


def test_grad_vertices_matches_central_differences():
    M, loops, Lx, P = _setup()
    d = synth.random_direction(4)
    gw = synth.rng(2).normal(size=len(P))
    _, gv = G.grad3d(Lx, P, gw)
    V = M.V.astype(np.float64)
    L = loops[0]
    h = 1e-4
    for j in (0, 3, 7):
        for k in range(3):
            Vp, Vm = V.copy(), V.copy()
            Vp[L[j], k] += h
            Vm[L[j], k] -= h
            fd = (gw @ W.wn3d(Vp, M.F, P, d, margins=False)["w"]
                  - gw @ W.wn3d(Vm, M.F, P, d, margins=False)["w"]) / (2 * h)
            assert abs(fd - gv[0][j, k]) < 1e-6 * max(1.0, np.abs(gv[0]).max())


def test_hat_weighted_integrals_by_gauss_legendre():
    # the closed form rests on int_0^1 (1-s)/|a+s(b-a)|^3 ds = K/|a| and
    # int_0^1 s/|a+s(b-a)|^3 ds = K/|b|, K = 1/(|a||b| + a.b)
    x, wq = np.polynomial.legendre.leggauss(200)
    s = 0.5 * (x + 1.0)
    wq = 0.5 * wq
    g = synth.rng(3)
    for _ in range(20):
        a, b = g.normal(size=3), g.normal(size=3)
        r = a[None, :] + s[:, None] * (b - a)[None, :]
        inv3 = 1.0 / np.linalg.norm(r, axis=1) ** 3
        K = 1.0 / (np.linalg.norm(a) * np.linalg.norm(b) + a @ b)
        if K > 50:          # segment passes too close to the origin for 200 nodes
            continue
        assert abs(np.sum(wq * (1 - s) * inv3) - K / np.linalg.norm(a)) < 1e-9 * K
        assert abs(np.sum(wq * s * inv3) - K / np.linalg.norm(b)) < 1e-9 * K


def test_gradient_identities():
    M, loops, Lx, P = _setup()
    for p in P[:10]:
        gp, gv = G.grad3d(Lx, p[None])
        gv = gv[0]
        rel = Lx[0] - p
        # translation: sum_v dw/dv + grad_p w = 0
        assert np.abs(gv.sum(0) + gp[0]).max() < 1e-14
        # uniform scaling about p leaves w unchanged
        assert abs(np.sum(rel * gv)) < 1e-13
        # rotation about p leaves w unchanged
        assert np.abs(np.cross(rel, gv).sum(0)).max() < 1e-13


def test_gradient_independent_of_direction_and_seeded_loss():
    M, loops, Lx, P = _setup()
    t = synth.targets01(len(P), 5).astype(np.float64)
    # L = sum (w - t)^2 ; dL/dw = 2 (w - t) ; with two directions the values
    # of w agree, hence so do the gradients
    w1 = W.wn3d(M.V, M.F, P, synth.random_direction(6), margins=False)["w"]
    w2 = W.wn3d(M.V, M.F, P, synth.random_direction(7), margins=False)["w"]
    np.testing.assert_allclose(w1, w2, atol=1e-12)
    gp, gv = G.grad3d(Lx, P, 2.0 * (w1 - t))
    assert np.all(np.isfinite(gp)) and np.all(np.isfinite(gv[0]))
    assert math.isfinite(float(np.abs(gv[0]).sum()))
