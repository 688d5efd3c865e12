"""Pins of the 2D gradient oracle (oracle.grad2d) against the 2D value
oracle (oracle.wn2d): central finite differences, zero response to interior
control points and closed loops, translation identity."""
import numpy as np

import synth
from oracle import grad2d as G
from oracle import wn2d as O


def _setup():
    C = synth.loops2d(seed=5, n_loops=5, seg_per_loop=6, n_open=3, dtype=np.float64)
    g = synth.rng(6)
    P = g.uniform(-0.9, 0.9, (40, 2))
    r = O.wn2d(C.ctrl, C.loop_off, C.closed, P)
    keep = ~r.degenerate & (r["m_x"] > 1e-3) & (r["m_joint"] > 1e-3)
    return C, P[keep][:25], g.normal(size=int(keep.sum()))[:25]


def _w(C, ctrl, P):
    return O.wn2d(ctrl, C.loop_off, C.closed, P, margins=False)["w"]


def test_query_gradient_matches_central_differences():
    C, P, gw = _setup()
    gq, _ = G.grad2d(C.ctrl, C.loop_off, C.closed, P, gw)
    h = 1e-6
    for k in range(2):
        e = np.zeros(2)
        e[k] = h
        fd = (_w(C, C.ctrl, P + e) - _w(C, C.ctrl, P - e)) / (2 * h)
        assert np.allclose(gw * fd, gq[:, k], rtol=1e-6, atol=1e-7)


def test_end_point_gradients_match_central_differences():
    C, P, gw = _setup()
    _, gc = G.grad2d(C.ctrl, C.loop_off, C.closed, P, gw)
    h = 1e-6
    checked = 0
    for l in range(len(C.closed)):
        if C.closed[l]:
            continue
        a, b = int(C.loop_off[l]), int(C.loop_off[l + 1])
        for seg, pt in ((a, 0), (b - 1, 3)):
            for k in range(2):
                cp, cm = C.ctrl.copy(), C.ctrl.copy()
                cp[seg, pt, k] += h
                cm[seg, pt, k] -= h
                fd = np.sum(gw * (_w(C, cp, P) - _w(C, cm, P))) / (2 * h)
                assert abs(fd - gc[seg, pt, k]) <= 1e-6 * max(1.0, abs(fd)), (l, seg, pt, k)
                checked += 1
    assert checked == 12


def test_interior_points_and_closed_loops_have_no_gradient():
    C, P, gw = _setup()
    _, gc = G.grad2d(C.ctrl, C.loop_off, C.closed, P, gw)
    h = 1e-6
    rng = synth.rng(7)
    for _ in range(12):
        seg = int(rng.integers(C.ctrl.shape[0]))
        pt = int(rng.integers(4))
        l = int(np.searchsorted(C.loop_off, seg, side="right") - 1)
        first, last = int(C.loop_off[l]), int(C.loop_off[l + 1]) - 1
        if not C.closed[l] and ((seg, pt) == (first, 0) or (seg, pt) == (last, 3)):
            continue
        cp, cm = C.ctrl.copy(), C.ctrl.copy()
        cp[seg, pt, 0] += h
        cm[seg, pt, 0] -= h
        # a closed loop's first/last points are a joint: move both copies together
        if C.closed[l] and (seg, pt) in ((first, 0), (last, 3)):
            for s2, p2 in ((first, 0), (last, 3)):
                cp[s2, p2, 0] = C.ctrl[s2, p2, 0] + h
                cm[s2, p2, 0] = C.ctrl[s2, p2, 0] - h
        fd = (_w(C, cp, P) - _w(C, cm, P)) / (2 * h)
        assert np.abs(fd).max() < 1e-8
        assert gc[seg, pt, 0] == 0.0


def test_translation_identity():
    C, P, gw = _setup()
    gq, gc = G.grad2d(C.ctrl, C.loop_off, C.closed, P, gw)
    assert np.allclose(gq.sum(0) + gc.reshape(-1, 2).sum(0), 0.0, atol=1e-10)
