"""GPU tests of the curve adjoint (wn_backward_curves): gradients with
respect to the queries and the Bezier control points against the FP64
oracle (oracle.gradcurves, pinned by finite differences of the curve-term
oracle) within 1e-3 relative; straight Beziers against the polyline adjoint
through the chain rule; fixed-order reductions bitwise reproducible; the
autograd path; edge cases; and 2^20 queries through the translation
identity."""
import numpy as np
import pytest
import torch

import synth
from oracle import gradcurves as GC

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2408_04466_amd as W
    from gpu_util import DevMesh

REL = 1e-3


def _q(P):
    P = np.ascontiguousarray(np.asarray(P, np.float32))
    return tuple(torch.from_numpy(np.ascontiguousarray(P[:, k])).cuda() for k in range(3))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


def _close(gpu, ref, what):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max()
    assert np.abs(gpu - ref).max() <= REL * scale + 1e-12, f"{what}: normwise {np.abs(gpu - ref).max() / scale:.3g}"
    tol = REL * np.maximum(np.abs(ref), 1e-3 * scale) + 1e-12
    bad = np.abs(gpu - ref) > tol
    assert not bad.any(), f"{what}: {int(bad.sum())} components off"


def _near(curves, n, seed):
    g = synth.rng(seed)
    out = []
    for k in range(n):
        c = curves[k % len(curves)]
        t = g.uniform(0.02, 0.98)
        s = 1 - t
        pt = s ** 3 * c[0] + 3 * s * s * t * c[1] + 3 * s * t * t * c[2] + t ** 3 * c[3]
        off = g.normal(size=3)
        out.append(pt + off / np.linalg.norm(off) * 10 ** g.uniform(-3, -1))
    return np.array(out)


@pytest.mark.parametrize("seed", [71, 72])
def test_matches_oracle(seed):
    M = synth.coons_surface(seed, 500, 32)
    curves = M.info["curves"].astype(np.float32).astype(np.float64)
    P = np.concatenate([synth.box_queries(M.V, 300, seed + 1), _near(curves, 100, seed + 2)])
    P = P.astype(np.float32).astype(np.float64)
    gw = synth.rng(seed + 3).normal(size=len(P)).astype(np.float32)
    gq, gc = W.backward_curves(_dev(curves), *_q(P), torch.from_numpy(gw).cuda())
    torch.cuda.synchronize()
    rq, rc = GC.grad_curves(curves, P, gw.astype(np.float64))
    _close(gq.cpu().numpy(), rq, "grad_q")
    _close(gc.cpu().numpy(), rc, "grad_ctrl")


def test_straight_beziers_equal_the_polyline_adjoint():
    M = synth.bumpy_cap()
    d = synth.random_direction(73)
    dm = DevMesh(M, d)
    B = dm.bnd.cpu().numpy().astype(np.float64)
    lo = dm.loop_off
    curves, ends = [], []
    for l in range(len(lo) - 1):
        a0, a1 = lo[l], lo[l + 1]
        for i in range(a0, a1):
            j = a0 + (i + 1 - a0) % (a1 - a0)
            curves.append([B[i], (2 * B[i] + B[j]) / 3, (B[i] + 2 * B[j]) / 3, B[j]])
            ends.append((i, j))
    curves = np.array(curves)
    P = synth.box_queries(M.V, 2000, 74)
    gw = torch.from_numpy(synth.rng(75).normal(size=len(P)).astype(np.float32)).cuda()
    gq, gc = W.backward_curves(_dev(curves), *_q(P), gw)
    pq, pb = W.backward(dm.bnd, dm.loop_off, *_q(P), gw)
    torch.cuda.synchronize()
    gc = gc.cpu().numpy().astype(np.float64)
    gv = np.zeros((len(B), 3))
    for (i, j), g4 in zip(ends, gc):
        gv[i] += g4[0] + (2 / 3) * g4[1] + (1 / 3) * g4[2]
        gv[j] += g4[3] + (1 / 3) * g4[1] + (2 / 3) * g4[2]
    _close(gq.cpu().numpy(), pq.cpu().numpy(), "grad_q vs polyline")
    _close(gv, pb.cpu().numpy(), "vertex gradients vs polyline")


def test_deterministic_autograd_and_edge_cases():
    M = synth.coons_surface(76, 500, 32)
    curves = _dev(M.info["curves"])
    d = synth.random_direction(77)
    dm = DevMesh(M, d)
    P = synth.box_queries(M.V, 3000, 78)
    gw = torch.from_numpy(synth.rng(79).normal(size=len(P)).astype(np.float32)).cuda()
    a = W.backward_curves(curves, *_q(P), gw)
    b = W.backward_curves(curves, *_q(P), gw)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    # autograd through winding_number_curves
    c = curves.clone().requires_grad_(True)
    qx, qy, qz = (t.clone().requires_grad_(True) for t in _q(P))
    w = W.winding_number_curves(dm.bvh, c, qx, qy, qz)
    (w * gw).sum().backward()
    torch.cuda.synchronize()
    assert torch.equal(c.grad, a[1]) and torch.equal(qx.grad, a[0][:, 0]) and torch.equal(qz.grad, a[0][:, 2])
    # non-finite queries: NaN gradient, no contribution to the control points
    P2 = P.copy()
    P2[:4] = np.nan
    g2q, g2c = W.backward_curves(curves, *_q(P2), gw)
    g3q, g3c = W.backward_curves(curves, *_q(P[4:]), gw[4:].contiguous())
    torch.cuda.synchronize()
    assert torch.isnan(g2q[:4]).all() and torch.isfinite(g2q[4:]).all()
    assert torch.allclose(g2c, g3c, rtol=1e-5, atol=1e-7)
    # no queries: zero control-point gradient; no curves: zero query gradient
    e = torch.empty(0, device="cuda")
    _, z = W.backward_curves(curves, e, e, e, e)
    zq, _ = W.backward_curves(torch.zeros((0, 4, 3), device="cuda"), *_q(P), gw)
    torch.cuda.synchronize()
    assert torch.count_nonzero(z) == 0 and torch.count_nonzero(zq) == 0


def test_full_size_translation_identity():
    """2^20 queries: moving every control point by delta changes L like moving
    every query by -delta, so sum grad_ctrl = -sum grad_q; grad_q on samples
    against the oracle."""
    M = synth.coons_surface(6, 4000, 64)
    curves = M.info["curves"].astype(np.float32).astype(np.float64)
    P = synth.box_queries(M.V, 1 << 20, 7)
    gw = synth.rng(80).normal(size=len(P)).astype(np.float32)
    gq, gc = W.backward_curves(_dev(curves), *_q(P), torch.from_numpy(gw).cuda())
    torch.cuda.synchronize()
    gq, gc = gq.cpu().numpy().astype(np.float64), gc.cpu().numpy().astype(np.float64)
    s_c, s_q = gc.sum((0, 1)), gq.sum(0)
    assert np.abs(s_c + s_q).max() <= 1e-3 * np.abs(s_q).max()
    sample = synth.rng(81).choice(len(P), 100, replace=False)
    rq, _ = GC.grad_curves(curves, P[sample].astype(np.float64), gw[sample].astype(np.float64))
    _close(gq[sample], rq, "grad_q (2^20 queries, sample)")
