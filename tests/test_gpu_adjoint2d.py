"""GPU tests of the 2D adjoint (wn_backward_2d): gradients with respect to
the queries and the control points against the FP64 oracle (oracle.grad2d,
pinned by finite differences of oracle.wn2d), in points and grid mode, at
the full 2048^2 grid size; closed curves give exact zeros; fixed-order
reductions are bitwise reproducible; the autograd path agrees."""
import numpy as np
import pytest
import torch

import synth
from oracle import grad2d as G

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2408_04466_amd as W

REL = 1e-3


def _close(gpu, ref, what):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max()
    assert np.abs(gpu - ref).max() <= REL * scale + 1e-12, f"{what}: normwise"
    tol = REL * np.maximum(np.abs(ref), 1e-3 * scale) + 1e-12
    bad = np.abs(gpu - ref) > tol
    assert not bad.any(), f"{what}: {int(bad.sum())} components off, worst {np.abs(gpu - ref)[bad].max()}"


def _upload(C, dt):
    return torch.from_numpy(C.ctrl.astype(dt)).cuda()


def test_points_mode_matches_oracle():
    C = synth.loops2d()                                   # 16 loops, 4 open, float32
    g = synth.rng(21)
    P = g.uniform(-1.2, 1.2, (20000, 2)).astype(np.float32)
    gw = g.normal(size=len(P)).astype(np.float32)
    ctrl = _upload(C, np.float32)
    x, y = (torch.from_numpy(np.ascontiguousarray(P[:, k])).cuda() for k in range(2))
    gq, gc = W.backward_2d(ctrl, C.loop_off, C.closed, x, y, torch.from_numpy(gw).cuda())
    torch.cuda.synchronize()
    rq, rc = G.grad2d(C.ctrl, C.loop_off, C.closed, P, gw)
    _close(gq.cpu().numpy(), rq, "grad_q")
    _close(gc.cpu().numpy(), rc, "grad_ctrl")
    nz = np.abs(rc) > 0
    assert nz.sum() == 4 * 4 and np.all(gc.cpu().numpy()[~nz] == 0.0)


def test_full_size_grid_matches_oracle_and_is_deterministic():
    C = synth.loops2d()
    ax = synth.grid_axis(-1.2, 1.2, 2048, np.float32)
    g = synth.rng(22)
    gw = g.normal(size=(2048, 2048)).astype(np.float32)
    ctrl = _upload(C, np.float32)
    xs = torch.from_numpy(ax).cuda()
    gwt = torch.from_numpy(gw).cuda()
    gq, gc = W.backward_2d(ctrl, C.loop_off, C.closed, xs, xs, gwt, grid=True)
    gq2, gc2 = W.backward_2d(ctrl, C.loop_off, C.closed, xs, xs, gwt, grid=True)
    torch.cuda.synchronize()
    assert torch.equal(gq, gq2) and torch.equal(gc, gc2)
    assert tuple(gq.shape) == (2048, 2048, 2)
    X, Y = np.meshgrid(ax, ax, indexing="xy")
    P = np.stack([X.ravel(), Y.ravel()], 1)
    rq, rc = G.grad2d(C.ctrl, C.loop_off, C.closed, P, gw.ravel())
    _close(gc.cpu().numpy(), rc, "grad_ctrl")
    rows = synth.rng(23).choice(2048, 16, replace=False)
    sel = (rows[:, None] * 2048 + np.arange(2048)[None, :]).ravel()
    _close(gq.cpu().numpy().reshape(-1, 2)[sel], rq[sel], "grad_q")


def test_closed_curves_have_zero_gradient_fp64():
    C = synth.star2d()                                    # one closed loop, float64
    ctrl = _upload(C, np.float64)
    ax = torch.from_numpy(synth.grid_axis(-1.5, 1.5, 128)).cuda()
    gw = torch.ones(128, 128, dtype=torch.float64, device="cuda")
    gq, gc = W.backward_2d(ctrl, C.loop_off, C.closed, ax, ax, gw, grid=True)
    torch.cuda.synchronize()
    assert torch.count_nonzero(gq) == 0 and torch.count_nonzero(gc) == 0


def test_fp64_open_curves_match_oracle_tightly():
    C = synth.loops2d(seed=9, n_loops=6, seg_per_loop=8, n_open=3, dtype=np.float64)
    g = synth.rng(24)
    P = g.uniform(-1.0, 1.0, (3000, 2))
    gw = g.normal(size=len(P))
    ctrl = _upload(C, np.float64)
    x, y = (torch.from_numpy(np.ascontiguousarray(P[:, k])).cuda() for k in range(2))
    gq, gc = W.backward_2d(ctrl, C.loop_off, C.closed, x, y, torch.from_numpy(gw).cuda())
    torch.cuda.synchronize()
    rq, rc = G.grad2d(C.ctrl, C.loop_off, C.closed, P, gw)
    assert np.allclose(gq.cpu().numpy(), rq, rtol=1e-9, atol=1e-9 * np.abs(rq).max())
    assert np.allclose(gc.cpu().numpy(), rc, rtol=1e-9, atol=1e-9 * np.abs(rc).max())


def test_autograd_and_edge_cases():
    C = synth.loops2d(seed=3, n_loops=4, seg_per_loop=10, n_open=2)
    ctrl = _upload(C, np.float32).requires_grad_(True)
    g = synth.rng(25)
    P = g.uniform(-1, 1, (4000, 2)).astype(np.float32)
    x = torch.from_numpy(np.ascontiguousarray(P[:, 0])).cuda().requires_grad_(True)
    y = torch.from_numpy(np.ascontiguousarray(P[:, 1])).cuda().requires_grad_(True)
    t = torch.from_numpy(synth.targets01(len(P), 26)).cuda()
    w = W.winding_number_2d(ctrl, C.loop_off, C.closed, x, y)
    loss = ((w - t) ** 2).sum()
    loss.backward()
    gq, gc = W.backward_2d(ctrl.detach(), C.loop_off, C.closed, x.detach(), y.detach(), (2 * (w - t)).detach())
    torch.cuda.synchronize()
    assert torch.equal(ctrl.grad, gc) and torch.equal(x.grad, gq[:, 0]) and torch.equal(y.grad, gq[:, 1])
    # non-finite queries: NaN gradient, excluded from the control-point sums
    P2 = P.copy()
    P2[:5] = np.nan
    x2, y2 = (torch.from_numpy(np.ascontiguousarray(P2[:, k])).cuda() for k in range(2))
    ones = torch.ones(len(P), device="cuda")
    gq2, gc2 = W.backward_2d(ctrl.detach(), C.loop_off, C.closed, x2, y2, ones)
    rq, rc = G.grad2d(C.ctrl, C.loop_off, C.closed, P2[5:], np.ones(len(P) - 5))
    torch.cuda.synchronize()
    assert torch.isnan(gq2[:5]).all() and torch.isfinite(gq2[5:]).all()
    _close(gc2.cpu().numpy(), rc, "grad_ctrl with NaN queries")
    # empty query set: grad_ctrl fully written with zeros
    e = torch.empty(0, device="cuda")
    _, gc3 = W.backward_2d(ctrl.detach(), C.loop_off, C.closed, e, e, e)
    torch.cuda.synchronize()
    assert torch.count_nonzero(gc3) == 0
