"""GPU tests of the query order (wn_spatial_order): the permutation equals a
stable argsort of Morton codes computed here in numpy from the definition in
the header (float32 cell arithmetic, 1024 cells per axis over the finite
queries' bounding box, non-finite last); it is deterministic; degenerate
inputs (one query, identical queries, a flat box); and evaluation is
independent of the order: the mesh, curve and patch paths give w[order],
chi[order] bit for bit on q[order], also at 2^20 queries."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2408_04466_amd as W
    from gpu_util import DevMesh


def _q(P):
    P = np.ascontiguousarray(np.asarray(P, np.float32))
    return tuple(torch.from_numpy(np.ascontiguousarray(P[:, k])).cuda() for k in range(3))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


def _spread(x):
    """Bits of x (< 1024) moved to positions 3i."""
    out = np.zeros_like(x, dtype=np.uint64)
    for b in range(10):
        out |= ((x.astype(np.uint64) >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
    return out


def _expected_order(P):
    P = np.asarray(P, np.float32)
    fin = np.isfinite(P).all(1)
    key = np.full(len(P), 0xFFFFFFFF, np.uint64)
    if fin.any():
        lo = P[fin].min(0)
        hi = P[fin].max(0)
        code = np.zeros(int(fin.sum()), np.uint64)
        for c in range(3):
            ext = np.float32(hi[c] - lo[c])
            if ext > 0:
                t = (P[fin, c] - lo[c]) / ext
                cell = np.clip(t * np.float32(1024), 0, 1023).astype(np.uint32)
            else:
                cell = np.zeros(int(fin.sum()), np.uint32)
            code |= _spread(cell) << np.uint64(c)
        key[fin] = code
    return np.argsort(key, kind="stable")


def _order(P):
    o = W.spatial_order(*_q(P))
    torch.cuda.synchronize()
    return o.cpu().numpy()


@pytest.mark.parametrize("n", [1, 2, 63, 3001, 40000])
def test_order_matches_the_definition(n):
    M = synth.coons_surface(90, 500, 32)
    P = synth.box_queries(M.V, n, 91 + n)
    if n > 10:
        P[::97] = np.nan          # non-finite queries go last, in index order
        P[5::101, 1] = np.inf
    o = _order(P)
    assert np.array_equal(np.sort(o), np.arange(n))
    assert np.array_equal(o, _expected_order(P))
    assert np.array_equal(o, _order(P))


def test_degenerate_boxes():
    assert np.array_equal(_order(np.tile([[0.5, -2.0, 3.0]], (700, 1))), np.arange(700))
    g = synth.rng(92)
    flat = np.c_[g.uniform(-1, 1, (2000, 2)), np.full(2000, 0.25)]      # zero extent in z
    assert np.array_equal(_order(flat), _expected_order(flat))
    allnan = np.full((300, 3), np.nan)
    assert np.array_equal(_order(allnan), np.arange(300))
    e = torch.empty(0, device="cuda")
    assert W.spatial_order(e, e, e).numel() == 0


def test_results_do_not_depend_on_the_order():
    M = synth.coons_surface(93, 4000, 64)
    d = synth.random_direction(94)
    dm = DevMesh(M, d)
    P = synth.box_queries(M.V, 1 << 20, 95)
    q = _q(P)
    o = W.spatial_order(*q).long()
    qo = tuple(t[o].contiguous() for t in q)
    # mesh path
    w, chi = W.eval_3d(dm.bvh, dm.bnd, dm.loop_off, *q)
    w2, chi2 = W.eval_3d(dm.bvh, dm.bnd, dm.loop_off, *qo)
    assert torch.equal(w2, w[o]) and torch.equal(chi2, chi[o])
    # curved boundary
    curves = _dev(M.info["curves"])
    w, chi = W.eval_3d_curves(dm.bvh, curves, *q)
    w2, chi2 = W.eval_3d_curves(dm.bvh, curves, *qo)
    assert torch.equal(w2, w[o]) and torch.equal(chi2, chi[o])
    # parametric patches
    net = _dev(M.info["net"][None])
    w, chi = W.eval_3d_patches(d, net, curves, *q)
    w2, chi2 = W.eval_3d_patches(d, net, curves, *qo)
    torch.cuda.synchronize()
    assert torch.equal(w2, w[o]) and torch.equal(chi2, chi[o])


def test_sorted_entry_points_match_the_unsorted_path():
    """From 2^16 queries the parametric path and the curve adjoint run on a
    coarse Morton-ordered copy of the queries: per-query results equal the
    unsorted kernels' bit for bit (the one-surface batch and calls below the
    threshold), and grad_ctrl equals the sum over halves to rounding."""
    M = synth.coons_surface(96, 4000, 64)
    d = synth.random_direction(97)
    n = (1 << 16) + 1001
    P = synth.box_queries(M.V, n, 98)
    P[17] = np.nan
    q = _q(P)
    net = _dev(M.info["net"][None])
    curves = _dev(M.info["curves"])
    w, chi = W.eval_3d_patches(d, net, curves, *q)
    _, chi_only = W.eval_3d_patches(d, net, curves, *q, want_w=False)
    b = W.PatchBatch([(1, 4, n, d)])
    wb, chib = b.eval(net, curves, *q)
    torch.cuda.synchronize()
    assert torch.equal(w.view(torch.int32), wb.view(torch.int32)) and torch.equal(chi, chib)
    assert torch.equal(chi_only, chib)
    gw = torch.from_numpy(synth.rng(99).normal(size=n).astype(np.float32)).cuda()
    gq, gc = W.backward_curves(curves, *q, gw)
    h = n // 2
    gq1, gc1 = W.backward_curves(curves, *(t[:h].contiguous() for t in q), gw[:h].contiguous())
    gq2, gc2 = W.backward_curves(curves, *(t[h:].contiguous() for t in q), gw[h:].contiguous())
    torch.cuda.synchronize()
    full = torch.cat([gq1, gq2])
    assert torch.equal(torch.isnan(gq), torch.isnan(full))
    ok = ~torch.isnan(full)
    assert torch.equal(gq[ok], full[ok])
    ref = (gc1.double() + gc2.double())
    assert torch.allclose(gc.double(), ref, rtol=1e-4, atol=1e-6 * ref.abs().max().item())


def test_sorted_curve_term_matches_the_unsorted_path():
    """wn_eval_3d_curves with chi_in from 2^16 queries runs on a sorted copy;
    per-query w and chi equal those of calls below the threshold."""
    M = synth.coons_surface(101, 4000, 64)
    d = synth.random_direction(102)
    dm = DevMesh(M, d)
    n = (1 << 16) + 77
    P = synth.box_queries(M.V, n, 103)
    P[5] = np.nan
    q = _q(P)
    curves = _dev(M.info["curves"])
    chi_in = W.crossings_3d(dm.bvh, *q)
    w, chi = W.eval_3d_curves(dm.bvh, curves, *q, chi_in=chi_in)
    h = n // 2
    parts = [W.eval_3d_curves(dm.bvh, curves, *(t[a:b].contiguous() for t in q), chi_in=chi_in[a:b].contiguous())
             for a, b in ((0, h), (h, n))]
    torch.cuda.synchronize()
    w2 = torch.cat([p[0] for p in parts])
    chi2 = torch.cat([p[1] for p in parts])
    assert torch.equal(w.view(torch.int32), w2.view(torch.int32)) and torch.equal(chi, chi2)
    # without chi_in (one kernel at every size): the same crossings and w
    w3, chi3 = W.eval_3d_curves(dm.bvh, curves, *q)
    w4, _ = W.eval_3d_curves(dm.bvh, curves, *q, want_chi=False)
    parts = [W.eval_3d_curves(dm.bvh, curves, *(t[a:b].contiguous() for t in q)) for a, b in ((0, h), (h, n))]
    torch.cuda.synchronize()
    w5 = torch.cat([p[0] for p in parts])
    chi5 = torch.cat([p[1] for p in parts])
    assert torch.equal(w3.view(torch.int32), w5.view(torch.int32)) and torch.equal(chi3, chi5)
    assert torch.equal(w4.view(torch.int32), w5.view(torch.int32)) and torch.equal(chi3, chi)
