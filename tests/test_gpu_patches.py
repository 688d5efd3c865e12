"""GPU tests of the exact parametric path (wn_eval_3d_patches): ray-patch
crossings of bicubic Bezier patches against the FP64 oracle
(oracle.patches3d) on random queries, queries near the surface and several
directions; w = chi + Theta/2pi against the patch and curve oracles; closed
pillows (w in {0, 1}, the same for every d); agreement with the tessellated
path away from the surface; edge cases; and 2^20 queries on samples."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import curves3d as OC
from oracle import patches3d as OP

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2408_04466_amd as W
    from gpu_util import DevMesh

TOL = 1e-4


def _q(P):
    P = np.ascontiguousarray(np.asarray(P, np.float32))
    return tuple(torch.from_numpy(np.ascontiguousarray(P[:, k])).cuda() for k in range(3))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


def _near_surface(net, d, n, seed):
    g = synth.rng(seed)
    out = []
    for _ in range(n):
        u, v = g.uniform(0, 1, 2)
        S, Su, Sv = OP.patch_eval(net, u, v)
        nrm = np.cross(Su, Sv)
        nrm /= np.linalg.norm(nrm)
        out.append(S + nrm * g.choice([-1, 1]) * 10 ** g.uniform(-4.5, -1) + d * g.uniform(-0.3, 0.3))
    return np.array(out)


@pytest.mark.parametrize("seed", [21, 24, 25])
def test_crossings_match_oracle(seed):
    M = synth.coons_surface(seed, 500, 32)
    net = M.info["net"].astype(np.float32).astype(np.float64)
    d = synth.random_direction(seed + 200)
    P = np.concatenate([synth.box_queries(M.V, 400, seed + 1), _near_surface(net, d, 150, seed + 2)])
    P = P.astype(np.float32).astype(np.float64)
    _, chi = W.eval_3d_patches(d, _dev(net[None]), None, *_q(P), want_w=False)
    torch.cuda.synchronize()
    chi = chi.cpu().numpy()
    r = OP.patch_crossings(net[None], P, d)
    ok = ~r.degenerate
    assert ok.mean() > 0.95 and np.count_nonzero(r.chi[ok]) > 50
    bad = np.nonzero(chi[ok] != r.chi[ok])[0]
    assert bad.size == 0, f"{bad.size} mismatches, e.g. {P[ok][bad[:3]]}"


def test_w_matches_oracles():
    M = synth.coons_surface(26, 500, 32)
    net = M.info["net"].astype(np.float32).astype(np.float64)
    curves = M.info["curves"].astype(np.float32).astype(np.float64)
    d = synth.random_direction(226)
    P = synth.box_queries(M.V, 300, 27).astype(np.float64)
    w, chi = W.eval_3d_patches(d, _dev(net[None]), _dev(curves), *_q(P))
    torch.cuda.synchronize()
    w, chi = w.cpu().numpy(), chi.cpu().numpy()
    r = OP.patch_crossings(net[None], P, d)
    ang, dist = OC.curve_margins(curves, P, d)
    ok = ~r.degenerate & (ang > 1e-5) & (dist > 1e-5)
    ref = r.chi + OC.curve_term(curves, P, d) / (2 * math.pi)
    assert np.array_equal(chi[ok], r.chi[ok])
    assert np.abs(w - ref)[ok].max() <= TOL


def test_closed_pillow_is_inside_outside_for_every_d():
    M = synth.coons_surface(23, 500, 32)
    net = M.info["net"]
    bump = net.copy()
    bump[1:3, 1:3] += np.array([0.0, 0.0, 0.8])
    nets = _dev(np.stack([np.swapaxes(net, 0, 1), bump]))
    g = synth.rng(60)
    P = synth.box_queries(M.V, 4000, 61)
    P[:, 2] = g.uniform(-0.6, 1.2, len(P))
    ws = []
    for k in range(4):
        d = synth.random_direction(int(g.integers(1 << 30)))
        w, _ = W.eval_3d_patches(d, nets, None, *_q(P))
        torch.cuda.synchronize()
        ws.append(w.cpu().numpy())
    ws = np.array(ws)
    assert set(np.unique(ws)) <= {0.0, 1.0}
    agree = np.all(ws == ws[0], axis=0)
    assert agree.mean() > 0.999 and ws[0].mean() > 0.05


def test_agrees_with_the_tessellated_path_away_from_the_surface():
    M = synth.coons_surface(28, 60000, 256)
    net = M.info["net"].astype(np.float32)
    d = synth.random_direction(228)
    dm = DevMesh(M, d)
    P = synth.box_queries(M.V, 20000, 29)
    _, chi_p = W.eval_3d_patches(d, _dev(net[None]), None, *_q(P), want_w=False)
    _, chi_m = dm.eval(P)
    torch.cuda.synchronize()
    chi_p = chi_p.cpu().numpy()
    # the tessellation deviates from the patch by well under 1e-3: compare the
    # queries whose crossings (per the patch oracle) keep 1e-2 from the patch
    # boundary, from tangency and from the query itself
    sample = synth.rng(30).choice(len(P), 1200, replace=False)
    r = OP.patch_crossings(M.info["net"][None], P[sample].astype(np.float64), d)
    sel = sample[r.margin > 1e-2]
    assert len(sel) > 600 and np.count_nonzero(chi_p[sel]) > 100
    assert np.array_equal(chi_p[sel], chi_m[sel])


def test_many_patches_sum():
    nets, Ps = [], []
    for s in range(40, 52):
        M = synth.coons_surface(s, 300, 16)
        nets.append(M.info["net"] + np.array([1.5 * (s % 4), 1.5 * (s // 4 % 3), 0.0]))
    nets = np.array(nets).astype(np.float32).astype(np.float64)
    d = synth.random_direction(240)
    lo, hi = nets.reshape(-1, 3).min(0), nets.reshape(-1, 3).max(0)
    P = (lo + (hi - lo) * synth.rng(41).uniform(0, 1, (300, 3))).astype(np.float32).astype(np.float64)
    _, chi = W.eval_3d_patches(d, _dev(nets), None, *_q(P), want_w=False)
    torch.cuda.synchronize()
    r = OP.patch_crossings(nets, P, d)
    ok = ~r.degenerate
    assert np.array_equal(chi.cpu().numpy()[ok], r.chi[ok]) and np.count_nonzero(r.chi[ok]) > 10


def test_many_chunks():
    """80 patches (three LDS chunks of staged patches): the counts equal the
    oracle's, and bit for bit those of the batched kernel."""
    nets = []
    for j in range(80):
        M = synth.coons_surface(500 + j, 300, 16)
        nets.append(M.info["net"] + np.array([1.2 * (j % 10), 1.2 * (j // 10), 0.0]))
    nets = np.array(nets).astype(np.float32).astype(np.float64)
    d = synth.random_direction(501)
    lo, hi = nets.reshape(-1, 3).min(0), nets.reshape(-1, 3).max(0)
    P = (lo + (hi - lo) * synth.rng(502).uniform(0, 1, (20000, 3))).astype(np.float32).astype(np.float64)
    P[11] = np.nan
    q = _q(P)
    _, chi = W.eval_3d_patches(d, _dev(nets), None, *q, want_w=False)
    b = W.PatchBatch([(80, 0, len(P), d)])
    _, chi_b = b.eval(_dev(nets), None, *q, want_w=False)
    torch.cuda.synchronize()
    chi, chi_b = chi.cpu().numpy(), chi_b.cpu().numpy()
    assert np.array_equal(chi, chi_b)
    assert chi[11] == W.WN_CHI_INVALID
    sample = np.arange(300)
    sample = sample[sample != 11]
    r = OP.patch_crossings(nets, P[sample], d)
    ok = ~r.degenerate
    assert ok.mean() > 0.95 and np.count_nonzero(r.chi[ok]) > 60
    assert np.array_equal(chi[sample][ok], r.chi[ok])


def test_edge_cases():
    M = synth.coons_surface(31, 300, 16)
    net = _dev(M.info["net"][None])
    curves = _dev(M.info["curves"])
    d = synth.random_direction(231)
    P = synth.box_queries(M.V, 64, 32)
    P[2] = np.nan
    P[9, 1] = -np.inf
    w, chi = W.eval_3d_patches(d, net, curves, *_q(P))
    torch.cuda.synchronize()
    w, chi = w.cpu().numpy(), chi.cpu().numpy()
    assert np.isnan(w[[2, 9]]).all() and (chi[[2, 9]] == W.WN_CHI_INVALID).all()
    good = np.isfinite(P).all(1)
    assert np.isfinite(w[good]).all()
    # no patches and no curves: w = chi = 0
    w0, c0 = W.eval_3d_patches(d, torch.zeros((0, 4, 4, 3), device="cuda"), None, *_q(P))
    torch.cuda.synchronize()
    assert np.all(c0.cpu().numpy()[good] == 0) and np.all(w0.cpu().numpy()[good] == 0)
    # w only (chi buffer allocated inside) equals w with chi
    w1, none = W.eval_3d_patches(d, net, curves, *_q(P), want_chi=False)
    torch.cuda.synchronize()
    assert none is None and np.array_equal(w1.cpu().numpy()[good], w[good])
    # bad direction
    with pytest.raises(W.WnError):
        W.eval_3d_patches([0.0, 0.0, 0.0], net, curves, *_q(P))
    # empty query set
    e = torch.empty(0, dtype=torch.float32, device="cuda")
    we, ce = W.eval_3d_patches(d, net, curves, e, e, e)
    assert we.numel() == 0 and ce.numel() == 0


def test_full_size_queries():
    M = synth.coons_surface(6, 4000, 64)
    net = M.info["net"].astype(np.float32).astype(np.float64)
    curves = M.info["curves"].astype(np.float32).astype(np.float64)
    d = synth.random_direction(106)
    P = synth.box_queries(M.V, 1 << 20, 7)
    w, chi = W.eval_3d_patches(d, _dev(net[None]), _dev(curves), *_q(P))
    torch.cuda.synchronize()
    w, chi = w.cpu().numpy(), chi.cpu().numpy()
    sample = synth.rng(8).choice(len(P), 150, replace=False)
    Ps = P[sample].astype(np.float64)
    r = OP.patch_crossings(net[None], Ps, d)
    ang, dist = OC.curve_margins(curves, Ps, d)
    ok = ~r.degenerate & (ang > 1e-5) & (dist > 1e-5)
    assert np.array_equal(chi[sample][ok], r.chi[ok])
    ref = r.chi + OC.curve_term(curves, Ps, d) / (2 * math.pi)
    assert np.abs(w[sample] - ref)[ok].max() <= TOL


def test_parametric_path_removes_the_discretization_error():
    """The accuracy experiment of Sec. 7 (parametric surfaces) in miniature:
    queries on a slice through a curved patch; the tessellated path (mesh
    chi + polyline boundary) against the exact parametric path, both against
    the FP64 oracles (patch crossings + curve integral)."""
    M = synth.coons_surface(33, 2000, 64)
    net = M.info["net"].astype(np.float32).astype(np.float64)
    curves = M.info["curves"].astype(np.float32).astype(np.float64)
    d = synth.random_direction(233)
    dm = DevMesh(M, d)
    lo, hi = M.V.min(0), M.V.max(0)
    g = synth.rng(34)
    n = 600
    P = np.stack([g.uniform(lo[0], hi[0], n), np.full(n, 0.5 * (lo[1] + hi[1])),
                  g.uniform(lo[2] - 0.2, hi[2] + 0.2, n)], 1).astype(np.float32)
    wm, _ = dm.eval(P)
    wp, _ = W.eval_3d_patches(d, _dev(net[None]), _dev(curves), *_q(P))
    torch.cuda.synchronize()
    wp = wp.cpu().numpy()
    P64 = P.astype(np.float64)
    r = OP.patch_crossings(net[None], P64, d)
    ang, dist = OC.curve_margins(curves, P64, d)
    ok = ~r.degenerate & (ang > 1e-5) & (dist > 1e-5)
    ref = r.chi + OC.curve_term(curves, P64, d) / (2 * math.pi)
    em, ep = np.abs(wm - ref)[ok], np.abs(wp - ref)[ok]
    print(f"slice, {ok.sum()} queries: tessellated (2000 triangles, 64 boundary edges) max {em.max():.3g} "
          f"mean {em.mean():.3g}, off by >= 0.5 at {(em >= 0.5).sum()}; parametric max {ep.max():.3g} mean {ep.mean():.3g}")
    assert ep.max() <= TOL and em.max() > 100 * ep.max()
