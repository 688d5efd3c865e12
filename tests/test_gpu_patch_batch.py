"""GPU tests of the batched parametric path (wn_patch_batch_create,
wn_eval_3d_patches_batched): every surface's w and chi equal the single-
surface call's bit for bit (mixed patch and curve counts, directions, query
counts from 0 to a few thousand across tile boundaries, non-finite queries,
surfaces without curves or without patches, a closed pillow); crossings
only and w only; a sample against the FP64 oracles; and 64 surfaces with
2^20 queries in total."""
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


def _bits(t):
    return t.view(torch.int32).cpu().numpy() if t.dtype == torch.float32 else t.cpu().numpy()


def _pillow(seed):
    M = synth.coons_surface(seed, 300, 16)
    net = M.info["net"]
    bump = net.copy()
    bump[1:3, 1:3] += np.array([0.0, 0.0, 0.8])
    return np.stack([np.swapaxes(net, 0, 1), bump]), M.V


def _surfaces(seed, sizes):
    """(nets [np,4,4,3], curves [nc,4,3] or empty, P [nq,3], d) per surface:
    Coons patches with their boundary curves, a 12-patch set without curves,
    a curves-only surface and a pillow, cycled over the query counts."""
    g = synth.rng(seed)
    out = []
    for k, nq in enumerate(sizes):
        kind = k % 4
        s = int(g.integers(1 << 20))
        M = synth.coons_surface(s, 300, 16)
        if kind == 0:
            nets, curves, V = M.info["net"][None], M.info["curves"], M.V
        elif kind == 1:
            nets = np.array([synth.coons_surface(s + j, 300, 16).info["net"] + np.array([1.5 * (j % 4), 1.5 * (j // 4), 0.0])
                             for j in range(12)])
            curves, V = np.zeros((0, 4, 3)), nets.reshape(-1, 3)
        elif kind == 2:
            nets, curves, V = np.zeros((0, 4, 4, 3)), M.info["curves"], M.V
        else:
            nets, V = _pillow(s)
            curves = np.zeros((0, 4, 3))
        P = synth.box_queries(V, nq, s + 1)
        if nq > 20:
            P[7] = np.nan
            P[13, 2] = np.inf
        out.append((nets, curves, P, synth.random_direction(s + 2)))
    return out


def _batched(surfs, want_w=True, want_chi=True):
    b = W.PatchBatch([(len(n), len(c), len(P), d) for n, c, P, d in surfs])
    nets = _dev(np.concatenate([n for n, _, _, _ in surfs]).reshape(-1, 4, 4, 3))
    curves = _dev(np.concatenate([c for _, c, _, _ in surfs]).reshape(-1, 4, 3))
    P = np.concatenate([P for _, _, P, _ in surfs]).reshape(-1, 3).astype(np.float32)
    q = [_dev(P[:, k]) for k in range(3)]
    w, chi = b.eval(nets, curves, *q, want_w=want_w, want_chi=want_chi)
    torch.cuda.synchronize()
    return b, w, chi


def _single(n, c, P, d, want_w=True):
    P = P.astype(np.float32)
    q = [_dev(P[:, k]) for k in range(3)]
    w, chi = W.eval_3d_patches(d, _dev(n).reshape(-1, 4, 4, 3), _dev(c).reshape(-1, 4, 3) if len(c) else None, *q,
                               want_w=want_w)
    torch.cuda.synchronize()
    return w, chi


def test_batched_equals_single_calls():
    surfs = _surfaces(300, [3000, 257, 0, 1, 256, 1500, 64, 700, 2049, 300, 5, 1000])
    b, w, chi = _batched(surfs)
    for k, ((n, c, P, d), wk, ck) in enumerate(zip(surfs, b.split(w), b.split(chi))):
        if len(P) == 0:
            assert wk.numel() == 0
            continue
        ws, cs = _single(n, c, P, d)
        assert np.array_equal(_bits(wk), _bits(ws)), f"surface {k}: w differs"
        assert np.array_equal(_bits(ck), _bits(cs)), f"surface {k}: chi differs"
    wn = w.cpu().numpy()
    assert np.isnan(wn).sum() == 2 * sum(len(P) > 20 for _, _, P, _ in surfs)
    # the pillows' w is 0 or 1 away from the surface
    for k in range(3, len(surfs), 4):
        v = b.split(w)[k].cpu().numpy()
        v = v[np.isfinite(v)]
        assert np.isin(v, [0.0, 1.0]).mean() > 0.99


def test_crossings_only_and_w_only():
    surfs = _surfaces(310, [900, 400, 650, 1200])
    _, w, chi = _batched(surfs)
    _, none_w, chi2 = _batched(surfs, want_w=False)
    _, w2, none_c = _batched(surfs, want_chi=False)
    assert none_w is None and none_c is None
    assert torch.equal(chi, chi2)
    assert np.array_equal(_bits(w), _bits(w2))


def test_sample_against_the_oracles():
    surfs = _surfaces(320, [400, 300])
    b, w, chi = _batched(surfs)
    n, c, P, d = surfs[0]
    P = P.astype(np.float32).astype(np.float64)
    fin = np.isfinite(P).all(1)
    idx = np.nonzero(fin)[0][:150]
    nets = n.astype(np.float32).astype(np.float64)
    curves = c.astype(np.float32).astype(np.float64)
    r = OP.patch_crossings(nets, P[idx], d)
    ang, dist = OC.curve_margins(curves, P[idx], d)
    ok = ~r.degenerate & (ang > 1e-5) & (dist > 1e-5)
    wk, ck = b.split(w)[0].cpu().numpy()[idx], b.split(chi)[0].cpu().numpy()[idx]
    assert ok.sum() > 100
    assert np.array_equal(ck[ok], r.chi[ok])
    ref = r.chi + OC.curve_term(curves, P[idx], d) / (2 * math.pi)
    assert np.abs(wk - ref)[ok].max() <= 1e-4
    # the 12-patch surface: crossings against the oracle
    n, _, P, d = surfs[1]
    P = P.astype(np.float32).astype(np.float64)
    idx = np.nonzero(np.isfinite(P).all(1))[0][:150]
    r = OP.patch_crossings(n.astype(np.float32).astype(np.float64), P[idx], d)
    ok = ~r.degenerate
    assert np.array_equal(b.split(chi)[1].cpu().numpy()[idx][ok], r.chi[ok])


def test_edge_cases():
    e = torch.empty(0, device="cuda")
    b = W.PatchBatch([])
    assert b.nq == 0
    w, chi = b.eval(None, None, e, e, e)
    assert w.numel() == 0 and chi.numel() == 0
    b = W.PatchBatch([(1, 0, 0, (0.0, 0.0, 1.0))])    # surfaces without queries: no launch
    M = synth.coons_surface(330, 300, 16)
    w, chi = b.eval(_dev(M.info["net"][None]), None, e, e, e)
    assert w.numel() == 0
    with pytest.raises(W.WnError):
        W.PatchBatch([(1, 4, 10, (0.0, 0.0, 1.0)), (1, 4, 10, (0.0, float("nan"), 1.0))])
    with pytest.raises(ValueError):
        b.eval(None, None, e, e, e, want_w=False, want_chi=False)


def test_full_size_64_surfaces():
    sizes = [16384] * 64
    surfs = _surfaces(340, sizes)
    b, w, chi = _batched(surfs)
    assert w.numel() == 1 << 20
    for k in [0, 1, 2, 3, 37, 62]:
        n, c, P, d = surfs[k]
        ws, cs = _single(n, c, P, d)
        assert np.array_equal(_bits(b.split(w)[k]), _bits(ws)), f"surface {k}"
        assert np.array_equal(_bits(b.split(chi)[k]), _bits(cs)), f"surface {k}"
