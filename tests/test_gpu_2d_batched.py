"""GPU tests of the batched 2D grid mode (wn_eval_2d_batched): every set equal
bit for bit to its own wn_eval_2d grid call (which runs the workgroup
histogram kernel, so small sets also check the wavefront kernel against it),
oracle parity on samples, empty and ragged sets on both kernels, the 21/22
segment boundary between them, and the full-size input shape of the 2D
experiment of Sec. 7 (1000 random cubics, each on a 250 x 250 grid over its
bounding box) with no point off by more than 1e-10 in float64."""
import numpy as np
import pytest
import torch

import synth
from oracle import wn2d as O2

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2408_04466_amd as W


def _run(sets, dtype, want_chi=True):
    """sets: list of (Curves2D, xs, ys).  Returns per-set (w, chi) numpy
    (one-off batch through eval_2d_batched)."""
    segs = [C.ctrl.astype(dtype).reshape(-1, 4, 2) for C, _, _ in sets]
    ctrl = torch.from_numpy(np.ascontiguousarray(np.concatenate(segs) if segs else np.zeros((0, 4, 2), dtype)))
    x = torch.from_numpy(np.concatenate([xs.astype(dtype) for _, xs, _ in sets]))
    y = torch.from_numpy(np.concatenate([ys.astype(dtype) for _, _, ys in sets]))
    desc = [(C.loop_off, C.closed, len(xs), len(ys)) for C, xs, ys in sets]
    ws, cs = W.eval_2d_batched(ctrl.cuda(), desc, x.cuda(), y.cuda(), want_chi=want_chi)
    torch.cuda.synchronize()
    return [w.cpu().numpy() for w in ws], ([c.cpu().numpy() for c in cs] if cs is not None else None)


def _single(C, xs, ys, dtype):
    ctrl = torch.from_numpy(np.ascontiguousarray(C.ctrl.astype(dtype))).cuda()
    w, chi = W.eval_2d(ctrl, C.loop_off, C.closed, torch.from_numpy(xs.astype(dtype)).cuda(),
                       torch.from_numpy(ys.astype(dtype)).cuda(), grid=True)
    torch.cuda.synchronize()
    return w.cpu().numpy(), chi.cpu().numpy()


def _endpoint_dist(C, P):
    d = np.full(len(P), np.inf)
    for l in range(len(C.closed)):
        if C.closed[l]:
            continue
        for pt in (C.ctrl[C.loop_off[l], 0], C.ctrl[C.loop_off[l + 1] - 1, 3]):
            d = np.minimum(d, np.linalg.norm(P - pt.astype(np.float64), axis=1))
    return d


def _oracle_check(C, xs, ys, w, chi, tol, n, seed):
    """n sampled grid points of one set against the FP64 oracle: chi exact on
    non-degenerate queries, w within tol away from open end points.
    Returns the number of points compared for w."""
    g = synth.rng(seed)
    r_i = g.integers(0, len(ys), n)
    c_i = g.integers(0, len(xs), n)
    P = np.stack([xs[c_i].astype(np.float64), ys[r_i].astype(np.float64)], 1)
    r = O2.wn2d(C.ctrl.astype(np.float64), C.loop_off, C.closed, P)
    ok = ~r.degenerate
    assert np.array_equal(chi[r_i, c_i][ok], r["chi"][ok])
    far = ok & (_endpoint_dist(C, P) > 1e-5)
    err = np.abs(w[r_i, c_i] - r["w"])[far]
    assert err.size == 0 or err.max() <= tol, err.max()
    return int(far.sum())


def _empty_set(nx, ny, dtype):
    return (synth.Curves2D(np.zeros((0, 4, 2), dtype), np.array([0], np.int64), np.zeros(0, np.uint8)),
            synth.grid_axis(-1, 1, nx, dtype), synth.grid_axis(-1, 1, ny, dtype))


def _mixed(dtype):
    L = synth.loops2d(dtype=dtype)                                # 16 loops, 4 open
    S = synth.star2d(dtype=dtype)                                 # one closed loop
    R = synth.random_cubics(seed=11, n=6, res=37, dtype=dtype)   # open single cubics
    L2 = synth.loops2d(seed=8, n_loops=3, seg_per_loop=5, n_open=2, dtype=dtype)
    L21 = synth.loops2d(seed=12, n_loops=3, seg_per_loop=7, n_open=1, dtype=dtype)   # 63 pieces: wavefront kernel
    L22 = synth.loops2d(seed=13, n_loops=2, seg_per_loop=11, n_open=1, dtype=dtype)  # 66 pieces: workgroup kernel
    L5 = synth.loops2d(seed=14, n_loops=1, seg_per_loop=5, n_open=1, dtype=dtype)    # 15 pieces: 4 rows per wavefront
    return [
        (L5, synth.grid_axis(-1.1, 1.1, 130, dtype), synth.grid_axis(-1.1, 1.1, 10, dtype)),
        (L21, synth.grid_axis(-1.1, 1.1, 700, dtype), synth.grid_axis(-1.1, 1.1, 50, dtype)),
        (L22, synth.grid_axis(-1.1, 1.1, 700, dtype), synth.grid_axis(-1.1, 1.1, 50, dtype)),
        (L, synth.grid_axis(-1.2, 1.2, 5000, dtype), synth.grid_axis(-1.2, 1.2, 3, dtype)),   # two workgroup tiles
        (L, synth.grid_axis(-1.2, 1.2, 300, dtype), synth.grid_axis(-1.2, 1.2, 200, dtype)),
        _empty_set(17, 9, dtype),                                 # no segments: w = 0
        (S, synth.grid_axis(-1.5, 1.5, 5000, dtype), synth.grid_axis(-1.5, 1.5, 7, dtype)),  # two column tiles
        R[0], R[1],
        (L2, synth.grid_axis(-1.1, 1.1, 1, dtype), synth.grid_axis(-1.1, 1.1, 33, dtype)),  # one column
        _empty_set(0, 5, dtype),                                  # no columns
        (L2, synth.grid_axis(-1.1, 1.1, 64, dtype), synth.grid_axis(-1.1, 1.1, 0, dtype)),  # no rows
        R[2], R[3], R[4], R[5],
        (L2, synth.grid_axis(-1.1, 1.1, 4097, dtype), synth.grid_axis(-1.1, 1.1, 3, dtype)),  # ragged tail tile
    ]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_mixed_batch_equals_single_calls_and_oracle(dtype):
    sets = _mixed(dtype)
    ws, cs = _run(sets, dtype)
    tol = 1e-4 if dtype == np.float32 else 1e-10
    for k, (C, xs, ys) in enumerate(sets):
        assert ws[k].shape == (len(ys), len(xs)) and cs[k].shape == ws[k].shape
        if ws[k].size == 0:
            continue
        if len(C.closed) == 0:
            assert np.all(ws[k] == 0) and np.all(cs[k] == 0), f"set {k}"
            continue
        w1, c1 = _single(C, xs, ys, dtype)
        assert np.array_equal(cs[k], c1), f"set {k}: chi differs from the single-set call"
        assert np.array_equal(ws[k].view(np.uint8), w1.view(np.uint8)), f"set {k}: w differs from the single-set call"
        _oracle_check(C, xs, ys, ws[k], cs[k], tol, 200, 100 + k)
    # without chi: identical w
    ws2, cs2 = _run(sets, dtype, want_chi=False)
    assert cs2 is None
    for a, b in zip(ws, ws2):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def test_non_finite_axis_values_and_empty_batch():
    C = synth.star2d()
    xs = synth.grid_axis(-1.5, 1.5, 40)
    ys = synth.grid_axis(-1.5, 1.5, 30)
    ys[3] = np.nan
    xs[-1] = np.inf
    ws, cs = _run([(C, xs, ys), _empty_set(4, 4, np.float64)], np.float64)
    w, chi = ws[0], cs[0]
    bad = np.zeros(w.shape, bool)
    bad[3, :] = True
    bad[:, -1] = True
    assert np.all(np.isnan(w[bad])) and np.all(chi[bad] == W.WN_CHI_INVALID)
    assert np.all(np.isfinite(w[~bad]))
    w1, c1 = _single(C, xs, ys, np.float64)
    assert np.array_equal(chi, c1) and np.array_equal(np.isnan(w), np.isnan(w1))
    assert np.array_equal(w[~bad], w1[~bad])
    ws, cs = W.eval_2d_batched(torch.zeros((0, 4, 2), dtype=torch.float64, device="cuda"), [],
                               torch.zeros(0, dtype=torch.float64, device="cuda"),
                               torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert ws == [] and cs == []


def test_batch_handle_reuse_with_new_curves():
    """One Batch2D evaluated twice with different control points (same
    topology): each result equals the single-set calls on its own curves."""
    A = synth.random_cubics(seed=31, n=40, res=60, dtype=np.float32)
    B = synth.random_cubics(seed=32, n=40, res=60, dtype=np.float32)
    b = W.Batch2D([(C.loop_off, C.closed, 60, 60) for C, _, _ in A], torch.float32)
    x = torch.from_numpy(np.concatenate([xs for _, xs, _ in A])).cuda()
    y = torch.from_numpy(np.concatenate([ys for _, _, ys in A])).cuda()
    for sets in (A, B, A):
        ctrl = torch.from_numpy(np.concatenate([C.ctrl for C, _, _ in sets])).cuda()
        w, chi = b.eval(ctrl, x, y)
        torch.cuda.synchronize()
        ws, cs = b.split(w), b.split(chi)
        for k in (0, 17, 39):
            C = sets[k][0]
            w1, c1 = _single(C, A[k][1], A[k][2], np.float32)
            assert np.array_equal(cs[k].cpu().numpy(), c1) and np.array_equal(ws[k].cpu().numpy(), w1)


def test_full_size_random_cubics_fp64():
    """1000 cubics with control points in [0, 1]^2, each on a 250^2 grid over
    its control-point bounding box, float64: a slice of sets equal to the
    single-set calls, sampled points of every 25th set against the oracle with
    no error above 1e-10 (the paper's misclassification threshold)."""
    sets = synth.random_cubics(seed=5, n=1000, res=250, dtype=np.float64)
    ws, cs = _run(sets, np.float64)
    assert len(ws) == 1000 and all(w.shape == (250, 250) for w in ws)
    for k in range(0, 1000, 100):
        C, xs, ys = sets[k]
        w1, c1 = _single(C, xs, ys, np.float64)
        assert np.array_equal(cs[k], c1) and np.array_equal(ws[k], w1), f"set {k}"
    compared = 0
    for k in range(0, 1000, 25):
        C, xs, ys = sets[k]
        compared += _oracle_check(C, xs, ys, ws[k], cs[k], 1e-10, 100, 1000 + k)
    assert compared > 3000
