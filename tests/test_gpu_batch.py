"""GPU tests of the batched persistent path (many surfaces of uneven size in
one launch, hipGraph replay, autotuner): bitwise agreement with the plain
per-surface calls, oracle parity on samples, replay correctness."""
import os

import numpy as np
import pytest
import torch

import synth
from oracle import wn3d as O

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2408_04466_amd as W
    from gpu_util import W_TOL, near_band


def _surfaces(seed, n, scale):
    CB = synth.coons_batch(seed, n_surf=n, scale=scale)
    meshes, queries = list(CB.meshes), list(CB.queries)
    # a closed surface and a surface without queries ride along
    meshes.append(synth.icosphere(2, radius=0.7))
    queries.append(synth.box_queries(meshes[-1].V, 3000, 9))
    meshes.append(synth.bumpy_cap())
    queries.append(np.zeros((0, 3), np.float32))
    # a long boundary (1200 edges) with few queries: the plain adjoint splits
    # it into vertex ranges
    meshes.append(synth.coons_surface(77, 4000, 1200))
    queries.append(synth.box_queries(meshes[-1].V, 3000, 78))
    return meshes, queries, CB.direction


def _upload(meshes, queries):
    surfs, plain = [], []
    for M, Q in zip(meshes, queries):
        V = torch.from_numpy(M.V).cuda()
        F = torch.from_numpy(M.F).cuda()
        idx, off = W.boundary_loops(M.F)
        bnd = V[torch.from_numpy(idx.astype(np.int64)).cuda()].contiguous()
        surfs.append({"V": V, "F": F, "bnd": bnd, "loop_off": off, "nq": len(Q), "idx": idx})
    P = np.concatenate(queries, 0).astype(np.float32)
    q = tuple(torch.from_numpy(np.ascontiguousarray(P[:, k])).cuda() for k in range(3))
    return surfs, P, q


def _plain(surfs, q, d):
    ws, cs, o = [], [], 0
    for s in surfs:
        n = s["nq"]
        if n == 0:
            continue
        bvh = W.BVH(s["V"], s["F"], d)
        w, chi = W.eval_3d(bvh, s["bnd"], s["loop_off"], q[0][o:o + n], q[1][o:o + n], q[2][o:o + n])
        torch.cuda.synchronize()
        ws.append(w.cpu().numpy())
        cs.append(chi.cpu().numpy())
        o += n
    return np.concatenate(ws), np.concatenate(cs)


@pytest.fixture(scope="module")
def small_batch():
    meshes, queries, d = _surfaces(31, 12, 0.05)
    surfs, P, q = _upload(meshes, queries)
    return meshes, queries, d, surfs, P, q


def test_batched_equals_plain_bitwise(small_batch):
    meshes, queries, d, surfs, P, q = small_batch
    B = W.Batch(surfs, d)
    w, chi = B.eval(*q)
    torch.cuda.synchronize()
    wp, cp = _plain(surfs, q, d)
    assert np.array_equal(chi.cpu().numpy(), cp)
    assert np.array_equal(w.cpu().numpy(), wp)
    info = B.info()
    assert info["total_q"] == len(P) and info["graph"] == 1
    B.free()


def test_batched_oracle_samples(small_batch):
    meshes, queries, d, surfs, P, q = small_batch
    B = W.Batch(surfs, d)
    w, chi = B.eval(*q)
    torch.cuda.synchronize()
    w, chi = w.cpu().numpy(), chi.cpu().numpy()
    import oracle_pool
    g = synth.rng(2)
    offs = np.concatenate([[0], np.cumsum([len(Q) for Q in queries])])
    sels = [g.choice(len(Q), min(len(Q), 64), replace=False) for Q in queries]
    rs = oracle_pool.map_wn3d((M.V, M.F, Q[sel], d, None) for M, Q, sel in zip(meshes, queries, sels))
    n_all = n_deg = 0
    for k, (r, sel) in enumerate(zip(rs, sels)):
        if len(sel) == 0:
            continue
        ok = ~r.degenerate
        n_all, n_deg = n_all + len(sel), n_deg + int((~ok).sum())
        assert np.array_equal(chi[offs[k] + sel][ok], r["chi"][ok]), k
        far = r["m_bnd"] > near_band(meshes[k].V, O.boundary_loops(meshes[k].F))
        wref = r["w"].copy()
        assert np.abs(w[offs[k] + sel][far & ok] - wref[far & ok]).max(initial=0.0) <= W_TOL, k
    print(f"batched oracle samples: {n_all} queries, {n_deg} degenerate", flush=True)
    assert n_deg <= 0.02 * n_all


def test_graph_replays_and_pointer_changes(small_batch):
    meshes, queries, d, surfs, P, q = small_batch
    B = W.Batch(surfs, d)
    ref_w, ref_c = B.eval(*q)
    torch.cuda.synchronize()
    ref_w, ref_c = ref_w.clone(), ref_c.clone()
    outs = [(torch.full_like(ref_w, float("nan")), torch.full_like(ref_c, -7)) for _ in range(3)]
    for rep in range(4):
        for w_o, c_o in outs:
            # eager work between replays touches the same memory pool
            junk = torch.randn(1 << 16, device="cuda").sum()
            w_o.fill_(float("nan"))
            B.eval(*q, w_out=w_o, chi_out=c_o)
            torch.cuda.synchronize()
            assert torch.equal(w_o, ref_w) and torch.equal(c_o, ref_c), f"replay {rep}"
            del junk
    # moved queries (new pointers): results follow the new inputs
    q2 = tuple(t.clone() for t in q)
    w2, c2 = B.eval(*q2)
    torch.cuda.synchronize()
    assert torch.equal(w2, ref_w) and torch.equal(c2, ref_c)
    B.free()


def test_direct_launch_mode_matches_graph(small_batch):
    meshes, queries, d, surfs, P, q = small_batch
    B = W.Batch(surfs, d)
    wg, cg = B.eval(*q)
    os.environ["WN_FORCE_NO_GRAPH"] = "1"
    try:
        B2 = W.Batch(surfs, d)
    finally:
        del os.environ["WN_FORCE_NO_GRAPH"]
    wd, cd = B2.eval(*q)
    torch.cuda.synchronize()
    assert B2.info()["graph"] == 0
    assert torch.equal(wg, wd) and torch.equal(cg, cd)


@pytest.mark.parametrize("mode", ["fused", "split"])
def test_forward_modes_match_plain(small_batch, mode):
    """Both forward modes (one fused kernel; crossing kernel then boundary
    kernel) give the plain path's bits, with and without chi_out, on graph
    replays with changed output pointers."""
    meshes, queries, d, surfs, P, q = small_batch
    os.environ["WN_BATCH_MODE"] = mode
    try:
        B = W.Batch(surfs, d)
    finally:
        del os.environ["WN_BATCH_MODE"]
    assert B.info()["mode"] == (1 if mode == "split" else 0)
    wp, cp = _plain(surfs, q, d)
    for rep in range(3):
        w, chi = B.eval(*q)
        w2, _ = B.eval(*q, want_chi=False)
        torch.cuda.synchronize()
        assert np.array_equal(chi.cpu().numpy(), cp), rep
        assert np.array_equal(w.cpu().numpy(), wp), rep
        assert np.array_equal(w2.cpu().numpy(), wp), rep
    B.free()


def test_autotuner_and_cache(small_batch, tmp_path):
    meshes, queries, d, surfs, P, q = small_batch
    cache = tmp_path / "tune.json"
    os.environ["WN_TUNE_CACHE"] = str(cache)
    try:
        B = W.Batch(surfs, d, tune_mode=1)
        w, chi = B.eval(*q)
        torch.cuda.synchronize()
        info = B.info()
        assert cache.exists() and info["tile"] in (256, 512, 1024, 2048) and info["wg_per_cu"] in (4, 8, 0)
        assert str(info["tile"]) in cache.read_text()
        B2 = W.Batch(surfs, d, tune_mode=2)
        w2, chi2 = B2.eval(*q)
        torch.cuda.synchronize()
        assert B2.info()["tile"] == info["tile"] and B2.info()["wg_per_cu"] == info["wg_per_cu"]
        assert B2.info()["mode"] == info["mode"] and info["mode"] in (0, 1)
    finally:
        del os.environ["WN_TUNE_CACHE"]
    B0 = W.Batch(surfs, d)
    w0, c0 = B0.eval(*q)
    torch.cuda.synchronize()
    assert torch.equal(w, w0) and torch.equal(chi, c0) and torch.equal(w2, w0)


def test_batched_backward_matches_plain(small_batch):
    meshes, queries, d, surfs, P, q = small_batch
    B = W.Batch(surfs, d)
    g = torch.from_numpy(synth.rng(3).normal(size=len(P)).astype(np.float32)).cuda()
    gq, gb = B.backward(*q, g)
    gq2, gb2 = B.backward(*q, g)
    torch.cuda.synchronize()
    assert torch.equal(gq, gq2) and torch.equal(gb, gb2)
    o, ob = 0, 0
    for s in surfs:
        n, nb = s["nq"], len(s["idx"])
        if n > 0 and nb > 0:
            pq, pb = W.backward(s["bnd"], s["loop_off"], q[0][o:o + n], q[1][o:o + n], q[2][o:o + n], g[o:o + n])
            torch.cuda.synchronize()
            if nb > 512:
                # the plain call splits a long boundary over few query tiles
                # into vertex ranges and sums grad_q over them: equal to rounding
                assert torch.allclose(gq[o:o + n], pq, rtol=1e-5, atol=1e-6 * float(pq.abs().max()))
            else:
                assert torch.equal(gq[o:o + n], pq)
            # the plain adjoint may hold fewer queries per lane for small query
            # counts, so its partial rows group the queries differently: the
            # float64 sums agree to rounding, not bit for bit
            assert torch.allclose(gb[ob:ob + nb], pb, rtol=1e-5, atol=1e-6 * float(pb.abs().max()))
        elif nb > 0:
            assert torch.count_nonzero(gb[ob:ob + nb]) == 0
        o += n
        ob += nb


@pytest.mark.slow
def test_full_size_batch_autotuned_parity():
    """The 256-surface workload at full size (11.2M triangles, 17.5M queries),
    in the configuration bench.py times (quick autotune, graph replay):
    crossing counts bit-exact and |dw| <= 1e-4 against the oracle on 16
    seeded queries of each of the 256 surfaces; batched equals plain bit for bit on
    every 16th surface; the batched backward is finite everywhere."""
    CB = synth.coons_batch(4)
    d = CB.direction
    surfs, P, q = _upload(CB.meshes, CB.queries)
    B = W.Batch(surfs, d, tune_mode=1)
    w, chi = B.eval(*q)
    w2, chi2 = B.eval(*q)                     # graph replay
    torch.cuda.synchronize()
    assert torch.equal(w, w2) and torch.equal(chi, chi2)
    wc, cc = w.cpu().numpy(), chi.cpu().numpy()
    offs = np.concatenate([[0], np.cumsum([len(Q) for Q in CB.queries])])
    import oracle_pool
    g = synth.rng(44)
    sels = [g.choice(len(Q), 16, replace=False) for Q in CB.queries]
    print("full batch: oracle on 16 queries of each of 256 surfaces", flush=True)
    rs = oracle_pool.map_wn3d((M.V, M.F, Q[sel], d, None) for M, Q, sel in zip(CB.meshes, CB.queries, sels))
    n_deg = 0
    for k, (r, sel) in enumerate(zip(rs, sels)):
        ok = ~r.degenerate
        n_deg += int((~ok).sum())
        assert np.array_equal(cc[offs[k] + sel][ok], r["chi"][ok]), k
        M = CB.meshes[k]
        far = ok & (r["m_bnd"] > near_band(M.V, O.boundary_loops(M.F)))
        assert np.abs(wc[offs[k] + sel][far] - r["w"][far]).max(initial=0.0) <= W_TOL, k
    print(f"full batch: {16 * 256} oracle queries, {n_deg} degenerate", flush=True)
    assert n_deg <= 0.02 * 16 * 256
    for k in range(0, 256, 16):
        s = surfs[k]
        a, b = int(offs[k]), int(offs[k + 1])
        bvh = W.BVH(s["V"], s["F"], d)
        wp, cp = W.eval_3d(bvh, s["bnd"], s["loop_off"], q[0][a:b], q[1][a:b], q[2][a:b])
        torch.cuda.synchronize()
        assert torch.equal(wp, w[a:b]) and torch.equal(cp, chi[a:b]), k
    gq, gb = B.backward(*q, torch.ones_like(w))
    torch.cuda.synchronize()
    assert bool(torch.isfinite(gq).all()) and bool(torch.isfinite(gb).all())
    B.free()
