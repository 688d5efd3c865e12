"""Helpers shared by the GPU tests: upload a synthetic mesh, evaluate through
the C ABI, and compare with the FP64 oracle on the same float32 arrays."""
from __future__ import annotations

import numpy as np
import torch

import paper_2408_04466_amd as W
from oracle import wn3d as O

W_TOL = 1e-4          # |w_gpu - w_oracle| for FP32 paths
NEAR_REL = 1e-4       # exempt: closer to the boundary than NEAR_REL x its longest edge


def near_band(V, loops):
    """Distance to the boundary below which w is exempt from W_TOL.  Across
    the boundary w turns through a full unit within a distance delta, so the
    float32 offsets of the boundary vertices (each rounded to 2^-24 of its
    distance, at most about the longest edge L for the edges that matter)
    perturb it by about 2^-24 L / delta: the float32 problem itself is that
    ill-conditioned there (measured: |dw| ~ 3e-9 L / delta).  Below
    NEAR_REL x L the tests check that bound instead
    (tests/test_gpu_3d.py::test_near_boundary_error_follows_float32_conditioning)."""
    V = np.asarray(V, np.float64)
    L = 0.0
    for lp in loops:
        lp = np.asarray(lp)
        if len(lp):
            L = max(L, float(np.linalg.norm(V[lp] - V[np.roll(lp, -1)], axis=1).max()))
    return NEAR_REL * L


class DevMesh:
    def __init__(self, M, d):
        self.M = M
        self.d = np.asarray(d, np.float64)
        self.V = torch.from_numpy(np.ascontiguousarray(M.V)).cuda()
        self.F = torch.from_numpy(np.ascontiguousarray(M.F)).cuda()
        self.bvh = W.BVH(self.V, self.F, self.d)
        idx, off = W.boundary_loops(M.F)
        self.bnd_idx, self.loop_off = idx, off
        self.bnd = self.V[torch.from_numpy(idx.astype(np.int64)).cuda()].contiguous()

    def queries(self, P):
        P = np.ascontiguousarray(np.asarray(P, np.float32))
        return tuple(torch.from_numpy(np.ascontiguousarray(P[:, k])).cuda() for k in range(3))

    def eval(self, P):
        qx, qy, qz = self.queries(P)
        w, chi = W.eval_3d(self.bvh, self.bnd, self.loop_off, qx, qy, qz)
        torch.cuda.synchronize()
        return w.cpu().numpy(), chi.cpu().numpy()


def compare_3d(dm: DevMesh, P, w_gpu, chi_gpu, sample=None, alt_dir_seed=12345,
               max_degenerate_frac=0.02, label=""):
    """Oracle parity on ``sample`` (indices into P).  chi must match bit for
    bit on non-degenerate queries; w within W_TOL away from the boundary.
    Degenerate queries are checked for w against the oracle with another
    direction (w does not depend on d).  "Away from the boundary": at least
    near_band() from it.  Large samples run in the oracle's
    process pool."""
    import oracle_pool
    P = np.asarray(P, np.float32)
    idx = np.arange(len(P)) if sample is None else np.asarray(sample)
    loops = [dm.bnd_idx[dm.loop_off[i]:dm.loop_off[i + 1]] for i in range(len(dm.loop_off) - 1)]
    r = oracle_pool.wn3d(dm.M.V, dm.M.F, P[idx], dm.d, loops=loops)
    deg = r.degenerate
    print(f"compare_3d{(' ' + label) if label else ''}: {len(idx)} queries, {int(deg.sum())} degenerate",
          flush=True)
    assert deg.mean() <= max_degenerate_frac, f"too many degenerate queries: {deg.sum()}/{len(idx)}"
    ok = ~deg
    bad = np.nonzero(chi_gpu[idx][ok] != r["chi"][ok])[0]
    assert bad.size == 0, f"chi mismatch at {idx[ok][bad][:10]}: gpu {chi_gpu[idx][ok][bad][:10]} oracle {r['chi'][ok][bad][:10]}"
    far = r["m_bnd"] >= near_band(dm.M.V, loops)
    wref = r["w"].copy()
    if deg.any():
        # w is independent of d: take a direction for which these are regular
        d2 = np.asarray(__import__("synth").random_direction(alt_dir_seed))
        r2 = oracle_pool.wn3d(dm.M.V, dm.M.F, P[idx][deg], d2, loops=loops)
        assert not r2.degenerate.any()
        wref[deg] = r2["w"]
    err = np.abs(w_gpu[idx] - wref)
    worst = np.argmax(np.where(far, err, 0))
    assert err[far].max() <= W_TOL, f"w error {err[far].max():.3g} at query {idx[worst]}"
    return {"n": len(idx), "degenerate": int(deg.sum()), "max_err": float(err[far].max())}
