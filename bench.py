#!/usr/bin/env python3
"""Benchmark of the one-shot winding number hot path on one MI355X.

One step = one forward + backward pass over the 3D open-mesh workload:
a noise-displaced unit sphere with a 30 degree polar cap removed (1,048,064
triangles, one boundary loop of 512 edges), 2^20 query points uniform in 1.2x
its bounding box, seeded ray direction.  Forward = crossing count through the
BVH + boundary integral (w); backward = adjoint with respect to the queries
and the boundary vertices for L = sum (w - t)^2.  Inputs are resident in HBM
before the timed region; the BVH build is timed separately.

Prints one JSON line (see the keys below).  ``--gpus N`` with N > 1 exits:
this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

FLOPS_PER_PAIR_FWD = 58      # boundary integral, per (query, boundary edge)
FLOPS_PER_PAIR_BWD = 40      # adjoint, per (query, boundary edge)
PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector peak
PEAK_HBM_GBS = 8000.0


def workload_c3():
    M = synth.open_sphere(3)
    P = synth.box_queries(M.V, 1 << 20, 7)
    d = synth.random_direction(3)
    t = synth.targets01(len(P), 8)
    return M, P, d, t


def _oracle_chunk(args):
    V, F, P, d, L, t = args
    from oracle import grad3d as G
    from oracle import wn3d as O
    r = O.wn3d(V, F, P, d, margins=False, loops=L)
    g = 2.0 * (r["w"] - t)
    Lx = O.loops_coords(V, L)
    G.grad3d(Lx, P, g)
    return len(P)


def cpu_baseline(M, P, d, t, nsample=64):
    """The FP64 oracle (forward + gradient) on a bounded sample of the same
    workload, on the host cores, before any GPU work in this process."""
    import multiprocessing as mp
    from oracle import wn3d as O
    cores = min(len(os.sched_getaffinity(0)), 16)
    idx = synth.rng(21).choice(len(P), nsample, replace=False)
    L = O.boundary_loops(M.F)
    chunks = np.array_split(idx, cores * 2)
    jobs = [(M.V, M.F, P[c], d, L, t[c]) for c in chunks if len(c)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        n = sum(pool.map(_oracle_chunk, jobs))
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "queries/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} random queries of the 2^20-query workload, forward w (brute-force "
                      f"crossings over all triangles + boundary term) and closed-form gradients, "
                      f"float64 numpy, multiprocessing over {cores} host cores; {dt:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--parity-sample", type=int, default=12)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on exactly one GPU (got --gpus {args.gpus}); "
              "multi-GPU runs are not part of it", file=sys.stderr)
        sys.exit(2)

    M, P, d, t = workload_c3()
    nq = len(P)
    cpu = None if args.no_cpu_baseline else cpu_baseline(M, P, d, t)

    import torch
    import paper_2408_04466_amd as W
    from oracle import wn3d as O

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    V = torch.from_numpy(M.V).to(dev)
    F = torch.from_numpy(M.F).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bvh = W.BVH(V, F, d)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    idx, off = W.boundary_loops(M.F)
    nb = len(idx)
    bnd = V[torch.from_numpy(idx.astype(np.int64)).to(dev)].contiguous()
    qx, qy, qz = (torch.from_numpy(np.ascontiguousarray(P[:, k])).to(dev) for k in range(3))
    tt = torch.from_numpy(t).to(dev)
    w = torch.empty(nq, dtype=torch.float32, device=dev)
    chi = torch.empty(nq, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        W.eval_3d(bvh, bnd, off, qx, qy, qz, want_chi=False, w_out=w)
        g = 2.0 * (w - tt)
        return W.backward(bnd, off, qx, qy, qz, g)

    # parity sample (the throughput below is reported only if it passes)
    W.eval_3d(bvh, bnd, off, qx, qy, qz, w_out=w, chi_out=chi)
    torch.cuda.synchronize()
    sidx = synth.rng(31).choice(nq, args.parity_sample, replace=False)
    r = O.wn3d(M.V, M.F, P[sidx], d)
    wc, cc = w.cpu().numpy(), chi.cpu().numpy()
    ok = ~r.degenerate
    chi_ok = bool(np.array_equal(cc[sidx][ok], r["chi"][ok]))
    werr = float(np.abs(wc[sidx] - r["w"])[ok & (r["m_bnd"] > 1e-5)].max())
    parity = {"sample": int(len(sidx)), "chi_bit_exact": chi_ok, "max_abs_w_err": werr,
              "degenerate": int((~ok).sum()), "pass": bool(chi_ok and werr <= 1e-4)}

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps

    # per-kernel timings on the same stream (HIP events around K launches)
    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    reps = max(args.steps, 10)
    chi_buf = torch.empty(nq, dtype=torch.int32, device=dev)
    W.crossings_3d(bvh, qx, qy, qz)
    ms_cross = timed(lambda: W.crossings_3d(bvh, qx, qy, qz), reps)
    chi_buf = W.crossings_3d(bvh, qx, qy, qz)
    ms_bnd = timed(lambda: W.eval_3d_boundary(bvh, bnd, off, qx, qy, qz, chi_buf), reps)
    gw = torch.ones(nq, dtype=torch.float32, device=dev)
    ms_bwd = timed(lambda: W.backward(bnd, off, qx, qy, qz, gw), reps)
    ms_fwd = timed(lambda: W.eval_3d(bvh, bnd, off, qx, qy, qz, want_chi=False, w_out=w), reps)

    pairs = nq * nb
    achieved = pairs * FLOPS_PER_PAIR_FWD / (ms_bnd * 1e-3) / 1e12
    out = {
        "metric": "winding queries/s fwd+bwd, batched vs plain, 3D mesh 2^20 pts at |err|<=1e-4",
        "value": nq / (ms_step * 1e-3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3D open mesh: noise-displaced sphere minus 30 deg cap, "
                               f"{M.F.shape[0]} triangles, {nb} boundary edges, 2^20 uniform queries "
                               "in 1.2x bbox, seeded random ray direction; fwd (crossings + boundary "
                               "integral) + bwd (adjoint w.r.t. queries and boundary vertices)",
                   "queries": nq, "triangles": int(M.F.shape[0]), "boundary_edges": nb,
                   "path": "plain"},
        "roofline": {"bound": "alu", "kernel": "k_bnd3d (boundary integral)",
                     "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "flops_per_pair": FLOPS_PER_PAIR_FWD, "pairs": pairs, "ms": ms_bnd},
        "kernels_ms": {"crossings": ms_cross, "boundary": ms_bnd, "forward": ms_fwd,
                       "backward": ms_bwd, "bvh_build": build_ms},
        "queries_per_s": {"fwd": nq / (ms_fwd * 1e-3), "fwd_bwd_plain": nq / (ms_step * 1e-3)},
        "parity": parity,
        "cpu_baseline": cpu,
    }
    if not parity["pass"]:
        out["value"] = None
        out["note"] = "parity sample failed: throughput withheld"
    print(json.dumps(out))


if __name__ == "__main__":
    main()
