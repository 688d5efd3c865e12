#!/usr/bin/env python3
"""Benchmark of the one-shot winding number hot path on one MI355X.

Headline step: one forward + backward pass over the 3D open-mesh workload,
through the batched persistent path (one hipGraph replay for the forward, one
persistent adjoint launch): a noise-displaced unit sphere with a 30 degree
polar cap removed (1,048,064 triangles, one boundary loop of 512 edges), 2^20
query points uniform in 1.2x its bounding box, seeded ray direction.
Forward = crossing count + boundary integral (w); backward = adjoint with
respect to the queries and the boundary vertices for L = sum (w - t)^2.
Inputs are resident in HBM before the timed region; BVH builds, graph
capture and autotuning are timed separately.

Also measured in the same run (reported beside the headline): the plain
path on the same workload, the 256-surface batch (batched vs a loop of plain
calls), the adjoint workload, and both 2D workloads.

Prints one JSON line.  ``--gpus N`` with N > 1 exits with status 2: the
library has no multi-GPU path, so the benchmark measures one GPU.
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
COUNTERS = os.path.join(ROOT, "profiles", "k_bnd3d_mesh_2p20_counters.md")
KERNEL_SOURCES = ("paper_2408_04466_amd/csrc/bnd3d.hip", "paper_2408_04466_amd/csrc/bndloop.hpp",
                  "paper_2408_04466_amd/csrc/geom.hpp")
# sources behind the other committed per-kernel VALU counts (the timed step's kernels)
STEP_KERNEL_SOURCES = {
    "k_batch_fwd": ("paper_2408_04466_amd/csrc/batch.hip", "paper_2408_04466_amd/csrc/bndloop.hpp",
                    "paper_2408_04466_amd/csrc/traverse.hpp", "paper_2408_04466_amd/csrc/geom.hpp",
                    "paper_2408_04466_amd/csrc/kernels.hpp", "paper_2408_04466_amd/csrc/bvh_build.hpp"),
    "k_batch_bwd": ("paper_2408_04466_amd/csrc/batch.hip", "paper_2408_04466_amd/csrc/adjloop.hpp",
                    "paper_2408_04466_amd/csrc/bndloop.hpp", "paper_2408_04466_amd/csrc/geom.hpp",
                    "paper_2408_04466_amd/csrc/kernels.hpp"),
}
FLOPS_PER_PAIR_BWD = 40      # adjoint, per (query, boundary edge)
PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector peak


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
    G.grad3d(O.loops_coords(V, L), P, g)
    return len(P)


def _parity_chunk(args):
    V, F, P, d, L = args
    from oracle import wn3d as O
    return dict(O.wn3d(V, F, P, d, loops=L))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pool, cores, M, P, d, t, nsample=64):
    """The FP64 oracle (forward + gradient) on a bounded sample of the same
    workload, on the host cores, before any GPU work in this process."""
    from oracle import wn3d as O
    idx = synth.rng(21).choice(len(P), nsample, replace=False)
    L = O.boundary_loops(M.F)
    chunks = np.array_split(idx, cores * 2)
    jobs = [(M.V, M.F, P[c], d, L, t[c]) for c in chunks if len(c)]
    t0 = time.perf_counter()
    n = sum(pool.map(_oracle_chunk, jobs))
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "queries/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{n} random queries of the 2^20-query mesh workload, forward w (brute-force "
                      f"crossings over all 1,048,064 triangles + boundary term) and closed-form "
                      f"gradients, float64 numpy, multiprocessing over {cores} host cores; "
                      f"{dt:.1f} s wall"}


def measured_counters():
    """(HBM bytes, VALU wavefront instructions) per k_bnd3d launch from the
    committed rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE scaled by
    a plain copy's counts; SQ_INSTS_VALU), or (None, None) when the kernel
    sources changed since the counters were taken."""
    import hashlib
    try:
        txt = open(COUNTERS).read()
    except OSError:
        return None, None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    vals = dict(line.split(": ", 1) for line in txt.splitlines()
                if line.startswith(("traffic_bytes_per_launch k_bnd3d", "source_sha256 k_bnd3d",
                                    "valu_wave_instructions_per_launch k_bnd3d")))
    if vals.get("source_sha256 k_bnd3d", "").strip() != h.hexdigest():
        return None, None
    valu = vals.get("valu_wave_instructions_per_launch k_bnd3d")
    return int(vals["traffic_bytes_per_launch k_bnd3d"]), (int(valu) if valu else None)


def step_kernel_valu():
    """{kernel: VALU wavefront instructions per launch} for the timed step's
    kernels from the committed counter summary, for those whose sources still
    hash to the value recorded with the count."""
    import hashlib
    try:
        txt = open(COUNTERS).read()
    except OSError:
        return {}
    vals = dict(line.split(": ", 1) for line in txt.splitlines()
                if line.startswith(("valu_wave_instructions_per_launch ", "source_sha256 ")))
    out = {}
    for k, files in STEP_KERNEL_SOURCES.items():
        h = hashlib.sha256()
        for f in files:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if vals.get(f"source_sha256 {k}", "").strip() == h.hexdigest() and f"valu_wave_instructions_per_launch {k}" in vals:
            out[k] = int(vals[f"valu_wave_instructions_per_launch {k}"])
    return out


def batch_path(info):
    """What the tuned one-surface batch runs, from its handle's settings."""
    mode = "split forward (crossing kernel, then boundary kernel)" if info["mode"] == 1 else \
        "fused forward (crossings + boundary integral in one kernel)"
    grid = (f"persistent grid of {info['wg_per_cu']} workgroups per CU pulling items"
            if info["wg_per_cu"] else "one workgroup per work item")
    launch = "replayed as a hipGraph" if info["graph"] else "launched directly"
    return (f"batched persistent path, 1 surface: {mode}, {grid}, tile {info['tile']} queries, "
            f"{launch}; backward: batched adjoint + fixed-order reduction")


# The paper's own timings for this path (Sec. 7, "3D Performance" and "2D
# Parametric Geometry"), as printed, on the CPU the paper names.  Context for
# the measured numbers, not a target: other machine, other meshes.
PAPER_CONTEXT = {
    "hardware": "Intel Core i7-9700X @ 4.900GHz as printed (no such part is listed; likely the 8-core "
                "i7-9700K), C++ with OpenMP",
    "mesh_one_shot_us_per_query": {"Piggy (F 11k, B 6, Q 600k)": 1.46, "Bunny (F 5k, B 9, Q 360k)": 2.12,
                                   "Camel (F 23k, B 56, Q 480k)": 8.99},
    "mesh_hierarchical_gwn_us_per_query": {"Piggy": 4.41, "Bunny": 2.69, "Camel": 4.71},
    "2d_1000_cubics_250x250_grid_total_ms": 5074,
    "2d_random_points_us_per_point": 0.08,
}


class Timer:
    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream

    def ms(self, fn, reps, warm=1):
        torch = self.torch
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(self.stream)
        for _ in range(reps):
            fn()
        b.record(self.stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps


def upload_mesh(torch, W, M, dev):
    V = torch.from_numpy(np.ascontiguousarray(M.V)).to(dev)
    F = torch.from_numpy(np.ascontiguousarray(M.F)).to(dev)
    idx, off = W.boundary_loops(M.F)
    bnd = V[torch.from_numpy(idx.astype(np.int64)).to(dev)].contiguous()
    return V, F, bnd, off, idx


def soa(torch, P, dev):
    return tuple(torch.from_numpy(np.ascontiguousarray(P[:, k])).to(dev) for k in range(3))


def copy_calibration():
    import torch
    n = 1 << 28                      # 2^28 float32 = 1 GiB each way
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))


def grid2d_only(args):
    """The 2D loops workload alone (16 loops x 64 cubics, float32, 2048^2 grid):
    grid-mode forward and backward, for profiling their kernels in isolation."""
    import torch
    import paper_2408_04466_amd as W
    dev = torch.device("cuda:0")
    T = Timer(torch, torch.cuda.current_stream())
    C2 = synth.loops2d()
    ctrl = torch.from_numpy(C2.ctrl).to(dev)
    xs = torch.from_numpy(synth.grid_axis(-1.2, 1.2, 2048, np.float32)).to(dev)
    g = torch.ones(2048, 2048, dtype=torch.float32, device=dev)
    ms = T.ms(lambda: W.eval_2d(ctrl, C2.loop_off, C2.closed, xs, xs, grid=True), args.steps)
    msb = T.ms(lambda: W.backward_2d(ctrl, C2.loop_off, C2.closed, xs, xs, g, grid=True), args.steps)
    print(json.dumps({"workload": "2d_loops_fp32_grid_2048^2", "forward_ms": ms, "backward_ms": msb,
                      "steps": args.steps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--parity-sample", type=int, default=256)
    ap.add_argument("--only-c3", action="store_true", help="skip the other workloads")
    ap.add_argument("--only-2d", action="store_true",
                    help="only time the 2D loops workload on its 2048^2 grid (forward and backward) and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 3 times (the reference kernel "
                         "for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.only_2d:
        grid2d_only(args)
        return
    if args.gpus != 1:
        print(f"bench.py: measures exactly one GPU (got --gpus {args.gpus}); "
              "the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    M, P, d, t = workload_c3()
    nq = len(P)
    # the oracle's worker processes are forked before this process touches
    # the GPU; they serve the CPU baseline and the parity sample
    import multiprocessing as mp
    cores = min(len(os.sched_getaffinity(0)), 16)
    pool = mp.get_context("fork").Pool(cores)
    cpu = None if args.no_cpu_baseline else cpu_baseline(pool, cores, M, P, d, t)
    others = None if args.only_c3 else {"c4": synth.coons_batch(4), "c5_mesh": synth.open_sphere(3, top_refine=4)}

    import torch
    import paper_2408_04466_amd as W
    from oracle import wn3d as O

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    T = Timer(torch, stream)
    V, F, bnd, off, idx = upload_mesh(torch, W, M, dev)
    nb = len(idx)
    qx, qy, qz = soa(torch, P, dev)
    tt = torch.from_numpy(t).to(dev)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    bvh = W.BVH(V, F, d)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    batch = W.Batch([{"V": V, "F": F, "bnd": bnd, "loop_off": off, "nq": nq}], d, tune_mode=1)
    torch.cuda.synchronize()
    batch_ms = (time.perf_counter() - t0) * 1e3

    w = torch.empty(nq, dtype=torch.float32, device=dev)
    chi = torch.empty(nq, dtype=torch.int32, device=dev)
    wb = torch.empty(nq, dtype=torch.float32, device=dev)

    # parity sample (the throughputs are reported only if it passes)
    batch.eval(qx, qy, qz, w_out=wb, chi_out=chi)
    W.eval_3d(bvh, bnd, off, qx, qy, qz, w_out=w, want_chi=False)
    torch.cuda.synchronize()
    sidx = synth.rng(31).choice(nq, args.parity_sample, replace=False)
    L = O.boundary_loops(M.F)
    t0 = time.perf_counter()
    parts = pool.map(_parity_chunk, [(M.V, M.F, P[c], d, L) for c in np.array_split(sidx, 2 * cores) if len(c)])
    r = O.Result(**{k: np.concatenate([p[k] for p in parts]) for k in parts[0]})
    parity_s = time.perf_counter() - t0
    pool.close()
    wc, cc = wb.cpu().numpy(), chi.cpu().numpy()
    ok = ~r.degenerate
    chi_ok = bool(np.array_equal(cc[sidx][ok], r["chi"][ok]))
    werr = float(np.abs(wc[sidx] - r["w"])[ok & (r["m_bnd"] > 1e-5)].max())
    same = bool(torch.equal(w, wb))
    parity = {"sample": int(len(sidx)), "chi_bit_exact": chi_ok, "max_abs_w_err": werr,
              "degenerate": int((~ok).sum()), "batched_equals_plain": same,
              "oracle_s": round(parity_s, 1),
              "pass": bool(chi_ok and werr <= 1e-4 and same)}

    n2t = -2.0 * tt              # dL/dw = 2 (w - t) = 2 w + (-2 t): one fused kernel per step

    def step_batched():
        batch.eval(qx, qy, qz, w_out=wb, want_chi=False)
        g = torch.add(n2t, wb, alpha=2.0)
        return batch.backward(qx, qy, qz, g)

    def step_plain():
        W.eval_3d(bvh, bnd, off, qx, qy, qz, want_chi=False, w_out=w)
        g = torch.add(n2t, w, alpha=2.0)
        return W.backward(bnd, off, qx, qy, qz, g)

    # untimed: alternate both steps for a while (clocks and allocator settle),
    # then the W warm-up steps of the timed path
    t_end = time.perf_counter() + 0.3
    while time.perf_counter() < t_end:
        step_batched()
        step_plain()
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        step_batched()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step_batched()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    ms_step_plain = T.ms(step_plain, args.steps, args.warmup)
    # per-step spread (events around each step; reported beside the value above)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for ea, eb in evs:
        ea.record(stream)
        step_batched()
        eb.record(stream)
    torch.cuda.synchronize()
    per_step = sorted(ea.elapsed_time(eb) for ea, eb in evs)

    # per-kernel timings on the same stream (HIP events around K launches)
    reps = max(args.steps, 10)
    chi_buf = W.crossings_3d(bvh, qx, qy, qz)
    ms_cross = T.ms(lambda: W.crossings_3d(bvh, qx, qy, qz), reps)
    ms_bnd = T.ms(lambda: W.eval_3d_boundary(bvh, bnd, off, qx, qy, qz, chi_buf), reps)
    gw = torch.ones(nq, dtype=torch.float32, device=dev)
    ms_bwd = T.ms(lambda: W.backward(bnd, off, qx, qy, qz, gw), reps)
    ms_fwd = T.ms(lambda: W.eval_3d(bvh, bnd, off, qx, qy, qz, want_chi=False, w_out=w), reps)
    ms_fwd_b = T.ms(lambda: batch.eval(qx, qy, qz, w_out=wb, want_chi=False), reps)
    ms_bwd_b = T.ms(lambda: batch.backward(qx, qy, qz, gw), reps)

    pairs = nq * nb
    achieved = pairs * FLOPS_PER_PAIR_FWD / (ms_bnd * 1e-3) / 1e12
    extra = {}
    if others is not None:
        extra = run_others(torch, W, T, others, d, args, dev)
    traffic, valu = measured_counters()
    step_valu = step_kernel_valu()
    step_ms = {"k_batch_fwd": ms_fwd_b, "k_batch_bwd": ms_bwd_b}
    step_counts = {k: {"ms": step_ms[k], "valu_wave_instructions": v} for k, v in step_valu.items()}

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
        "config": {"workload": "3D open mesh: noise-displaced unit sphere minus a 30 deg polar cap, "
                               f"{M.F.shape[0]} triangles, {nb} boundary edges, 2^20 uniform queries "
                               "in 1.2x bbox, seeded random ray direction; step = forward (crossings + "
                               "boundary integral) + backward (adjoint w.r.t. queries and boundary "
                               "vertices) through the batched persistent path",
                   "queries": nq, "triangles": int(M.F.shape[0]), "boundary_edges": nb,
                   "path": batch_path(batch.info()),
                   "batch_tuning": {k: batch.info()[k] for k in ("tile", "wg_per_cu", "mode", "graph")}},
        "roofline": {"bound": "alu", "kernel": "k_bnd3d (boundary integral)",
                     "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1, "
                                     "factors from a 1 GiB copy)",
                     "flops_per_pair": FLOPS_PER_PAIR_FWD, "pairs_per_launch": pairs,
                     "avg_launch_ms": ms_bnd,
                     # the committed SQ_INSTS_VALU count per launch (wavefront
                     # instructions) and per (query, edge) pair; not an issue
                     # fraction: float32 operations issue every 2 cycles per
                     # wavefront, float64, conversions and bit-field operations
                     # every 4, square root and reciprocal every 8
                     "valu": ({"wave_instructions_per_launch": valu, "per_pair": valu * 64 / pairs}
                              if valu else None)},
        "batched_vs_plain": {
            "mesh_2^20": {"batched_fwd_bwd_qps": nq / (ms_step * 1e-3),
                          "plain_fwd_bwd_qps": nq / (ms_step_plain * 1e-3),
                          "batched_fwd_qps": nq / (ms_fwd_b * 1e-3),
                          "plain_fwd_qps": nq / (ms_fwd * 1e-3),
                          "ratio_fwd_bwd": ms_step_plain / ms_step},
            **extra.get("c4", {})},
        "step_ms": {"mean": ms_step, "median": per_step[len(per_step) // 2], "min": per_step[0]},
        "device": {**W.device_info(), "name": torch.cuda.get_device_name(dev)},
        # the timed step's two kernels against the same vector-issue limit
        "step_valu": step_counts or None,
        "kernels_ms": {"crossings": ms_cross, "boundary": ms_bnd, "plain_forward": ms_fwd,
                       "plain_backward": ms_bwd, "batched_forward": ms_fwd_b, "batched_backward": ms_bwd_b,
                       "bvh_build": build_ms, "batch_create": batch_ms},
        "workloads": {k: v for k, v in extra.items() if k != "c4"},
        "parity": parity,
        "cpu_baseline": cpu,
        "paper_context": PAPER_CONTEXT,
    }
    if not parity["pass"]:
        out["value"] = None
        out["note"] = "parity sample failed: throughput withheld"
    print(json.dumps(out))


def run_others(torch, W, T, others, d3, args, dev):
    res = {}
    reps = max(3, args.steps // 4)
    # --- 256-surface batch: batched persistent launch vs a loop of plain calls
    CB = others["c4"]
    surfs, P = [], []
    for Mk, Qk in zip(CB.meshes, CB.queries):
        V, F, bnd, off, idx = upload_mesh(torch, W, Mk, dev)
        surfs.append({"V": V, "F": F, "bnd": bnd, "loop_off": off, "nq": len(Qk), "nb": len(idx)})
        P.append(Qk)
    P = np.concatenate(P, 0)
    q = soa(torch, P, dev)
    nq = len(P)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B = W.Batch(surfs, CB.direction, tune_mode=1)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    w = torch.empty(nq, dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    B.eval(*q, w_out=w, want_chi=False)          # autotunes, then captures
    torch.cuda.synchronize()
    first_ms = (time.perf_counter() - t0) * 1e3
    info = B.info()
    bvhs = [W.BVH(s["V"], s["F"], CB.direction) for s in surfs]
    offs = np.concatenate([[0], np.cumsum([s["nq"] for s in surfs])])
    wp = torch.empty(nq, dtype=torch.float32, device=dev)
    g = torch.ones(nq, dtype=torch.float32, device=dev)

    def plain_fwd():
        for k, s in enumerate(surfs):
            a, b = int(offs[k]), int(offs[k + 1])
            W.eval_3d(bvhs[k], s["bnd"], s["loop_off"], q[0][a:b], q[1][a:b], q[2][a:b],
                      want_chi=False, w_out=wp[a:b])

    def plain_bwd():
        for k, s in enumerate(surfs):
            a, b = int(offs[k]), int(offs[k + 1])
            W.backward(s["bnd"], s["loop_off"], q[0][a:b], q[1][a:b], q[2][a:b], g[a:b])

    ms_bf = T.ms(lambda: B.eval(*q, w_out=w, want_chi=False), reps)
    ms_bb = T.ms(lambda: B.backward(*q, g), reps)
    ms_pf = T.ms(plain_fwd, reps)
    ms_pb = T.ms(plain_bwd, reps)
    same = bool(torch.equal(w, wp))
    pairs = info["total_pairs"]
    res["c4"] = {"surfaces_256": {
        "queries": nq, "pairs": pairs, "triangles": int(sum(m.F.shape[0] for m in CB.meshes)),
        "batched_fwd_ms": ms_bf, "plain_fwd_ms": ms_pf, "batched_bwd_ms": ms_bb, "plain_bwd_ms": ms_pb,
        "batched_fwd_bwd_qps": nq / ((ms_bf + ms_bb) * 1e-3), "plain_fwd_bwd_qps": nq / ((ms_pf + ms_pb) * 1e-3),
        "ratio_fwd": ms_pf / ms_bf, "ratio_fwd_bwd": (ms_pf + ms_pb) / (ms_bf + ms_bb),
        "boundary_TFLOPs_batched_fwd": pairs * FLOPS_PER_PAIR_FWD / (ms_bf * 1e-3) / 1e12,
        "tile": info["tile"], "wg_per_cu": info["wg_per_cu"], "graph": info["graph"],
        "forward_mode": "split" if info["mode"] else "fused",
        "create_ms": create_ms, "first_eval_ms_incl_tuning": first_ms, "tune_ms": info["tune_us"] / 1e3,
        "batched_equals_plain": same}}
    B.free()
    del bvhs
    # --- adjoint workload: boundary refined to 2048 edges, 2^18 queries
    M5 = others["c5_mesh"]
    P5 = synth.box_queries(M5.V, 1 << 18, 13)
    t5 = torch.from_numpy(synth.targets01(len(P5), 14)).to(dev)
    V, F, bnd, off, idx = upload_mesh(torch, W, M5, dev)
    bvh5 = W.BVH(V, F, d3)
    q5 = soa(torch, P5, dev)
    w5 = torch.empty(len(P5), dtype=torch.float32, device=dev)

    def step5():
        W.eval_3d(bvh5, bnd, off, *q5, want_chi=False, w_out=w5)
        return W.backward(bnd, off, *q5, 2.0 * (w5 - t5))

    ms5 = T.ms(step5, reps)
    gw5 = torch.ones(len(P5), dtype=torch.float32, device=dev)
    ms5b = T.ms(lambda: W.backward(bnd, off, *q5, gw5), reps)
    p5 = len(P5) * len(idx)
    res["adjoint_2048_edges_2^18"] = {"fwd_bwd_ms": ms5, "bwd_ms": ms5b, "queries_per_s": len(P5) / (ms5 * 1e-3),
                                      "bwd_TFLOPs": p5 * FLOPS_PER_PAIR_BWD / (ms5b * 1e-3) / 1e12}
    # --- 3D grid mode: 128^3 voxel grid over the mesh, d = +z, one ray per column
    M3 = synth.open_sphere(3)
    dz = np.array([0.0, 0.0, 1.0])
    V, F, bnd, off, idx = upload_mesh(torch, W, M3, dev)
    bvhz = W.BVH(V, F, dz)
    lo, hi = M3.V.min(0).astype(np.float64), M3.V.max(0).astype(np.float64)
    c, h = (lo + hi) / 2, (hi - lo) / 2 * 1.2
    ax = [synth.grid_axis(c[k] - h[k], c[k] + h[k], 128, np.float32) for k in range(3)]
    gx, gy, gz = (torch.from_numpy(a).to(dev) for a in ax)
    Xg, Yg, Zg = np.meshgrid(*ax, indexing="ij")
    qg = tuple(torch.from_numpy(np.ascontiguousarray(a.ravel())).to(dev) for a in (Xg, Yg, Zg))
    wg = torch.empty(128 ** 3, dtype=torch.float32, device=dev)
    perm = torch.from_numpy(synth.rng(17).permutation(128 ** 3)).to(dev)
    qs = tuple(t[perm].contiguous() for t in qg)          # the same points in random order
    ws = torch.empty_like(wg)
    ms_g = T.ms(lambda: W.eval_3d_grid(bvhz, bnd, off, gx, gy, gz, want_chi=False), reps)
    ms_gq = T.ms(lambda: W.eval_3d(bvhz, bnd, off, *qg, want_chi=False, w_out=wg), reps)
    ms_gs = T.ms(lambda: W.eval_3d(bvhz, bnd, off, *qs, want_chi=False, w_out=ws), reps)
    wgrid, _ = W.eval_3d_grid(bvhz, bnd, off, gx, gy, gz, want_chi=False)
    torch.cuda.synchronize()
    res["3d_voxel_grid_128^3_dz"] = {
        "grid_ms": ms_g, "points_in_column_order_ms": ms_gq, "points_in_random_order_ms": ms_gs,
        "queries_per_s": 128 ** 3 / (ms_g * 1e-3),
        "grid_equals_per_query": bool(torch.equal(wgrid.view(-1), wg) and torch.equal(ws, wg[perm]))}
    del bvhz
    # --- 2D workloads
    C1 = synth.star2d()
    ctrl = torch.from_numpy(C1.ctrl).to(dev)
    xs = torch.from_numpy(synth.grid_axis(-1.5, 1.5, 128)).to(dev)
    ms1 = T.ms(lambda: W.eval_2d(ctrl, C1.loop_off, C1.closed, xs, xs, grid=True), reps)
    res["2d_star_fp64_grid_128^2"] = {"ms": ms1, "queries_per_s": 128 * 128 / (ms1 * 1e-3)}
    C2 = synth.loops2d()
    ctrl2 = torch.from_numpy(C2.ctrl).to(dev)
    xs2 = torch.from_numpy(synth.grid_axis(-1.2, 1.2, 2048, np.float32)).to(dev)
    ms2 = T.ms(lambda: W.eval_2d(ctrl2, C2.loop_off, C2.closed, xs2, xs2, grid=True), reps)
    g2 = torch.ones(2048, 2048, dtype=torch.float32, device=dev)
    ms2b = T.ms(lambda: W.backward_2d(ctrl2, C2.loop_off, C2.closed, xs2, xs2, g2, grid=True), reps)
    res["2d_loops_fp32_grid_2048^2"] = {"ms": ms2, "queries_per_s": 2048 * 2048 / (ms2 * 1e-3),
                                        "hbm_GBs_outputs": 2048 * 2048 * 8 / (ms2 * 1e-3) / 1e9,
                                        "backward_ms": ms2b,
                                        "backward_hbm_GBs": 2048 * 2048 * 12 / (ms2b * 1e-3) / 1e9}
    # --- curved boundary: a Coons surface (~1M triangles) bounded by 4 cubic
    # Beziers, 2^20 queries; boundary term along the curves vs the 512-edge
    # polyline through the same boundary vertices
    MC = synth.coons_surface(6, 1 << 20, 512)
    dmc = synth.random_direction(106)
    Vc = torch.from_numpy(MC.V).to(dev)
    bvhc = W.BVH(Vc, torch.from_numpy(MC.F).to(dev), dmc)
    idxc, offc = W.boundary_loops(MC.F)
    bndc = Vc[torch.from_numpy(idxc.astype(np.int64)).to(dev)].contiguous()
    Pc = synth.box_queries(MC.V, 1 << 20, 7)
    qc = [torch.from_numpy(np.ascontiguousarray(Pc[:, k])).to(dev) for k in range(3)]
    ctrlc = torch.from_numpy(np.ascontiguousarray(MC.info["curves"].astype(np.float32))).to(dev)
    zc = torch.zeros(1 << 20, dtype=torch.int32, device=dev)
    ms_cb = T.ms(lambda: W.eval_3d_curves(bvhc, ctrlc, *qc, chi_in=zc), reps)
    ms_cw = T.ms(lambda: W.eval_3d_curves(bvhc, ctrlc, *qc), reps)
    ms_pb = T.ms(lambda: W.eval_3d_boundary(bvhc, bndc, offc, *qc, zc), reps)
    ms_tw = T.ms(lambda: W.eval_3d(bvhc, bndc, offc, *qc), reps)
    gwc = torch.ones(1 << 20, dtype=torch.float32, device=dev)
    ms_cbw = T.ms(lambda: W.backward_curves(ctrlc, *qc, gwc), reps)
    netc = torch.from_numpy(np.ascontiguousarray(MC.info["net"][None].astype(np.float32))).to(dev)
    ms_pc = T.ms(lambda: W.eval_3d_patches(dmc, netc, None, *qc, want_w=False), reps)
    ms_pw = T.ms(lambda: W.eval_3d_patches(dmc, netc, ctrlc, *qc), reps)
    # the same queries once put in Morton order (results are the same values, permuted)
    ms_ord = T.ms(lambda: W.spatial_order(*qc), reps)
    oc = W.spatial_order(*qc).long()
    qs = [t[oc].contiguous() for t in qc]
    ms_cws = T.ms(lambda: W.eval_3d_curves(bvhc, ctrlc, *qs), reps)
    ms_pws = T.ms(lambda: W.eval_3d_patches(dmc, netc, ctrlc, *qs), reps)
    ms_tws = T.ms(lambda: W.eval_3d(bvhc, bndc, offc, *qs), reps)
    ms_cbws = T.ms(lambda: W.backward_curves(ctrlc, *qs, gwc), reps)
    res["3d_spatial_order_2p20"] = {
        "order_ms": ms_ord, "curves_w_sorted_ms": ms_cws, "patches_w_sorted_ms": ms_pws,
        "tessellated_w_sorted_ms_1M_triangles": ms_tws, "curves_backward_sorted_ms": ms_cbws}
    res["3d_parametric_coons_2p20"] = {
        "patches": 1, "curves": 4, "crossings_ms": ms_pc, "w_ms": ms_pw,
        "tessellated_w_ms_1M_triangles": ms_tw, "queries_per_s": (1 << 20) / (ms_pw * 1e-3)}
    res["3d_curved_boundary_coons_2p20"] = {
        "curves": 4, "curves_boundary_ms": ms_cb, "curves_with_bvh_chi_ms": ms_cw,
        "polyline_512_boundary_ms": ms_pb, "curves_backward_ms": ms_cbw,
        "queries_per_s": (1 << 20) / (ms_cw * 1e-3)}
    del bvhc
    # --- 64 parametric surfaces (1 patch + 4 boundary curves each, own
    # direction, 2^14 queries each): one batched launch vs 64 single calls
    ps_nets, ps_curves, ps_q, ps_desc = [], [], [], []
    for k in range(64):
        Mk = synth.coons_surface(1000 + k, 300, 16)
        dk = synth.random_direction(2000 + k)
        ps_nets.append(Mk.info["net"][None])
        ps_curves.append(Mk.info["curves"])
        ps_q.append(synth.box_queries(Mk.V, 1 << 14, 3000 + k))
        ps_desc.append((1, 4, 1 << 14, dk))
    pb = W.PatchBatch(ps_desc)
    pnets = torch.from_numpy(np.ascontiguousarray(np.concatenate(ps_nets).astype(np.float32))).to(dev)
    pcurv = torch.from_numpy(np.ascontiguousarray(np.concatenate(ps_curves).astype(np.float32))).to(dev)
    pq = np.concatenate(ps_q).astype(np.float32)
    pqs = [torch.from_numpy(np.ascontiguousarray(pq[:, k])).to(dev) for k in range(3)]
    ms_pbat = T.ms(lambda: pb.eval(pnets, pcurv, *pqs), reps)
    views = [(pnets[k:k + 1], pcurv[4 * k:4 * k + 4], [t[k << 14:(k + 1) << 14] for t in pqs], ps_desc[k][3])
             for k in range(64)]

    def loop_ps():
        for n_k, c_k, q_k, d_k in views:
            W.eval_3d_patches(d_k, n_k, c_k, *q_k)

    ms_ploop = T.ms(loop_ps, reps)
    res["3d_parametric_batched_64x2p14"] = {
        "surfaces": 64, "queries": 1 << 20, "batched_ms": ms_pbat, "loop_of_single_calls_ms": ms_ploop,
        "queries_per_s": (1 << 20) / (ms_pbat * 1e-3)}
    # --- the 2D experiment's shape: 1000 random cubics, each on its own 250^2
    # grid, float64; one batched launch vs a loop of single-set calls
    E1 = synth.random_cubics(seed=5, n=1000, res=250, dtype=np.float64)
    ctrl3 = torch.from_numpy(np.concatenate([C.ctrl for C, _, _ in E1])).to(dev)
    xe = torch.from_numpy(np.concatenate([xs for _, xs, _ in E1])).to(dev)
    ye = torch.from_numpy(np.concatenate([ys for _, _, ys in E1])).to(dev)
    b2 = W.Batch2D([(C.loop_off, C.closed, 250, 250) for C, _, _ in E1], torch.float64)
    w3 = torch.empty(b2.nout, dtype=torch.float64, device=dev)
    c3 = torch.empty(b2.nout, dtype=torch.int32, device=dev)
    ms3 = T.ms(lambda: b2.eval(ctrl3, xe, ye, out=(w3, c3)), reps)
    ms3w = T.ms(lambda: b2.eval(ctrl3, xe, ye, out=(w3, None)), reps)
    singles = [(ctrl3[k:k + 1], C.loop_off, C.closed, xe[250 * k:250 * (k + 1)], ye[250 * k:250 * (k + 1)])
               for k, (C, _, _) in enumerate(E1)]

    def loop_e1():
        for c, lo, cl, xk, yk in singles:
            W.eval_2d(c, lo, cl, xk, yk, grid=True)
    ms3l = T.ms(loop_e1, 2)
    nq3 = 1000 * 250 * 250
    res["2d_random_cubics_fp64_1000x250^2"] = {
        "batched_ms": ms3, "queries_per_s": nq3 / (ms3 * 1e-3),
        "hbm_GBs_outputs": nq3 * 12 / (ms3 * 1e-3) / 1e9,
        "batched_w_only_ms": ms3w, "w_only_hbm_GBs": nq3 * 8 / (ms3w * 1e-3) / 1e9,
        "loop_of_single_calls_ms": ms3l}
    return res


if __name__ == "__main__":
    main()
