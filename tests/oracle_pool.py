"""A process pool for running the FP64 oracle on large parity samples.

The workers are forked when this module is first imported, before any test
initialises the GPU (conftest imports it first), so they hold no GPU state
and never touch the device.  Each task carries its own inputs.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))
_pool = None


def start():
    """Fork the workers (call before the GPU is initialised)."""
    return _start()


def _start():
    global _pool
    if _pool is None:
        _pool = mp.get_context("fork").Pool(WORKERS)
    return _pool


def _wn3d_chunk(args):
    V, F, P, d, loops = args
    from oracle import wn3d as O
    r = O.wn3d(V, F, P, d, loops=loops)
    return dict(r)


def wn3d(V, F, P, d, loops=None):
    """oracle.wn3d over the rows of P, split across the workers (same result
    as one call: every query is independent)."""
    from oracle import wn3d as O
    P = np.atleast_2d(np.asarray(P))
    if loops is None:
        loops = O.boundary_loops(F)
    if len(P) < 2 * WORKERS:
        return O.wn3d(V, F, P, d, loops=loops)
    chunks = [c for c in np.array_split(np.arange(len(P)), 2 * WORKERS) if len(c)]
    parts = _start().map(_wn3d_chunk, [(V, F, P[c], d, loops) for c in chunks])
    out = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    return O.Result(**out)


def map_wn3d(jobs):
    """[oracle.wn3d(V, F, P, d, loops=loops) for (V, F, P, d, loops) in jobs],
    one job per task."""
    from oracle import wn3d as O
    jobs = list(jobs)
    parts = _start().map(_wn3d_chunk, jobs, chunksize=1)
    return [O.Result(**p) for p in parts]


def _grad3d_chunk(args):
    Lx, P, g = args
    from oracle import grad3d as G
    return G.grad3d(Lx, P, g)


def grad3d(Lx, P, g):
    """oracle.grad3d over the rows of P split across the workers: the query
    gradients concatenated, the boundary gradients summed over chunks in
    chunk order."""
    from oracle import grad3d as G
    P = np.atleast_2d(np.asarray(P, np.float64))
    g = np.asarray(g, np.float64)
    if len(P) < 2 * WORKERS:
        return G.grad3d(Lx, P, g)
    # at most 2048 queries per task: the oracle holds [queries, edges, 3] arrays
    n = max(2 * WORKERS, -(-len(P) // 2048))
    chunks = [c for c in np.array_split(np.arange(len(P)), n) if len(c)]
    parts = _start().map(_grad3d_chunk, [(Lx, P[c], g[c]) for c in chunks])
    gq = np.concatenate([p[0] for p in parts])
    gv = [sum(p[1][k] for p in parts) for k in range(len(Lx))]
    return gq, gv


def shutdown():
    global _pool
    if _pool is not None:
        _pool.terminate()
        _pool.join()
        _pool = None


def _wn2d_chunk(args):
    ctrl, loop_off, closed, P = args
    from oracle import wn2d as O2
    return dict(O2.wn2d(ctrl, loop_off, closed, P))


def wn2d(ctrl, loop_off, closed, P):
    """oracle.wn2d over the rows of P split across the workers, queries
    grouped by ordinate so that the points of one ray line stay together
    (the oracle solves each line's roots once)."""
    from oracle import wn2d as O2
    P = np.atleast_2d(np.asarray(P, np.float64))
    if len(P) < 2 * WORKERS:
        return O2.wn2d(ctrl, loop_off, closed, P)
    order = np.argsort(P[:, 1], kind="stable")
    chunks = [c for c in np.array_split(order, 4 * WORKERS) if len(c)]
    parts = _start().map(_wn2d_chunk, [(ctrl, loop_off, closed, P[c]) for c in chunks])
    out = {}
    for k in parts[0]:
        v = np.empty(len(P), dtype=np.asarray(parts[0][k]).dtype)
        for c, part in zip(chunks, parts):
            v[c] = part[k]
        out[k] = v
    return O2.Result2D(**out)
