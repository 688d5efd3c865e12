"""wn_backward_noalloc (the adjoint with its workspace in the library's own
device array) against wn_backward through the C ABI: same kernels and the
same fixed-order reductions, so the outputs must agree bit for bit.  Two
calls in a row, the second with a smaller input, so that the second reads
only what it wrote itself; a call with few queries over a long boundary
(split into vertex ranges); and a workspace beyond the array's size, which
must be refused before anything is enqueued."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2408_04466_amd as W
    from gpu_util import DevMesh


def _inputs(dm, M, n, seed):
    P = synth.box_queries(M.V, n, seed)
    qx, qy, qz = dm.queries(P)
    g = torch.from_numpy(synth.rng(seed + 1).normal(size=n).astype(np.float32)).cuda()
    return qx, qy, qz, g


def _both(dm, qx, qy, qz, g):
    ref = W.backward(dm.bnd, dm.loop_off, qx, qy, qz, g)
    # outputs prefilled with NaN: every entry must be written by the call
    gq = torch.full((qx.numel(), 3), float("nan"), device="cuda")
    gb = torch.full(tuple(dm.bnd.shape), float("nan"), device="cuda")
    out = W.backward(dm.bnd, dm.loop_off, qx, qy, qz, g, grad_q=gq, grad_bnd=gb, noalloc=True)
    torch.cuda.synchronize()
    return ref, out


@pytest.mark.parametrize("mesh,sizes", [("open_sphere", (1 << 18, 5000)),
                                        ("refined", (1 << 16, 3000))])
def test_noalloc_matches_backward_twice(mesh, sizes):
    M = synth.open_sphere(3) if mesh == "open_sphere" else synth.open_sphere(3, top_refine=4)
    dm = DevMesh(M, synth.random_direction(3))
    for k, n in enumerate(sizes):
        print(f"noalloc {mesh}: call {k}, {n} queries, {len(dm.bnd_idx)} boundary vertices", flush=True)
        (rq, rb), (nq_, nb_) = _both(dm, *_inputs(dm, M, n, 40 + k))
        assert torch.equal(rq, nq_), f"grad_q differs on call {k}"
        assert torch.equal(rb, nb_), f"grad_bnd differs on call {k}"
        assert torch.isfinite(nq_).all() and torch.isfinite(nb_).all()


def test_noalloc_one_output_and_empty():
    M = synth.bumpy_cap()
    dm = DevMesh(M, synth.random_direction(3))
    qx, qy, qz, g = _inputs(dm, M, 777, 50)
    rq, _ = W.backward(dm.bnd, dm.loop_off, qx, qy, qz, g, want_bnd=False)
    nq_, nb_ = W.backward(dm.bnd, dm.loop_off, qx, qy, qz, g, want_bnd=False, noalloc=True)
    _, rb = W.backward(dm.bnd, dm.loop_off, qx, qy, qz, g, want_q=False)
    _, nb2 = W.backward(dm.bnd, dm.loop_off, qx, qy, qz, g, want_q=False, noalloc=True)
    torch.cuda.synchronize()
    assert nb_ is None and torch.equal(rq, nq_) and torch.equal(rb, nb2)
    e = torch.empty(0, device="cuda")
    gq, gb = W.backward(dm.bnd, dm.loop_off, e, e, e, e, noalloc=True)
    torch.cuda.synchronize()
    assert gq.shape == (0, 3) and torch.equal(gb, torch.zeros_like(gb))


def test_noalloc_refuses_oversized_workspace():
    M = synth.open_sphere(3, top_refine=4)
    dm = DevMesh(M, synth.random_direction(3))
    n = 1 << 22      # about 400 MB of vertex partials over 2048 boundary vertices
    q = torch.zeros(n, device="cuda")
    gq = torch.full((n, 3), 7.0, device="cuda")
    with pytest.raises(W.WnError) as ei:
        W.backward(dm.bnd, dm.loop_off, q, q, q, q, grad_q=gq, noalloc=True)
    assert ei.value.status == 2 and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((gq == 7.0).all())   # nothing was enqueued
