"""GPU tests of the diagnostic counters (wn_diagnose) and the device query
(wn_device_info): counts of non-finite queries and of finite queries with
an invalid crossing count, on a call's real outputs and on a chi array
written here; exact at sizes across the grid-stride boundary."""
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


def test_counts_on_a_real_call():
    M = synth.bumpy_cap()
    dm = DevMesh(M, synth.random_direction(400))
    P = synth.box_queries(M.V, 5000, 401)
    P[::37, 0] = np.nan
    P[5::101, 2] = -np.inf
    nonfin = int((~np.isfinite(P).all(1)).sum())
    q = _q(P)
    w, chi = W.eval_3d(dm.bvh, dm.bnd, dm.loop_off, *q)
    c = W.diagnose(*q, chi)
    torch.cuda.synchronize()
    assert c.tolist() == [nonfin, 0]


@pytest.mark.parametrize("n", [1, 255, 257, 4096 * 256 + 3, 3 << 20])
def test_counts_are_exact(n):
    g = synth.rng(402 + n % 97)
    P = g.uniform(-1, 1, (n, 3)).astype(np.float32)
    bad = g.uniform(0, 1, n) < 0.01
    P[bad, g.integers(0, 3, int(bad.sum()))] = np.nan
    chi = np.zeros(n, np.int32)
    inval = g.uniform(0, 1, n) < 0.02
    chi[inval] = W.WN_CHI_INVALID
    c = W.diagnose(*_q(P), torch.from_numpy(chi).cuda())
    torch.cuda.synchronize()
    assert c.tolist() == [int(bad.sum()), int((inval & ~bad).sum())]
    # the counters are overwritten, not accumulated
    c2 = W.diagnose(*_q(P), torch.from_numpy(chi).cuda())
    torch.cuda.synchronize()
    assert torch.equal(c, c2)


def test_empty_and_device_info():
    e = torch.empty(0, device="cuda")
    c = W.diagnose(e, e, e, torch.empty(0, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    assert c.tolist() == [0, 0]
    info = W.device_info()
    assert info["compute_units"] > 0 and info["clock_mhz"] > 0
