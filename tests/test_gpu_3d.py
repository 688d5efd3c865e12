"""GPU parity of the 3D path (crossings + boundary integral) against the FP64
oracle, through the C ABI.  chi bit-exact on non-degenerate queries, w within
1e-4 away from the boundary (Alg. 1; Eq. chi; Eq. wn_discrete_sum)."""
import math

import os

import numpy as np
import pytest
import torch

import synth
from oracle import wn3d as O

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2408_04466_amd as W
    from gpu_util import DevMesh, compare_3d, W_TOL


def _rand_queries(M, n, seed, scale=1.2):
    P = synth.box_queries(M.V, n, seed, scale=scale)
    ext = np.ptp(M.V.astype(np.float64), axis=0)
    if ext.min() < 1e-3 * ext.max():
        # flat mesh: spread the queries off its plane as well
        k = int(np.argmin(ext))
        P[:, k] = synth.rng(seed + 1).uniform(-0.6, 0.6, n) * ext.max()
    return P


SMALL = {
    "bumpy_cap": lambda: synth.bumpy_cap(),
    "twisted_sheet": lambda: synth.random_open_mesh(3, n=6),
    "coons": lambda: synth.coons_surface(11, 2000, 96),
    "disk": lambda: synth.disk_fan(64),
    "sphere_small": lambda: synth.open_sphere(4, n_lon=48, n_rings=40, top_refine=2),
}


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("dseed", [3, 17])
def test_small_meshes_match_oracle(name, dseed):
    M = SMALL[name]()
    dm = DevMesh(M, synth.random_direction(dseed))
    P = _rand_queries(M, 1500, 100 + dseed)
    w, chi = dm.eval(P)
    compare_3d(dm, P, w, chi)


def _union(meshes, offsets):
    Vs, Fs, n = [], [], 0
    for M, o in zip(meshes, offsets):
        Vs.append(M.V + np.asarray(o, np.float32))
        Fs.append(M.F + n)
        n += len(M.V)
    return synth.Mesh(np.concatenate(Vs), np.concatenate(Fs).astype(np.int32))


def test_many_loops_across_lds_chunks():
    # five disjoint patches: 5 boundary loops of 200-260 edges, so loops
    # straddle the 512-vertex LDS chunks of the boundary kernel
    parts = [synth.coons_surface(40 + k, 1500, 200 + 16 * k) for k in range(5)]
    M = _union(parts, [(1.3 * k, 0.2 * k, 0.0) for k in range(5)])
    dm = DevMesh(M, synth.random_direction(23))
    assert len(dm.loop_off) == 6 and dm.loop_off[-1] > 1024
    P = _rand_queries(M, 2000, 24)
    w, chi = dm.eval(P)
    compare_3d(dm, P, w, chi)
    # and the union equals the sum of the parts (Sec. 7, Fig. bool: union = sum of w)
    tot = np.zeros(len(P))
    for Mk, o in zip(parts, [(1.3 * k, 0.2 * k, 0.0) for k in range(5)]):
        Mk = synth.Mesh(Mk.V + np.asarray(o, np.float32), Mk.F)
        tot += DevMesh(Mk, synth.random_direction(23)).eval(P)[0]
    assert np.abs(tot - w).max() <= 5 * W_TOL


def test_closed_mesh_inside_outside():
    M = synth.icosphere(3)
    dm = DevMesh(M, synth.random_direction(5))
    assert len(dm.loop_off) == 1     # no boundary loops
    P = synth.rng(3).uniform(-1.5, 1.5, (20000, 3)).astype(np.float32)
    w, chi = dm.eval(P)
    r = np.linalg.norm(P.astype(np.float64), axis=1)
    far = np.abs(r - 1.0) > 0.02
    assert np.array_equal(w[far], (r[far] < 1.0).astype(np.float32))
    assert np.array_equal(chi[far], (r[far] < 1.0).astype(np.int32))


@pytest.fixture(scope="module")
def c3():
    """The 3D open-mesh workload: noise-displaced unit sphere (amplitude 0.05)
    with a 30 degree polar cap removed, 512 x 1024 rings (1,048,064
    triangles, one boundary loop of 512 edges), 2^20 queries uniform in 1.2x
    its bounding box, seeded random direction."""
    M = synth.open_sphere(3)
    d = synth.random_direction(3)
    dm = DevMesh(M, d)
    P = _rand_queries(M, 1 << 20, 7)
    w, chi = dm.eval(P)
    return dm, P, w, chi


def test_c3_full_size_sampled_parity(c3):
    """1024 seeded queries of the 2^20 (plus the first and the last) against
    the FP64 oracle over all 1,048,064 triangles."""
    dm, P, w, chi = c3
    assert dm.M.F.shape[0] == 1048064 and len(dm.bnd_idx) == 512
    sample = synth.rng(11).choice(len(P), 1024, replace=False)
    sample = np.concatenate([sample, [0, len(P) - 1]])
    info = compare_3d(dm, P, w, chi, sample, label="mesh 2^20")
    print("c3 sample", info)


def test_c3_full_size_batched_path_matches(c3):
    """The headline configuration: the mesh workload as a one-surface batch
    with quick autotuning and graph replay gives the plain path's bits
    (which the oracle samples above pin)."""
    dm, P, w, chi = c3
    q = dm.queries(P)
    B = W.Batch([{"V": dm.V, "F": dm.F, "bnd": dm.bnd, "loop_off": dm.loop_off, "nq": len(P)}],
                dm.d, tune_mode=1)
    for _ in range(2):
        wb, cb = B.eval(*q)
        torch.cuda.synchronize()
        assert np.array_equal(wb.cpu().numpy(), w) and np.array_equal(cb.cpu().numpy(), chi)
    B.free()


def test_c3_properties_at_full_size(c3):
    dm, P, w, chi = c3
    assert np.all(np.isfinite(w))
    assert chi.min() >= -2 and chi.max() <= 3
    # a second direction gives the same w (d-invariance) everywhere except
    # next to the boundary curve
    dm2 = DevMesh(dm.M, synth.random_direction(99))
    w2, chi2 = dm2.eval(P)
    from scipy.spatial import cKDTree
    L = dm.M.V[dm.bnd_idx].astype(np.float64)
    t = np.linspace(0, 1, 64, endpoint=False)[:, None, None]
    dense = (L[None] * (1 - t) + np.roll(L, -1, 0)[None] * t).reshape(-1, 3)
    dist, _ = cKDTree(dense).query(P.astype(np.float64), distance_upper_bound=1e-4)
    far = np.isinf(dist)
    diff = np.abs(w - w2)
    assert diff[far].max() <= 2 * W_TOL, diff[far].max()
    # the crossing counts differ, the winding numbers agree
    assert np.any(chi != chi2)


def test_near_boundary_queries():
    M = synth.open_sphere(3, n_lon=128, n_rings=64)
    d = synth.random_direction(21)
    dm = DevMesh(M, d)
    V = M.V.astype(np.float64)
    L = dm.bnd_idx
    g = synth.rng(5)
    pts = []
    for k, dist in enumerate([1e-5, 3e-5, 1e-4, 1e-3, 1e-2]):
        for _ in range(40):
            i = int(g.integers(len(L)))
            a, b = V[L[i]], V[L[(i + 1) % len(L)]]
            m = a + g.uniform(0.1, 0.9) * (b - a)
            e = (b - a) / np.linalg.norm(b - a)
            u = g.normal(size=3)
            u -= (u @ e) * e
            u /= np.linalg.norm(u)
            pts.append(m + dist * u * 1.5)
    P = np.array(pts, np.float32)
    w, chi = dm.eval(P)
    compare_3d(dm, P, w, chi, max_degenerate_frac=0.2)


def test_near_boundary_error_follows_float32_conditioning():
    """Queries 1e-6 to 1e-2 from boundary edges of meshes whose boundary
    edges are long (0.07 to 0.8).  Away from the boundary (at least
    near_band = 1e-4 x the longest edge L) w is within W_TOL of the oracle;
    closer, the error stays below 2^-24 L / delta, the float32 conditioning of
    w there (delta: the oracle's distance to the boundary).  chi is bit-exact
    wherever the oracle calls the query regular."""
    import oracle_pool
    from gpu_util import NEAR_REL, near_band
    cases = [(synth.bumpy_cap(), 3), (synth.coons_surface(11, 300, 40), 4), (synth.random_open_mesh(3, n=5), 5)]
    for M, seed in cases:
        d = synth.random_direction(seed)
        dm = DevMesh(M, d)
        V = M.V.astype(np.float64)
        loops = [dm.bnd_idx[dm.loop_off[k]:dm.loop_off[k + 1]] for k in range(len(dm.loop_off) - 1)]
        L = loops[0]
        g = synth.rng(30 + seed)
        pts = []
        for dl in (1e-6, 1e-5, 3e-5, 1e-4, 3e-4, 1e-3, 1e-2):
            for _ in range(32):
                i = int(g.integers(len(L)))
                a, b = V[L[i]], V[L[(i + 1) % len(L)]]
                e = (b - a) / np.linalg.norm(b - a)
                u = g.normal(size=3)
                u -= (u @ e) * e
                pts.append(a + g.uniform(0.1, 0.9) * (b - a) + dl * u / np.linalg.norm(u))
        P = np.asarray(pts, np.float32)
        w, chi = dm.eval(P)
        r = oracle_pool.wn3d(M.V, M.F, P, d, loops=loops)
        deg = r.degenerate
        assert np.array_equal(chi[~deg], r["chi"][~deg])
        wref, valid = r["w"].copy(), ~deg
        if deg.any():
            r2 = oracle_pool.wn3d(M.V, M.F, P[deg], synth.random_direction(12345), loops=loops)
            wref[deg] = r2["w"]
            valid[np.nonzero(deg)[0][~r2.degenerate]] = True
        err = np.abs(w - wref)
        band = near_band(M.V, loops)
        delta = r["m_bnd"]
        out, near = valid & (delta >= band), valid & (delta < band)
        print(f"near boundary (L = {band / NEAR_REL:.3g}): {int(out.sum())} queries beyond the band, max err "
              f"{err[out].max():.2e}; {int(near.sum())} inside, max err x delta / L "
              f"{(err[near] * delta[near]).max() / (band / NEAR_REL):.2e}", flush=True)
        assert out.sum() > 100 and near.sum() > 30
        assert err[out].max() <= W_TOL
        assert np.all(err[near] <= 2.0 ** -24 * (band / NEAR_REL) / delta[near])


def test_w_continuous_across_boundary_crossing():
    M = synth.bumpy_cap()
    d = synth.random_direction(17)
    dm = DevMesh(M, d)
    V = M.V.astype(np.float64)
    L = dm.bnd_idx
    pts = []
    for i in range(len(L)):
        a, b = V[L[i]], V[L[(i + 1) % len(L)]]
        mid = 0.5 * (a + b)
        side = np.cross(d, b - a)
        side /= np.linalg.norm(side)
        base = mid - 0.7 * d
        for s in (1e-5, -1e-5):
            pts.append(base + s * side)
    P = np.array(pts, np.float32)
    w, chi = dm.eval(P)
    w, chi = w.reshape(-1, 2), chi.reshape(-1, 2)
    assert np.all(np.abs(chi[:, 0] - chi[:, 1]) == 1)
    assert np.abs(w[:, 0] - w[:, 1]).max() < 1e-3


def test_entry_points_agree_and_are_deterministic():
    """wn_eval_3d (one fused kernel) gives the bits of crossings + boundary
    term, also with non-finite and far-outside queries mixed in."""
    M = synth.coons_surface(5, 5000, 256)
    dm = DevMesh(M, synth.random_direction(8))
    P = _rand_queries(M, 50000, 9)
    g = synth.rng(10)
    P[g.choice(len(P), 40, replace=False)] = np.nan
    P[g.choice(len(P), 40, replace=False)] = g.uniform(-1e4, 1e4, (40, 3)).astype(np.float32)
    qx, qy, qz = dm.queries(P)
    w1, chi1 = W.eval_3d(dm.bvh, dm.bnd, dm.loop_off, qx, qy, qz)
    w2, _ = W.eval_3d(dm.bvh, dm.bnd, dm.loop_off, qx, qy, qz, want_chi=False)
    chi3 = W.crossings_3d(dm.bvh, qx, qy, qz)
    w4 = W.eval_3d_boundary(dm.bvh, dm.bnd, dm.loop_off, qx, qy, qz, chi3)
    w5, chi5 = W.eval_3d(dm.bvh, dm.bnd, dm.loop_off, qx, qy, qz)
    torch.cuda.synchronize()
    same = lambda a, b: torch.equal(torch.nan_to_num(a, nan=7.0), torch.nan_to_num(b, nan=7.0))
    assert same(w1, w2) and torch.equal(chi1, chi3) and same(w1, w4)
    assert same(w1, w5) and torch.equal(chi1, chi5)
    assert int(torch.isnan(w1).sum()) == 40


def test_edge_cases():
    M = synth.bumpy_cap()
    dm = DevMesh(M, synth.random_direction(4))
    # empty query set
    e = torch.empty(0, dtype=torch.float32, device="cuda")
    w, chi = W.eval_3d(dm.bvh, dm.bnd, dm.loop_off, e, e, e)
    assert w.numel() == 0
    # non-finite queries
    P = np.array([[np.nan, 0, 0], [0, np.inf, 0], [0.1, 0.2, 0.3]], np.float32)
    w, chi = dm.eval(P)
    assert np.isnan(w[0]) and np.isnan(w[1]) and np.isfinite(w[2])
    assert chi[0] == W.WN_CHI_INVALID and chi[1] == W.WN_CHI_INVALID
    # far away: w -> 0
    w, chi = dm.eval(np.array([[300.0, -200.0, 500.0]], np.float32))
    assert abs(w[0]) < 1e-4
    # one triangle
    T = synth.Mesh(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32), np.array([[0, 1, 2]], np.int32))
    dmt = DevMesh(T, synth.random_direction(6))
    P = synth.rng(1).uniform(-1, 2, (500, 3)).astype(np.float32)
    w, chi = dmt.eval(P)
    compare_3d(dmt, P, w, chi)


def test_far_queries():
    """Queries 2^10 to 2^100 scene sizes away.  Half sit far below the open
    cap on vertical rays through its hole (d = +z): each such ray crosses the
    surface once, so the boundary term has to cancel chi exactly; the others
    lie in random directions.  They are interleaved with near queries so that
    wavefronts mix both kinds (the far path rescales after every edge, and
    beyond 2^56 frame units w is returned as 0).  Far away |w| <= area / (4
    pi dist^2) (Sec. 3: w is the solid angle over 4 pi); near, the oracle
    decides.  The fused, split and batched entry points agree bit for bit."""
    M = synth.bumpy_cap()
    d = np.array([0.0, 0.0, 1.0])
    dm = DevMesh(M, d)
    g = synth.rng(24)
    n = 384
    xy = g.uniform(-0.4, 0.4, (n, 2))
    below = np.stack([xy[:, 0], xy[:, 1], -np.exp2(g.uniform(10.0, 100.0, n))], 1)
    u = g.normal(size=(n, 3))
    rand = u / np.linalg.norm(u, axis=1, keepdims=True) * np.exp2(g.uniform(10.0, 100.0, n))[:, None]
    Pfar = np.concatenate([below, rand]).astype(np.float32)
    P = np.empty((2 * len(Pfar), 3), np.float32)
    P[0::2] = Pfar
    P[1::2] = _rand_queries(M, len(Pfar), 25)
    qx, qy, qz = dm.queries(P)
    w, chi = W.eval_3d(dm.bvh, dm.bnd, dm.loop_off, qx, qy, qz)
    chi3 = W.crossings_3d(dm.bvh, qx, qy, qz)
    w4 = W.eval_3d_boundary(dm.bvh, dm.bnd, dm.loop_off, qx, qy, qz, chi3)
    B = W.Batch([{"V": dm.V, "F": dm.F, "bnd": dm.bnd, "loop_off": dm.loop_off, "nq": len(P)}], d)
    wb, cb = B.eval(qx, qy, qz)
    torch.cuda.synchronize()
    w, chi = w.cpu().numpy(), chi.cpu().numpy()
    assert np.array_equal(w4.cpu().numpy(), w) and np.array_equal(chi3.cpu().numpy(), chi)
    assert np.array_equal(wb.cpu().numpy(), w) and np.array_equal(cb.cpu().numpy(), chi)
    far = np.arange(0, len(P), 2)
    V = M.V.astype(np.float64)
    area = 0.5 * np.linalg.norm(np.cross(V[M.F[:, 1]] - V[M.F[:, 0]], V[M.F[:, 2]] - V[M.F[:, 0]]), axis=1).sum()
    dist = np.linalg.norm(P[far].astype(np.float64), axis=1) - np.linalg.norm(V, axis=1).max()
    assert np.all(np.abs(w[far]) <= area / (4.0 * math.pi * dist * dist) + 2e-7), np.abs(w[far]).max()
    assert np.all(np.abs(chi[far][:n]) == 1)          # the vertical rays cross the cap once
    compare_3d(dm, P, w, chi, sample=np.arange(1, len(P), 2), label="near, mixed with far")


def test_invalid_arguments_raise():
    M = synth.bumpy_cap()
    dm = DevMesh(M, synth.random_direction(4))
    q = torch.zeros(4, dtype=torch.float32, device="cuda")
    with pytest.raises(W.WnError):
        W.eval_3d(dm.bvh, dm.bnd[:2].contiguous(), np.array([0, 2]), q, q, q)   # a 2-vertex loop
    with pytest.raises(TypeError):
        W.eval_3d(dm.bvh, dm.bnd, dm.loop_off, q.double(), q, q)


def test_quantised_tree_on_clustered_and_elongated_meshes():
    """The four-wide tree stores child boxes as 8-bit cells of each node's
    grid, assigned with the monotone cell function the traversal applies to
    the query.  Meshes that stress that grid: a disk of radius
    1e-3 beside a unit disk 50 units away (nodes near the root span both,
    so the small disk sits in a handful of cells), and a 100 x 0.002 strip
    of 400 triangles (boxes of aspect 1e4 to 1e5).  chi must stay
    bit-exact against the oracle near the small and thin parts, and the
    fused, split and batched entry points must agree bit for bit."""
    small = synth.disk_fan(64, radius=1e-3, z=0.0)
    big = synth.disk_fan(64, radius=1.0, z=0.5)
    Vb = big.V.copy()
    Vb[:, :2] += 50.0
    M1 = synth.Mesh(np.concatenate([small.V, Vb]).astype(np.float32),
                    np.concatenate([small.F, big.F + len(small.V)]).astype(np.int32))
    n = 200
    xs = np.linspace(-50.0, 50.0, n + 1)
    top = np.stack([xs, np.full(n + 1, 0.001), 0.01 * np.sin(xs)], 1)
    bot = np.stack([xs, np.full(n + 1, -0.001), 0.01 * np.sin(xs)], 1)
    V2 = np.concatenate([top, bot]).astype(np.float32)
    k = np.arange(n)
    F2 = np.concatenate([np.stack([k, n + 1 + k, k + 1], 1), np.stack([k + 1, n + 1 + k, n + 2 + k], 1)])
    M2 = synth.Mesh(V2, F2.astype(np.int32))
    g = synth.rng(31)
    cases = [
        (M1, g.uniform([-1.5e-3, -1.5e-3, -1e-3], [1.5e-3, 1.5e-3, 1e-3], (400, 3)), 7),
        (M2, np.stack([g.uniform(-49.0, 49.0, 400), g.uniform(-0.003, 0.003, 400),
                       g.uniform(-0.05, 0.05, 400)], 1), 8),
    ]
    for M, P, seed in cases:
        d = synth.random_direction(seed)
        dm = DevMesh(M, d)
        P = P.astype(np.float32)
        qx, qy, qz = dm.queries(P)
        w, chi = W.eval_3d(dm.bvh, dm.bnd, dm.loop_off, qx, qy, qz)
        chi3 = W.crossings_3d(dm.bvh, qx, qy, qz)
        B = W.Batch([{"V": dm.V, "F": dm.F, "bnd": dm.bnd, "loop_off": dm.loop_off, "nq": len(P)}], d)
        wb, cb = B.eval(qx, qy, qz)
        torch.cuda.synchronize()
        w, chi = w.cpu().numpy(), chi.cpu().numpy()
        assert np.array_equal(chi3.cpu().numpy(), chi)
        assert np.array_equal(wb.cpu().numpy(), w) and np.array_equal(cb.cpu().numpy(), chi)
        assert np.any(chi != 0)
        compare_3d(dm, P, w, chi, max_degenerate_frac=0.05, label=f"quantised tree {seed}")


def test_more_boundary_loops_than_the_kernel_argument_table():
    """300 small disks scattered in the unit box: 300 boundary loops, more than
    the WN_MAX_LOOPS that travel in the kernel arguments, so the plain calls
    read the loop table from device memory.  The fused, split and batched
    forward and the grid mode agree bit for bit, and with the oracle on a
    sample; plain and batched backward agree to rounding; the no-allocation
    backward refuses the table."""
    g = synth.rng(33)
    nd = 300
    Vs, Fs, o = [], [], 0
    for k in range(nd):
        D = synth.disk_fan(6, radius=0.04, z=0.0)
        V = D.V.astype(np.float64)
        c, s = np.cos(g.uniform(0, np.pi)), np.sin(g.uniform(0, np.pi))
        V = V @ np.array([[1, 0, 0], [0, c, -s], [0, s, c]]).T + g.uniform(-1, 1, 3)
        Vs.append(V)
        Fs.append(D.F + o)
        o += len(V)
    M = synth.Mesh(np.concatenate(Vs).astype(np.float32), np.concatenate(Fs).astype(np.int32))
    for d in (synth.random_direction(34), np.array([0.0, 0.0, 1.0])):
        dm = DevMesh(M, d)
        assert len(dm.loop_off) - 1 == nd > W.WN_MAX_LOOPS
        P = g.uniform(-1.1, 1.1, (2048, 3)).astype(np.float32)
        qx, qy, qz = dm.queries(P)
        w, chi = W.eval_3d(dm.bvh, dm.bnd, dm.loop_off, qx, qy, qz)
        chi3 = W.crossings_3d(dm.bvh, qx, qy, qz)
        w3 = W.eval_3d_boundary(dm.bvh, dm.bnd, dm.loop_off, qx, qy, qz, chi3)
        B = W.Batch([{"V": dm.V, "F": dm.F, "bnd": dm.bnd, "loop_off": dm.loop_off, "nq": len(P)}], d)
        wb, cb = B.eval(qx, qy, qz)
        torch.cuda.synchronize()
        w, chi = w.cpu().numpy(), chi.cpu().numpy()
        assert np.array_equal(w3.cpu().numpy(), w) and np.array_equal(chi3.cpu().numpy(), chi)
        assert np.array_equal(wb.cpu().numpy(), w) and np.array_equal(cb.cpu().numpy(), chi)
        assert np.any(chi != 0)
        compare_3d(dm, P, w, chi, sample=synth.rng(35).choice(len(P), 200, replace=False),
                   label="300 loops")
        gw = torch.from_numpy(g.uniform(-1, 1, len(P)).astype(np.float32)).cuda()
        gq, gbnd = W.backward(dm.bnd, dm.loop_off, qx, qy, qz, gw)
        gq2, gbnd2 = B.backward(qx, qy, qz, gw)
        torch.cuda.synchronize()
        # few queries over 1800 boundary vertices: the plain call splits the
        # boundary into ranges, the batch does not, so the sums differ in order
        for a, b in ((gq, gq2), (gbnd, gbnd2)):
            assert float((a - b).abs().max()) <= 1e-5 * float(b.abs().max())
        assert float(gbnd.abs().sum()) > 0
        with pytest.raises(W.WnError) as ei:
            W.backward(dm.bnd, dm.loop_off, qx, qy, qz, gw, noalloc=True)
        assert "at most" in str(ei.value)
        if d[2] == 1.0:
            ax = [synth.grid_axis(-1.0, 1.0, n, np.float32) for n in (10, 12, 16)]
            wg, cg = W.eval_3d_grid(dm.bvh, dm.bnd, dm.loop_off, *[torch.from_numpy(a).cuda() for a in ax])
            X, Y, Z = np.meshgrid(*ax, indexing="ij")
            Pg = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1).astype(np.float32)
            wp, cp = dm.eval(Pg)
            assert np.array_equal(wg.cpu().numpy().ravel(), wp) and np.array_equal(cg.cpu().numpy().ravel(), cp)


@pytest.mark.parametrize("n_tri", [2, 3, 4, 5, 9])
def test_trees_of_a_few_triangles(n_tri):
    """Fans of 2-9 triangles: the four-wide root then holds two to four
    slots, leaves and nodes mixed; chi and w against the oracle."""
    if n_tri == 2:   # a fan of two is flat: take a quad
        D = synth.Mesh(np.array([[-1, -1, 0], [1, -1, 0], [1, 1, 0], [-1, 1, 0]], np.float32),
                       np.array([[0, 1, 2], [0, 2, 3]], np.int32))
    else:
        D = synth.disk_fan(n_tri, radius=1.0, z=0.0)
    V = D.V.astype(np.float64)
    V[:, 2] += 0.3 * np.sin(3.0 * V[:, 0]) * np.cos(2.0 * V[:, 1])   # not flat
    M = synth.Mesh(V.astype(np.float32), D.F)
    dm = DevMesh(M, synth.random_direction(40 + n_tri))
    P = synth.rng(41 + n_tri).uniform(-1.2, 1.2, (600, 3)).astype(np.float32)
    w, chi = dm.eval(P)
    assert np.any(chi != 0)
    compare_3d(dm, P, w, chi, max_degenerate_frac=0.05, label=f"{n_tri} triangles")
