"""GPU tests of the 3D grid mode (queries on lines along the ray share the
ray, Sec. 5 "Optimization"): bit-identical to the per-query path on the
same float32 points, oracle parity on samples, deep stacks of surfaces,
edge cases, and the full-size voxel grid over the 1M-triangle mesh."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2408_04466_amd as W
    from gpu_util import DevMesh, compare_3d

DZ = np.array([0.0, 0.0, 1.0])


def _axes(M, n, scale=1.2, seed=0, shift=0.0):
    lo, hi = M.V.min(0).astype(np.float64), M.V.max(0).astype(np.float64)
    c, h = (lo + hi) / 2, (hi - lo) / 2 * scale
    c = c + shift * h   # off the mesh's centre lines (odd point counts)
    return [synth.grid_axis(c[k] - h[k], c[k] + h[k], n[k], np.float32) for k in range(3)]


def _points(ax):
    X, Y, Z = np.meshgrid(ax[0], ax[1], ax[2], indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1).astype(np.float32)


def _grid(dm, ax, want_chi=True):
    g = [torch.from_numpy(a).cuda() for a in ax]
    w, chi = W.eval_3d_grid(dm.bvh, dm.bnd, dm.loop_off, *g, want_chi=want_chi)
    torch.cuda.synchronize()
    return w, chi


def _stack_of_disks(n_layers, n_tri=48):
    Vs, Fs, o = [], [], 0
    for k in range(n_layers):
        D = synth.disk_fan(n_tri, radius=1.0, z=-1.0 + 2.0 * k / max(n_layers - 1, 1))
        Vs.append(D.V)
        Fs.append(D.F + o)
        o += len(D.V)
    return synth.Mesh(np.concatenate(Vs).astype(np.float32), np.concatenate(Fs).astype(np.int32))


# nz = 16: wavefronts span several columns (the per-lane walk); nz = 128 and
# 256: two and four wavefronts share a column's walk (5 x 3 x 128: the last
# workgroup holds half a column)
@pytest.mark.parametrize("shape", [(24, 20, 16), (6, 5, 128), (5, 3, 128), (4, 3, 256)])
@pytest.mark.parametrize("name", ["bumpy_cap", "coons", "sphere"])
def test_grid_equals_per_query_path_and_oracle(name, shape):
    M = {"bumpy_cap": synth.bumpy_cap(), "coons": synth.coons_surface(3, 3000, 96),
         "sphere": synth.icosphere(3, radius=0.8)}[name]
    dm = DevMesh(M, DZ)
    ax = _axes(M, shape, shift=0.0123 if shape[0] % 2 else 0.0)
    w, chi = _grid(dm, ax)
    assert tuple(w.shape) == shape
    P = _points(ax)
    wp, cp = dm.eval(P)
    assert np.array_equal(chi.cpu().numpy().ravel(), cp)
    assert np.array_equal(w.cpu().numpy().ravel(), wp)
    sample = synth.rng(3).choice(len(P), 150, replace=False)
    compare_3d(dm, P, wp, cp, sample)


@pytest.mark.parametrize("shape", [(10, 12, 30), (6, 4, 64)])
@pytest.mark.parametrize("layers", [12, 40])
def test_deep_stack_of_surfaces(layers, shape):
    # stacked disks: columns through the stack cross every layer (12: kept in
    # the column lists; 40: more than a list holds, those columns' points
    # traverse the tree themselves).  Their 576 or 1920 boundary vertices in
    # 12 or 40 loops take two or four staged chunks, with loops running
    # across chunk ends (nz = 64: the column's shared walk carries the last
    # vertex of a chunk into the next).  Even x and y counts keep the columns
    # off the disks' projected edges through the centre.
    M = _stack_of_disks(layers)
    dm = DevMesh(M, DZ)
    ax = _axes(M, shape)
    w, chi = _grid(dm, ax)
    P = _points(ax)
    wp, cp = dm.eval(P)
    assert np.array_equal(chi.cpu().numpy().ravel(), cp)
    assert np.array_equal(w.cpu().numpy().ravel(), wp)
    assert np.abs(cp).max() >= layers // 2   # columns inside the stack cross many disks
    compare_3d(dm, P, wp, cp, synth.rng(4).choice(len(P), 60, replace=False))


def test_grid_edge_cases():
    M = synth.bumpy_cap()
    dm = DevMesh(M, DZ)
    ax = _axes(M, (5, 4, 3))
    # empty axes
    e = torch.empty(0, dtype=torch.float32, device="cuda")
    g = [torch.from_numpy(a).cuda() for a in ax]
    w, chi = W.eval_3d_grid(dm.bvh, dm.bnd, dm.loop_off, g[0], e, g[2])
    assert tuple(w.shape) == (5, 0, 3)
    # a non-finite axis value makes exactly its points invalid (nz = 64, 128: a
    # non-finite x or y takes the wavefront, or the workgroup, off the shared
    # walk)
    for nzk in (3, 64, 128):
        ax2 = _axes(M, (5, 4, nzk))
        ax2[1][2] = np.nan
        ax2[2][0] = np.inf
        w, chi = _grid(dm, ax2)
        w, chi = w.cpu().numpy(), chi.cpu().numpy()
        bad = np.zeros((5, 4, nzk), bool)
        bad[:, 2, :] = True
        bad[:, :, 0] = True
        assert np.all(np.isnan(w[bad])) and np.all(chi[bad] == W.WN_CHI_INVALID)
        assert np.all(np.isfinite(w[~bad]))
        if nzk >= 64:
            P = _points(ax2)
            ok = ~bad.ravel()
            wp, cp = dm.eval(P[ok])
            assert np.array_equal(w.ravel()[ok], wp) and np.array_equal(chi.ravel()[ok], cp)
    # a BVH for another direction is refused
    dm2 = DevMesh(M, synth.random_direction(2))
    with pytest.raises(W.WnError) as ei:
        W.eval_3d_grid(dm2.bvh, dm2.bnd, dm2.loop_off, *g)
    assert "+z" in str(ei.value)
    # a closed surface without boundary
    S = synth.icosphere(2, radius=0.5)
    ds = DevMesh(S, DZ)
    ax3 = _axes(S, (6, 6, 6))
    w, chi = _grid(ds, ax3)
    assert set(np.unique(w.cpu().numpy())) <= {0.0, 1.0}


def test_voxel_grid_over_full_size_mesh():
    """The 1M-triangle mesh on a 128^3 grid over 1.2x its bounding box with
    d = +z: oracle samples, and bit-identical to the per-query path on a
    slab of columns."""
    M = synth.open_sphere(3)
    dm = DevMesh(M, DZ)
    ax = _axes(M, (128, 128, 128))
    w, chi = _grid(dm, ax)
    w, chi = w.cpu().numpy(), chi.cpu().numpy()
    P = _points(ax)
    sample = synth.rng(8).choice(len(P), 30, replace=False)
    compare_3d(dm, P, w.ravel(), chi.ravel(), sample)
    slab = slice(60 * 128 * 128, 61 * 128 * 128)        # all points with x index 60
    wp, cp = dm.eval(P[slab])
    assert np.array_equal(chi.ravel()[slab], cp) and np.array_equal(w.ravel()[slab], wp)
