"""CPU checks of the C ABI: the library builds and loads without a GPU,
exports every function that include/wn.h declares, and its host-side parts
(boundary extraction, argument validation) behave as documented.  No kernel
is launched here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from oracle import wn3d as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def W():
    from paper_2408_04466_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2408_04466_amd import build
        build.build()
    import paper_2408_04466_amd as W
    W.lib()
    return W


def header_functions():
    src = open(os.path.join(ROOT, "include", "wn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wn_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_function(W):
    names = header_functions()
    assert len(names) >= 10
    lib = C.CDLL(W._lib.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    # the binding declares a signature for every exported entry point
    assert set(names) <= set(W._lib.exported_symbols())


def test_version_and_status_strings(W):
    L = W.lib()
    assert L.wn_version() >= 10000
    assert L.wn_status_string(0) == b"WN_OK"
    assert L.wn_status_string(3) == b"WN_ERR_OUT_OF_MEMORY"
    assert L.wn_status_string(99) == b"WN_ERR_UNKNOWN"


@pytest.mark.parametrize("mesh", ["bumpy_cap", "sphere_refined", "coons", "icosphere", "two_patches"])
def test_boundary_loops_match_oracle(W, mesh):
    if mesh == "bumpy_cap":
        M = synth.bumpy_cap()
    elif mesh == "sphere_refined":
        M = synth.open_sphere(5, n_lon=24, n_rings=8, top_refine=4)
    elif mesh == "coons":
        M = synth.coons_surface(3, 600, 64)
    elif mesh == "icosphere":
        M = synth.icosphere(1)
    else:
        A, B = synth.coons_surface(1, 300, 40), synth.coons_surface(2, 300, 48)
        M = synth.Mesh(np.concatenate([A.V, B.V]), np.concatenate([A.F, B.F + len(A.V)]))
    idx, off = W.boundary_loops(M.F)
    mine = [idx[off[i]:off[i + 1]].tolist() for i in range(len(off) - 1)]
    assert mine == [L.tolist() for L in O.boundary_loops(M.F)]


def test_boundary_loops_rejects_bad_input(W):
    with pytest.raises(W.WnError):
        W.boundary_loops(np.array([[0, 1, -1]], np.int32))      # index out of range
    # a vertex with two outgoing boundary edges (two triangles touching at a vertex)
    bow = np.array([[0, 1, 2], [0, 3, 4]], np.int32)
    with pytest.raises(W.WnError):
        W.boundary_loops(bow)


def _err(W):
    return W.lib().wn_last_error().decode()


def test_validation_happens_on_the_host(W):
    L = W.lib()
    P = C.c_void_p
    fake = P(16)   # never dereferenced: validation fails first
    # NULL handle
    assert L.wn_eval_3d(None, fake, None, 0, fake, fake, fake, 4, fake, None, None) == 1
    assert "bvh" in _err(W)
    # more loops than the no-allocation adjoint takes (wn_backward copies such
    # a table to device memory instead)
    off = np.arange(0, 3 * 300, 3, dtype=np.int64)
    assert L.wn_backward_noalloc(fake, off.ctypes.data_as(C.POINTER(C.c_int64)), 299, fake, fake, fake, 4,
                                 fake, fake, fake, None) == 2
    assert "at most" in _err(W)
    # a two-vertex loop
    off = np.array([0, 2], np.int64)
    assert L.wn_backward(fake, off.ctypes.data_as(C.POINTER(C.c_int64)), 1, fake, fake, fake, 4,
                         fake, fake, fake, None) == 1
    # negative query count
    assert L.wn_backward(None, None, 0, fake, fake, fake, -1, fake, None, None, None) == 1
    # bad direction
    h = P()
    d = (C.c_double * 3)(0.0, 0.0, 0.0)
    assert L.wn_build_bvh(fake, 3, fake, 1, d, None, C.byref(h)) == 1
    # 2D: unsupported dtype, loops that do not cover the segments
    assert L.wn_eval_2d(7, fake, 1, None, None, 0, 0, fake, fake, 1, 1, fake, None, None) == 2
    off = np.array([0, 2], np.int64)
    cl = np.array([1], np.uint8)
    assert L.wn_eval_2d(0, fake, 3, off.ctypes.data_as(C.POINTER(C.c_int64)), cl.ctypes.data_as(P), 1, 0,
                        fake, fake, 1, 1, fake, None, None) == 1
    assert "nseg" in _err(W)
    # 2D batched: the failing set is named; an all-empty batch does nothing
    from paper_2408_04466_amd._lib import CurveSet2D
    sets = (CurveSet2D * 3)()
    offs = [np.array([0, 1], np.int64), np.array([0, 2], np.int64), np.array([0, 1], np.int64)]
    cls = np.array([0], np.uint8)
    for k, o in enumerate(offs):
        sets[k].nseg, sets[k].nloops, sets[k].nx, sets[k].ny = 1, 1, 4, 4
        sets[k].loop_off = o.ctypes.data_as(C.POINTER(C.c_int64))
        sets[k].loop_closed = cls.ctypes.data_as(P)
    h = P()
    assert L.wn_batch2d_create(1, sets, 3, None, C.byref(h)) == 1 and not h.value
    assert "set 1" in _err(W) and "nseg" in _err(W)
    sets[1].nseg = 2
    sets[2].ny = -1
    assert L.wn_batch2d_create(1, sets, 3, None, C.byref(h)) == 1
    assert "set 2" in _err(W)
    sets[2].ny = 1 << 40
    assert L.wn_batch2d_create(1, sets, 3, None, C.byref(h)) == 2
    sets[2].ny = 1 << 30                     # 2^30 wavefront tiles: more than one launch holds
    assert L.wn_batch2d_create(1, sets, 3, None, C.byref(h)) == 2
    assert "too large" in _err(W)
    assert L.wn_batch2d_create(5, sets, 3, None, C.byref(h)) == 2
    assert L.wn_eval_2d_batched(None, fake, fake, fake, fake, None, None) == 1
    assert "batch" in _err(W)
    assert L.wn_batch2d_free(None) == 0
    # parametric path: bad direction, NULL nets, nothing requested
    d0 = (C.c_double * 3)(0.0, 0.0, 0.0)
    d1 = (C.c_double * 3)(0.0, 0.0, 1.0)
    assert L.wn_eval_3d_patches(d0, fake, 1, None, 0, fake, fake, fake, 4, fake, None, None) == 1
    assert L.wn_eval_3d_patches(d1, None, 1, None, 0, fake, fake, fake, 4, fake, None, None) == 1
    assert "nets" in _err(W)
    assert L.wn_eval_3d_patches(d1, fake, 1, None, 0, fake, fake, fake, 4, None, None, None) == 1
    assert L.wn_eval_3d_patches(d1, fake, 1, None, 0, fake, fake, fake, 0, None, None, None) == 0
    assert L.wn_eval_3d_curves(None, fake, 1, fake, fake, fake, 4, None, fake, None, None) == 1
    # batched parametric surfaces: the failing surface is named; NULL batch;
    # nothing requested
    from paper_2408_04466_amd._lib import PatchSurface
    ps = (PatchSurface * 2)()
    ps[0].npatch, ps[0].ncurves, ps[0].nq = 1, 4, 10
    ps[0].dir[2] = 1.0
    ps[1].npatch, ps[1].ncurves, ps[1].nq = 1, -4, 10
    ps[1].dir[2] = 1.0
    h = P()
    assert L.wn_patch_batch_create(ps, 2, None, C.byref(h)) == 1 and not h.value
    assert "surface 1" in _err(W)
    ps[1].ncurves = 4
    ps[1].dir[2] = 0.0
    assert L.wn_patch_batch_create(ps, 2, None, C.byref(h)) == 1
    assert "surface 1" in _err(W) and "dir" in _err(W)
    ps[1].dir[2] = 1.0
    ps[1].npatch = 1 << 30
    assert L.wn_patch_batch_create(ps, 2, None, C.byref(h)) == 2
    ps[1].npatch = 1
    ps[1].nq = 1 << 40
    assert L.wn_patch_batch_create(ps, 2, None, C.byref(h)) == 2
    assert L.wn_patch_batch_create(ps, -1, None, C.byref(h)) == 1
    assert L.wn_patch_batch_create(None, 1, None, C.byref(h)) == 1
    assert L.wn_patch_batch_create(ps, 0, None, None) == 1
    assert L.wn_eval_3d_patches_batched(None, fake, fake, fake, fake, fake, fake, None, None) == 1
    assert "batch" in _err(W)
    assert L.wn_patch_batch_free(None) == 0
    # diagnostics: NULL counts, NULL chi with queries, negative count
    assert L.wn_diagnose(fake, fake, fake, fake, 4, None, None) == 1
    assert "counts_out" in _err(W)
    assert L.wn_diagnose(fake, fake, fake, None, 4, fake, None) == 1
    assert L.wn_diagnose(fake, fake, fake, fake, -1, fake, None) == 1
    assert L.wn_device_info(None, None) == 1
    # spatial order: NULL output, too many queries, negative and empty counts
    assert L.wn_spatial_order(fake, fake, fake, 4, None, None) == 1
    assert "order_out" in _err(W)
    assert L.wn_spatial_order(fake, fake, fake, 1 << 31, fake, None) == 2
    assert L.wn_spatial_order(fake, fake, fake, -1, fake, None) == 1
    assert L.wn_spatial_order(None, None, None, 0, None, None) == 0


def test_missing_library_fails_loudly(tmp_path):
    import subprocess
    import sys
    code = ("import os; os.environ['WN_LIBRARY']='/nonexistent/libwn.so'\n"
            "import paper_2408_04466_amd as W\n"
            "try:\n    W.lib()\nexcept RuntimeError as e:\n    print('raised', 'no fallback' in str(e))\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert "raised True" in r.stdout, r.stdout + r.stderr


def test_bench_measures_one_gpu_only():
    """bench.py --gpus N with N > 1 exits with status 2 and a message, before
    any device work (the library has no multi-GPU path)."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr and r.stdout == ""
