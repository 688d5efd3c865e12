"""Python entry points: marshal torch tensors and the current stream into the
C ABI of ``libwn.so``.  No arithmetic of the method happens here."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from ._lib import CurveSet2D, PatchSurface, check, lib, WN_MAX_LOOPS

__all__ = ["boundary_loops", "BVH", "eval_3d", "eval_3d_boundary", "eval_3d_grid", "eval_3d_curves", "eval_3d_patches", "backward_curves", "spatial_order", "PatchBatch", "diagnose", "device_info",
           "WindingNumberCurves", "winding_number_curves", "crossings_3d",
           "backward", "WindingNumber3D", "winding_number", "eval_2d", "eval_2d_batched", "Batch2D", "backward_2d",
           "WindingNumber2D", "winding_number_2d", "Batch"]


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev(t: torch.Tensor, dtype, name: str, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr()) if t.numel() else C.c_void_p(0)


def _loops(loop_off, limit: bool = False) -> tuple[np.ndarray, int]:
    """Host loop offsets as int64 and the loop count (``limit``: the 2D
    adjoint, whose loop table travels in the kernel arguments only)."""
    lo = np.ascontiguousarray(np.asarray(loop_off, dtype=np.int64))
    n = max(lo.size - 1, 0)
    if limit and n > WN_MAX_LOOPS:
        raise ValueError(f"at most {WN_MAX_LOOPS} loops per call")
    return lo, n


def _ptr64(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int64)) if a.size else None


def boundary_loops(F) -> tuple[np.ndarray, np.ndarray]:
    """Boundary loops of an oriented triangle mesh (host).  Returns
    (bnd_idx int32 [nb], loop_off int64 [nloops + 1])."""
    if isinstance(F, torch.Tensor):
        F = F.detach().cpu().numpy()
    F = np.ascontiguousarray(np.asarray(F, dtype=np.int32))
    nf = F.shape[0]
    nv = int(F.max()) + 1 if nf else 0
    cap = 3 * nf
    idx = np.zeros(max(cap, 1), np.int32)
    off = np.zeros(max(cap, 1) + 1, np.int64)
    nb = C.c_int64(0)
    nl = C.c_int32(0)
    st = lib().wn_boundary_loops(F.ctypes.data_as(C.c_void_p) if nf else None, nf, nv,
                                 idx.ctypes.data_as(C.c_void_p), off.ctypes.data_as(C.c_void_p),
                                 cap, C.byref(nb), C.byref(nl))
    check(st, "wn_boundary_loops")
    return idx[: nb.value].copy(), off[: nl.value + 1].copy()


class BVH:
    """Handle of ``wn_build_bvh``: frame of the ray direction and the BVH of
    the mesh projections.  ``V`` float32 [nv, 3], ``F`` int32 [nf, 3] on the
    GPU.  The build synchronises the current stream once."""

    def __init__(self, V: torch.Tensor, F: torch.Tensor, direction, stream=None):
        nv, nf = V.shape[0], F.shape[0]
        pv = _dev(V, torch.float32, "V", (nv, 3))
        pf = _dev(F, torch.int32, "F", (nf, 3))
        d = (C.c_double * 3)(*[float(x) for x in np.asarray(direction, np.float64).ravel()[:3]])
        h = C.c_void_p()
        check(lib().wn_build_bvh(pv, nv, pf, nf, d, _stream(stream), C.byref(h)), "wn_build_bvh")
        self._h = h
        self.nv, self.nf = nv, nf

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("BVH already freed")
        return self._h

    @property
    def direction(self) -> np.ndarray:
        d = (C.c_double * 3)()
        check(lib().wn_bvh_direction(self.handle, d), "wn_bvh_direction")
        return np.array(d[:])

    def free(self):
        if getattr(self, "_h", None) is not None:
            torch.cuda.synchronize()
            lib().wn_free_bvh(self._h)
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None) is not None:
                lib().wn_free_bvh(self._h)
                self._h = None
        except Exception:
            pass


def _queries(qx, qy, qz):
    nq = qx.shape[0]
    return (_dev(qx, torch.float32, "qx", (nq,)), _dev(qy, torch.float32, "qy", (nq,)),
            _dev(qz, torch.float32, "qz", (nq,)), nq)


def eval_3d(bvh: BVH, bnd_xyz: torch.Tensor, loop_off, qx, qy, qz, want_chi: bool = True,
            w_out=None, chi_out=None, stream=None):
    """w (and chi) for queries (qx, qy, qz) against the mesh of ``bvh`` whose
    boundary is ``bnd_xyz`` [nb, 3] with host loop offsets ``loop_off``."""
    lo, nl = _loops(loop_off)
    nb = int(lo[-1]) if nl else 0
    pb = _dev(bnd_xyz, torch.float32, "bnd_xyz", (nb, 3))
    px, py, pz, nq = _queries(qx, qy, qz)
    w = torch.empty(nq, dtype=torch.float32, device=qx.device) if w_out is None else w_out
    chi = None
    if want_chi:
        chi = torch.empty(nq, dtype=torch.int32, device=qx.device) if chi_out is None else chi_out
    pw = _dev(w, torch.float32, "w_out", (nq,))
    pc = _dev(chi, torch.int32, "chi_out", (nq,)) if chi is not None else None
    check(lib().wn_eval_3d(bvh.handle, pb, _ptr64(lo), nl, px, py, pz, nq, pw, pc, _stream(stream)),
          "wn_eval_3d")
    return w, chi


def eval_3d_curves(bvh: BVH, ctrl: torch.Tensor, qx, qy, qz, chi_in=None, want_chi: bool = True, stream=None):
    """w for a surface bounded by loops of cubic Beziers ``ctrl`` [nc, 4, 3]
    (float32, boundary orientation): chi_d from ``chi_in`` (int32 [nq]) or,
    if None, from ``bvh`` (the surface's tessellation), plus the boundary
    integral along the curves in the frame of ``bvh``.  Returns (w, chi)."""
    nc = ctrl.shape[0]
    pcurve = _dev(ctrl, torch.float32, "ctrl", (nc, 4, 3))
    px, py, pz, nq = _queries(qx, qy, qz)
    pin = _dev(chi_in, torch.int32, "chi_in", (nq,)) if chi_in is not None else None
    w = torch.empty(nq, dtype=torch.float32, device=qx.device)
    chi = torch.empty(nq, dtype=torch.int32, device=qx.device) if want_chi else None
    check(lib().wn_eval_3d_curves(bvh.handle, pcurve, nc, px, py, pz, nq, pin, _dev(w, torch.float32, "w"),
                                  _dev(chi, torch.int32, "chi") if chi is not None else None, _stream(stream)),
          "wn_eval_3d_curves")
    return w, chi


def eval_3d_patches(direction, nets: torch.Tensor, curves, qx, qy, qz, want_w: bool = True,
                    want_chi: bool = True, stream=None):
    """w (and chi) of a surface of bicubic Bezier patches ``nets`` [np, 4, 4, 3]
    (float32) with boundary curves ``curves`` [nc, 4, 3] (or None), for the
    ray direction ``direction`` (3 floats): exact ray-patch crossings plus the
    boundary integral along the curves.  Returns (w or None, chi or None)."""
    npatch = nets.shape[0]
    pn = _dev(nets, torch.float32, "nets", (npatch, 4, 4, 3))
    nc = 0 if curves is None else curves.shape[0]
    pcv = _dev(curves, torch.float32, "curves", (nc, 4, 3)) if curves is not None else None
    px, py, pz, nq = _queries(qx, qy, qz)
    if not (want_w or want_chi):
        raise ValueError("nothing requested")
    w = torch.empty(nq, dtype=torch.float32, device=qx.device) if want_w else None
    chi = torch.empty(nq, dtype=torch.int32, device=qx.device) if want_chi else None
    d = (C.c_double * 3)(*[float(x) for x in direction])
    check(lib().wn_eval_3d_patches(d, pn, npatch, pcv, nc, px, py, pz, nq,
                                   _dev(w, torch.float32, "w") if w is not None else None,
                                   _dev(chi, torch.int32, "chi") if chi is not None else None, _stream(stream)),
          "wn_eval_3d_patches")
    return w, chi


def diagnose(qx, qy, qz, chi, stream=None) -> torch.Tensor:
    """int64 device tensor [2]: queries with a non-finite coordinate, and
    finite queries whose chi is WN_CHI_INVALID (``wn_diagnose``)."""
    px, py, pz, nq = _queries(qx, qy, qz)
    pc = _dev(chi, torch.int32, "chi", (nq,))
    out = torch.empty(2, dtype=torch.int64, device=qx.device)
    check(lib().wn_diagnose(px, py, pz, pc, nq, _dev(out, torch.int64, "counts"), _stream(stream)),
          "wn_diagnose")
    return out


def device_info() -> dict:
    """Compute units and peak shader clock of the current device, as the HIP
    runtime reports them."""
    cus, clk = C.c_int32(), C.c_int32()
    check(lib().wn_device_info(C.byref(cus), C.byref(clk)), "wn_device_info")
    return {"compute_units": cus.value, "clock_mhz": clk.value / 1000.0}


def spatial_order(qx, qy, qz, stream=None) -> torch.Tensor:
    """int32 permutation [nq] that sorts the queries by Morton code over their
    bounding box (``wn_spatial_order``): deterministic, non-finite queries
    last.  Evaluating the permuted queries gives the permuted results bit for
    bit, and neighbouring lanes then take similar paths."""
    px, py, pz, nq = _queries(qx, qy, qz)
    order = torch.empty(nq, dtype=torch.int32, device=qx.device)
    check(lib().wn_spatial_order(px, py, pz, nq, _dev(order, torch.int32, "order"), _stream(stream)),
          "wn_spatial_order")
    return order


def eval_3d_grid(bvh: BVH, bnd_xyz: torch.Tensor, loop_off, gx, gy, gz, want_chi: bool = True, stream=None):
    """w (and chi) on the grid gx[nx] x gy[ny] x gz[nz] (float32 device
    vectors), output shape [nx, ny, nz] (z fastest); the BVH must be built for
    the direction +z (columns along the ray share it)."""
    lo, nl = _loops(loop_off)
    nb = int(lo[-1]) if nl else 0
    pb = _dev(bnd_xyz, torch.float32, "bnd_xyz", (nb, 3))
    nx, ny, nz = gx.shape[0], gy.shape[0], gz.shape[0]
    px = _dev(gx, torch.float32, "gx", (nx,))
    py = _dev(gy, torch.float32, "gy", (ny,))
    pz = _dev(gz, torch.float32, "gz", (nz,))
    w = torch.empty((nx, ny, nz), dtype=torch.float32, device=gx.device)
    chi = torch.empty((nx, ny, nz), dtype=torch.int32, device=gx.device) if want_chi else None
    check(lib().wn_eval_3d_grid(bvh.handle, pb, _ptr64(lo), nl, px, py, pz, nx, ny, nz,
                                _dev(w, torch.float32, "w"), _dev(chi, torch.int32, "chi") if chi is not None else None,
                                _stream(stream)), "wn_eval_3d_grid")
    return w, chi


def eval_3d_boundary(bvh: BVH, bnd_xyz, loop_off, qx, qy, qz, chi_in, stream=None):
    lo, nl = _loops(loop_off)
    nb = int(lo[-1]) if nl else 0
    pb = _dev(bnd_xyz, torch.float32, "bnd_xyz", (nb, 3))
    px, py, pz, nq = _queries(qx, qy, qz)
    pc = _dev(chi_in, torch.int32, "chi_in", (nq,))
    w = torch.empty(nq, dtype=torch.float32, device=qx.device)
    check(lib().wn_eval_3d_boundary(bvh.handle, pb, _ptr64(lo), nl, px, py, pz, nq, pc,
                                    _dev(w, torch.float32, "w"), _stream(stream)),
          "wn_eval_3d_boundary")
    return w


def crossings_3d(bvh: BVH, qx, qy, qz, stream=None):
    px, py, pz, nq = _queries(qx, qy, qz)
    chi = torch.empty(nq, dtype=torch.int32, device=qx.device)
    check(lib().wn_crossings_3d(bvh.handle, px, py, pz, nq, _dev(chi, torch.int32, "chi"),
                                _stream(stream)), "wn_crossings_3d")
    return chi


def backward(bnd_xyz, loop_off, qx, qy, qz, grad_w, want_q: bool = True, want_bnd: bool = True,
             stream=None, grad_q=None, grad_bnd=None, noalloc: bool = False):
    """(dL/dq [nq, 3] or None, dL/d bnd_xyz [nb, 3] or None) for dL/dw = grad_w.

    ``grad_q`` / ``grad_bnd`` may be given as preallocated outputs.  With
    ``noalloc`` the call goes to ``wn_backward_noalloc``: the library then
    allocates nothing (its workspace is a library-held device array)."""
    lo, nl = _loops(loop_off)
    nb = int(lo[-1]) if nl else 0
    pb = _dev(bnd_xyz, torch.float32, "bnd_xyz", (nb, 3))
    px, py, pz, nq = _queries(qx, qy, qz)
    pg = _dev(grad_w, torch.float32, "grad_w", (nq,))
    dev = qx.device
    gq = grad_q if grad_q is not None else (
        torch.empty((nq, 3), dtype=torch.float32, device=dev) if want_q else None)
    gb = grad_bnd if grad_bnd is not None else (
        torch.empty((nb, 3), dtype=torch.float32, device=dev) if want_bnd else None)
    name = "wn_backward_noalloc" if noalloc else "wn_backward"
    check(getattr(lib(), name)(pb, _ptr64(lo), nl, px, py, pz, nq, pg,
                               _dev(gq, torch.float32, "grad_q", (nq, 3)) if gq is not None else None,
                               _dev(gb, torch.float32, "grad_bnd", (nb, 3)) if gb is not None else None,
                               _stream(stream)), name)
    return gq, gb


class WindingNumber3D(torch.autograd.Function):
    """w = winding number of the mesh of ``bvh`` at the queries; gradients
    flow to the boundary vertices ``bnd_xyz`` and to the query coordinates
    (chi_d is piecewise constant and contributes none)."""

    @staticmethod
    def forward(ctx, bnd_xyz, qx, qy, qz, bvh, loop_off):
        w, _ = eval_3d(bvh, bnd_xyz.detach(), loop_off, qx.detach(), qy.detach(), qz.detach(),
                       want_chi=False)
        ctx.save_for_backward(bnd_xyz, qx, qy, qz)
        ctx.loop_off = loop_off
        return w

    @staticmethod
    def backward(ctx, grad_w):
        bnd_xyz, qx, qy, qz = ctx.saved_tensors
        need_b = ctx.needs_input_grad[0]
        need_q = any(ctx.needs_input_grad[1:4])
        gq, gb = backward(bnd_xyz.detach(), ctx.loop_off, qx.detach(), qy.detach(), qz.detach(),
                          grad_w.contiguous().float(), want_q=need_q, want_bnd=need_b)
        gx = gy = gz = None
        if gq is not None:
            gx, gy, gz = gq[:, 0], gq[:, 1], gq[:, 2]
        return gb, gx, gy, gz, None, None


def winding_number(bvh, bnd_xyz, loop_off, qx, qy, qz):
    return WindingNumber3D.apply(bnd_xyz, qx, qy, qz, bvh, loop_off)


def eval_2d(ctrl: torch.Tensor, loop_off, loop_closed, x: torch.Tensor, y: torch.Tensor,
            grid: bool = False, want_chi: bool = True, stream=None):
    """w (and chi) of loops of cubic Beziers ``ctrl`` [nseg, 4, 2] (float32 or
    float64) at points (x[i], y[i]) or on the grid x[nx] by y[ny] (row-major
    [ny, nx] output).  Ray direction +x."""
    if ctrl.dtype == torch.float64:
        dt, code = torch.float64, 1
    elif ctrl.dtype == torch.float32:
        dt, code = torch.float32, 0
    else:
        raise TypeError("ctrl must be float32 or float64")
    nseg = ctrl.shape[0]
    pc = _dev(ctrl, dt, "ctrl", (nseg, 4, 2))
    lo, nl = _loops(loop_off)
    cl = np.ascontiguousarray(np.asarray(loop_closed, np.uint8))
    if cl.size != nl:
        raise ValueError("loop_closed must have one entry per loop")
    nx = x.shape[0]
    ny = y.shape[0]
    px = _dev(x, dt, "x", (nx,))
    py = _dev(y, dt, "y", (ny,))
    if not grid and nx != ny:
        raise ValueError("points mode needs len(x) == len(y)")
    shape = (ny, nx) if grid else (nx,)
    w = torch.empty(shape, dtype=dt, device=x.device)
    chi = torch.empty(shape, dtype=torch.int32, device=x.device) if want_chi else None
    check(lib().wn_eval_2d(code, pc, nseg, _ptr64(lo), cl.ctypes.data_as(C.c_void_p) if cl.size else None,
                           nl, 1 if grid else 0, px, py, nx, ny if grid else nx,
                           _dev(w, dt, "w"), _dev(chi, torch.int32, "chi") if chi is not None else None,
                           _stream(stream)), "wn_eval_2d")
    return w, chi


class Batch2D:
    """Many 2D curve sets, each evaluated on its own grid in one launch.

    ``sets`` is a sequence of ``(loop_off, loop_closed, nx, ny)`` (loop
    offsets relative to the set's first segment).  The batch holds the set
    descriptors and loop tables on the device; ``eval`` takes the segments of
    every set concatenated (``ctrl`` [sum nseg, 4, 2]) and the axes
    concatenated (``x`` [sum nx], ``y`` [sum ny]).  Every set's output equals
    eval_2d(..., grid=True) on that set alone, bit for bit."""

    def __init__(self, sets, dtype=torch.float32, stream=None):
        if dtype == torch.float64:
            self.dtype, self._code = torch.float64, 1
        elif dtype == torch.float32:
            self.dtype, self._code = torch.float32, 0
        else:
            raise TypeError("dtype must be float32 or float64")
        self._h = None
        n = len(sets)
        desc = (CurveSet2D * max(n, 1))()
        keep = []
        self.shapes = []
        self.nseg = self.nx = self.ny = 0
        for k, (loop_off, loop_closed, nx, ny) in enumerate(sets):
            lo = np.ascontiguousarray(np.asarray(loop_off, dtype=np.int64))
            cl = np.ascontiguousarray(np.asarray(loop_closed, np.uint8))
            nl = max(lo.size - 1, 0)
            if cl.size != nl:
                raise ValueError(f"set {k}: loop_closed must have one entry per loop")
            nseg = int(lo[-1]) if lo.size else 0
            keep += [lo, cl]
            d = desc[k]
            d.nseg, d.nloops, d.nx, d.ny = nseg, nl, int(nx), int(ny)
            d.loop_off = _ptr64(lo)
            d.loop_closed = cl.ctypes.data_as(C.c_void_p) if cl.size else None
            self.nseg += nseg
            self.nx += int(nx)
            self.ny += int(ny)
            self.shapes.append((int(ny), int(nx)))
        self.nout = sum(a * b for a, b in self.shapes)
        h = C.c_void_p()
        check(lib().wn_batch2d_create(self._code, desc if n else None, n, _stream(stream), C.byref(h)),
              "wn_batch2d_create")
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().wn_batch2d_free(self._h)
            self._h = None

    def eval(self, ctrl: torch.Tensor, x: torch.Tensor, y: torch.Tensor, want_chi: bool = True,
             out=None, stream=None):
        """(w, chi) as flat [sum nx*ny] tensors (each set's [ny, nx] grid in set
        order; chi None if not wanted).  ``out`` may pass preallocated
        (w, chi) tensors.  ``split`` turns them into per-set views."""
        dt = self.dtype
        pc = _dev(ctrl, dt, "ctrl", (self.nseg, 4, 2))
        px = _dev(x, dt, "x", (self.nx,))
        py = _dev(y, dt, "y", (self.ny,))
        if out is not None:
            w, chi = out
        else:
            w = torch.empty(self.nout, dtype=dt, device=x.device)
            chi = torch.empty(self.nout, dtype=torch.int32, device=x.device) if want_chi else None
        check(lib().wn_eval_2d_batched(self._h, pc, px, py, _dev(w, dt, "w", (self.nout,)),
                                       _dev(chi, torch.int32, "chi", (self.nout,)) if chi is not None else None,
                                       _stream(stream)), "wn_eval_2d_batched")
        return w, chi

    def split(self, flat: torch.Tensor):
        """Per-set [ny, nx] views of a flat output."""
        views, o = [], 0
        for ny, nx in self.shapes:
            views.append(flat[o:o + ny * nx].view(ny, nx))
            o += ny * nx
        return views


class PatchBatch:
    """Many parametric surfaces (bicubic patches + boundary curves), each with
    its own ray direction and queries, evaluated in one launch.

    ``surfaces`` is a sequence of ``(npatch, ncurves, nq, direction)``.
    ``eval`` takes every surface's patch nets concatenated (``nets``
    [sum npatch, 4, 4, 3]), their curves concatenated (``curves``
    [sum ncurves, 4, 3]) and their queries concatenated; each surface's
    results equal eval_3d_patches on that surface alone, bit for bit."""

    def __init__(self, surfaces, stream=None):
        self._h = None
        n = len(surfaces)
        desc = (PatchSurface * max(n, 1))()
        self.counts = []
        for k, (npatch, ncurves, nq, direction) in enumerate(surfaces):
            d = desc[k]
            d.npatch, d.ncurves, d.nq = int(npatch), int(ncurves), int(nq)
            for j, v in enumerate(direction):
                d.dir[j] = float(v)
            self.counts.append((int(npatch), int(ncurves), int(nq)))
        self.npatch = sum(c[0] for c in self.counts)
        self.ncurves = sum(c[1] for c in self.counts)
        self.nq = sum(c[2] for c in self.counts)
        h = C.c_void_p()
        check(lib().wn_patch_batch_create(desc if n else None, n, _stream(stream), C.byref(h)),
              "wn_patch_batch_create")
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().wn_patch_batch_free(self._h)
            self._h = None

    def eval(self, nets, curves, qx, qy, qz, want_w: bool = True, want_chi: bool = True, stream=None):
        """(w or None, chi or None) as flat [sum nq] tensors in surface order."""
        if not (want_w or want_chi):
            raise ValueError("nothing requested")
        pn = _dev(nets, torch.float32, "nets", (self.npatch, 4, 4, 3)) if self.npatch else None
        pc = _dev(curves, torch.float32, "curves", (self.ncurves, 4, 3)) if self.ncurves else None
        n = self.nq
        px, py, pz = (_dev(t, torch.float32, name, (n,)) for t, name in ((qx, "qx"), (qy, "qy"), (qz, "qz")))
        w = torch.empty(n, dtype=torch.float32, device=qx.device) if want_w else None
        chi = torch.empty(n, dtype=torch.int32, device=qx.device) if want_chi else None
        check(lib().wn_eval_3d_patches_batched(self._h, pn, pc, px, py, pz,
                                               _dev(w, torch.float32, "w") if w is not None else None,
                                               _dev(chi, torch.int32, "chi") if chi is not None else None,
                                               _stream(stream)), "wn_eval_3d_patches_batched")
        return w, chi

    def split(self, flat: torch.Tensor):
        """Per-surface views of a flat output."""
        views, o = [], 0
        for _, _, nq in self.counts:
            views.append(flat[o:o + nq])
            o += nq
        return views


def eval_2d_batched(ctrl: torch.Tensor, sets, x: torch.Tensor, y: torch.Tensor, want_chi: bool = True,
                    stream=None):
    """One-off Batch2D evaluation: lists of per-set [ny, nx] w (and chi)
    views; see Batch2D for the layout of ``ctrl``, ``sets``, ``x``, ``y``."""
    b = Batch2D(sets, ctrl.dtype, stream)
    w, chi = b.eval(ctrl, x, y, want_chi, stream=stream)
    return b.split(w), (b.split(chi) if chi is not None else None)


def backward_2d(ctrl: torch.Tensor, loop_off, loop_closed, x: torch.Tensor, y: torch.Tensor,
                grad_w: torch.Tensor, grid: bool = False, want_q: bool = True, want_ctrl: bool = True,
                stream=None):
    """(dL/dp, dL/dctrl) for dL/dw = grad_w on the queries of eval_2d (same
    layout: points [n] or grid [ny, nx]); dL/dp has a trailing axis of 2, dL/dctrl
    the shape of ctrl.  Only the open loops' end points get nonzero entries."""
    if ctrl.dtype == torch.float64:
        dt, code = torch.float64, 1
    elif ctrl.dtype == torch.float32:
        dt, code = torch.float32, 0
    else:
        raise TypeError("ctrl must be float32 or float64")
    nseg = ctrl.shape[0]
    pc = _dev(ctrl, dt, "ctrl", (nseg, 4, 2))
    lo, nl = _loops(loop_off, limit=True)
    cl = np.ascontiguousarray(np.asarray(loop_closed, np.uint8))
    if cl.size != nl:
        raise ValueError("loop_closed must have one entry per loop")
    nx, ny = x.shape[0], y.shape[0]
    if not grid and nx != ny:
        raise ValueError("points mode needs len(x) == len(y)")
    shape = (ny, nx) if grid else (nx,)
    pg = _dev(grad_w, dt, "grad_w", shape)
    gq = torch.empty(shape + (2,), dtype=dt, device=x.device) if want_q else None
    gc = torch.empty((nseg, 4, 2), dtype=dt, device=x.device) if want_ctrl else None
    check(lib().wn_backward_2d(code, pc, nseg, _ptr64(lo), cl.ctypes.data_as(C.c_void_p) if cl.size else None, nl,
                               1 if grid else 0, _dev(x, dt, "x", (nx,)), _dev(y, dt, "y", (ny,)), nx,
                               ny if grid else nx, pg, _dev(gq, dt, "grad_q") if gq is not None else None,
                               _dev(gc, dt, "grad_ctrl") if gc is not None else None, _stream(stream)),
          "wn_backward_2d")
    return gq, gc


class WindingNumber2D(torch.autograd.Function):
    """w of cubic Bezier loops at points (x[i], y[i]); gradients flow to the
    control points (only open loops' end points move w) and to x, y."""

    @staticmethod
    def forward(ctx, ctrl, x, y, loop_off, loop_closed):
        w, _ = eval_2d(ctrl.detach(), loop_off, loop_closed, x.detach(), y.detach(), want_chi=False)
        ctx.save_for_backward(ctrl, x, y)
        ctx.loops = (loop_off, loop_closed)
        return w

    @staticmethod
    def backward(ctx, grad_w):
        ctrl, x, y = ctx.saved_tensors
        need_c = ctx.needs_input_grad[0]
        need_q = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        gq, gc = backward_2d(ctrl.detach(), ctx.loops[0], ctx.loops[1], x.detach(), y.detach(),
                             grad_w.contiguous().to(ctrl.dtype), want_q=need_q, want_ctrl=need_c)
        gx = gy = None
        if gq is not None:
            gx, gy = gq[:, 0], gq[:, 1]
        return gc, gx, gy, None, None


def winding_number_2d(ctrl, loop_off, loop_closed, x, y):
    return WindingNumber2D.apply(ctrl, x, y, loop_off, loop_closed)


def backward_curves(ctrl: torch.Tensor, qx, qy, qz, grad_w: torch.Tensor, want_q: bool = True,
                    want_ctrl: bool = True, stream=None):
    """(dL/dp [nq, 3], dL/dctrl [nc, 4, 3]) for dL/dw = grad_w of the curve
    boundary term (``wn_backward_curves``); either may be None.  A control
    point shared by two curves gets one entry per curve."""
    nc = ctrl.shape[0]
    pcv = _dev(ctrl, torch.float32, "ctrl", (nc, 4, 3))
    px, py, pz, nq = _queries(qx, qy, qz)
    pg = _dev(grad_w, torch.float32, "grad_w", (nq,))
    gq = torch.empty((nq, 3), dtype=torch.float32, device=qx.device) if want_q else None
    gc = torch.empty((nc, 4, 3), dtype=torch.float32, device=qx.device) if want_ctrl else None
    if gq is None and gc is None:
        return None, None
    check(lib().wn_backward_curves(pcv, nc, px, py, pz, nq, pg,
                                   _dev(gq, torch.float32, "grad_q") if gq is not None else None,
                                   _dev(gc, torch.float32, "grad_ctrl") if gc is not None else None,
                                   _stream(stream)), "wn_backward_curves")
    return gq, gc


class WindingNumberCurves(torch.autograd.Function):
    """w of a surface bounded by Bezier curves (chi_d from the BVH of its
    tessellation, or from ``chi`` if given); gradients flow to the control
    points and the queries through the curve boundary term."""

    @staticmethod
    def forward(ctx, ctrl, qx, qy, qz, bvh, chi):
        w, _ = eval_3d_curves(bvh, ctrl.detach(), qx.detach(), qy.detach(), qz.detach(), chi_in=chi,
                              want_chi=False)
        ctx.save_for_backward(ctrl, qx, qy, qz)
        return w

    @staticmethod
    def backward(ctx, grad_w):
        ctrl, qx, qy, qz = ctx.saved_tensors
        need_c = ctx.needs_input_grad[0]
        need_q = any(ctx.needs_input_grad[1:4])
        gq, gc = backward_curves(ctrl.detach(), qx.detach(), qy.detach(), qz.detach(),
                                 grad_w.contiguous().float(), want_q=need_q, want_ctrl=need_c)
        if gq is None:
            return gc, None, None, None, None, None
        return gc, gq[:, 0], gq[:, 1], gq[:, 2], None, None


def winding_number_curves(bvh, ctrl, qx, qy, qz, chi=None):
    return WindingNumberCurves.apply(ctrl, qx, qy, qz, bvh, chi)


class Batch:
    """Many surfaces, each with its own queries, in one persistent launch
    (``wn_batch_create`` / ``wn_eval_batched`` / ``wn_backward_batched``).

    ``surfaces`` is a list of dicts with device tensors ``V`` [nv, 3]
    float32, ``F`` [nf, 3] int32, ``bnd`` [nb, 3] float32 (copies of
    boundary vertices), host ``loop_off`` and the query count ``nq``.
    Queries are passed concatenated in surface order."""

    def __init__(self, surfaces, direction, tune_mode: int = 0, stream=None):
        from ._lib import Surface
        self._keep = []
        arr = (Surface * max(len(surfaces), 1))()
        nb_tot = 0
        for i, s in enumerate(surfaces):
            V, F, bnd = s["V"], s["F"], s["bnd"]
            lo, nl = _loops(s["loop_off"])
            nb = int(lo[-1]) if nl else 0
            self._keep.append(lo)
            arr[i].V = _dev(V, torch.float32, "V", (V.shape[0], 3))
            arr[i].nv = V.shape[0]
            arr[i].F = _dev(F, torch.int32, "F", (F.shape[0], 3))
            arr[i].nf = F.shape[0]
            arr[i].bnd_xyz = _dev(bnd, torch.float32, "bnd", (nb, 3))
            arr[i].loop_off = _ptr64(lo)
            arr[i].nloops = nl
            arr[i].nq = int(s["nq"])
            nb_tot += nb
        d = (C.c_double * 3)(*[float(x) for x in np.asarray(direction, np.float64).ravel()[:3]])
        h = C.c_void_p()
        check(lib().wn_batch_create(arr, len(surfaces), d, int(tune_mode), _stream(stream), C.byref(h)),
              "wn_batch_create")
        self._h = h
        self.total_q = sum(int(s["nq"]) for s in surfaces)
        self.total_b = nb_tot

    def info(self) -> dict:
        v = (C.c_int64 * 9)()
        check(lib().wn_batch_info(self._h, v), "wn_batch_info")
        keys = ["total_q", "total_b", "total_pairs", "n_items", "tile", "wg_per_cu", "graph", "tune_us", "mode"]
        return dict(zip(keys, v[:]))

    def eval(self, qx, qy, qz, want_chi: bool = True, w_out=None, chi_out=None, stream=None):
        nq = self.total_q
        px = _dev(qx, torch.float32, "qx", (nq,))
        py = _dev(qy, torch.float32, "qy", (nq,))
        pz = _dev(qz, torch.float32, "qz", (nq,))
        w = torch.empty(nq, dtype=torch.float32, device=qx.device) if w_out is None else w_out
        chi = None
        if want_chi:
            chi = torch.empty(nq, dtype=torch.int32, device=qx.device) if chi_out is None else chi_out
        check(lib().wn_eval_batched(self._h, px, py, pz, _dev(w, torch.float32, "w_out", (nq,)),
                                    _dev(chi, torch.int32, "chi_out", (nq,)) if chi is not None else None,
                                    _stream(stream)), "wn_eval_batched")
        return w, chi

    def backward(self, qx, qy, qz, grad_w, want_q: bool = True, want_bnd: bool = True, stream=None):
        nq = self.total_q
        dev = qx.device
        gq = torch.empty((nq, 3), dtype=torch.float32, device=dev) if want_q else None
        gb = torch.empty((self.total_b, 3), dtype=torch.float32, device=dev) if want_bnd else None
        check(lib().wn_backward_batched(
            self._h, _dev(qx, torch.float32, "qx", (nq,)), _dev(qy, torch.float32, "qy", (nq,)),
            _dev(qz, torch.float32, "qz", (nq,)), _dev(grad_w, torch.float32, "grad_w", (nq,)),
            _dev(gq, torch.float32, "grad_q") if gq is not None else None,
            _dev(gb, torch.float32, "grad_bnd") if gb is not None else None, _stream(stream)),
            "wn_backward_batched")
        return gq, gb

    def free(self):
        if getattr(self, "_h", None) is not None:
            torch.cuda.synchronize()
            lib().wn_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None) is not None:
                lib().wn_batch_free(self._h)
                self._h = None
        except Exception:
            pass
