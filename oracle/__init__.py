"""FP64 CPU oracle for the one-shot generalized winding number.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call or
link this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, headers,
tables or constants with the HIP path; the only common module is ``synth``
(seeded input generators, no method arithmetic).

Contents
--------
- ``wn3d``   : 3D meshes.  Boundary half-edges (Sec. 5.1 "Multiple Boundaries";
               Sec. 6.1 "Preprocessing"), brute-force signed crossing count
               (Eq. chi; the ray-casting step of Alg. 1), boundary line integral relative to
               one fixed ray direction (Eq. wn_discrete_sum with Lemma 2, see
               the module docstring), degeneracy margins.
- ``wn2d``   : 2D cubic Bezier loops (Sec. 3 definition of w_C, Sec. 7 "2D
               parametric geometry"): crossings of the +d ray with every cubic,
               plus the open-loop endpoint angles.
- ``grad3d`` : closed-form derivatives of the boundary integral with respect to
               the query point and the boundary vertices (the crossing count is
               piecewise constant, so it contributes nothing).
- ``grad2d`` : the same for 2D loops: only the open loops' end points (and the
               query) carry a gradient.
- ``curves3d``   : the boundary term along cubic Bezier boundary curves
               (Sec. 5.1 "Exact Computations", region areas from boundary integrals), adaptive
               Gauss-Legendre on the form whose edge integral is the polyline
               edge term.
- ``patches3d``  : signed ray crossings of bicubic Bezier patches (Eq. chi;
               Sec. 5.1 "Parametric Surfaces") by subdivision, convex-hull pruning
               and Newton, with duplicate roots merged.
- ``gradcurves`` : derivatives of the curve boundary term with respect to
               the query and the control points (Biot-Savart integrals).

Every floating-point computation is float64 on inputs promoted exactly from
the kernel's float32 arrays.  Parity status of each function is stated in its
module header ("pinned by ..." or "parity unpinned").
"""
from . import wn3d, wn2d, grad3d, grad2d, curves3d, patches3d, gradcurves  # noqa: F401
