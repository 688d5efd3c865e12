"""One-shot generalized winding numbers on AMD Instinct MI355X.

Thin Python binding over ``libwn.so`` (C ABI in ``include/wn.h``): argument
checks and marshalling of torch device tensors and the current HIP stream.
All computation runs in the library's HIP kernels.
"""
from .api import (  # noqa: F401
    BVH,
    Batch,
    Batch2D,
    PatchBatch,
    WindingNumber2D,
    WindingNumber3D,
    WindingNumberCurves,
    backward_2d,
    backward_curves,
    backward,
    boundary_loops,
    crossings_3d,
    eval_2d,
    eval_2d_batched,
    eval_3d,
    eval_3d_boundary,
    eval_3d_curves,
    eval_3d_patches,
    eval_3d_grid,
    diagnose,
    device_info,
    spatial_order,
    winding_number,
    winding_number_2d,
    winding_number_curves,
)
from ._lib import WN_CHI_INVALID, WN_MAX_LOOPS, WnError, lib  # noqa: F401
