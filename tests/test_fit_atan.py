"""The arctangent polynomials of the two device atan2 functions are the ones
paper_2408_04466_amd/fit_atan.py derives (CPU only): the float64 Chebyshev
set in csrc/wn2d.hip and the float32 minimax set in csrc/geom.hpp, each
within its error budget when evaluated in its own precision."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                "paper_2408_04466_amd"))
import fit_atan  # noqa: E402


def test_float64_set_is_derived():
    c, _ = fit_atan.fit_f64()
    assert fit_atan.source_f64() == c
    assert fit_atan.max_error(c, np.float64) < 2e-16


def test_float32_set_is_derived():
    c, e = fit_atan.fit_f32()
    assert e < 1e-13
    assert fit_atan.source_f32() == c
    assert fit_atan.max_error(c, np.float32) < 6e-8
