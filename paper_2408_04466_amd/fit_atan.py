"""Derivation and check of the arctangent polynomials in the kernels.

Both device atan2 functions reduce to |t| <= tan(pi/8) and evaluate
atan(t) = t P(t^2).

* float64 (``atan2_f64`` in csrc/wn2d.hip): P of degree 10 from a Chebyshev
  fit of atan(t)/t on [0, tan(pi/8)^2] in 40-digit arithmetic, coefficients
  rounded to float64.
* float32 (``atan2_f32`` in csrc/geom.hpp): P of degree 4 with P(0) = 1, the
  minimax fit of atan(t) by t P(t^2) on a grid of 8000 points of
  (0, tan(pi/8)] (a linear program: minimise E subject to |t P(t^2) -
  atan(t)| <= E at every grid point; reference values from mpmath),
  coefficients rounded to float32.  The fit's own error is ~5e-14; what
  remains, ~5e-8, is float32 rounding in the evaluation.

Running this file derives both sets, checks that they are the constants in
the two sources, and reports each polynomial's largest error over the reduced
range, evaluated by Horner's rule with fused multiply-adds in its own
precision, against mpmath's atan.  Needs mpmath and scipy.
"""
import os
import re

import mpmath as mp
import numpy as np

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def fit_f64():
    mp.mp.dps = 40
    tmax = mp.tan(mp.pi / 8)

    def g(s):
        if s == 0:
            return mp.mpf(1)
        r = mp.sqrt(s)
        return mp.atan(r) / r

    poly, err = mp.chebyfit(g, [0, tmax ** 2], 11, error=True)
    return [float(x) for x in poly[::-1]], float(err)


def fit_f32(n=8000):
    from scipy.optimize import linprog
    mp.mp.dps = 30
    tmax = float(mp.tan(mp.pi / 8))
    t = np.linspace(0.0, tmax, n + 1)[1:]
    s = t * t
    ref = np.array([float(mp.atan(mp.mpf(float(x)))) for x in t])
    # unknowns c1..c4, E; residual t (1 + sum_k c_k s^k) - atan(t)
    A = np.stack([t * s ** k for k in range(1, 5)], 1)
    b = ref - t
    one = np.ones((len(t), 1))
    res = linprog(np.r_[np.zeros(4), 1.0],
                  A_ub=np.vstack([np.hstack([A, -one]), np.hstack([-A, -one])]),
                  b_ub=np.concatenate([b, -b]), bounds=[(None, None)] * 5, method="highs")
    if not res.success:
        raise RuntimeError(res.message)
    return [1.0] + [float(np.float32(c)) for c in res.x[:4]], float(res.x[4])


def source_f64():
    src = open(os.path.join(CSRC, "wn2d.hip")).read()
    body = re.search(r"constexpr double kP\[11\] = \{(.*?)\};", src, re.S).group(1)
    return [float(x) for x in body.replace("\n", " ").split(",")]


def source_f32():
    src = open(os.path.join(CSRC, "geom.hpp")).read()
    body = src[src.index("float atan2_f32("):]
    body = body[:body.index("float r = ")]
    first = re.search(r"float p = ([-0-9.e]+)f;", body).group(1)
    rest = re.findall(r"p = __fmaf_rn\(p, s, ([-0-9.e]+)f\);", body)
    return [float(x) for x in (rest[::-1] + [first])]


def max_error(coef, dtype, n=200001):
    """Largest |t P(t^2) - atan(t)| on the reduced range, P by Horner's rule
    with one rounding per step (a fused multiply-add) in ``dtype``."""
    t = np.linspace(0, np.tan(np.pi / 8), n).astype(dtype)
    s = t * t
    p = np.full(t.shape, coef[-1], dtype=np.longdouble)
    for c in coef[-2::-1]:
        p = (p * s.astype(np.longdouble) + np.longdouble(c)).astype(dtype).astype(np.longdouble)
    approx = (t.astype(np.longdouble) * p).astype(dtype)
    ref = np.arctan(t.astype(np.longdouble))
    return float(np.abs(approx.astype(np.longdouble) - ref).max())


def main():
    c64, e64 = fit_f64()
    c32, e32 = fit_f32()
    print("float64 coefficients (increasing powers of t^2):")
    for c in c64:
        print(f"  {c!r}")
    print(f"  fit error {e64:.3g}; evaluated in float64: max abs error {max_error(c64, np.float64):.3g}")
    print("float32 coefficients (increasing powers of t^2):")
    for c in c32:
        print(f"  {c!r}")
    print(f"  fit error {e32:.3g}; evaluated in float32: max abs error {max_error(c32, np.float32):.3g}")
    assert source_f64() == c64, "csrc/wn2d.hip kP differs from the derived float64 set"
    assert source_f32() == c32, "csrc/geom.hpp atan2_f32 differs from the derived float32 set"
    print("both sets match the sources")


if __name__ == "__main__":
    main()
