"""Derivation and check of the arctangent polynomials in the kernels.

Both device atan2 functions reduce to |t| <= tan(pi/8) and evaluate
atan(t) = t P(t^2).

* float64 (``atan2_f64`` in csrc/wn2d.hip): P of degree 10 from a Chebyshev
  fit of atan(t)/t on [0, tan(pi/8)^2] in 40-digit arithmetic.  Running this
  file prints those coefficients rounded to float64, as they appear in the
  source.
* float32 (``atan2_f32`` in csrc/geom.hpp): P of degree 4.

It then reports each polynomial's largest error over the reduced range,
evaluated by Horner's rule in its own precision, against mpmath's atan.
Needs mpmath.
"""
import mpmath as mp
import numpy as np

F32 = [1.0, -0.3333280682563782, 0.199747234582901, -0.1385444849729538, 0.07993615418672562]


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


def max_error(coef, dtype, n=200001):
    t = np.linspace(0, np.tan(np.pi / 8), n).astype(dtype)
    s = t * t
    p = np.full_like(s, coef[-1], dtype=dtype)
    for c in coef[-2::-1]:
        p = (p * s + dtype(c)).astype(dtype)
    approx = (t * p).astype(dtype)
    ref = np.arctan(t.astype(np.longdouble))
    return float(np.abs(approx.astype(np.longdouble) - ref).max())


if __name__ == "__main__":
    c64, fit_err = fit_f64()
    print("float64 coefficients (increasing powers of t^2):")
    for c in c64:
        print(f"  {c!r}")
    print(f"fit error {fit_err:.3g}; float64 Horner max abs error {max_error(c64, np.float64):.3g}")
    print(f"float32 polynomial: float32 Horner max abs error {max_error(F32, np.float32):.3g}")
