"""Coefficients of small_rot (oat_geom.hpp): sin d and cos d - 1 for the
rotation of a ring point from its segment's reference point, |d| <= pi/8
(a segment of 2^s points, 2^s <= N_j / 8, has |j - j_ref| <= 2^(s-1)).

    sin d     ~ d (1 + a1 d^2 + a2 d^4)
    cos d - 1 ~ d^2 (-1/2 + b1 d^2 + b2 d^4)

The leading terms are kept exact and (a1, a2), (b1, b2) minimise the largest
RELATIVE error over (0, pi/8], so the position error, ring radius times
|d| times that error, stays below about 5e-7 cell for every ring size.  The
minimax fit is Lawson's iteratively reweighted least squares on a dense
grid.  Run as a script it prints the FP32 literals written in the header.
"""
import math

import numpy as np

D_MAX = math.pi / 8


def _lawson(c, cols, iters=3000):
    """Minimise max_i |c_i + X_i . a| (Lawson's algorithm)."""
    X = np.column_stack(cols)
    w = np.full(len(c), 1.0 / len(c))
    for _ in range(iters):
        sw = np.sqrt(w)
        a, *_ = np.linalg.lstsq(X * sw[:, None], -c * sw, rcond=None)
        e = np.abs(c + X @ a)
        w = w * e
        w /= w.sum()
    return a


def coefficients():
    """(a1, a2, b1, b2) rounded to FP32, as Python floats."""
    d = np.linspace(D_MAX / 20000, D_MAX, 20000)
    u = d * d
    s = np.sin(d)
    # relative error of sin: d (1 + u (a1 + a2 u)) / sin d - 1
    a = _lawson(d / s - 1, [d * u / s, d * u * u / s])
    cm = -2.0 * np.sin(d / 2) ** 2          # cos d - 1 without cancellation
    # relative error of cos - 1: u (-1/2 + u (b1 + b2 u)) / (cos d - 1) - 1
    b = _lawson(-0.5 * u / cm - 1, [u * u / cm, u ** 3 / cm])
    return tuple(float(np.float32(x)) for x in (a[0], a[1], b[0], b[1]))


def max_relative_errors(coefs, n=400001):
    """Largest relative errors of the two polynomials (FP64 evaluation)."""
    a1, a2, b1, b2 = coefs
    d = np.linspace(1e-7, D_MAX, n)
    u = d * d
    es = d * (1 + u * (a1 + a2 * u)) / np.sin(d) - 1
    ec = u * (-0.5 + u * (b1 + b2 * u)) / (-2.0 * np.sin(d / 2) ** 2) - 1
    return float(np.abs(es).max()), float(np.abs(ec).max())


if __name__ == "__main__":
    c = coefficients()
    print("a1 a2 b1 b2 =", ", ".join(str(np.float32(x)) + "f" for x in c))
    print("max relative error: sin %.3g, cos - 1 %.3g" % max_relative_errors(c))
