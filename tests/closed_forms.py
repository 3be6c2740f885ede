"""Closed forms used to pin the oracle (derived from the continuous model).

Spherical Radon transform, Eq. (srt): g(r_s, t) = integral of A over the
sphere |r - r_s| = c0 t.

Uniform ball (amplitude A, radius a, centre at distance d from r_s): the
sphere of radius rho meets the ball in a cap of area
2 pi rho^2 (1 - cos theta*), cos theta* = (rho^2 + d^2 - a^2) / (2 rho d),
which simplifies to  g = A pi rho (a^2 - (d - rho)^2) / d  for |d - rho| <= a.

Isotropic Gaussian exp(-|r-c|^2 / (2 s^2)): integrating over the sphere in
polar coordinates about the line r_s -> c gives
g = (2 pi rho s^2 / d) [exp(-(rho-d)^2/(2 s^2)) - exp(-(rho+d)^2/(2 s^2))].
"""
import numpy as np


def srt_ball(rho, d, a, A=1.0):
    rho = np.asarray(rho, dtype=np.float64)
    inside = np.abs(d - rho) <= a
    return np.where(inside, A * np.pi * rho * (a * a - (d - rho) ** 2) / d, 0.0)


def srt_gaussian(rho, d, s, A=1.0):
    rho = np.asarray(rho, dtype=np.float64)
    return A * 2.0 * np.pi * rho * s * s / d * (
        np.exp(-(rho - d) ** 2 / (2 * s * s)) - np.exp(-(rho + d) ** 2 / (2 * s * s)))
