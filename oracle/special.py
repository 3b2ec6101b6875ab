"""Special functions for the oracle (float64, scipy-backed).

* spherical Bessel j_l and Legendre P_l: the ingredients of the plane-wave
  expansion (Sec. 2.1, Eq. plane-sph-harmonics) and of the rotation average
  of two plane waves (Sec. 2.2, Eq. double-e-expansion; Appendix A).
* complex orthonormal spherical harmonics Y_lm with the Condon-Shortley
  phase: the angular part of the multipole window (Sec. 2.2,
  Eq. 3PCF-multipole-window).
* the radial-bin average of j_l: the binning window applied to each
  secondary vertex (Sec. 2.2, the paragraph after Eq. nL-2fold), read as the
  r^2-weighted mean over a shell r_lo <= r < r_hi.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy.special import spherical_jn, sph_harm_y, eval_legendre

__all__ = ["sph_jn", "legendre", "ylm", "jbar", "jbar_l0_closed", "gauss_legendre", "tophat_window",
           "thin_shell"]

# Gauss-Legendre order for the bin average.  A bin spans at most a few
# oscillations of j_l(k r) at the grid's largest k, where 64 nodes converge to
# rounding (checked against 128 nodes by the tests).
JBAR_NODES = 64


def sph_jn(l: int, x):
    """Spherical Bessel function of the first kind j_l(x)."""
    return spherical_jn(l, x)


def legendre(l: int, mu):
    """Legendre polynomial P_l(mu)."""
    return eval_legendre(l, mu)


def ylm(l: int, m: int, theta, phi):
    """Y_l^m(theta, phi): polar angle theta, azimuth phi, Condon-Shortley phase."""
    return sph_harm_y(l, m, theta, phi)


def gauss_legendre(n: int):
    """Nodes and weights of the n-point Gauss-Legendre rule on [-1, 1]."""
    return leggauss(n)


def jbar(l: int, edges, k, nodes: int = JBAR_NODES) -> np.ndarray:
    """Bin-averaged spherical Bessel function.

    jbar_{l,b}(k) = 3 / (r_{b+1}^3 - r_b^3) * int_{r_b}^{r_{b+1}} r^2 j_l(k r) dr

    Returns an array [nbins, k.size].
    """
    k = np.asarray(k, dtype=np.float64).ravel()
    edges = np.asarray(edges, dtype=np.float64)
    xg, wg = leggauss(nodes)
    out = np.empty((edges.size - 1, k.size))
    for b in range(edges.size - 1):
        r1, r2 = edges[b], edges[b + 1]
        r = 0.5 * (r2 - r1) * xg + 0.5 * (r2 + r1)
        wr = 0.5 * (r2 - r1) * wg * r * r
        vals = spherical_jn(l, np.multiply.outer(k, r))
        out[b] = vals @ wr * (3.0 / (r2 ** 3 - r1 ** 3))
    return out


def jbar_l0_closed(edges, k) -> np.ndarray:
    """Closed form of the l = 0 bin average: int r^2 j_0(k r) dr = [sin kr - kr cos kr] / k^3."""
    k = np.asarray(k, dtype=np.float64).ravel()
    edges = np.asarray(edges, dtype=np.float64)
    out = np.empty((edges.size - 1, k.size))
    for b in range(edges.size - 1):
        r1, r2 = edges[b], edges[b + 1]
        with np.errstate(divide="ignore", invalid="ignore"):
            prim = lambda r: (np.sin(k * r) - k * r * np.cos(k * r)) / k ** 3  # noqa: E731
            v = (prim(r2) - prim(r1)) * 3.0 / (r2 ** 3 - r1 ** 3)
        out[b] = np.where(k == 0, 1.0, v)
    return out


def thin_shell(l: int, edges, k) -> np.ndarray:
    """Infinitely thin shell at each bin's mid radius: j_l(k r_b), r_b = (edges[b] + edges[b+1]) / 2
    (the radial factor of Eq. 3PCF-multipole-window).  Returns [nbins, k.size]."""
    k = np.asarray(k, dtype=np.float64).ravel()
    edges = np.asarray(edges, dtype=np.float64)
    mid = 0.5 * (edges[:-1] + edges[1:])
    return spherical_jn(l, np.multiply.outer(mid, k))


def tophat_window(x):
    """Fourier transform of the unit-volume sphere at x = k R: 3 j_1(x) / x
    (the spherical top-hat binning window of Sec. 3), 1 at x = 0."""
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        v = 3.0 * spherical_jn(1, x) / x
    return np.where(x == 0.0, 1.0, v)
