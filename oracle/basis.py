"""Cubic B-spline basis: deposit, interpolation, connection coefficients.

The paper reconstructs the density on a multiresolution basis of compactly
supported scaling functions (Sec. 2.1, the equation after
Eq. window-sphshell-real) and uses the connection coefficients of three basis
functions for the grid summation (Sec. 2.2, Eq. con-coeff).  The basis here
is the centred cubic B-spline B3 (support 4 cells per axis, D_sup = 4):

    B3(u) = (4 - 6u^2 + 3|u|^3) / 6   for |u| < 1
          = (2 - |u|)^3 / 6           for 1 <= |u| < 2
          = 0                         otherwise,

in cell units u = x / a, a = box / n, nodes at integer u, periodic wrap.  The
coefficient of node l from a catalogue is sum_i w_i prod_d B3(u_{i,d} - l_d)
(Sec. 3, the decomposition step of the workflow); the density contrast is
delta = n / nbar - 1 (Sec. 3, the periodic-box paragraph) with
nbar = W / n^3 per cell and W = sum_i w_i.

Connection coefficients are computed exactly in rational arithmetic by
integrating products of the spline's polynomial pieces.
"""
from __future__ import annotations

from fractions import Fraction
import numpy as np

__all__ = ["b3", "taps", "deposit", "density_contrast", "gather",
           "gamma_1d", "gamma_matrix", "b7_samples", "b7_hat"]


def b3(u):
    """Centred cubic B-spline."""
    u = np.abs(np.asarray(u, dtype=np.float64))
    out = np.zeros_like(u)
    m1 = u < 1.0
    m2 = (u >= 1.0) & (u < 2.0)
    out[m1] = (4.0 - 6.0 * u[m1] ** 2 + 3.0 * u[m1] ** 3) / 6.0
    out[m2] = (2.0 - u[m2]) ** 3 / 6.0
    return out


def taps(pos, n: int, box: float):
    """Per-particle stencil of the basis: first node and weights per axis.

    u = x n / box in float64 (x as given, e.g. float32); the four nodes
    floor(u) - 1 .. floor(u) + 2 carry weights B3(u - node).
    Returns (base [P,3] int64, weights [P,3,4] float64).
    """
    u = np.asarray(pos, dtype=np.float64) * (float(n) / float(box))
    fl = np.floor(u)
    base = fl.astype(np.int64) - 1
    offs = np.arange(4, dtype=np.float64)
    wts = b3(u[:, :, None] - (base[:, :, None].astype(np.float64) + offs))
    return base, wts


def _tap_terms(pos, n, box):
    """Yield (flat node index [P], weight [P]) for each of the 64 stencil taps."""
    base, wts = taps(pos, n, box)
    for jx in range(4):
        ix = (base[:, 0] + jx) % n
        for jy in range(4):
            iy = (base[:, 1] + jy) % n
            wxy = wts[:, 0, jx] * wts[:, 1, jy]
            for jz in range(4):
                iz = (base[:, 2] + jz) % n
                yield (ix * n + iy) * n + iz, wxy * wts[:, 2, jz]


def deposit(pos, w, n: int, box: float):
    """Basis coefficients eps_l = sum_i w_i prod_d B3(u_{i,d} - l_d) on the n^3 grid."""
    w = np.ones(len(pos)) if w is None else np.asarray(w, dtype=np.float64)
    eps = np.zeros(n ** 3)
    for idx, wt in _tap_terms(pos, n, box):
        eps += np.bincount(idx, weights=w * wt, minlength=n ** 3)
    return eps.reshape(n, n, n)


def density_contrast(eps, total_weight: float):
    """delta = eps n^3 / W - 1."""
    n3 = eps.size
    return eps * (n3 / total_weight) - 1.0


def gather(field, pos, n: int, box: float):
    """Interpolate grid coefficients at particle positions: sum_l f_l prod_d B3(u_d - l_d).

    ``field`` may carry leading batch axes: shape [..., n, n, n].
    Returns [..., P].
    """
    field = np.asarray(field)
    flat = field.reshape(field.shape[:-3] + (n ** 3,))
    out = None
    for idx, wt in _tap_terms(pos, n, box):
        term = flat[..., idx] * wt
        out = term if out is None else out + term
    return out


# ---------------------------------------------------------------------------
# exact piecewise-polynomial integration for connection coefficients
# ---------------------------------------------------------------------------

def _poly_mul(p, q):
    out = [Fraction(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def _poly_shift(p, s):
    """Coefficients of p(u - s) given those of p(u) (ascending powers)."""
    out = [Fraction(0)] * len(p)
    # (u - s)^k = sum_j C(k,j) u^j (-s)^(k-j)
    from math import comb
    for k, c in enumerate(p):
        for j in range(k + 1):
            out[j] += c * comb(k, j) * Fraction(-s) ** (k - j)
    return out


def _poly_integrate(p, a, b):
    tot = Fraction(0)
    for k, c in enumerate(p):
        tot += c * (Fraction(b) ** (k + 1) - Fraction(a) ** (k + 1)) / (k + 1)
    return tot


def _b3_piece(j):
    """Polynomial (ascending coefficients) of B3 on the unit interval [j, j+1]."""
    six = Fraction(6)
    if j == -2:   # (2 + u)^3 / 6
        return [Fraction(8) / six, Fraction(12) / six, Fraction(6) / six, Fraction(1) / six]
    if j == -1:   # (4 - 6u^2 - 3u^3) / 6
        return [Fraction(4) / six, Fraction(0), Fraction(-6) / six, Fraction(-3) / six]
    if j == 0:    # (4 - 6u^2 + 3u^3) / 6
        return [Fraction(4) / six, Fraction(0), Fraction(-6) / six, Fraction(3) / six]
    if j == 1:    # (2 - u)^3 / 6
        return [Fraction(8) / six, Fraction(-12) / six, Fraction(6) / six, Fraction(-1) / six]
    return [Fraction(0)]


def _b3_shifted_piece(j, s):
    """Polynomial of B3(u - s) on [j, j+1]."""
    return _poly_shift(_b3_piece(j - s), s)


def gamma_1d(s: int, t: int) -> Fraction:
    """gamma(s, t) = int B3(u) B3(u - s) B3(u - t) du, exactly (one axis of Eq. con-coeff)."""
    tot = Fraction(0)
    for j in range(-2, 2):
        p = _poly_mul(_poly_mul(_b3_piece(j), _b3_shifted_piece(j, s)), _b3_shifted_piece(j, t))
        tot += _poly_integrate(p, j, j + 1)
    return tot


def gamma_matrix() -> np.ndarray:
    """gamma(s, t) for s, t in -3..3 as a float64 [7, 7] array (index s + 3, t + 3)."""
    g = np.zeros((7, 7))
    for s in range(-3, 4):
        for t in range(-3, 4):
            g[s + 3, t + 3] = float(gamma_1d(s, t))
    return g


def b7_samples() -> dict:
    """Autocorrelation of B3 at integer lags, exactly: int B3(u) B3(u - s) du, s in -3..3."""
    out = {}
    for s in range(-3, 4):
        tot = Fraction(0)
        for j in range(-2, 2):
            tot += _poly_integrate(_poly_mul(_b3_piece(j), _b3_shifted_piece(j, s)), j, j + 1)
        out[s] = tot
    return out


def b7_hat(theta) -> np.ndarray:
    """Discrete-time Fourier transform of the B3 autocorrelation samples, sum_s B7(s) e^{-i theta s}."""
    smp = b7_samples()
    theta = np.asarray(theta, dtype=np.float64)
    out = np.full(theta.shape, float(smp[0]))
    for s in range(1, 4):
        out = out + 2.0 * float(smp[s]) * np.cos(s * theta)
    return out
