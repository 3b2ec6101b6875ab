"""Daubechies-4 scaling-function basis: tabulation, deposit, interpolation,
autocorrelation, power spectrum and connection coefficients.

The paper's runs use the Daubechies scaling function of genus D_g = 4 (four
filter taps, support D_sup = D_g - 1 = 3 cells; Sec. 2.2, the complexity
remark after the grid-summation equations, and Sec. 3, the basis paragraph).
It is defined by the two-scale relation

    phi(x) = sqrt(2) sum_{k=0}^{3} h_k phi(2x - k),   int phi = 1,

with the orthonormal filter h = [1 + s, 3 + s, 3 - s, 1 - s] / (4 sqrt 2),
s = sqrt 3.  phi has no closed form; this module

  * finds phi at the integers as the eigenvector of eigenvalue 1 of the
    two-scale relation restricted to x = 1, 2 (phi(0) = phi(3) = 0), scaled
    to phi(1) + phi(2) = 1 (partition of unity), then fills the dyadic points
    k / 2^r level by level from the same relation (the cascade algorithm);
  * takes as the basis function the linear interpolant phi_R of the values at
    level R = LEVEL (spacing 2^-R), the definition both the deposit and the
    interpolation use;
  * indexes the basis so that node l carries phi(u - l + 1) (support
    [l - 1, l + 2] in cell units u = x / a): the stencil of a particle is then
    the four nodes floor(u) - 1 .. floor(u) + 2 as for the cubic B-spline, the
    last weight phi(f - 1) being zero (f = u - floor(u)).  A whole-cell
    relabelling of the nodes leaves every estimator unchanged.

The power spectrum |phi_hat(w)|^2 follows the infinite product
phi_hat(w) = prod_{j>=1} m0(w / 2^j), m0(w) = 2^-1/2 sum_k h_k e^{-i k w};
the connection coefficients gamma(s, t) = int phi(x) phi(x - s) phi(x - t) dx
(Eq. con-coeff, one axis) solve the linear system the two-scale relation
imposes on them, normalised by sum_{s,t} gamma = int phi = 1.  Both are of the
exact scaling function; the autocorrelation samples used for the particle
form's volume mean are those of phi_R, integrated exactly (products of
piecewise-linear functions).
"""
from __future__ import annotations

import numpy as np

from . import basis as _b3

__all__ = ["FILTER", "LEVEL", "integer_values", "table", "phi", "taps", "deposit", "density_contrast", "gather",
           "autocorr_samples", "autocorr_hat", "phi_hat_sq", "phi_hat_axis", "gamma_matrix"]

_S3 = np.sqrt(3.0)
FILTER = np.array([1.0 + _S3, 3.0 + _S3, 3.0 - _S3, 1.0 - _S3]) / (4.0 * np.sqrt(2.0))
LEVEL = 10
SUPPORT = 3

density_contrast = _b3.density_contrast


def integer_values() -> np.ndarray:
    """[phi(0), phi(1), phi(2), phi(3)]: the two-scale relation at x = 1, 2 is
    phi(k) = sqrt2 sum_j h_j phi(2k - j), a 2x2 eigenproblem with eigenvalue 1."""
    r2 = np.sqrt(2.0)
    # phi(1) = sqrt2 (h1 phi(1) + h0 phi(2)),  phi(2) = sqrt2 (h3 phi(1) + h2 phi(2))
    M = r2 * np.array([[FILTER[1], FILTER[0]], [FILTER[3], FILTER[2]]])
    w, v = np.linalg.eig(M)
    k = int(np.argmin(np.abs(w - 1.0)))
    vec = np.real(v[:, k])
    vec = vec / vec.sum()
    return np.array([0.0, vec[0], vec[1], 0.0])


def table(level: int = LEVEL) -> np.ndarray:
    """phi at x = i / 2^level, i = 0 .. 3 2^level, by the cascade algorithm."""
    r2 = np.sqrt(2.0)
    cur = integer_values()
    for r in range(1, level + 1):
        nxt = np.zeros(SUPPORT * 2 ** r + 1)
        nxt[0::2] = cur                               # points already known at level r - 1
        half = 2 ** (r - 1)
        for i in range(1, nxt.size, 2):
            # 2x - j = (i - j 2^(r-1)) / 2^(r-1): index i - j half of level r - 1
            acc = 0.0
            for j in range(4):
                idx = i - j * half
                if 0 <= idx < cur.size:
                    acc += FILTER[j] * cur[idx]
            nxt[i] = r2 * acc
        cur = nxt
    return cur


_TABLE = None


def _tab() -> np.ndarray:
    global _TABLE
    if _TABLE is None:
        _TABLE = table(LEVEL)
    return _TABLE


def phi(x) -> np.ndarray:
    """phi_R(x): linear interpolation of the level-R dyadic values, zero outside [0, 3]."""
    t = _tab()
    x = np.asarray(x, dtype=np.float64)
    s = x * float(2 ** LEVEL)
    i0 = np.floor(s)
    frac = s - i0
    i0 = i0.astype(np.int64)
    inside = (x >= 0.0) & (x < SUPPORT)
    ic = np.clip(i0, 0, t.size - 2)
    val = (1.0 - frac) * t[ic] + frac * t[ic + 1]
    return np.where(inside, val, 0.0)


def taps(pos, n: int, box: float):
    """Per-particle stencil: first node floor(u) - 1 and the weights phi_R(u - l + 1) of the
    nodes l = floor(u) - 1 .. floor(u) + 2 per axis.  Returns (base [P,3], weights [P,3,4])."""
    u = np.asarray(pos, dtype=np.float64) * (float(n) / float(box))
    fl = np.floor(u)
    base = fl.astype(np.int64) - 1
    offs = np.arange(4, dtype=np.float64)
    wts = phi(u[:, :, None] - (base[:, :, None].astype(np.float64) + offs) + 1.0)
    return base, wts


def _tap_terms(pos, n, box):
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
    """Basis coefficients eps_l = sum_i w_i prod_d phi_R(u_{i,d} - l_d + 1)."""
    w = np.ones(len(pos)) if w is None else np.asarray(w, dtype=np.float64)
    eps = np.zeros(n ** 3)
    for idx, wt in _tap_terms(pos, n, box):
        eps += np.bincount(idx, weights=w * wt, minlength=n ** 3)
    return eps.reshape(n, n, n)


def gather(field, pos, n: int, box: float):
    """sum_l f_l prod_d phi_R(u_d - l_d + 1) at the particle positions; field [..., n, n, n] -> [..., P]."""
    field = np.asarray(field)
    flat = field.reshape(field.shape[:-3] + (n ** 3,))
    out = None
    for idx, wt in _tap_terms(pos, n, box):
        term = flat[..., idx] * wt
        out = term if out is None else out + term
    return out


def autocorr_samples() -> np.ndarray:
    """A(s) = int phi_R(x) phi_R(x - s) dx for s = 0, 1, 2 (A(-s) = A(s), zero beyond),
    exactly: on each interval of the level-R grid both factors are linear."""
    t = _tab()
    h = 1.0 / 2 ** LEVEL
    out = np.zeros(3)
    for s in range(3):
        sh = s * 2 ** LEVEL
        a0 = t[sh:-1]                     # phi_R on [x_i, x_i+1], x_i >= s
        a1 = t[sh + 1:]
        b0 = t[:t.size - 1 - sh]          # phi_R(x - s) at the same points
        b1 = t[1:t.size - sh]
        out[s] = np.sum(h / 6.0 * (2.0 * a0 * b0 + a0 * b1 + a1 * b0 + 2.0 * a1 * b1))
    return out


def autocorr_hat(theta) -> np.ndarray:
    """sum_s A(s) e^{-i theta s} = A0 + 2 A1 cos(theta) + 2 A2 cos(2 theta)."""
    a = autocorr_samples()
    theta = np.asarray(theta, dtype=np.float64)
    return a[0] + 2.0 * a[1] * np.cos(theta) + 2.0 * a[2] * np.cos(2.0 * theta)


def phi_hat_sq(w, terms: int = 64) -> np.ndarray:
    """|phi_hat(w)|^2 = prod_{j=1}^{terms} |m0(w / 2^j)|^2, m0(w) = 2^-1/2 sum_k h_k e^{-i k w}
    (the factors reach 1 to double precision long before 64 terms)."""
    w = np.asarray(w, dtype=np.float64)
    out = np.ones_like(w)
    k = np.arange(4)
    for j in range(1, terms + 1):
        xi = w / 2.0 ** j
        m0 = (FILTER[None, :] * np.exp(-1j * k[None, :] * xi.reshape(-1, 1))).sum(-1) / np.sqrt(2.0)
        out = out * (np.abs(m0) ** 2).reshape(w.shape)
    return out


def phi_hat_axis(n: int) -> np.ndarray:
    """|phi_hat(2 pi q / n)|^2 over the DFT frequencies q of one axis (fftfreq order)."""
    q = np.fft.fftfreq(n, d=1.0 / n)
    return phi_hat_sq(2.0 * np.pi * q / n)


def gamma_matrix() -> np.ndarray:
    """gamma(s, t) for s, t in -3..3 as [7, 7] (index s + 3, t + 3); zero unless |s|, |t|, |s - t| <= 2.

    The two-scale relation gives gamma(s, t) = sqrt2 sum_{k,l,m} h_k h_l h_m gamma(2s + l - k, 2t + m - k);
    on the 19 admissible (s, t) this is gamma = T gamma, solved as the null vector of (T - I)
    together with sum_{s,t} gamma(s, t) = 1."""
    pairs = [(s, t) for s in range(-2, 3) for t in range(-2, 3) if abs(s - t) <= 2]
    index = {p: i for i, p in enumerate(pairs)}
    T = np.zeros((len(pairs), len(pairs)))
    r2 = np.sqrt(2.0)
    for (s, t), i in index.items():
        for k in range(4):
            for l in range(4):
                for m in range(4):
                    key = (2 * s + l - k, 2 * t + m - k)
                    if key in index:
                        T[i, index[key]] += r2 * FILTER[k] * FILTER[l] * FILTER[m]
    A = np.vstack([T - np.eye(len(pairs)), np.ones((1, len(pairs)))])
    rhs = np.zeros(len(pairs) + 1)
    rhs[-1] = 1.0
    sol, *_ = np.linalg.lstsq(A, rhs, rcond=None)
    g = np.zeros((7, 7))
    for (s, t), i in index.items():
        g[s + 3, t + 3] = sol[i]
    return g
