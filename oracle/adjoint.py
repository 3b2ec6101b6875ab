"""Gradients of J = sum_l sum_{b1,b2} lam_l[b1,b2] zeta_l[b1,b2] (float64).

The paper has no gradient; these are the chain rule applied to the nodal
summation of ``estimator`` and to the deposit of ``basis``.

Nodal form.  With a_{lm,b} = ifftn(fftn(delta) K_{lm,b}) linear in delta and
lam^s = (lam + lam^T) / 2,

  dJ/ddelta_y = (4 pi / n^3) [ sum_{l,m} sum_{b1,b2} lam_l[b1,b2] Re(a_{b1} conj(a_{b2}))(y)
                               + 2 Re fftn( sum_{l,m,b} K_{lm,b} ifftn(c_{lm,b}) )(y) ],
  c_{lm,b}(x) = delta_x sum_{b'} lam^s_l[b,b'] conj(a_{lm,b'}(x)),

with m over -l..l: the first term is the explicit dependence on the primary
vertex, the second the transpose of the filter-and-transform map applied to
the secondary vertices.

Deposit.  delta_l = eps_l n^3 / W - 1 with eps_l = sum_i w_i B_i(l) and
W = sum_i w_i, so for a grid gradient g = dJ/ddelta,

  dJ/dw_i = (n^3 / W) sum_l B_i(l) g_l - (n^3 / W^2) sum_l eps_l g_l.
"""
from __future__ import annotations

import numpy as np

from . import basis
from .estimator import Plan, fields, FOUR_PI

__all__ = ["zeta_nodal_grad", "deposit_weight_grad", "zeta_nodal_objective"]


def zeta_nodal_objective(plan: Plan, delta, lam) -> float:
    """J = sum_l <lam_l, zeta_l> for the nodal form (used by finite differences)."""
    from .estimator import zeta_nodal
    return float(np.sum(np.asarray(lam) * zeta_nodal(plan, delta)))


def zeta_nodal_grad(plan: Plan, delta, lam, ls=None, bins=None) -> np.ndarray:
    """dJ/ddelta for the nodal form.

    lam has shape [lmax+1, nbins, nbins]; with ``ls`` / ``bins`` only those
    multipoles and bins enter J (lam then indexed [len(ls), len(bins), len(bins)]).
    """
    delta = np.asarray(delta, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    n = plan.n
    dhat = np.fft.fftn(delta)
    direct = np.zeros_like(delta)
    acc = np.zeros(delta.shape, dtype=np.complex128)
    bl = plan.bins(bins)
    for li, l in enumerate(plan.ls(ls)):
        lam_l = lam[li]
        lam_s = 0.5 * (lam_l + lam_l.T)
        for m in range(-l, l + 1):
            A = fields(plan, dhat, l, m, bl)                      # [nb, n, n, n]
            direct += np.einsum("ij,ixyz,jxyz->xyz", lam_l, A, A.conj()).real
            C = delta[None] * np.einsum("ij,jxyz->ixyz", lam_s, A.conj())
            yc = plan.ylm_conj_grid(l, m)
            for bi, b in enumerate(bl):
                acc += plan.kernel(l, m, b, yc) * np.fft.ifftn(C[bi])
    grad = direct + 2.0 * np.fft.fftn(acc).real
    return grad * (FOUR_PI / n ** 3)


def deposit_weight_grad(pos, w, n: int, box: float, g) -> np.ndarray:
    """dJ/dw_i given g = dJ/ddelta on the grid (delta from the deposit of (pos, w))."""
    w = np.ones(len(pos)) if w is None else np.asarray(w, dtype=np.float64)
    W = w.sum()
    eps = basis.deposit(pos, w, n, box)
    g = np.asarray(g, dtype=np.float64)
    interp = basis.gather(g, pos, n, box)
    return (n ** 3 / W) * interp - (n ** 3 / W ** 2) * float(np.sum(eps * g))
