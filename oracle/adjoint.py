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

Particle form (primary on the catalogue, volume mean subtracted).  With
atilde = gather(a) at the particles, F_J(u) = sum_{l,m} sum_{b1,b2}
lam_l[b1,b2] atilde_{b1}(u) conj(atilde_{b2}(u)) and
H(q) = B7hat(q) sum_l (2l+1) sum_{b1,b2} lam_l[b1,b2] jbar_{b1} jbar_{b2}
(zero on the Nyquist planes), the dependence on delta at fixed primary
weights is

  dJ/ddelta = (4 pi / n^3) 2 Re fftn( sum_{l,m,b} K_{lm,b} ifftn(c_{lm,b}) )
              - (2 / n^3) Re ifftn(H dhat),
  c_{lm,b} = n^3 scatter_i[ (w_i / W) sum_{b'} lam^s_l[b,b'] conj(atilde_{lm,b'}(u_i)) ],

the scatter being the transpose of the gather (the deposit's stencil).  The
weights enter through delta (deposit, below) and through the primary:

  dJ/dw_i += 4 pi [ F_J(u_i) / W - sum_j w_j F_J(u_j) / W^2 ].

Grid summation with connection coefficients.  zeta_l is the bilinear form
sum lam a_{b1}^T M conj(a_{b2}) with the symmetric operator
M(x, y) = sum_w delta_w Gamma(x - w, y - w); with G_Delta(x) =
sum_s delta(x - s) Gamma(s, s + Delta) (the stencil fields of
estimator.zeta_gamma),

  dJ/ddelta_x = (4 pi / n^3) [ Re sum_{l,m} sum_{s,t} Gamma(s,t) sum_{b1,b2} lam[b1,b2] a_{b1}(x+s) conj(a_{b2}(x+t))
                               + 2 Re fftn( sum_{l,m,b} K_{lm,b} ifftn(c_{lm,b}) )(x) ],
  c_{lm,b}(x) = sum_Delta G_Delta(x) V_b(x + Delta),  V_b = sum_{b'} lam^s[b,b'] conj(a_{b'}):

the nodal formula with every pointwise product replaced by its Gamma
stencil (the nodal form is Gamma(s,t) = delta_{s0} delta_{t0}).

Deposit.  delta_l = eps_l n^3 / W - 1 with eps_l = sum_i w_i B_i(l) and
W = sum_i w_i, so for a grid gradient g = dJ/ddelta,

  dJ/dw_i = (n^3 / W) sum_l B_i(l) g_l - (n^3 / W^2) sum_l eps_l g_l.
"""
from __future__ import annotations

import numpy as np

from . import basis
from .estimator import Plan, fields, FOUR_PI, BASES

__all__ = ["zeta_nodal_grad", "deposit_weight_grad", "zeta_nodal_objective",
           "zeta_particle_objective", "zeta_particle_grad", "zeta_gamma_objective", "zeta_gamma_grad"]


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
    prim = plan.primary(delta)
    direct = np.zeros_like(delta)
    acc = np.zeros(delta.shape, dtype=np.complex128)
    bl = plan.bins(bins)
    for li, l in enumerate(plan.ls(ls)):
        lam_l = lam[li]
        lam_s = 0.5 * (lam_l + lam_l.T)
        for m in range(-l, l + 1):
            A = fields(plan, dhat, l, m, bl)                      # [nb, n, n, n]
            direct += np.einsum("ij,ixyz,jxyz->xyz", lam_l, A, A.conj()).real
            C = prim[None] * np.einsum("ij,jxyz->ixyz", lam_s, A.conj())
            yc = plan.ylm_conj_grid(l, m)
            for bi, b in enumerate(bl):
                acc += plan.kernel(l, m, b, yc) * np.fft.ifftn(C[bi])
    # the primary is delta filtered by a real, even window: its transpose is the same filter
    grad = plan.primary(direct) + 2.0 * np.fft.fftn(acc).real
    return grad * (FOUR_PI / n ** 3)


def deposit_weight_grad(pos, w, n: int, box: float, g, basis_name: str = "b3") -> np.ndarray:
    """dJ/dw_i given g = dJ/ddelta on the grid (delta from the deposit of (pos, w))."""
    w = np.ones(len(pos)) if w is None else np.asarray(w, dtype=np.float64)
    W = w.sum()
    B = BASES[basis_name]
    eps = B.deposit(pos, w, n, box)
    g = np.asarray(g, dtype=np.float64)
    interp = B.gather(g, pos, n, box)
    return (n ** 3 / W) * interp - (n ** 3 / W ** 2) * float(np.sum(eps * g))


def zeta_particle_objective(plan: Plan, pos, w, lam) -> float:
    """J = sum_l <lam_l, zeta_l> for the particle form (used by finite differences)."""
    from .estimator import zeta_particle
    return float(np.sum(np.asarray(lam) * zeta_particle(plan, pos, w)))


def _scatter(vals, pos, n: int, box: float, B=basis) -> np.ndarray:
    """Transpose of the basis' gather for complex per-particle values: sum_i v_i B(u_i - l)."""
    return (B.deposit(pos, vals.real, n, box) + 1j * B.deposit(pos, vals.imag, n, box))


def zeta_particle_grad(plan: Plan, pos, w, lam, ls=None, bins=None):
    """(dJ/ddelta at fixed primary weights, dJ/dw) for the particle form.

    lam has shape [lmax+1, nbins, nbins], or [len(ls), len(bins), len(bins)]
    with ``ls`` / ``bins``.
    """
    from .estimator import fields
    n, box = plan.n, plan.box
    w = np.ones(len(pos)) if w is None else np.asarray(w, dtype=np.float64)
    W = w.sum()
    lam = np.asarray(lam, dtype=np.float64)
    delta = basis.density_contrast(plan.B.deposit(pos, w, n, box), W)
    dhat = np.fft.fftn(delta)
    acc = np.zeros(delta.shape, dtype=np.complex128)
    FJ = np.zeros(len(pos))
    bl = plan.bins(bins)
    b7 = plan.autocorr_hat_axis()
    H = np.zeros(delta.shape)
    for li, l in enumerate(plan.ls(ls)):
        lam_l = lam[li]
        lam_s = 0.5 * (lam_l + lam_l.T)
        J = np.stack([plan.jbar_grid(l, b) for b in bl])               # [nb, n, n, n]
        H += (2 * l + 1) * np.einsum("ij,ixyz,jxyz->xyz", lam_l, J, J)
        for m in range(-l, l + 1):
            A = fields(plan, dhat, l, m, bl)
            At = plan.B.gather(A, pos, n, box)                         # [nb, P]
            FJ += np.einsum("ij,ip,jp->p", lam_l, At, At.conj()).real
            S = (w / W)[None, :] * (lam_s @ At.conj())
            yc = plan.ylm_conj_grid(l, m)
            for bi, b in enumerate(bl):
                c = float(n) ** 3 * _scatter(S[bi], pos, n, box, plan.B)
                acc += plan.kernel(l, m, b, yc) * np.fft.ifftn(c)
    H *= b7[:, None, None] * b7[None, :, None] * b7[None, None, :] * plan.phi_hat_grid() ** 2
    H[plan.nyquist] = 0.0
    g = (FOUR_PI / n ** 3) * 2.0 * np.fft.fftn(acc).real - (2.0 / n ** 3) * np.fft.ifftn(H * dhat).real
    dw = deposit_weight_grad(pos, w, n, box, g, plan.basis) + FOUR_PI * (FJ / W - float(np.dot(w, FJ)) / W ** 2)
    return g, dw


def zeta_gamma_objective(plan: Plan, delta, lam) -> float:
    """J = sum_l <lam_l, zeta_l> for the grid-Gamma form (used by finite differences)."""
    from .estimator import zeta_gamma
    return float(np.sum(np.asarray(lam) * zeta_gamma(plan, delta)))


def _gamma_stencil_field_t(q, gmat, shift):
    """Transpose in delta of G_Delta(y) = sum_s delta(y - s) Gamma(s, s + Delta):
    sum_s q(x + s) Gamma(s, s + Delta), per axis (Gamma separable).  No reflection symmetry of
    Gamma is assumed (the Daubechies-4 scaling function is not symmetric)."""
    g = q
    for axis in range(3):
        d = shift[axis]
        acc = np.zeros_like(g)
        for s in range(-3, 4):
            t = s + d
            if -3 <= t <= 3:
                c = gmat[s + 3, t + 3]
                if c != 0.0:
                    acc = acc + c * np.roll(g, -s, axis=axis)       # g(x + s)
        g = acc
    return g


def zeta_gamma_grad(plan: Plan, delta, lam, ls=None, bins=None) -> np.ndarray:
    """dJ/ddelta for the grid summation with connection coefficients.

    lam has shape [lmax+1, nbins, nbins], or [len(ls), len(bins), len(bins)]
    with ``ls`` / ``bins``.
    """
    from .estimator import _gamma_stencil_field
    delta = np.asarray(delta, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    n = plan.n
    dhat = np.fft.fftn(delta)
    gmat = plan.B.gamma_matrix()
    shifts = [(dx, dy, dz) for dx in range(-3, 4) for dy in range(-3, 4) for dz in range(-3, 4)]
    gfields = {sh: _gamma_stencil_field(plan.primary(delta), gmat, sh) for sh in shifts}
    direct = np.zeros(delta.shape, dtype=np.complex128)
    acc = np.zeros(delta.shape, dtype=np.complex128)
    bl = plan.bins(bins)
    for li, l in enumerate(plan.ls(ls)):
        lam_l = lam[li]
        lam_s = 0.5 * (lam_l + lam_l.T)
        for m in range(-l, l + 1):
            A = fields(plan, dhat, l, m, bl)                                 # [nb, n, n, n]
            V = np.einsum("ij,jxyz->ixyz", lam_s, A.conj())
            C = np.zeros_like(A)
            for sh, G in gfields.items():
                rolled = (-sh[0], -sh[1], -sh[2])
                Ash = np.roll(A, shift=rolled, axis=(1, 2, 3))              # a(x + Delta)
                Q = np.einsum("ij,ixyz,jxyz->xyz", lam_l, A, Ash.conj())     # sum lam a_b1(y) conj(a_b2(y + Delta))
                direct += _gamma_stencil_field_t(Q, gmat, sh)
                C += G[None] * np.roll(V, shift=rolled, axis=(1, 2, 3))      # G_Delta(x) V_b(x + Delta)
            yc = plan.ylm_conj_grid(l, m)
            for bi, b in enumerate(bl):
                acc += plan.kernel(l, m, b, yc) * np.fft.ifftn(C[bi])
    grad = plan.primary(direct.real) + 2.0 * np.fft.fftn(acc).real
    return grad * (FOUR_PI / n ** 3)
