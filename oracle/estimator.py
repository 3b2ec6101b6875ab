"""In-situ multipole 3PCF: kernel, fields and the three summation forms (float64).

Conventions (cell units; the paper's passages in brackets):

* grid: n^3 periodic nodes, cell a = box / n; density contrast delta on the
  nodes [Sec. 3, periodic-box paragraph].
* DFT: dhat(q) = sum_x delta_x exp(-2 pi i q.x / n), inverse with 1/n^3 and
  the + sign, integer frequencies q_d in [-n/2, n/2), k = 2 pi q / box
  [Sec. 2.1, Eq. trans-field-FT].
* multipole window [Sec. 2.2, Eq. 3PCF-multipole-window, with the binning
  window of the paragraph after Eq. nL-2fold]:
      K_{lm,b}(q) = i^l jbar_{l,b}(|k|) conj(Y_lm(k_hat)),
  set to zero on every Nyquist plane (any q_d = -n/2, which has no +n/2
  partner); at q = 0 the direction is immaterial because jbar_{l>0}(0) = 0
  and Y_00 is constant.
* fields a_{lm,b} = ifftn(dhat K_{lm,b})  [Eq. SFC-3PCF-vertex].
* nodal (grid) summation [Eqs. 3PCF-multipole-sum, SFC-3PCF with the
  connection coefficients lumped onto the primary node]:
      zeta_l[b1,b2] = (4 pi / n^3) sum_x delta_x sum_{m=-l}^{l} a_{lm,b1}(x) conj(a_{lm,b2}(x)).
* grid-Gamma summation [Eqs. con-coeff, SFC-3PCF]:
      zeta_l = (4 pi / n^3) sum_x delta_x sum_m sum_{s,t} Gamma_{s,t} a_{b1}(x+s) conj(a_{b2}(x+t)),
  Gamma_{s,t} = prod_d gamma(s_d, t_d) from ``basis.gamma_1d``.
* particle summation [Eq. DDD-sum-privertex and the particle sum at the end
  of Sec. 2.2], primary vertex delta = n / nbar - 1 with n the catalogue:
      zeta_l = 4 pi [ (1/W) sum_i w_i F_l(u_i) - Fbar_l ],
      F_l(u) = sum_m atilde_{lm,b1}(u) conj(atilde_{lm,b2}(u)),
  atilde the B3 interpolant of the field coefficients, Fbar_l the exact
  volume mean of F_l (it carries the "-1" of the primary's contrast).

The factor 4 pi is the product of the two sqrt(4 pi) of the paper's window;
with it zeta(r1, r2, theta) = sum_l zeta_l P_l(cos theta) [Eq. triplet-counting].
"""
from __future__ import annotations

import numpy as np

from . import special, basis, basis_d4

BASES = {"b3": basis, "d4": basis_d4}

__all__ = ["Plan", "zeta_nodal", "zeta_gamma", "zeta_gamma_quadrature",
           "zeta_particle", "fields", "volume_mean_pair", "xi", "zeta_theta", "reduced_3pcf", "xi_multipoles",
           "ss_fields", "ss_multipoles"]

FOUR_PI = 4.0 * np.pi


class Plan:
    """Grid, bins and the tabulated window functions for one configuration.

    binning "shell": r^2-weighted average of j_l over [edges[b], edges[b+1]);
    "thin": j_l(k r_b) at the mid radius (Eq. 3PCF-multipole-window).
    smoothing R > 0: the spherical top-hat window W_TH(kR) on every vertex
    (Sec. 3): both secondaries' radial window, and the grid forms' primary
    delta_p = ifftn(fftn(delta) W_TH).  phi_hat: the secondaries' window
    also carries the power spectrum of the scaling function (Eq. SFC-3PCF-vertex):
    prod_d sinc^8(pi q_d / n) for the cubic B-spline, prod_d |phi_hat(2 pi q_d / n)|^2 by the
    infinite product for Daubechies-4.  basis "b3" (cubic B-spline, module ``basis``) or "d4"
    (Daubechies-4, module ``basis_d4``): the deposit, the interpolation at particles, the volume
    mean's autocorrelation and the connection coefficients follow it.
    """

    def __init__(self, n: int, box: float, lmax: int, edges, binning: str = "shell", smoothing: float = 0.0,
                 phi_hat: bool = False, basis: str = "b3"):
        if basis not in BASES:
            raise ValueError("basis must be 'b3' or 'd4'")
        self.basis = basis
        self.B = BASES[basis]
        self.n = int(n)
        self.box = float(box)
        self.lmax = int(lmax)
        self.edges = np.asarray(edges, dtype=np.float64)
        self.nbins = self.edges.size - 1
        if binning not in ("shell", "thin"):
            raise ValueError("binning must be 'shell' or 'thin'")
        self.binning = binning
        self.smoothing = float(smoothing)
        self.phi_hat = bool(phi_hat)
        q = np.fft.fftfreq(self.n, d=1.0 / self.n)                     # integers
        self.q1 = q
        qx, qy, qz = q[:, None, None], q[None, :, None], q[None, None, :]
        q2 = (qx ** 2 + qy ** 2 + qz ** 2)
        self.kf = 2.0 * np.pi / self.box
        uniq, inv = np.unique(q2.ravel(), return_inverse=True)
        self._q2_uniq = uniq
        self._q2_inv = inv.reshape(q2.shape)
        self.kmag_uniq = self.kf * np.sqrt(uniq)
        half = -self.n // 2
        self.nyquist = (qx == half) | (qy == half) | (qz == half)
        qn = np.sqrt(q2)
        with np.errstate(invalid="ignore", divide="ignore"):
            ct = np.where(qn > 0, qz / np.where(qn > 0, qn, 1.0), 1.0)
        self.theta = np.arccos(np.clip(ct, -1.0, 1.0))
        self.phi = np.arctan2(np.broadcast_to(qy, q2.shape), np.broadcast_to(qx, q2.shape))
        self.kgrid = self.kf * qn
        self._jbar = {}

    # -- window tables ---------------------------------------------------
    def jbar_uniq(self, l: int) -> np.ndarray:
        """Radial window of a secondary vertex on the distinct |k| of the grid: [nbins, n_unique]
        (bin average or thin shell, times the top-hat window when smoothing)."""
        if l not in self._jbar:
            if self.binning == "shell":
                r = special.jbar(l, self.edges, self.kmag_uniq)
            else:
                r = special.thin_shell(l, self.edges, self.kmag_uniq)
            if self.smoothing > 0.0:
                r = r * special.tophat_window(self.kmag_uniq * self.smoothing)[None, :]
            self._jbar[l] = r
        return self._jbar[l]

    def phi_hat_grid(self) -> np.ndarray:
        """The basis power spectrum on the k-grid (ones without the phi_hat option):
        prod_d sinc^8(pi q_d / n) (B3), prod_d |phi_hat(2 pi q_d / n)|^2 (D4)."""
        if not self.phi_hat:
            return np.ones((self.n,) * 3)
        if self.basis == "d4":
            s = basis_d4.phi_hat_axis(self.n)
        else:
            h = np.pi * self.q1 / self.n
            s = np.ones_like(h)
            nz = h != 0
            s[nz] = np.sin(h[nz]) / h[nz]
            s = s ** 8
        return s[:, None, None] * s[None, :, None] * s[None, None, :]

    def autocorr_hat_axis(self) -> np.ndarray:
        """sum_s A(s) e^{-i theta s} of the basis autocorrelation samples A(s), theta = 2 pi q / n."""
        th = 2.0 * np.pi * self.q1 / self.n
        return basis.b7_hat(th) if self.basis == "b3" else basis_d4.autocorr_hat(th)

    def primary(self, delta) -> np.ndarray:
        """The grid forms' primary vertex: delta, or delta filtered by the top-hat window."""
        delta = np.asarray(delta, dtype=np.float64)
        if self.smoothing <= 0.0:
            return delta
        return np.fft.ifftn(np.fft.fftn(delta) * special.tophat_window(self.kgrid * self.smoothing)).real

    def jbar_grid(self, l: int, b: int) -> np.ndarray:
        return self.jbar_uniq(l)[b][self._q2_inv]

    def ylm_conj_grid(self, l: int, m: int) -> np.ndarray:
        return np.conj(special.ylm(l, m, self.theta, self.phi))

    def kernel(self, l: int, m: int, b: int, ylm_conj=None) -> np.ndarray:
        """K_{lm,b}(q) on the full k-grid (complex128 [n, n, n])."""
        yc = self.ylm_conj_grid(l, m) if ylm_conj is None else ylm_conj
        k = (1j ** l) * self.jbar_grid(l, b) * yc
        if self.phi_hat:
            k = k * self.phi_hat_grid()
        k[self.nyquist] = 0.0
        return k

    # -- helpers ----------------------------------------------------------
    def ls(self, ls):
        return list(range(self.lmax + 1)) if ls is None else [int(l) for l in ls]

    def bins(self, bins):
        return list(range(self.nbins)) if bins is None else [int(b) for b in bins]


def fields(plan: Plan, dhat: np.ndarray, l: int, m: int, bins=None) -> np.ndarray:
    """a_{lm,b}(x) = ifftn(dhat K_{lm,b}) for the requested bins: [nb, n, n, n] complex."""
    yc = plan.ylm_conj_grid(l, m)
    return np.stack([np.fft.ifftn(dhat * plan.kernel(l, m, b, yc)) for b in plan.bins(bins)])


def _pair_sum(A: np.ndarray, weight: np.ndarray) -> np.ndarray:
    """sum_x weight_x A_{b1}(x) conj(A_{b2}(x)) as an [nb, nb] complex matrix."""
    nb = A.shape[0]
    flat = A.reshape(nb, -1)
    return (flat * weight.ravel()) @ flat.conj().T


def zeta_nodal(plan: Plan, delta: np.ndarray, ls=None, bins=None) -> np.ndarray:
    """Nodal grid summation; returns real zeta [len(ls), nb, nb].

    The imaginary part, which cancels between m and -m, is checked to be at
    rounding level before it is dropped.
    """
    delta = np.asarray(delta, dtype=np.float64)
    dhat = np.fft.fftn(delta)
    prim = plan.primary(delta)
    out = []
    for l in plan.ls(ls):
        z = 0.0
        for m in range(-l, l + 1):
            z = z + _pair_sum(fields(plan, dhat, l, m, bins), prim)
        z = z * (FOUR_PI / plan.n ** 3)
        _check_real(z)
        out.append(z.real)
    return np.array(out)


def _check_real(z, floor: float = 0.0):
    """The m-sum must be real up to rounding; ``floor`` is the size of the summed
    terms for sums that cancel exactly (then |z| itself is rounding noise)."""
    scale = max(np.abs(z).max(), floor, 1e-300)
    if np.abs(z.imag).max() > 1e-9 * scale:
        raise AssertionError(f"zeta has an imaginary part {np.abs(z.imag).max():.3e} (scale {scale:.3e})")


# ---------------------------------------------------------------------------
# grid summation with connection coefficients
# ---------------------------------------------------------------------------

def _gamma_stencil_field(delta, gmat, shift):
    """G_Delta(y) = sum_s delta(y - s) Gamma(s, s + Delta), Gamma = prod_d gamma (separable)."""
    g = delta
    for axis in range(3):
        d = shift[axis]
        acc = np.zeros_like(g)
        for s in range(-3, 4):
            t = s + d
            if -3 <= t <= 3:
                c = gmat[s + 3, t + 3]
                if c != 0.0:
                    acc = acc + c * np.roll(g, s, axis=axis)        # g(y - s)
        g = acc
    return g


def zeta_gamma(plan: Plan, delta: np.ndarray, ls=None, bins=None) -> np.ndarray:
    """Grid summation with the connection coefficients of B3 (Eq. SFC-3PCF).

    The double sum over (s, t) is re-indexed by Delta = t - s:
        sum_x delta_x sum_{s,t} Gamma(s,t) a(x+s) b*(x+t)
      = sum_Delta sum_y G_Delta(y) a(y) b*(y + Delta),
    with G_Delta(y) = sum_s delta(y - s) Gamma(s, s + Delta).
    """
    delta = np.asarray(delta, dtype=np.float64)
    dhat = np.fft.fftn(delta)
    gmat = plan.B.gamma_matrix()
    shifts = [(dx, dy, dz) for dx in range(-3, 4) for dy in range(-3, 4) for dz in range(-3, 4)]
    prim = plan.primary(delta)
    gfields = {sh: _gamma_stencil_field(prim, gmat, sh) for sh in shifts}
    out = []
    for l in plan.ls(ls):
        z = 0.0
        for m in range(-l, l + 1):
            A = fields(plan, dhat, l, m, bins)
            nb = A.shape[0]
            flat = A.reshape(nb, -1)
            for sh, G in gfields.items():
                Bs = np.roll(A, shift=(-sh[0], -sh[1], -sh[2]), axis=(1, 2, 3)).reshape(nb, -1)
                z = z + (flat * G.ravel()) @ Bs.conj().T
        z = z * (FOUR_PI / plan.n ** 3)
        _check_real(z)
        out.append(z.real)
    return np.array(out)


def _node_interp_matrix(n: int, order: int = 5):
    """Values of B3-interpolated data at Gauss-Legendre nodes of every cell (one axis).

    Returns (M [order*n, n], weights [order*n]) with node j of cell c at
    u = c + (xi_j + 1) / 2.
    """
    xi, wi = special.gauss_legendre(order)
    u = (np.arange(n)[:, None] + 0.5 * (xi[None, :] + 1.0)).ravel()
    M = np.zeros((u.size, n))
    for l in range(n):
        for wrap in (-n, 0, n):
            M[:, l] += basis.b3(u - (l + wrap))
    return M, np.tile(0.5 * wi, n)


def zeta_gamma_quadrature(plan: Plan, delta: np.ndarray, ls=None, bins=None) -> np.ndarray:
    """Grid-Gamma summation evaluated as the integral of three B3 interpolants.

    sum_{x,s,t} delta_x Gamma(s,t) a(x+s) b*(x+t) = int delta_B(u) a_B(u) b_B*(u) d^3u,
    with f_B(u) = sum_l f_l B3(u - l); the integrand is a degree-9 polynomial
    per axis on each cell, which 5-point Gauss-Legendre integrates exactly.
    Cubic B-spline only (the Daubechies-4 products are not piecewise polynomial).
    """
    if plan.basis != "b3":
        raise ValueError("the quadrature form needs the cubic B-spline basis")
    n = plan.n
    M, wq = _node_interp_matrix(n)

    def interp(f):
        g = np.tensordot(M, f, axes=(1, 0))                 # axis 0
        g = np.tensordot(M, g, axes=(1, 1)).transpose(1, 0, 2)
        g = np.tensordot(M, g, axes=(1, 2)).transpose(1, 2, 0)
        return g

    delta = np.asarray(delta, dtype=np.float64)
    dhat = np.fft.fftn(delta)
    W = wq[:, None, None] * wq[None, :, None] * wq[None, None, :]
    wd = W * interp(plan.primary(delta))
    out = []
    for l in plan.ls(ls):
        z = 0.0
        for m in range(-l, l + 1):
            A = fields(plan, dhat, l, m, bins)
            At = np.stack([interp(a) for a in A])
            z = z + _pair_sum(At, wd)
        z = z * (FOUR_PI / n ** 3)
        _check_real(z)
        out.append(z.real)
    return np.array(out)


# ---------------------------------------------------------------------------
# particle summation
# ---------------------------------------------------------------------------

def volume_mean_pair(plan: Plan, dhat: np.ndarray, l: int, bins=None) -> np.ndarray:
    """Fbar_l[b1,b2] = (1/n^3) int sum_m atilde_{b1} conj(atilde_{b2}) d^3u.

    By Parseval on the periodic interpolants (aliases folded into the
    autocorrelation of the basis) and the addition theorem
    sum_m conj(Y_lm) Y_lm = (2l+1)/(4 pi):
        Fbar_l = (2l+1) / (4 pi n^6) sum_q |dhat|^2 Ahat(q) jbar_{b1} jbar_{b2},
    Ahat = prod_d sum_s A(s) e^{-i theta_d s} (B7hat for the cubic B-spline),
    Nyquist planes excluded (the window vanishes there).
    """
    n = plan.n
    b7 = plan.autocorr_hat_axis()
    b7g = b7[:, None, None] * b7[None, :, None] * b7[None, None, :]
    p = np.abs(dhat) ** 2 * b7g * plan.phi_hat_grid() ** 2
    p[plan.nyquist] = 0.0
    bl = plan.bins(bins)
    J = np.stack([plan.jbar_grid(l, b).ravel() for b in bl])
    return (2 * l + 1) / (FOUR_PI * float(n) ** 6) * ((J * p.ravel()) @ J.T)


def zeta_particle(plan: Plan, pos, w, ls=None, bins=None, mode: str = "delta", delta=None) -> np.ndarray:
    """Particle summation over the catalogue (primary vertex on the particles).

    mode "delta": secondaries from delta = n/nbar - 1 and primary n/nbar - 1
                  (volume mean of F subtracted);
    mode "ddd":   secondaries from n/nbar and primary n/nbar (plain triplet
                  counting, the q = 0 mode kept, nothing subtracted).
    ``delta`` (mode "delta" only) replaces the deposit of the catalogue as the
    secondaries' grid, the primary staying on the weighted particles.
    """
    n, box = plan.n, plan.box
    w = np.ones(len(pos)) if w is None else np.asarray(w, dtype=np.float64)
    W = w.sum()
    if delta is not None:
        if mode != "delta":
            raise ValueError("an explicit delta needs mode 'delta'")
        src = np.asarray(delta, dtype=np.float64)
    else:
        eps = plan.B.deposit(pos, w, n, box)
        rho = eps * (n ** 3 / W)
        src = rho - 1.0 if mode == "delta" else rho
    dhat = np.fft.fftn(src)
    out = []
    for l in plan.ls(ls):
        z = 0.0
        floor = 0.0
        for m in range(-l, l + 1):
            A = fields(plan, dhat, l, m, bins)
            At = plan.B.gather(A, pos, n, box)                # [nb, P]
            z = z + (At * (w / W)) @ At.conj().T
            floor += float(np.abs(A).max()) ** 2
        _check_real(z, floor)
        z = z.real
        if mode == "delta":
            z = z - volume_mean_pair(plan, dhat, l, bins)
        out.append(FOUR_PI * z)
    return np.array(out)


# ---------------------------------------------------------------------------
# two-point function and the reconstructed 3PCF
# ---------------------------------------------------------------------------

def xi(plan: Plan, delta, radii) -> np.ndarray:
    """xi(r) = n^-3 sum_x delta_p(x) (W_r o delta)(x) for each radius [Sec. 2.1, Eqs. pair-counting and
    window-sphshell]: the secondary filtered by the thin shell j_0(k r) (times the top-hat and phi-hat
    windows of the plan, Nyquist planes zeroed as for the 3PCF's secondaries), the primary delta_p the
    grid forms' primary (plan.primary)."""
    delta = np.asarray(delta, dtype=np.float64)
    dhat = np.fft.fftn(delta)
    prim = plan.primary(delta)
    w = plan.phi_hat_grid()
    if plan.smoothing > 0.0:
        w = w * special.tophat_window(plan.kgrid * plan.smoothing)
    out = []
    for r in np.asarray(radii, dtype=np.float64).ravel():
        k = w * special.sph_jn(0, plan.kgrid * r)
        k[plan.nyquist] = 0.0
        sec = np.fft.ifftn(dhat * k)
        out.append(float(np.mean(prim * sec.real)))
    return np.array(out)


def zeta_theta(zeta, mu, lt: int) -> np.ndarray:
    """zeta(r1, r2, theta) = sum_{l=0}^{lt} zeta_l(r1, r2) P_l(cos theta) [Eq. triplet-counting],
    the multipole sum truncated at lt.  zeta [L+1, nb, nb] -> [nb, nb, len(mu)]."""
    zeta = np.asarray(zeta, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64).ravel()
    out = np.zeros(zeta.shape[1:] + mu.shape)
    for l in range(lt + 1):
        out += zeta[l][:, :, None] * special.legendre(l, mu)[None, None, :]
    return out


def reduced_3pcf(plan: Plan, delta, zeta, mu, lt: int) -> np.ndarray:
    """Q = zeta(theta) / [xi(r1) xi(r2) + xi(r2) xi(r3) + xi(r3) xi(r1)] [Eq. Q-factor], with the
    triangle's third side r3^2 = r1^2 + r2^2 - 2 r1 r2 cos theta and r_b the bins' mid radii."""
    mu = np.asarray(mu, dtype=np.float64).ravel()
    rb = 0.5 * (plan.edges[:-1] + plan.edges[1:])
    zt = zeta_theta(zeta, mu, lt)
    xb = xi(plan, delta, rb)
    nb = plan.nbins
    q = np.zeros_like(zt)
    for i in range(nb):
        for j in range(nb):
            r3 = np.sqrt(np.maximum(rb[i] ** 2 + rb[j] ** 2 - 2.0 * rb[i] * rb[j] * mu, 0.0))
            x3 = xi(plan, delta, r3)
            q[i, j] = zt[i, j] / (xb[i] * xb[j] + xb[j] * x3 + x3 * xb[i])
    return q


def xi_multipoles(plan: Plan, delta, radii, ells) -> np.ndarray:
    """Line-of-sight multipoles of the two-point function [Sec. 2.1, Eqs. DD-multipole and
    DD-windowfunction], the line of sight along the grid's z axis:

        xi_ell(r) = n^-3 sum_x delta_p(x) (W^ell_r o delta)(x),
        W^ell_r(k) = (2 ell + 1) i^ell j_ell(k r) P_ell(cos theta_k),

    so that the azimuthal average of the pair correlation at separation r and polar angle theta_r
    is sum_ell xi_ell(r) P_ell(cos theta_r).  The plan's top-hat and phi-hat windows apply as in
    ``xi`` (Nyquist planes zeroed).  Returns [len(ells), len(radii)] (real part; the imaginary
    part vanishes for real delta)."""
    delta = np.asarray(delta, dtype=np.float64)
    dhat = np.fft.fftn(delta)
    prim = plan.primary(delta)
    w = plan.phi_hat_grid()
    if plan.smoothing > 0.0:
        w = w * special.tophat_window(plan.kgrid * plan.smoothing)
    mu = np.cos(plan.theta)
    out = np.zeros((len(ells), np.size(radii)))
    for i, ell in enumerate(ells):
        ang = (2 * ell + 1) * (1j ** ell) * special.legendre(ell, mu)
        for j, r in enumerate(np.asarray(radii, dtype=np.float64).ravel()):
            k = w * ang * special.sph_jn(ell, plan.kgrid * r)
            k[plan.nyquist] = 0.0
            sec = np.fft.ifftn(dhat * k)
            out[i, j] = float(np.mean(prim * sec.real))
    return out


# ---------------------------------------------------------------------------
# edge-corrected estimator with a random catalogue
# ---------------------------------------------------------------------------

def ss_fields(pos_d, w_d, pos_r, w_r, n: int, box: float, basis_name: str = "b3"):
    """The two fields of the Szapudi-Szalay estimator [Sec. 3, Eq. SSestimator]: the data and random
    catalogues deposited on the basis, each normalised to unit mean, and

        f = n_D / nbar_D - n_R / nbar_R   (the field of D - R, from the coefficient differences),
        r = n_R / nbar_R                  (the field of R).

    Returns (f, r) as float64 [n, n, n]."""
    w_d = np.ones(len(pos_d)) if w_d is None else np.asarray(w_d, dtype=np.float64)
    w_r = np.ones(len(pos_r)) if w_r is None else np.asarray(w_r, dtype=np.float64)
    B = BASES[basis_name]
    rd = B.deposit(pos_d, w_d, n, box) * (n ** 3 / w_d.sum())
    rr = B.deposit(pos_r, w_r, n, box) * (n ** 3 / w_r.sum())
    return rd - rr, rr


def ss_multipoles(zeta_n, zeta_r, lt: int, nquad: int) -> np.ndarray:
    """Multipoles of the edge-corrected 3PCF zeta = (D - R)^3 / R^3 [Eq. SSestimator]:

        zeta_l = (2l + 1) / 2 int_{-1}^{1} N(mu) / R(mu) P_l(mu) dmu,  l = 0 .. lt,

    with N and R the triplet correlations of f and r reconstructed from their multipoles truncated
    at lt [Eq. triplet-counting], the integral by nquad-point Gauss-Legendre quadrature.
    zeta_n, zeta_r: [L+1, nb, nb] -> [lt+1, nb, nb]."""
    xg, wg = special.gauss_legendre(nquad)
    num = zeta_theta(zeta_n, xg, lt)
    den = zeta_theta(zeta_r, xg, lt)
    ratio = num / den
    out = np.zeros((lt + 1,) + ratio.shape[:2])
    for l in range(lt + 1):
        out[l] = 0.5 * (2 * l + 1) * (ratio * (wg * special.legendre(l, xg))[None, None, :]).sum(-1)
    return out
