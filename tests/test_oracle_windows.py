"""Pins of the oracle's vertex windows, two-point function and 3PCF reconstruction.

Each check compares the oracle with something other than itself: a quadrature
of the defining integral, a limit, a closed form of a few-mode field, or an
orientation average of plane waves evaluated by brute-force quadrature.
"""
import numpy as np
import pytest
from scipy.integrate import quad

from mockgen import random_field
from oracle import basis, special
from oracle import estimator as E


def test_tophat_window_is_the_sphere_transform():
    """W_TH(kR) = (3 / R^3) int_0^R r^2 j_0(k r) dr, the unit-volume sphere's transform (Sec. 3)."""
    R = 7.5
    for k in (1e-4, 0.03, 0.2, 0.9, 2.5):
        num = 3.0 / R ** 3 * quad(lambda r: r * r * np.sin(k * r) / (k * r), 0.0, R, epsabs=1e-15, epsrel=1e-14)[0]
        assert abs(float(special.tophat_window(k * R)) - num) < 1e-12
    assert float(special.tophat_window(0.0)) == 1.0


def test_thin_shell_is_the_narrow_bin_limit():
    """The bin average tends to j_l(k r_mid) as the bin narrows (the two use different code paths)."""
    k = np.linspace(0.0, 0.6, 41)
    for l in (0, 1, 4, 9):
        for w in (1e-3, 1e-4):
            edges = np.array([30.0 - w / 2, 30.0 + w / 2])
            avg = special.jbar(l, edges, k)
            thin = special.thin_shell(l, edges, k)
            # the bin average differs from the mid-point value at second order in the width
            assert np.max(np.abs(avg - thin)) < 50 * w * w


def test_phi_hat_is_the_b3_power_spectrum():
    """phi-hat per axis = |int B3(u) exp(-i theta u) du|^2 at theta = 2 pi q / n (Eq. SFC-3PCF-vertex)."""
    n = 16
    plan = E.Plan(n, 100.0, 1, [10.0, 20.0], phi_hat=True)
    g = plan.phi_hat_grid()
    for q in range(-n // 2, n // 2):
        th = 2.0 * np.pi * q / n
        re = quad(lambda u: basis.b3(np.array([u]))[0] * np.cos(th * u), -2, 2, points=[-1, 0, 1], epsabs=1e-15)[0]
        im = quad(lambda u: basis.b3(np.array([u]))[0] * np.sin(th * u), -2, 2, points=[-1, 0, 1], epsabs=1e-15)[0]
        assert abs(g[q % n, 0, 0] - (re * re + im * im)) < 1e-13


def _triple_sum(plan, delta, l, wp=None):
    """zeta_l = (2l+1)(-1)^l / n^9 sum_{q1,q2} d(q1) d(q2) Wp(q3) d(q3) R(q1) R(q2) P_l(q1.q2), q3 = -q1-q2,

    the Fourier form of Eq. DDD-3PCF-DFT with the first equality of Eq. double-e-expansion, the
    secondaries' radial window R of the plan and the primary's window Wp (no Y_lm, no m-sum)."""
    n = plan.n
    dh = np.fft.fftn(delta).ravel()
    q = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    Q = np.stack(np.meshgrid(q, q, q, indexing="ij"), -1).reshape(-1, 3)
    keep = ~(Q == -(n // 2)).any(1)
    Qk, idx = Q[keep], np.arange(n ** 3)[keep]
    jb = np.stack([plan.jbar_grid(l, b).ravel() for b in range(plan.nbins)])[:, idx]
    m3 = (-(Qk[:, None, :] + Qk[None, :, :])) % n
    i3 = (m3[..., 0] * n + m3[..., 1]) * n + m3[..., 2]
    d3 = dh[i3]
    if wp is not None:
        d3 = d3 * wp.ravel()[i3]
    qq = np.linalg.norm(Qk, axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        mu = np.nan_to_num((Qk @ Qk.T) / np.outer(qq, qq), nan=1.0)
    T = dh[idx][:, None] * dh[idx][None, :] * d3 * special.legendre(l, mu)
    return ((2 * l + 1) * (-1) ** l / float(n) ** 9 * (jb @ T @ jb.T)).real


@pytest.mark.parametrize("binning,R", [("thin", 0.0), ("thin", 9.0), ("shell", 6.0)])
def test_thin_shell_and_tophat_triple_sum(binning, R):
    """Thin-shell windows and the top-hat on every vertex (primary included) against the Fourier
    triple sum with the primary's window on the third wave vector."""
    n = 8
    delta = random_field(n, 21)
    plan = E.Plan(n, 100.0, 3, np.linspace(8.0, 40.0, 4), binning=binning, smoothing=R)
    z = E.zeta_nodal(plan, delta)
    wp = special.tophat_window(plan.kgrid * R) if R > 0 else None
    for l in range(plan.lmax + 1):
        zt = _triple_sum(plan, delta, l, wp)
        assert np.max(np.abs(zt - z[l])) < 1e-12 * np.max(np.abs(z[l]))


def test_phi_hat_triple_sum():
    """The phi-hat option multiplies each secondary's window by phi-hat(q)."""
    n = 8
    delta = random_field(n, 22)
    plan = E.Plan(n, 100.0, 2, np.linspace(8.0, 40.0, 3), phi_hat=True)
    z = E.zeta_nodal(plan, delta)
    ph = plan.phi_hat_grid()

    class Windows:
        pass

    win = Windows()
    win.n, win.nbins = n, plan.nbins
    win.jbar_grid = lambda l, b: plan.jbar_grid(l, b) * ph
    for l in range(plan.lmax + 1):
        zt = _triple_sum(win, delta, l)
        assert np.max(np.abs(zt - z[l])) < 1e-12 * np.max(np.abs(z[l]))


def _cos_mode(n, q0):
    x = np.arange(n)
    X = np.stack(np.meshgrid(x, x, x, indexing="ij"), -1)
    return np.cos(2.0 * np.pi * (X @ np.asarray(q0, dtype=np.float64)) / n)


@pytest.mark.parametrize("R", [0.0, 5.0])
def test_xi_of_one_cosine_mode(R):
    """delta = cos(k0.x): xi(r) = (1/2) W_TH(k0 R)^2 j_0(k0 r) (with the top-hat on both vertices)."""
    n, box = 16, 160.0
    q0 = (2, 1, 3)
    delta = _cos_mode(n, q0)
    plan = E.Plan(n, box, 0, [10.0, 20.0], smoothing=R)
    k0 = 2.0 * np.pi / box * np.linalg.norm(q0)
    r = np.array([0.0, 3.0, 17.5, 41.0])
    w = float(special.tophat_window(k0 * R)) if R > 0 else 1.0
    ref = 0.5 * w * w * np.sinc(k0 * r / np.pi)
    assert np.max(np.abs(E.xi(plan, delta, r) - ref)) < 1e-14


def test_xi_zero_lag_is_the_variance():
    """Without smoothing xi(0) = mean(delta^2) for a band-limited field (Parseval)."""
    n = 16
    from mockgen import band_limited_field
    delta = band_limited_field(n, 4)
    plan = E.Plan(n, 160.0, 0, [10.0, 20.0])
    assert abs(E.xi(plan, delta, [0.0])[0] - np.mean(delta ** 2)) < 1e-13 * np.mean(delta ** 2)


def _orientation_average(dh_modes, r1, r2, mu, nodes=48):
    """< sum_{(a,b,c)} d_a d_b d_c exp(i k_a.R r1) exp(i k_b.R r2) >_R over rotations R, by
    Gauss-Legendre quadrature in cos(theta_1) and trapezoids in phi_1 and the roll psi of r2 about r1."""
    xg, wg = special.gauss_legendre(nodes)
    ph = np.linspace(0.0, 2.0 * np.pi, 2 * nodes, endpoint=False)
    ps = np.linspace(0.0, 2.0 * np.pi, 2 * nodes, endpoint=False)
    st = np.sqrt(1.0 - xg ** 2)
    # unit vectors e1 (r1 direction) and two perpendicular ones
    c1, s1 = xg[:, None], st[:, None]
    e1 = np.stack([s1 * np.cos(ph)[None, :], s1 * np.sin(ph)[None, :], np.broadcast_to(c1, (nodes, 2 * nodes))], -1)
    u = np.stack([c1 * np.cos(ph)[None, :], c1 * np.sin(ph)[None, :], np.broadcast_to(-s1, (nodes, 2 * nodes))], -1)
    v = np.cross(e1, u)
    sn = np.sqrt(max(1.0 - mu * mu, 0.0))
    acc = 0.0
    for coef, ka, kb in dh_modes:
        pa = np.einsum("ijk,k->ij", e1, ka) * r1
        base = np.einsum("ijk,k->ij", e1, kb) * mu
        ub = np.einsum("ijk,k->ij", u, kb) * sn
        vb = np.einsum("ijk,k->ij", v, kb) * sn
        pb = r2 * (base[..., None] + ub[..., None] * np.cos(ps) + vb[..., None] * np.sin(ps))
        val = np.exp(1j * pa)[..., None] * np.exp(1j * pb)
        acc += coef * np.sum(val.mean(-1).mean(-1) * wg) / 2.0
    return acc


def test_zeta_theta_is_the_orientation_average():
    """sum_l zeta_l P_l(cos theta) (thin shells, l <= 14) equals the orientation-averaged triplet
    correlation <delta(x) delta(x + r1) delta(x + r2)> of a three-mode field (Eq. triplet-counting
    with Eq. double-e-expansion summed over all L), computed by quadrature over rotations."""
    n, box = 16, 400.0
    qa, qb = np.array([1, 0, 0]), np.array([0, 1, 1])
    qc = -(qa + qb)
    x = np.arange(n)
    X = np.stack(np.meshgrid(x, x, x, indexing="ij"), -1)
    delta = sum(np.cos(2.0 * np.pi * (X @ q) / n) for q in (qa, qb, qc))
    r1, r2 = 30.0, 45.0
    edges = np.array([r1 - 1.0, r1 + 1.0, r2 - 1.0, r2 + 1.0])      # thin shells at 30 (bin 0) and 45 (bin 2)
    # k r <= 1.3 here: the terms beyond l = 14 are below 1e-15 of the sum
    plan = E.Plan(n, box, 14, edges, binning="thin")
    z = E.zeta_nodal(plan, delta, bins=[0, 2])
    mu = np.array([-0.9, -0.3, 0.2, 0.75])
    zt = E.zeta_theta(z, mu, 14)
    # the same triple by brute force: delta = sum_j (e^{i k_j.x} + e^{-i k_j.x}) / 2 with k_a + k_b + k_c = 0;
    # <d(x) d(x + s1) d(x + s2)>_x keeps the mode triples summing to zero
    kf = 2.0 * np.pi / box
    ks = [kf * qa, kf * qb, kf * qc]
    modes = []
    for sgn in (1, -1):
        for i in range(3):
            for j in range(3):
                if i != j:
                    # primary carries the third mode; secondaries modes i, j (with the overall sign)
                    modes.append((1.0 / 8.0, sgn * ks[i], sgn * ks[j]))
    for t, m in enumerate(mu):
        ref = _orientation_average(modes, r1, r2, m).real
        assert abs(zt[0, 1, t] - ref) < 1e-9 * max(1.0, abs(ref)), (m, zt[0, 1, t], ref)


def test_reduced_3pcf_definition():
    """Q at theta is zeta(theta) / (xi1 xi2 + xi2 xi3 + xi3 xi1) with xi from the pinned xi() at the
    third side; the hierarchical amplitude of zeta = xi-products is 1."""
    n = 8
    delta = random_field(n, 23)
    plan = E.Plan(n, 100.0, 2, np.linspace(8.0, 40.0, 3), binning="thin", smoothing=4.0)
    rb = 0.5 * (plan.edges[:-1] + plan.edges[1:])
    mu = np.array([-0.5, 0.1, 0.8])
    xb = E.xi(plan, delta, rb)
    # a zeta whose monopole-only sum equals the hierarchical product at mu[0]
    r3 = np.sqrt(rb[:, None] ** 2 + rb[None, :] ** 2 - 2 * rb[:, None] * rb[None, :] * mu[0])
    x3 = np.stack([E.xi(plan, delta, r3[i]) for i in range(plan.nbins)])
    zh = xb[:, None] * xb[None, :] + xb[None, :] * x3 + x3 * xb[:, None]
    zeta = np.zeros((plan.lmax + 1, plan.nbins, plan.nbins))
    zeta[0] = zh
    q = E.reduced_3pcf(plan, delta, zeta, mu[:1], 2)
    assert np.max(np.abs(q[..., 0] - 1.0)) < 1e-12


def test_xi_multipoles_of_one_cosine_mode():
    """delta = cos(k0.x): xi_ell(r) = (1/2)(2 ell + 1) i^ell j_ell(k0 r) P_ell(mu0) W^2, mu0 the cosine of
    k0 with the line of sight (odd ell vanish: the two modes +-k0 cancel)."""
    n, box = 16, 160.0
    q0 = np.array([2, 1, 3])
    delta = _cos_mode(n, q0)
    plan = E.Plan(n, box, 0, [10.0, 20.0], smoothing=4.0)
    k0 = 2.0 * np.pi / box * np.linalg.norm(q0)
    mu0 = q0[2] / np.linalg.norm(q0)
    r = np.array([3.0, 17.5, 41.0])
    ells = [0, 1, 2, 4, 6]
    got = E.xi_multipoles(plan, delta, r, ells)
    w = float(special.tophat_window(k0 * 4.0))
    for i, ell in enumerate(ells):
        ref = 0.0 if ell % 2 else 0.5 * w * w * (2 * ell + 1) * ((-1) ** (ell // 2)) * special.sph_jn(ell, k0 * r) \
            * special.legendre(ell, mu0)
        assert np.max(np.abs(got[i] - ref)) < 1e-14


def test_xi_multipoles_resum_the_azimuthal_average():
    """sum_ell xi_ell(r) P_ell(cos theta_r) equals the azimuthal average of the pair correlation
    n^-6 sum_q |dhat|^2 exp(i k.r) over phi_r (Eq. DD-multipole), by quadrature in phi_r."""
    n, box = 8, 400.0
    delta = random_field(n, 24)
    plan = E.Plan(n, box, 0, [10.0, 20.0])
    r = 35.0
    ells = list(range(0, 21, 2))
    xl = E.xi_multipoles(plan, delta, [r], ells)[:, 0]
    dh = np.fft.fftn(delta)
    p2 = np.abs(dh) ** 2
    p2[plan.nyquist] = 0.0
    q = np.fft.fftfreq(n, 1.0 / n)
    Q = np.stack(np.meshgrid(q, q, q, indexing="ij"), -1).reshape(-1, 3) * (2.0 * np.pi / box)
    for ct in (-0.8, 0.0, 0.45, 0.95):
        st = np.sqrt(1.0 - ct * ct)
        ph = np.linspace(0.0, 2.0 * np.pi, 256, endpoint=False)
        rv = r * np.stack([st * np.cos(ph), st * np.sin(ph), np.full_like(ph, ct)], -1)
        avg = (p2.ravel()[None, :] * np.exp(1j * rv @ Q.T)).sum(1).mean().real / float(n) ** 6
        res = sum(xl[i] * special.legendre(ell, ct) for i, ell in enumerate(ells))
        assert abs(res - avg) < 1e-12 * np.abs(xl).max(), (ct, res, avg)


def test_ss_estimator_of_identical_catalogues_vanishes():
    """D = R: the field of D - R is zero, and so is every multipole of (D - R)^3 / R^3."""
    from mockgen import lognormal_catalogue
    n, box = 16, 160.0
    pos, w = lognormal_catalogue(n, box, 3000, 8.0, 31, 32, 33, (0.5, 1.5))
    f, r = E.ss_fields(pos, w, pos, w, n, box)
    assert np.abs(f).max() == 0.0
    assert abs(r.mean() - 1.0) < 1e-14


def test_ss_estimator_with_uniform_randoms_is_the_plain_3pcf():
    """A random field that is exactly uniform (r = 1) has R_0 = 1 and R_{l>0} = 0, so the estimator's
    multipoles are those of f, recovered exactly by the Gauss-Legendre projection (polynomial in mu)."""
    n = 8
    f = random_field(n, 25)
    r = np.ones((n,) * 3)
    plan = E.Plan(n, 100.0, 4, np.linspace(8.0, 40.0, 4))
    zn, zr = E.zeta_nodal(plan, f), E.zeta_nodal(plan, r)
    assert abs(zr[0] - 1.0).max() < 1e-13 and np.abs(zr[1:]).max() < 1e-13
    zs = E.ss_multipoles(zn, zr, 4, 12)
    assert np.max(np.abs(zs - zn)) < 1e-12 * np.abs(zn).max()


def test_ss_projection_against_adaptive_quadrature():
    """The projection of N(mu) / R(mu) for a non-uniform random field against scipy's adaptive
    quadrature of the same ratio (independent of the Gauss-Legendre rule)."""
    n = 8
    f = random_field(n, 26)
    r = 1.0 + 0.3 * random_field(n, 27)
    plan = E.Plan(n, 100.0, 3, np.linspace(8.0, 40.0, 3))
    zn, zr = E.zeta_nodal(plan, f), E.zeta_nodal(plan, r)
    zs = E.ss_multipoles(zn, zr, 3, 64)
    for l in range(4):
        for i in range(2):
            for j in range(2):
                g = lambda m: float(E.zeta_theta(zn[:, i:i + 1, j:j + 1], [m], 3)[0, 0, 0]
                                    / E.zeta_theta(zr[:, i:i + 1, j:j + 1], [m], 3)[0, 0, 0]
                                    * special.legendre(l, m))
                ref = 0.5 * (2 * l + 1) * quad(g, -1.0, 1.0, epsabs=1e-14, epsrel=1e-12)[0]
                assert abs(zs[l, i, j] - ref) < 1e-10 * max(1.0, np.abs(zs).max())
