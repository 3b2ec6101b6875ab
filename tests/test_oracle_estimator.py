"""Pins of the oracle's estimator: closed forms, special cases, invariances, brute force."""
import numpy as np
import pytest

from mockgen import random_field, band_limited_field, uniform_catalogue, lognormal_catalogue
from oracle import basis, special
from oracle import estimator as E


def _fourier_triple_sum(plan, delta, l):
    """zeta_l = (2l+1)(-1)^l / n^9 sum_{q1,q2} d(q1) d(q2) d(-q1-q2) jb(q1) jb(q2) P_l(q1.q2).

    Derived from the first equality of Eq. double-e-expansion inserted in
    Eq. DDD-3PCF-DFT (no Y_lm, no i^l phases, no m-sum); Nyquist modes of the
    two secondary vertices excluded.
    """
    n = plan.n
    dh = np.fft.fftn(delta).ravel()
    q = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    Q = np.stack(np.meshgrid(q, q, q, indexing="ij"), -1).reshape(-1, 3)
    keep = ~(Q == -(n // 2)).any(1)
    Qk, idx = Q[keep], np.arange(n ** 3)[keep]
    jb = np.stack([plan.jbar_grid(l, b).ravel() for b in range(plan.nbins)])[:, idx]
    m3 = (-(Qk[:, None, :] + Qk[None, :, :])) % n
    d3 = dh[(m3[..., 0] * n + m3[..., 1]) * n + m3[..., 2]]
    qq = np.linalg.norm(Qk, axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        mu = np.nan_to_num((Qk @ Qk.T) / np.outer(qq, qq), nan=1.0)
    T = dh[idx][:, None] * dh[idx][None, :] * d3 * special.legendre(l, mu)
    z = (2 * l + 1) * (-1) ** l / float(n) ** 9 * (jb @ T @ jb.T)
    return z


@pytest.mark.parametrize("n", [8, 6])
def test_fourier_triple_sum(n):
    delta = random_field(n, 11 + n)
    plan = E.Plan(n, 100.0, 4, np.linspace(5.0, 45.0, 4))
    z = E.zeta_nodal(plan, delta)
    for l in range(plan.lmax + 1):
        zt = _fourier_triple_sum(plan, delta, l)
        assert np.max(np.abs(zt.imag)) < 1e-13 * np.max(np.abs(zt))
        assert np.max(np.abs(zt.real - z[l])) < 1e-12 * np.max(np.abs(z[l]))


def test_zero_bin_special_cases():
    """A vanishing bin at r = 0 makes jbar_0 = 1: zeta_0(0,0) = mean(delta^3), zeta_{l>0}(0,0) = 0,
    zeta_0(b,0) = n^-3 sum_x delta_x^2 (ifftn(dhat jbar_{0,b}))_x  (band-limited delta)."""
    n = 8
    delta = band_limited_field(n, 5)
    edges = np.array([0.0, 1e-7, 20.0, 35.0])
    plan = E.Plan(n, 100.0, 3, edges)
    z = E.zeta_nodal(plan, delta)
    assert abs(z[0, 0, 0] - np.mean(delta ** 3)) < 1e-12 * np.mean(np.abs(delta) ** 3)
    for l in range(1, 4):
        assert abs(z[l, 0, 0]) < 1e-12 * abs(z[0, 0, 0])
    dh = np.fft.fftn(delta)
    for b in (1, 2):
        f = np.fft.ifftn(dh * plan.jbar_grid(0, b)).real
        assert abs(z[0, b, 0] - np.mean(delta ** 2 * f)) < 1e-12 * np.mean(np.abs(delta ** 2 * f))


def test_real_and_symmetric():
    n = 16
    delta = random_field(n, 3)
    plan = E.Plan(n, 200.0, 3, np.linspace(20.0, 80.0, 5))
    z = E.zeta_nodal(plan, delta)          # the oracle itself asserts |Im| at rounding level
    assert np.max(np.abs(z - z.transpose(0, 2, 1))) < 1e-13 * np.max(np.abs(z))


def test_nyquist_rule_needed_for_realness():
    """Keeping the unpaired Nyquist planes would make zeta complex (the reason they are zeroed)."""
    n = 8
    delta = random_field(n, 4)
    plan = E.Plan(n, 100.0, 2, np.linspace(5.0, 40.0, 3))
    dh = np.fft.fftn(delta)
    z = 0.0
    l = 1
    for m in range(-l, l + 1):
        yc = plan.ylm_conj_grid(l, m)
        A = np.stack([np.fft.ifftn(dh * (1j ** l) * plan.jbar_grid(l, b) * yc) for b in range(plan.nbins)])
        flat = A.reshape(plan.nbins, -1)
        z = z + (flat * delta.ravel()) @ flat.conj().T
    assert np.max(np.abs(z.imag)) > 1e-3 * np.max(np.abs(z))


def _cube_ops(d):
    yield np.transpose(d, (1, 0, 2))
    yield np.transpose(d, (2, 1, 0))
    yield np.transpose(d, (1, 2, 0))
    yield np.roll(d[::-1], 1, axis=0)                      # x -> -x
    yield np.roll(d[:, ::-1], 1, axis=1)                   # y -> -y
    yield np.roll(d[:, :, ::-1], 1, axis=2)                # z -> -z
    yield np.roll(d, (3, -2, 5), axis=(0, 1, 2))           # integer translation


def test_invariances():
    n = 8
    delta = random_field(n, 6)
    plan = E.Plan(n, 100.0, 3, np.linspace(5.0, 40.0, 4))
    z = E.zeta_nodal(plan, delta)
    s = np.max(np.abs(z))
    for d2 in _cube_ops(delta):
        assert np.max(np.abs(E.zeta_nodal(plan, np.ascontiguousarray(d2)) - z)) < 1e-13 * s
    assert np.max(np.abs(E.zeta_nodal(plan, -delta) + z)) < 1e-13 * s
    assert np.max(np.abs(E.zeta_nodal(plan, 1.7 * delta) - 1.7 ** 3 * z)) < 1e-13 * s * 5


def test_real_harmonics_give_same_zeta():
    """Contracting real spherical harmonics instead of complex ones leaves zeta_l unchanged."""
    n = 8
    delta = random_field(n, 8)
    plan = E.Plan(n, 100.0, 3, np.linspace(5.0, 40.0, 3))
    z = E.zeta_nodal(plan, delta)
    dh = np.fft.fftn(delta)
    for l in range(plan.lmax + 1):
        acc = 0.0
        for m in range(-l, l + 1):
            y = special.ylm(l, abs(m), plan.theta, plan.phi)
            if m > 0:
                yr = np.sqrt(2) * (-1) ** m * y.real
            elif m < 0:
                yr = np.sqrt(2) * (-1) ** m * y.imag
            else:
                yr = y.real
            A = []
            for b in range(plan.nbins):
                k = (1j ** l) * plan.jbar_grid(l, b) * yr
                k[plan.nyquist] = 0.0
                A.append(np.fft.ifftn(dh * k).ravel())
            A = np.array(A)
            acc = acc + (A * delta.ravel()) @ A.conj().T
        zr = (4 * np.pi / n ** 3) * acc
        assert np.max(np.abs(zr.real - z[l])) < 1e-13 * np.max(np.abs(z))


def _gamma_literal(delta, A, B, g=None):
    """sum_x delta_x sum_{s,t in [-3,3]^3} Gamma(s,t) A(x+s) conj(B(x+t)), literally over all (s, t)."""
    g = basis.gamma_matrix() if g is None else g
    offs = [(i, j, k) for i in range(-3, 4) for j in range(-3, 4) for k in range(-3, 4)]
    As = np.stack([np.roll(A, (-o[0], -o[1], -o[2]), axis=(0, 1, 2)).ravel() for o in offs])
    Bs = np.stack([np.roll(B, (-o[0], -o[1], -o[2]), axis=(0, 1, 2)).ravel() for o in offs])
    M = (As * delta.ravel()) @ Bs.conj().T                 # [343, 343]
    G = np.array([[g[s[0] + 3, t[0] + 3] * g[s[1] + 3, t[1] + 3] * g[s[2] + 3, t[2] + 3] for t in offs] for s in offs])
    return np.sum(G * M)


def test_gamma_forms_agree_with_literal_sum():
    """Eq. SFC-3PCF summed literally over (s,t) = the Delta-stencil oracle = the quadrature oracle."""
    n = 8
    delta = random_field(n, 9)
    plan = E.Plan(n, 100.0, 2, np.linspace(10.0, 40.0, 3))
    zg = E.zeta_gamma(plan, delta)
    zq = E.zeta_gamma_quadrature(plan, delta)
    assert np.max(np.abs(zg - zq)) < 1e-13 * np.max(np.abs(zg))
    dh = np.fft.fftn(delta)
    l = 2
    tot = 0.0
    for m in range(-l, l + 1):
        A = E.fields(plan, dh, l, m)
        tot = tot + _gamma_literal(delta, A[0], A[1])
    tot *= 4 * np.pi / n ** 3
    assert abs(tot.imag) < 1e-13 * abs(tot)
    assert abs(tot.real - zg[l, 0, 1]) < 1e-13 * np.max(np.abs(zg[l]))


def test_gamma_d4_agrees_with_literal_sum():
    """The Delta-stencil oracle with the Daubechies-4 connection coefficients (not reflection
    symmetric) equals Eq. SFC-3PCF summed literally over (s, t)."""
    from oracle import basis_d4
    n = 8
    delta = random_field(n, 19)
    plan = E.Plan(n, 100.0, 1, np.linspace(10.0, 40.0, 3), basis="d4")
    zg = E.zeta_gamma(plan, delta)
    dh = np.fft.fftn(delta)
    l = 1
    tot = 0.0
    for m in range(-l, l + 1):
        A = E.fields(plan, dh, l, m)
        tot = tot + _gamma_literal(delta, A[0], A[1], basis_d4.gamma_matrix())
    tot *= 4 * np.pi / n ** 3
    assert abs(tot.imag) < 1e-13 * abs(tot)
    assert abs(tot.real - zg[l, 0, 1]) < 1e-13 * np.max(np.abs(zg[l]))


def test_gamma_equals_nodal_for_constant_fields():
    """With constant secondaries the connection coefficients sum to one: Gamma form = nodal form."""
    n = 8
    delta = random_field(n, 10)
    c1, c2 = 0.7 - 0.2j, -1.1 + 0.4j
    A = np.full((n, n, n), c1)
    B = np.full((n, n, n), c2)
    lit = _gamma_literal(delta, A, B)
    nodal = np.sum(delta * A * np.conj(B))
    assert abs(lit - nodal) < 1e-13 * max(1.0, abs(nodal))


def test_volume_mean_by_quadrature():
    """Fbar_l (Parseval + B7hat) equals the 5-point Gauss-Legendre volume integral of F_l."""
    n = 8
    delta = random_field(n, 12)
    plan = E.Plan(n, 100.0, 2, np.linspace(10.0, 40.0, 3))
    dh = np.fft.fftn(delta)
    M, wq = E._node_interp_matrix(n)

    def interp(f):
        g = np.tensordot(M, f, axes=(1, 0))
        g = np.tensordot(M, g, axes=(1, 1)).transpose(1, 0, 2)
        return np.tensordot(M, g, axes=(1, 2)).transpose(1, 2, 0)

    W = (wq[:, None, None] * wq[None, :, None] * wq[None, None, :]).ravel()
    for l in range(3):
        tot = 0.0
        for m in range(-l, l + 1):
            A = np.stack([interp(a).ravel() for a in E.fields(plan, dh, l, m)])
            tot = tot + (A * W) @ A.conj().T
        tot = tot.real / n ** 3
        ref = E.volume_mean_pair(plan, dh, l)
        assert np.max(np.abs(tot - ref)) < 1e-13 * np.max(np.abs(ref))


def _brute_force(pos, w, box, lmax, edges):
    """Triplet count (2l+1)/(nbar^3 V V_b1 V_b2) sum_{ijk} w w w 1_b1(r_ij) 1_b2(r_ik) P_l(rhat_ij . rhat_ik),
    minimum-image separations, j = k included (the definition of Eq. 3PCF-spatial-average
    projected on Legendre polynomials)."""
    x = pos.astype(np.float64)
    w = w.astype(np.float64)
    V = box ** 3
    nbar = w.sum() / V
    nb = len(edges) - 1
    vb = 4 * np.pi / 3 * (edges[1:] ** 3 - edges[:-1] ** 3)
    out = np.zeros((lmax + 1, nb, nb))
    for i in range(len(x)):
        d = x - x[i]
        d -= box * np.round(d / box)
        r = np.linalg.norm(d, axis=1)
        b = np.searchsorted(edges, r, side="right") - 1
        ok = (b >= 0) & (b < nb) & (r > 0)
        if not ok.any():
            continue
        u = d[ok] / r[ok, None]
        bb = b[ok]
        ww = w[ok]
        mu = np.clip(u @ u.T, -1, 1)
        H = np.zeros((nb, ok.sum()))
        H[bb, np.arange(ok.sum())] = ww
        for l in range(lmax + 1):
            out[l] += w[i] * (H @ special.legendre(l, mu) @ H.T)
    for l in range(lmax + 1):
        out[l] *= (2 * l + 1) / (nbar ** 3 * V) / np.outer(vb, vb)
    return out


@pytest.mark.slow
def test_brute_force_triplets_convergence():
    """Particle summation in triplet-counting mode approaches the O(N^3) triplet count as the grid refines."""
    box = 250.0
    edges = np.linspace(10.0, 60.0, 7)
    pos, w = lognormal_catalogue(32, box, 2000, 4.0, 1001, 1002)
    sub = np.random.default_rng(1005).permutation(2000)[:300]
    pos, w = pos[sub], w[sub]
    lmax = 2
    bf = _brute_force(pos, w, box, lmax, edges)
    errs = []
    for n in (32, 64, 128):
        plan = E.Plan(n, box, lmax, edges)
        z = E.zeta_particle(plan, pos, w, mode="ddd")
        errs.append([np.linalg.norm(z[l] - bf[l]) / np.linalg.norm(bf[l]) for l in range(lmax + 1)])
    errs = np.array(errs)
    assert np.all(errs[2] < errs[1]) and np.all(errs[1] < errs[0])
    assert errs[2, 0] < 0.1 and np.all(errs[2] < 0.35)


def test_uniform_randoms_consistent_with_shot_noise():
    """Uniform randoms: zeta_l equals its Poisson expectation within the scatter of 16 seeds.

    For N_R iid uniform points, delta = sum_i f_i with f_i = (n^3/N_R)(B(u_i - x) - n^-3), and
    E[delta_x delta_y delta_z] = N_R E[f f f] (only the one-particle cumulant survives), so
    E[zeta_l] = (n^9 / N_R^2) E_u[zeta_l(g_u)] with g_u = B(u - x) - n^-3, averaged over
    sub-cell offsets u (periodic trapezoid rule, exact for this smooth periodic average).
    """
    n, box, nr = 16, 125.0, 4000
    edges = np.linspace(15.0, 55.0, 4)
    plan = E.Plan(n, box, 2, edges)
    zs = []
    for seed in range(16):
        pos, w = uniform_catalogue(nr, box, 7000 + seed)
        eps = basis.deposit(pos, w, n, box)
        zs.append(E.zeta_nodal(plan, basis.density_contrast(eps, w.sum())))
    zs = np.array(zs)
    a = box / n
    acc = 0.0
    t = (np.arange(4) + 0.5) / 4
    for ux in t:
        for uy in t:
            for uz in t:
                p = (np.array([[ux, uy, uz]]) * a + 40.0).astype(np.float32)
                g = basis.deposit(p, None, n, box) - 1.0 / n ** 3
                acc = acc + E.zeta_nodal(plan, g)
    expect = acc / 64 * float(n) ** 9 / nr ** 2
    mean = zs.mean(0)
    sig = zs.std(0, ddof=1) / np.sqrt(len(zs))
    zscore = np.abs(mean - expect) / sig
    assert np.mean(zscore < 3.0) >= 0.9
    assert np.all(zscore < 5.0)
    # the estimate is consistent with zero once the one-particle term is removed,
    # and the one-particle term scales as N_R^-2
    assert np.all(np.abs(expect) < 10 * np.abs(zs).max())


def test_uniform_randoms_particle_form_consistent_with_shot_noise():
    """The particle summation in its default mode (primary on the weighted particles, secondaries from
    the deposited contrast, volume mean subtracted) on uniform randoms equals its Poisson expectation
    within the scatter of 16 seeds.

    With delta = sum_j f_j, f_j = (n^3/N_R)(B(u_j - x) - n^-3), the primary's average over particles i
    of F(u_i) - Fbar keeps in expectation only the terms whose two secondaries both come from particle
    i: a secondary from another particle j has zero mean over u_j, and for i outside {j, k} the mean
    over u_i is the volume mean that Fbar removes.  Hence
        E[zeta_l] = (n^3/N_R)^2 E_u[zeta1_l(u)],
    zeta1(u) the same form for one unit-weight particle at u with secondaries g_u = B(u - x) - n^-3,
    averaged over sub-cell offsets (the form is invariant under whole-cell shifts).  Dropping the
    volume mean, or scaling it or the primary's weights wrongly, moves the mean by O(N_R) times this."""
    n, box, nr = 16, 125.0, 4000
    edges = np.linspace(15.0, 55.0, 4)
    plan = E.Plan(n, box, 2, edges)
    zs, fbar = [], []
    for seed in range(16):
        pos, w = uniform_catalogue(nr, box, 7100 + seed)
        zs.append(E.zeta_particle(plan, pos, w))
        dh = np.fft.fftn(basis.density_contrast(basis.deposit(pos, w, n, box), float(w.astype(np.float64).sum())))
        fbar.append([4 * np.pi * E.volume_mean_pair(plan, dh, l) for l in range(3)])
    zs, fbar = np.array(zs), np.array(fbar)
    a = box / n
    acc = 0.0
    t = (np.arange(4) + 0.5) / 4
    for ux in t:
        for uy in t:
            for uz in t:
                p = (np.array([[ux, uy, uz]]) * a + 40.0).astype(np.float32)
                g = basis.deposit(p, None, n, box) - 1.0 / n ** 3
                acc = acc + E.zeta_particle(plan, p, None, delta=g)
    expect = acc / 64 * (float(n) ** 3 / nr) ** 2
    mean = zs.mean(0)
    sig = zs.std(0, ddof=1) / np.sqrt(len(zs))
    zscore = np.abs(mean - expect) / sig
    assert np.mean(zscore < 3.0) >= 0.9
    assert np.all(zscore < 5.0)
    # power: without the volume mean the same means would sit many sigma away
    assert np.min(np.abs(mean + fbar.mean(0) - expect) / sig) > 10.0


def test_lognormal_skewness_positive():
    """A log-normal field has positive three-point amplitude on small bins; its Gaussian parent is odd."""
    n, box = 32, 250.0
    pos, w = lognormal_catalogue(n, box, 20000, 4.0, 1001, 1002)
    eps = basis.deposit(pos, w, n, box)
    delta = basis.density_contrast(eps, w.sum())
    plan = E.Plan(n, box, 0, np.array([10.0, 20.0, 30.0]))
    z = E.zeta_nodal(plan, delta)
    assert z[0, 0, 0] > 0 and z[0, 1, 1] > 0
    assert np.allclose(E.zeta_nodal(plan, -delta), -z, rtol=1e-12, atol=0)
