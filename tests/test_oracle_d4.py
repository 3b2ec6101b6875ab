"""Pins of the Daubechies-4 basis of the oracle (oracle.basis_d4) against what the
mathematics of the scaling function fixes independently of the cascade and the
linear systems that compute it: closed-form values at the integers, partition of
unity and reproduction of linear functions (two vanishing moments), the closed
form of |m0|^2, the Strang-Fix zeros of phi_hat, orthonormality of the integer
translates, the symmetries and sum rules of the connection coefficients, and
brute-force quadrature of the tabulated function."""
import numpy as np
import pytest

from mockgen import lognormal_catalogue
from oracle import basis_d4 as D
from oracle import estimator as E

S3 = np.sqrt(3.0)
M1 = (3.0 - S3) / 2.0          # first moment int x phi(x) dx of the Daubechies-4 scaling function


def test_filter_is_orthonormal():
    h = D.FILTER
    assert abs(h.sum() - np.sqrt(2.0)) < 1e-15
    assert abs((h * h).sum() - 1.0) < 1e-15
    assert abs(h[0] * h[2] + h[1] * h[3]) < 1e-15          # double-shift orthogonality


def test_integer_values_closed_form():
    v = D.integer_values()
    assert np.allclose(v, [0.0, (1.0 + S3) / 2.0, (1.0 - S3) / 2.0, 0.0], rtol=0, atol=1e-14)


def test_table_consistent_across_levels():
    """A coarser table is the even-indexed subsample of a finer one (dyadic values are exact)."""
    a = D.table(6)
    b = D.table(8)
    assert np.abs(b[::4] - a).max() < 1e-14


@pytest.mark.parametrize("seed", [1, 2])
def test_partition_of_unity_and_linear_reproduction(seed):
    x = np.random.default_rng(seed).uniform(0.0, 1.0, 200)
    k = np.arange(-3, 4)
    vals = D.phi(x[:, None] - k[None, :])
    assert np.abs(vals.sum(1) - 1.0).max() < 1e-13
    # sum_k k phi(x - k) = x - M1 (two vanishing moments)
    assert np.abs((vals * k[None, :]).sum(1) - (x - M1)).max() < 1e-12


def test_translates_are_orthonormal():
    """A_R(s) = int phi_R phi_R(. - s) is delta_{s0} up to the interpolation error of the table,
    and equals a brute-force midpoint quadrature of the tabulated function."""
    a = D.autocorr_samples()
    assert abs(a[0] - 1.0) < 2e-3 and abs(a[1]) < 2e-3 and abs(a[2]) < 2e-3
    x = (np.arange(3 * 2 ** 15) + 0.5) / 2 ** 15
    for s in range(3):
        brute = np.sum(D.phi(x) * D.phi(x - s)) / 2 ** 15
        assert abs(brute - a[s]) < 1e-7


def test_m0_closed_form_and_phi_hat():
    xi = np.linspace(-4.0, 4.0, 33)
    k = np.arange(4)
    m0 = (D.FILTER[None, :] * np.exp(-1j * k[None, :] * xi[:, None])).sum(-1) / np.sqrt(2.0)
    closed = np.cos(xi / 2) ** 4 * (1.0 + 2.0 * np.sin(xi / 2) ** 2)
    assert np.abs(np.abs(m0) ** 2 - closed).max() < 1e-14
    # phi_hat(0) = 1 (to the rounding of 64 factors) and the Strang-Fix zeros phi_hat(2 pi k) = 0, k != 0
    assert abs(D.phi_hat_sq(np.array([0.0]))[0] - 1.0) < 1e-13
    assert D.phi_hat_sq(2.0 * np.pi * np.arange(1, 6)).max() < 1e-20
    # against the transform of the tabulated function (dense midpoint sum)
    xm = (np.arange(3 * 2 ** 14) + 0.5) / 2 ** 14
    pm = D.phi(xm)
    for w in (0.3, 1.0, 2.5):
        ft = np.sum(pm * np.exp(-1j * w * xm)) / 2 ** 14
        assert abs(abs(ft) ** 2 - D.phi_hat_sq(np.array([w]))[0]) < 2e-3


def test_connection_coefficients_sum_rules_and_symmetry():
    g = D.gamma_matrix()
    idx = np.arange(-3, 4)
    # sum_t gamma(s, t) = int phi(x) phi(x - s) dx = delta_{s0} (partition of unity, orthonormality)
    rows = g.sum(1)
    assert np.abs(rows - (idx == 0)).max() < 1e-12
    # gamma(s, t) = gamma(t, s) and gamma(s, t) = gamma(-s, t - s) (shift of the integration variable)
    assert np.abs(g - g.T).max() < 1e-12
    for s in range(-2, 3):
        for t in range(-2, 3):
            if abs(t - s) <= 2:
                assert abs(g[s + 3, t + 3] - g[-s + 3, t - s + 3]) < 1e-12
    # zero outside |s|, |t|, |s - t| <= 2
    for s in range(-3, 4):
        for t in range(-3, 4):
            if max(abs(s), abs(t), abs(s - t)) > 2:
                assert g[s + 3, t + 3] == 0.0


def test_connection_coefficients_against_quadrature():
    """gamma(s, t) of the exact scaling function against a midpoint quadrature of the tabulated one."""
    g = D.gamma_matrix()
    x = (np.arange(3 * 2 ** 14) + 0.5) / 2 ** 14
    p0 = D.phi(x)
    for s in range(-2, 3):
        for t in range(-2, 3):
            if abs(s - t) <= 2:
                q = np.sum(p0 * D.phi(x - s) * D.phi(x - t)) / 2 ** 14
                assert abs(q - g[s + 3, t + 3]) < 3e-3


def test_deposit_moments():
    """Sum of the coefficients is the total weight; their first moment is sum w (u - M1 + 1) per axis
    (node l carries phi(u - l + 1)), for particles away from the periodic seam."""
    n, box = 16, 160.0
    rng = np.random.default_rng(7)
    pos = rng.uniform(40.0, 120.0, (300, 3)).astype(np.float32)
    w = rng.uniform(0.5, 1.5, 300)
    eps = D.deposit(pos, w, n, box)
    assert abs(eps.sum() - w.sum()) < 1e-11 * w.sum()
    u = pos.astype(np.float64) * n / box
    l = np.arange(n)
    for d in range(3):
        marg = eps.sum(axis=tuple(a for a in range(3) if a != d))
        assert abs((marg * l).sum() - np.sum(w * (u[:, d] - M1 + 1.0))) < 1e-9 * w.sum()


def test_gather_is_the_transpose_of_the_deposit():
    n, box = 8, 80.0
    pos, w = lognormal_catalogue(n, box, 400, 12.0, 51, 52, 53, (0.5, 1.5))
    f = np.random.default_rng(54).standard_normal((n, n, n))
    v = np.random.default_rng(55).standard_normal(len(pos))
    lhs = np.sum(D.deposit(pos, v, n, box) * f)
    rhs = np.sum(v * D.gather(f, pos, n, box))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_volume_mean_by_monte_carlo():
    """Fbar_l with the Daubechies-4 autocorrelation against the average of F(u) over random points."""
    n, box = 8, 80.0
    plan = E.Plan(n, box, 1, np.array([10.0, 20.0, 30.0]), basis="d4")
    delta = np.random.default_rng(61).standard_normal((n, n, n))
    dh = np.fft.fftn(delta)
    pts = np.random.default_rng(62).uniform(0.0, box, (200000, 3))
    for l in range(2):
        F = 0.0
        for m in range(-l, l + 1):
            At = D.gather(E.fields(plan, dh, l, m), pts, n, box)
            F = F + np.einsum("ip,jp->ijp", At, At.conj()).real
        mc = F.mean(-1)
        err = F.std(-1) / np.sqrt(F.shape[-1])
        ref = E.volume_mean_pair(plan, dh, l)
        assert np.all(np.abs(mc - ref) < 5 * err + 1e-12)
