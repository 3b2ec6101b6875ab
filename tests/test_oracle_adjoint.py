"""Pins of the oracle's gradients: central finite differences and dot-product tests."""
import numpy as np
import pytest

from mockgen import random_field, lognormal_catalogue
from oracle import basis
from oracle import estimator as E
from oracle import adjoint as A


def test_nodal_grad_matches_finite_differences():
    n = 8
    delta = random_field(n, 21)
    plan = E.Plan(n, 100.0, 2, np.linspace(5.0, 40.0, 4))
    lam = np.random.default_rng(22).standard_normal((plan.lmax + 1, plan.nbins, plan.nbins))
    g = A.zeta_nodal_grad(plan, delta, lam)
    rng = np.random.default_rng(23)
    for _ in range(3):
        v = rng.standard_normal(delta.shape)
        v /= np.sqrt(np.mean(v * v))
        h = 1e-4
        fd = (A.zeta_nodal_objective(plan, delta + h * v, lam)
              - A.zeta_nodal_objective(plan, delta - h * v, lam)) / (2 * h)
        an = np.sum(g * v)
        assert abs(fd - an) < 1e-7 * max(abs(fd), 1e-30) + 1e-14


def test_nodal_grad_single_entry():
    """The gradient of one zeta entry, checked coordinate-wise on a tiny grid."""
    n = 4
    delta = random_field(n, 24)
    plan = E.Plan(n, 40.0, 1, np.array([5.0, 15.0, 25.0]))
    lam = np.zeros((2, 2, 2))
    lam[1, 0, 1] = 1.0
    g = A.zeta_nodal_grad(plan, delta, lam)
    h = 1e-5
    for idx in [(0, 0, 0), (1, 2, 3), (3, 3, 1)]:
        e = np.zeros_like(delta)
        e[idx] = 1.0
        fd = (A.zeta_nodal_objective(plan, delta + h * e, lam)
              - A.zeta_nodal_objective(plan, delta - h * e, lam)) / (2 * h)
        assert abs(fd - g[idx]) < 1e-8 * max(1.0, abs(fd))


def test_weight_grad_matches_finite_differences():
    n, box = 16, 250.0
    pos, w = lognormal_catalogue(16, box, 500, 8.0, 31, 32, 33, (0.5, 1.5))
    w = w.astype(np.float64)
    plan = E.Plan(n, box, 1, np.linspace(20.0, 60.0, 3))
    lam = np.random.default_rng(34).standard_normal((2, 2, 2))

    def J(wv):
        eps = basis.deposit(pos, wv, n, box)
        return A.zeta_nodal_objective(plan, basis.density_contrast(eps, wv.sum()), lam)

    eps = basis.deposit(pos, w, n, box)
    delta = basis.density_contrast(eps, w.sum())
    g = A.zeta_nodal_grad(plan, delta, lam)
    gw = A.deposit_weight_grad(pos, w, n, box, g)
    rng = np.random.default_rng(35)
    for _ in range(2):
        v = rng.standard_normal(w.shape)
        v /= np.linalg.norm(v)
        h = 1e-4
        fd = (J(w + h * v) - J(w - h * v)) / (2 * h)
        assert abs(fd - np.sum(gw * v)) < 1e-7 * abs(fd)


def test_fft_filter_dot_products():
    """<ifftn(K fftn(x)), c> = <x, fftn(K ifftn(c))> (bilinear), the transpose used by the adjoint."""
    n = 8
    rng = np.random.default_rng(40)
    plan = E.Plan(n, 100.0, 3, np.linspace(5.0, 40.0, 3))
    x = rng.standard_normal((n, n, n))
    c = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    K = plan.kernel(3, 2, 1)
    lhs = np.sum(np.fft.ifftn(K * np.fft.fftn(x)) * c)
    rhs = np.sum(x * np.fft.fftn(K * np.fft.ifftn(c)))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def _particle_case(basis_name="b3"):
    n, box = 8, 80.0
    pos, w = lognormal_catalogue(n, box, 1500, 12.0, 31, 32, 33, (0.5, 1.5))
    plan = E.Plan(n, box, 2, np.array([8.0, 16.0, 24.0, 32.0]), basis=basis_name)
    lam = np.random.default_rng(34).standard_normal((plan.lmax + 1, plan.nbins, plan.nbins))
    return plan, pos, w.astype(np.float64), lam


@pytest.mark.parametrize("basis_name", ["b3", "d4"])
def test_particle_grad_delta_matches_finite_differences(basis_name):
    """dJ/ddelta of the particle form (primary weights fixed) against central differences."""
    plan, pos, w, lam = _particle_case(basis_name)
    g, _ = A.zeta_particle_grad(plan, pos, w, lam)
    delta = basis.density_contrast(plan.B.deposit(pos, w, plan.n, plan.box), w.sum())
    rng = np.random.default_rng(35)
    for _ in range(3):
        v = rng.standard_normal(delta.shape)
        v /= np.sqrt(np.mean(v * v))
        h = 1e-4
        jp = np.sum(lam * E.zeta_particle(plan, pos, w, delta=delta + h * v))
        jm = np.sum(lam * E.zeta_particle(plan, pos, w, delta=delta - h * v))
        fd = (jp - jm) / (2 * h)
        assert abs(fd - np.sum(g * v)) < 1e-7 * abs(fd)


@pytest.mark.parametrize("basis_name", ["b3", "d4"])
def test_particle_grad_weights_matches_finite_differences(basis_name):
    """dJ/dw of the particle form (through the deposit and the primary) against central differences."""
    plan, pos, w, lam = _particle_case(basis_name)
    _, dw = A.zeta_particle_grad(plan, pos, w, lam)
    rng = np.random.default_rng(36)
    for _ in range(3):
        v = rng.standard_normal(w.shape)
        v /= np.linalg.norm(v)
        h = 1e-4
        fd = (A.zeta_particle_objective(plan, pos, w + h * v, lam)
              - A.zeta_particle_objective(plan, pos, w - h * v, lam)) / (2 * h)
        assert abs(fd - np.dot(dw, v)) < 1e-7 * abs(fd)


def test_particle_grad_subset_equals_masked_full():
    """Restricting to some (l, bins) equals the full gradient with lam zero elsewhere."""
    plan, pos, w, lam = _particle_case()
    ls, bins = [0, 2], [0, 2]
    masked = np.zeros_like(lam)
    masked[np.ix_(ls, bins, bins)] = lam[np.ix_(ls, bins, bins)]
    g_full, dw_full = A.zeta_particle_grad(plan, pos, w, masked)
    g_sub, dw_sub = A.zeta_particle_grad(plan, pos, w, lam[np.ix_(ls, bins, bins)], ls=ls, bins=bins)
    assert np.abs(g_full - g_sub).max() <= 1e-12 * np.abs(g_full).max()
    assert np.abs(dw_full - dw_sub).max() <= 1e-12 * np.abs(dw_full).max()


@pytest.mark.parametrize("basis_name", ["b3", "d4"])
def test_gamma_grad_matches_finite_differences(basis_name):
    """dJ/ddelta of the grid summation with connection coefficients against central differences."""
    n = 8
    delta = random_field(n, 41)
    plan = E.Plan(n, 100.0, 2, np.linspace(5.0, 40.0, 4), basis=basis_name)
    lam = np.random.default_rng(42).standard_normal((plan.lmax + 1, plan.nbins, plan.nbins))
    g = A.zeta_gamma_grad(plan, delta, lam)
    rng = np.random.default_rng(43)
    for _ in range(3):
        v = rng.standard_normal(delta.shape)
        v /= np.sqrt(np.mean(v * v))
        h = 1e-4
        fd = (A.zeta_gamma_objective(plan, delta + h * v, lam)
              - A.zeta_gamma_objective(plan, delta - h * v, lam)) / (2 * h)
        assert abs(fd - np.sum(g * v)) < 1e-7 * abs(fd)


def test_gamma_grad_with_point_stencil_is_nodal():
    """With Gamma(s,t) replaced by delta_{s0} delta_{t0} the gradient is the nodal one (structure check)."""
    from oracle import basis as B
    n = 8
    delta = random_field(n, 44)
    plan = E.Plan(n, 100.0, 1, np.linspace(5.0, 40.0, 3))
    lam = np.random.default_rng(45).standard_normal((plan.lmax + 1, plan.nbins, plan.nbins))
    point = np.zeros((7, 7))
    point[3, 3] = 1.0
    orig = B.gamma_matrix
    try:
        B.gamma_matrix = lambda: point
        g = A.zeta_gamma_grad(plan, delta, lam)
    finally:
        B.gamma_matrix = orig
    gn = A.zeta_nodal_grad(plan, delta, lam)
    assert np.abs(g - gn).max() <= 1e-12 * np.abs(gn).max()
