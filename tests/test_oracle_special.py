"""Pins of the oracle's special functions against identities the paper relies on."""
import numpy as np
import pytest

from oracle import special


def _dirs(rng, count):
    v = rng.standard_normal((count, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    th = np.arccos(np.clip(v[:, 2], -1, 1))
    ph = np.arctan2(v[:, 1], v[:, 0])
    return v, th, ph


@pytest.mark.parametrize("l", range(0, 11))
def test_addition_theorem(l):
    """sum_m Y_lm(k1) conj(Y_lm(k2)) = (2l+1)/(4 pi) P_l(k1.k2)  (Appendix A, addition theorem)."""
    rng = np.random.default_rng(10 + l)
    v1, t1, p1 = _dirs(rng, 200)
    v2, t2, p2 = _dirs(rng, 200)
    s = sum(special.ylm(l, m, t1, p1) * np.conj(special.ylm(l, m, t2, p2)) for m in range(-l, l + 1))
    ref = (2 * l + 1) / (4 * np.pi) * special.legendre(l, np.sum(v1 * v2, axis=1))
    assert np.max(np.abs(s - ref)) < 1e-13


def test_addition_theorem_on_grid_directions():
    """Same identity at directions of integer wavevectors, as used on the k-grid."""
    q = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [-3, 2, 5], [7, -7, 1], [0, 0, -4], [2, -1, -1]], float)
    u = q / np.linalg.norm(q, axis=1, keepdims=True)
    th = np.arccos(u[:, 2])
    ph = np.arctan2(u[:, 1], u[:, 0])
    for l in range(11):
        for i in range(len(q)):
            for j in range(len(q)):
                s = sum(special.ylm(l, m, th[i], ph[i]) * np.conj(special.ylm(l, m, th[j], ph[j]))
                        for m in range(-l, l + 1))
                assert abs(s - (2 * l + 1) / (4 * np.pi) * special.legendre(l, u[i] @ u[j])) < 1e-13


def test_plane_wave_expansion():
    """exp(i k.r) = 4 pi sum_l i^l j_l(kr) sum_m conj(Y_lm(k)) Y_lm(r)  (Sec. 2.1, Eq. plane-sph-harmonics)."""
    rng = np.random.default_rng(3)
    for kr in (0.3, 4.0, 25.0):
        v1, t1, p1 = _dirs(rng, 20)
        v2, t2, p2 = _dirs(rng, 20)
        lt = int(kr) + 40
        tot = 0.0
        for l in range(lt + 1):
            ang = sum(np.conj(special.ylm(l, m, t1, p1)) * special.ylm(l, m, t2, p2) for m in range(-l, l + 1))
            tot = tot + 4 * np.pi * (1j ** l) * special.sph_jn(l, kr) * ang
        ref = np.exp(1j * kr * np.sum(v1 * v2, axis=1))
        assert np.max(np.abs(tot - ref)) < 1e-12


def test_double_plane_wave_gegenbauer():
    """sum_L (-1)^L (2L+1) j_L(a) j_L(b) P_L(mu) = j_0(sqrt(a^2 + b^2 + 2ab mu)).

    This is the rotation average of two plane waves (Sec. 2.2, Eq. double-e-expansion)
    taken at collinear secondary vertices; it pins the (-1)^L sign and j_L at large L.
    """
    for a, b in ((0.5, 1.7), (10.0, 3.0), (40.0, 55.0)):
        for mu in (-1.0, -0.3, 0.2, 0.95):
            L = int(max(a, b)) + 60
            s = sum((-1) ** l * (2 * l + 1) * special.sph_jn(l, a) * special.sph_jn(l, b) * special.legendre(l, mu)
                    for l in range(L + 1))
            ref = special.sph_jn(0, np.sqrt(a * a + b * b + 2 * a * b * mu))
            assert abs(s - ref) < 1e-13


def test_rotation_average_monte_carlo_free():
    """Rotation average of two plane waves by exact quadrature over one direction.

    For r1 parallel to r2 the average over orientations of exp(i(k1.r1 + k2.r2))
    equals j_0(|k1 r1 + k2 r2|); Eq. double-e-expansion with P_L(1) = 1 must agree.
    """
    rng = np.random.default_rng(7)
    v1, _, _ = _dirs(rng, 5)
    v2, _, _ = _dirs(rng, 5)
    for i in range(5):
        k1, k2, r1, r2 = 0.3, 0.45, 20.0, 35.0
        mu = v1[i] @ v2[i]
        series = sum((-1) ** l * (2 * l + 1) * special.legendre(l, mu) * special.sph_jn(l, k1 * r1)
                     * special.sph_jn(l, k2 * r2) for l in range(90))
        ref = special.sph_jn(0, np.linalg.norm(k1 * r1 * v1[i] + k2 * r2 * v2[i]))
        assert abs(series - ref) < 1e-13


def test_jbar_l0_closed_form():
    """l = 0 bin average equals [sin kr - kr cos kr]/k^3 between the edges, over the bin volume."""
    edges = np.linspace(20.0, 200.0, 21)
    k = np.linspace(0.01, 0.9, 300)
    assert np.max(np.abs(special.jbar(0, edges, k) - special.jbar_l0_closed(edges, k))) < 1e-13


def test_jbar_quadrature_converged():
    """64 Gauss-Legendre nodes per bin agree with 128 at the largest |k| of a 512^3, box 3000 grid."""
    edges = np.linspace(20.0, 200.0, 21)
    kmax = 2 * np.pi / 3000.0 * 256 * np.sqrt(3.0)
    k = np.linspace(0.0, kmax, 400)
    for l in (0, 3, 10):
        a = special.jbar(l, edges, k, nodes=64)
        b = special.jbar(l, edges, k, nodes=128)
        assert np.max(np.abs(a - b)) < 1e-14


def test_jbar_thin_shell_limit():
    """As the bin width goes to zero the bin average tends to j_l(k r)  (the thin shell of Eq. 3PCF-multipole-window)."""
    k = np.linspace(0.0, 0.8, 50)
    for l in (0, 2, 7):
        r = 60.0
        for h, tol in ((1e-2, 1e-5), (1e-3, 1e-7)):
            jb = special.jbar(l, [r - h, r + h], k)[0]
            assert np.max(np.abs(jb - special.sph_jn(l, k * r))) < tol


def test_jbar_at_zero():
    edges = np.linspace(10.0, 60.0, 7)
    assert np.allclose(special.jbar(0, edges, [0.0])[:, 0], 1.0, atol=1e-15)
    for l in range(1, 6):
        assert np.all(special.jbar(l, edges, [0.0]) == 0.0)
