"""Pins of the oracle's B-spline basis: deposit, interpolation, connection coefficients."""
import os
from fractions import Fraction

import numpy as np
from scipy.integrate import quad

from oracle import basis

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gamma_b3.txt")


def _golden():
    gam, b7 = {}, {}
    for line in open(GOLDEN):
        if not line.strip() or line.startswith("#"):
            continue
        p = line.split()
        if p[0] == "B7":
            b7[int(p[1])] = Fraction(int(p[2]), int(p[3]))
        else:
            gam[(int(p[0]), int(p[1]))] = Fraction(int(p[2]), int(p[3]))
    return gam, b7


def test_b3_partition_of_unity_and_mass():
    u = np.linspace(-0.999, 0.999, 101)
    tot = sum(basis.b3(u - l) for l in range(-3, 4))
    assert np.max(np.abs(tot - 1.0)) < 1e-15
    assert abs(quad(lambda x: basis.b3(np.array([x]))[0], -2, 2, points=[-1, 0, 1])[0] - 1.0) < 1e-14


def test_gamma_golden_values():
    """Exact rationals of Eq. con-coeff (one axis) for the cubic B-spline."""
    gam, b7 = _golden()
    full = {}
    for (s, t), v in gam.items():
        for a, b in ((s, t), (t, s), (-s, -t), (-t, -s)):
            full[(a, b)] = v
    nz = 0
    for s in range(-3, 4):
        for t in range(-3, 4):
            g = basis.gamma_1d(s, t)
            assert g == full.get((s, t), Fraction(0)), (s, t)
            nz += g != 0
    assert nz == 37
    smp = basis.b7_samples()
    for s, v in b7.items():
        assert smp[s] == v and smp[-s] == v


def test_gamma_by_numerical_quadrature():
    """Independent check of the rational integration by adaptive quadrature."""
    for s in range(-3, 4):
        for t in range(-3, 4):
            f = lambda x: (basis.b3(np.array([x]))[0] * basis.b3(np.array([x - s]))[0]  # noqa: E731
                           * basis.b3(np.array([x - t]))[0])
            val = quad(f, -2, 2, points=list(range(-2, 3)), epsabs=1e-16, epsrel=1e-14, limit=200)[0]
            assert abs(val - float(basis.gamma_1d(s, t))) < 1e-15


def test_gamma_sum_rules():
    """sum_t gamma(s,t) = B7(s) (partition of unity), sum_{s,t} gamma = 1, symmetries."""
    smp = basis.b7_samples()
    assert sum(smp.values()) == 1
    for s in range(-3, 4):
        assert sum(basis.gamma_1d(s, t) for t in range(-3, 4)) == smp[s]
        for t in range(-3, 4):
            assert basis.gamma_1d(s, t) == basis.gamma_1d(t, s) == basis.gamma_1d(-s, -t)
    assert sum(basis.gamma_1d(s, t) for s in range(-3, 4) for t in range(-3, 4)) == 1


def test_b7_hat_matches_aliased_sinc():
    """DTFT of the autocorrelation samples equals sum_p sinc^8 over aliases (Poisson summation)."""
    th = np.linspace(-np.pi, np.pi, 37)
    s = np.zeros_like(th)
    for p in range(-400, 401):
        x = (th + 2 * np.pi * p) / 2
        s += np.sinc(x / np.pi) ** 8
    assert np.max(np.abs(basis.b7_hat(th) - s)) < 1e-13


def test_deposit_partition_of_unity_and_node_weights():
    n, box = 16, 100.0
    rng = np.random.default_rng(0)
    pos = (rng.random((500, 3)) * box).astype(np.float32)
    w = rng.uniform(0.5, 1.5, 500)
    eps = basis.deposit(pos, w, n, box)
    assert abs(eps.sum() - w.sum()) < 1e-12 * w.sum()
    # a particle on a node spreads (1/6, 4/6, 1/6) per axis
    a = box / n
    p = np.array([[3 * a, 7 * a, 15 * a]], dtype=np.float32)
    e = basis.deposit(p, None, n, box)
    one = np.array([1, 4, 1]) / 6.0
    ref = np.zeros((n, n, n))
    for i, x in enumerate((2, 3, 4)):
        for j, y in enumerate((6, 7, 8)):
            for k, z in enumerate((14, 15, 0)):
                ref[x, y, z] = one[i] * one[j] * one[k]
    assert np.max(np.abs(e - ref)) < 1e-15


def test_deposit_linear_reproduction():
    """sum_l l eps_l = sum_i w_i u_i for particles away from the periodic seam."""
    n, box = 32, 100.0
    rng = np.random.default_rng(1)
    pos = (20.0 + rng.random((300, 3)) * 60.0).astype(np.float32)
    w = rng.uniform(0.5, 1.5, 300)
    eps = basis.deposit(pos, w, n, box)
    l = np.arange(n)
    u = pos.astype(np.float64) * n / box
    for ax in range(3):
        shape = [1, 1, 1]
        shape[ax] = n
        assert abs(np.sum(eps * l.reshape(shape)) - np.sum(w * u[:, ax])) < 1e-10


def test_deposit_gather_adjoint():
    """<deposit(w), g> = <w, gather(g)>."""
    n, box = 16, 50.0
    rng = np.random.default_rng(2)
    pos = (rng.random((400, 3)) * box).astype(np.float32)
    w = rng.standard_normal(400)
    g = rng.standard_normal((n, n, n))
    lhs = np.sum(basis.deposit(pos, w, n, box) * g)
    rhs = np.sum(w * basis.gather(g, pos, n, box))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gather_reproduces_linear_field():
    """Cubic B-spline interpolation of the node values of a linear ramp is the ramp (off the seam)."""
    n, box = 32, 32.0
    x = np.arange(n, dtype=np.float64)
    f = np.broadcast_to(x[:, None, None], (n, n, n)) * 1.0
    pos = np.array([[5.25, 3.0, 9.0], [17.7, 30.0, 1.0], [26.5, 12.0, 4.0]], dtype=np.float32)
    v = basis.gather(f, pos, n, box)
    assert np.max(np.abs(v - pos[:, 0].astype(np.float64))) < 1e-13
