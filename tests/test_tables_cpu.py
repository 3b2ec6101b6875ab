"""The library's host-side float64 tables (exported through the C ABI) against the oracle.

No GPU is needed: mp3_sph_bessel and mp3_window_table run on the host.
"""
import ctypes

import numpy as np
import pytest

from oracle import special
from oracle import estimator as E
from tests._common import ensure_library


@pytest.fixture(scope="module")
def lib():
    ensure_library()
    from paper_2507_15209_amd import _lib
    return _lib.load()


def _bessel(lib, lmax, x):
    out = np.zeros(lmax + 1)
    st = lib.mp3_sph_bessel(lmax, float(x), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert st == 0
    return out


@pytest.mark.parametrize("lmax", [4, 10, 20])
def test_sph_bessel_near_zeros_of_j0(lib, lmax):
    """Miller's branch (x <= lmax) around x = n pi, where j_0 vanishes and cannot normalise the
    recurrence, and elsewhere, against the oracle's j_l: within 1e-12 of max(|j_l|, j_l scale)."""
    xs = [1e-4, 0.3, 1.0, 2.5]
    for k in range(1, 7):
        for eps in (0.0, 1e-12, 1e-9, 1e-6, 1e-3, -1e-12, -1e-6):
            xs.append(k * np.pi + eps)
    xs += [lmax + 0.5, lmax * 1.7 + 3.0, 150.0]
    for x in xs:
        got = _bessel(lib, lmax, x)
        ref = np.array([special.sph_jn(l, x) for l in range(lmax + 1)])
        # relative where the function is not tiny, absolute against the l = 0..1 scale otherwise
        scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref[:2]).max())
        err = np.abs(got - ref) / scale
        assert err.max() < 1e-11, (x, err.max(), int(err.argmax()))


def _desc(n, box, lmax, edges, binning=0, smoothing=0.0):
    from paper_2507_15209_amd import _lib
    edges = np.ascontiguousarray(edges, dtype=np.float64)
    d = _lib.PlanDesc(n, box, lmax, edges.size - 1, edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0, 0, 1,
                      0, 0, binning, smoothing)
    return d, edges


@pytest.mark.parametrize("binning,R", [(0, 0.0), (1, 0.0), (1, 6.0), (0, 9.0)])
def test_window_table_matches_oracle(lib, binning, R):
    """The plan's radial window on every |q|^2 of a 16^3 grid (bin average or thin shell, top-hat
    smoothing) against the oracle's window on the same |k|, within 1e-12 of the table's scale."""
    n, box, lmax = 16, 160.0, 6
    edges = np.array([3.0, 11.0, 20.0, 34.0, 52.0])
    d, keep = _desc(n, box, lmax, edges, binning, R)
    nq2 = 3 * (n // 2) ** 2 + 1
    out = np.zeros((lmax + 1) * nq2 * 4)
    st = lib.mp3_window_table(ctypes.byref(d), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size)
    assert st == 0
    tab = out.reshape(lmax + 1, nq2, 4)
    plan = E.Plan(n, box, lmax, edges, binning="thin" if binning else "shell", smoothing=R)
    k = 2.0 * np.pi / box * np.sqrt(np.arange(nq2, dtype=np.float64))
    for l in range(lmax + 1):
        if binning:
            ref = special.thin_shell(l, edges, k)
        else:
            ref = special.jbar(l, edges, k)
        if R > 0:
            ref = ref * special.tophat_window(k * R)[None, :]
        assert np.abs(tab[l].T - ref).max() < 1e-12, l
        # the oracle plan's own table on the grid's distinct |q|^2 agrees too
        uq = np.round(plan._q2_uniq).astype(int)
        assert np.abs(tab[l][uq].T - plan.jbar_uniq(l)).max() < 1e-12


def test_window_table_rejects_bad_arguments(lib):
    d, keep = _desc(16, 160.0, 2, [5.0, 10.0])
    out = np.zeros(8)
    assert lib.mp3_window_table(ctypes.byref(d), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 8) == -1
    bad, keep2 = _desc(16, float("inf"), 2, [5.0, 10.0])
    assert lib.mp3_window_table(ctypes.byref(bad), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 8) == -6
    assert lib.mp3_sph_bessel(3, float("nan"), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == -6
    assert lib.mp3_sph_bessel(3, -1.0, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == -1


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@pytest.mark.parametrize("n", [16, 64, 256])
def test_basis_tables_match_oracle(lib, n):
    """Daubechies-4 table (cascade), autocorrelation of its interpolant and |phi_hat|^2 (infinite
    product) from the library's host code against the oracle's independent computation; the cubic
    B-spline's autocorrelation and sinc^8 likewise."""
    from oracle import basis as B3
    from oracle import basis_d4 as D4
    tab = np.zeros(3 * 1024 + 1)
    acf = np.zeros(4)
    ph = np.zeros(n)
    gam = np.zeros(49)
    assert lib.mp3_basis_tables(1, n, _dp(tab), tab.size, _dp(acf), _dp(ph), _dp(gam)) == 0
    assert np.abs(tab - D4.table(10)).max() < 1e-14
    assert np.abs(acf[:3] - D4.autocorr_samples()).max() < 1e-14 and acf[3] == 0.0
    assert np.abs(ph - D4.phi_hat_axis(n)).max() < 1e-13
    assert np.abs(gam.reshape(7, 7) - D4.gamma_matrix()).max() < 1e-13
    assert lib.mp3_basis_tables(0, n, None, 0, _dp(acf), _dp(ph), _dp(gam)) == 0
    assert np.abs(gam.reshape(7, 7) - B3.gamma_matrix()).max() < 1e-15
    b7 = B3.b7_samples()
    assert np.abs(acf - np.array([float(b7[s]) for s in range(4)])).max() < 1e-16
    plan = E.Plan(n, 100.0, 0, [1.0, 2.0], phi_hat=True)
    assert np.abs(ph - plan.phi_hat_grid()[:, 0, 0]).max() < 1e-14


def test_basis_tables_reject_bad_arguments(lib):
    tab = np.zeros(10)
    assert lib.mp3_basis_tables(2, 16, None, 0, None, None, None) == -1
    assert lib.mp3_basis_tables(1, 16, _dp(tab), tab.size, None, None, None) == -1       # wrong count
    assert lib.mp3_basis_tables(0, 16, _dp(tab), tab.size, None, None, None) == -1       # no table for B3
    ph = np.zeros(24)
    assert lib.mp3_basis_tables(1, 24, None, 0, None, _dp(ph), None) == -4               # unsupported n
