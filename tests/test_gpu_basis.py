"""GPU: the Daubechies-4 basis (deposit, nodal and particle forms, their gradients, the Phi-hat
window) against the oracle's Daubechies-4 module, at 1e-10 (float64) / 1e-4 (float32) relative
per multipole and per gradient (L2 and element-wise), the deposit at 1e-13 / 1e-6."""
import numpy as np
import pytest

from mockgen import lognormal_catalogue, random_field
from oracle import basis_d4 as D
from oracle import estimator as E
from oracle import adjoint as A
from tests._common import assert_zeta_close, assert_grad_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-4}


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def mp3():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_15209_amd as m
    return m


def _dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _ref_delta(pos, w, n, box):
    return D.density_contrast(D.deposit(pos, w, n, box), float(np.sum(np.asarray(w, dtype=np.float64))))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [16, 32, 64])
def test_deposit_d4(mp3, prec, n):
    """Daubechies-4 deposit and contrast, including particles on the periodic seam and at x = box.
    float32 bar 2e-6 of the largest value: the LDS and global float atomics add ~30 weights per node
    in arbitrary order, and the scaling function's negative lobe makes the sum of their magnitudes
    exceed the result (about 1e-6 measured at n = 16)."""
    _say("deposit d4", prec, n)
    box = 8.0 * n
    pos, w = lognormal_catalogue(n, box, 30000, 0.05 * box, 201, 202, 203, (0.5, 1.5))
    pos[:4] = np.array([[0.0, 0.0, 0.0], [box, 1.0, 2.0], [box - 1e-3, box * 0.5, 0.0],
                        [3.0, box, box - 2.0]], dtype=np.float32)
    plan = mp3.Plan(n, box, 0, [1.0, 2.0], precision=prec, basis="d4")
    d = plan.deposit(_dev(pos, torch.float32), _dev(w, torch.float32)).cpu().numpy()[0]
    ref = _ref_delta(pos, w, n, box)
    tol = 1e-13 if prec == "f64" else 2e-6
    assert np.abs(d - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("phi_hat", [False, True])
def test_nodal_d4_value_and_gradient(mp3, prec, phi_hat):
    """Nodal form on a Daubechies-4 deposit: zeta (one sweep and forward alone), dJ/ddelta and dJ/dw
    (through the Daubechies-4 deposit) against the oracle; with and without the basis' Phi-hat window."""
    _say("nodal d4", prec, phi_hat)
    n, lmax, nb = 32, 3, 6
    box = 10.0 * n
    edges = np.linspace(0.08 * box, 0.35 * box, nb + 1)
    pos, w = lognormal_catalogue(n, box, 8000, 0.05 * box, 211, 212, 213, (0.5, 1.5))
    lam = np.random.default_rng(214).standard_normal((lmax + 1, nb, nb))
    plan = mp3.Plan(n, box, lmax, edges, precision=prec, basis="d4", phi_hat=phi_hat)
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    delta = plan.deposit(pt, wt)
    z, dd, dw = plan.zeta_value_and_grad(delta, _dev(lam[None], torch.float64), pt, wt)
    z2 = plan.zeta(delta)
    dref = _ref_delta(pos, w, n, box)
    op = E.Plan(n, box, lmax, edges, basis="d4", phi_hat=phi_hat)
    zref = E.zeta_nodal(op, dref)
    assert_zeta_close(z.cpu().numpy()[0], zref, TOL[prec])
    assert_zeta_close(z2.cpu().numpy()[0], zref, TOL[prec])
    gref = A.zeta_nodal_grad(op, dref, lam)
    wref = A.deposit_weight_grad(pos, w, n, box, gref, "d4")
    eg = assert_grad_close(dd.cpu().numpy()[0], gref, TOL[prec], "dJ/ddelta")
    ew = assert_grad_close(dw.cpu().numpy(), wref, TOL[prec], "dJ/dw")
    print("grad errors (L2, max)", eg, ew)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nb", [4, 12])
def test_particle_d4_value_and_gradient(mp3, prec, nb):
    """Particle form with the Daubechies-4 basis (27 non-zero taps, the volume mean with the
    basis' own autocorrelation): zeta, and dJ/ddelta, dJ/dw by the backward and by the one sweep."""
    _say("particle d4", prec, nb)
    n, lmax, npart = 32, 3, 20000
    box = 8.0 * n
    edges = np.linspace(0.06 * box, 0.35 * box, nb + 1)
    pos, w = lognormal_catalogue(n, box, npart, 0.04 * box, 221, 222, 223, (0.5, 1.5))
    lam = np.random.default_rng(224 + nb).standard_normal((lmax + 1, nb, nb))
    plan = mp3.Plan(n, box, lmax, edges, precision=prec, summation="particle", basis="d4")
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    delta = plan.deposit(pt, wt)
    lt = _dev(lam[None], torch.float64)
    z = plan.zeta(delta, pt, wt)
    z1, g1, w1 = plan.zeta_value_and_grad(delta, lt, pt, wt)
    g2, w2 = plan.zeta_backward(delta, lt, pt, wt)
    op = E.Plan(n, box, lmax, edges, basis="d4")
    zref = E.zeta_particle(op, pos, w)
    assert_zeta_close(z.cpu().numpy()[0], zref, TOL[prec])
    assert_zeta_close(z1.cpu().numpy()[0], zref, TOL[prec])
    gref, wref = A.zeta_particle_grad(op, pos, w, lam)
    for g, dw in ((g1, w1), (g2, w2)):
        assert_grad_close(g.cpu().numpy()[0], gref, TOL[prec], "dJ/ddelta")
        assert_grad_close(dw.cpu().numpy(), wref, TOL[prec], "dJ/dw")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nb", [3, 12, 20])
def test_gamma_d4_value_and_gradient(mp3, prec, nb):
    """Grid summation with the Daubechies-4 connection coefficients (the 125-shift stencil): zeta
    from the forward and from the one sweep, and dJ/ddelta from the backward and the one sweep,
    against the oracle's stencil form; 12 and 20 bins take the bins in chunks (pairs of chunks in
    the forward, single chunks in the adjoint) at float64."""
    _say("gamma d4", prec, nb)
    n, box, lmax = 16, 160.0, 2
    edges = np.linspace(15.0, 55.0, nb + 1)
    delta = random_field(n, 241 + nb)
    lam = np.random.default_rng(242 + nb).standard_normal((lmax + 1, nb, nb))
    plan = mp3.Plan(n, box, lmax, edges, precision=prec, summation="gamma", basis="d4")
    dd = _dev(delta[None], torch.float64 if prec == "f64" else torch.float32)
    lt = _dev(lam[None], torch.float64)
    z = plan.zeta(dd)
    z1, g1, _ = plan.zeta_value_and_grad(dd, lt)
    g2, _ = plan.zeta_backward(dd, lt)
    op = E.Plan(n, box, lmax, edges, basis="d4")
    zref = E.zeta_gamma(op, delta)
    for zz in (z, z1):
        zz = zz.cpu().numpy()[0]
        assert_zeta_close(zz, zref, TOL[prec])
        assert np.abs(zz - zz.transpose(0, 2, 1)).max() <= 1e-12 * np.abs(zz).max()
    gref = A.zeta_gamma_grad(op, delta, lam)
    for g in (g1, g2):
        assert_grad_close(g.cpu().numpy()[0], gref, TOL[prec], "dJ/ddelta")


def test_gamma_d4_smoothing_and_batch(mp3):
    """The stencil form with the top-hat primary (its transposed filter in the gradient) on a batch
    of two fields, float64."""
    _say("gamma d4 smoothing batch")
    n, box, lmax, nb = 16, 160.0, 1, 4
    edges = np.linspace(15.0, 55.0, nb + 1)
    d = np.stack([random_field(n, 251), random_field(n, 252)])
    lam = np.random.default_rng(253).standard_normal((2, lmax + 1, nb, nb))
    plan = mp3.Plan(n, box, lmax, edges, precision="f64", summation="gamma", basis="d4", smoothing=12.0, batch=2)
    z, g, _ = plan.zeta_value_and_grad(_dev(d, torch.float64), _dev(lam, torch.float64))
    op = E.Plan(n, box, lmax, edges, basis="d4", smoothing=12.0)
    for j in range(2):
        assert_zeta_close(z.cpu().numpy()[j], E.zeta_gamma(op, d[j]), 1e-10)
        assert_grad_close(g.cpu().numpy()[j], A.zeta_gamma_grad(op, d[j], lam[j]), 1e-10, f"dJ/ddelta mock {j}")


def test_gamma_d4_bf16x3_is_unsupported(mp3):
    _say("gamma d4 bf16x3 unsupported")
    with pytest.raises(mp3.Mp3Error):
        mp3.Plan(16, 160.0, 1, [10.0, 20.0], summation="gamma", basis="d4", precision="bf16x3")


def test_d4_differs_from_b3(mp3):
    """The basis option reaches the kernels: the same catalogue deposits differently."""
    _say("d4 vs b3")
    n, box = 16, 128.0
    pos, w = lognormal_catalogue(n, box, 5000, 8.0, 231, 232, 233, (0.5, 1.5))
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    a = mp3.Plan(n, box, 0, [1.0, 2.0], precision="f64").deposit(pt, wt).cpu().numpy()
    b = mp3.Plan(n, box, 0, [1.0, 2.0], precision="f64", basis="d4").deposit(pt, wt).cpu().numpy()
    assert np.abs(a - b).max() > 1e-3 * np.abs(a).max()
