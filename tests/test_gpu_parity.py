"""GPU parity: the HIP path through the C ABI against the CPU float64 oracle.

Bars: the float64 form within 1e-10 relative, the float32 form within 1e-4
per multipole (see tests/_common.per_l_errors).  Inputs are seeded mocks and
random fields from ``mockgen``; expected values come only from ``oracle``.
"""
import numpy as np
import pytest

from mockgen import random_field, lognormal_catalogue, WORKLOADS, workload_catalogue, batch_sizes
from oracle import basis
from oracle import estimator as E
from oracle import adjoint as A
from tests._common import assert_zeta_close, per_l_errors, assert_grad_close

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


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,l,m,nb", [(16, 0, 0, 3), (16, 3, 2, 5), (32, 4, 4, 6), (64, 2, 1, 2), (128, 5, 3, 1)])
def test_multipole_fields(mp3, prec, n, l, m, nb):
    _say("fields", prec, n, l, m, nb)
    box = 10.0 * n
    edges = np.linspace(0.1 * box, 0.35 * box, nb + 1)
    delta = random_field(n, 100 + n + l)
    plan = mp3.Plan(n, box, max(l, 1), edges, precision=prec)
    rd = torch.float64 if prec == "f64" else torch.float32
    a = plan.multipole_fields(_dev(delta[None], rd), l, m).cpu().numpy()[0]
    oplan = E.Plan(n, box, max(l, 1), edges)
    ref = E.fields(oplan, np.fft.fftn(delta), l, m)
    err = np.linalg.norm(a - ref) / np.linalg.norm(ref)
    assert err < (1e-12 if prec == "f64" else 2e-6), err


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_deposit(mp3, prec):
    _say("deposit", prec)
    n, box = 32, 250.0
    pos, w = lognormal_catalogue(n, box, 20000, 4.0, 1001, 1002, 1003, (0.5, 1.5))
    plan = mp3.Plan(n, box, 1, [10.0, 20.0], precision=prec)
    d = plan.deposit(_dev(pos, torch.float32), _dev(w, torch.float32)).cpu().numpy()[0]
    ref = basis.density_contrast(basis.deposit(pos, w, n, box), float(np.sum(w.astype(np.float64))))
    err = np.abs(d - ref).max() / np.abs(ref).max()
    assert err < (1e-13 if prec == "f64" else 1e-6), err


def test_deposit_wraps_edge_positions(mp3):
    """Positions on the seam, at 0 and just below box, and outside [0, box) wrap periodically."""
    _say("deposit seam")
    n, box = 16, 100.0
    pos = np.array([[0.0, 0.0, 0.0], [np.nextafter(np.float32(box), np.float32(0)), 50.0, 99.9],
                    [6.25, 6.25, 6.25], [-3.0, 103.0, 250.0]], dtype=np.float32)
    plan = mp3.Plan(n, box, 0, [10.0, 20.0], precision="f64")
    d = plan.deposit(_dev(pos, torch.float32)).cpu().numpy()[0]
    wrapped = np.mod(pos.astype(np.float64), box).astype(np.float32)
    ref = basis.density_contrast(basis.deposit(wrapped, None, n, box), 4.0)
    assert np.abs(d - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,lmax,nb", [(16, 3, 4), (32, 4, 6), (64, 2, 5), (32, 6, 1)])
def test_zeta_random_field(mp3, prec, n, lmax, nb):
    _say("zeta random", prec, n, lmax, nb)
    box = 8.0 * n
    edges = np.linspace(0.05 * box, 0.4 * box, nb + 1)
    delta = random_field(n, 7 + n + nb)
    plan = mp3.Plan(n, box, lmax, edges, precision=prec)
    rd = torch.float64 if prec == "f64" else torch.float32
    z = plan.zeta(_dev(delta[None], rd)).cpu().numpy()[0]
    ref = E.zeta_nodal(E.Plan(n, box, lmax, edges), delta)
    e = assert_zeta_close(z, ref, TOL[prec])
    print("per-l errors", e)
    assert np.abs(z - z.transpose(0, 2, 1)).max() <= 1e-12 * np.abs(z).max()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_zeta_small_workload(mp3, prec):
    """Box 250, 32^3, L = 4, 6 bins, 2000-particle log-normal mock: deposit + nodal zeta."""
    wl = WORKLOADS["box250_n32_l4"]
    _say("zeta workload", wl.name, prec)
    pos, w = workload_catalogue(wl)
    plan = mp3.Plan(wl.n, wl.box, wl.lmax, wl.edges, precision=prec)
    delta = plan.deposit(_dev(pos, torch.float32), _dev(w, torch.float32))
    z = plan.zeta(delta).cpu().numpy()[0]
    dref = basis.density_contrast(basis.deposit(pos, w, wl.n, wl.box), float(len(w)))
    ref = E.zeta_nodal(E.Plan(wl.n, wl.box, wl.lmax, wl.edges), dref)
    e = assert_zeta_close(z, ref, TOL[prec])
    print("per-l errors", e)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_zeta_batch_uneven(mp3, prec):
    """Three mocks of uneven size in one call equal three separate oracle evaluations."""
    _say("batch", prec)
    n, box, lmax = 32, 500.0, 3
    edges = np.linspace(30.0, 150.0, 5)
    cats = [lognormal_catalogue(n, box, npart, 8.0, 5000 + 10 * j + 1, 5000 + 10 * j + 2)
            for j, npart in enumerate((3000, 11000, 500))]
    pos = np.concatenate([c[0] for c in cats])
    w = np.concatenate([c[1] for c in cats])
    off = np.cumsum([0] + [len(c[1]) for c in cats])
    plan = mp3.Plan(n, box, lmax, edges, precision=prec, batch=3)
    delta = plan.deposit(_dev(pos, torch.float32), _dev(w, torch.float32), off)
    z = plan.zeta(delta).cpu().numpy()
    op = E.Plan(n, box, lmax, edges)
    for j, (p, ww) in enumerate(cats):
        ref = E.zeta_nodal(op, basis.density_contrast(basis.deposit(p, ww, n, box), float(len(ww))))
        assert_zeta_close(z[j], ref, TOL[prec])


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,lmax,nb", [(16, 2, 3), (32, 3, 5)])
def test_backward_delta_and_weights(mp3, prec, n, lmax, nb):
    _say("backward", prec, n, lmax, nb)
    box = 10.0 * n
    edges = np.linspace(0.08 * box, 0.35 * box, nb + 1)
    pos, w = lognormal_catalogue(n, box, 4000, 0.05 * box, 61, 62, 63, (0.5, 1.5))
    lam = np.random.default_rng(64).standard_normal((lmax + 1, nb, nb))
    plan = mp3.Plan(n, box, lmax, edges, precision=prec)
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    delta = plan.deposit(pt, wt)
    dd, dw = plan.zeta_backward(delta, _dev(lam[None], torch.float64), pt, wt)
    dref = basis.density_contrast(basis.deposit(pos, w, n, box), float(np.sum(w.astype(np.float64))))
    op = E.Plan(n, box, lmax, edges)
    gref = A.zeta_nodal_grad(op, dref, lam)
    wref = A.deposit_weight_grad(pos, w, n, box, gref)
    tol = 1e-10 if prec == "f64" else 1e-4
    eg = assert_grad_close(dd.cpu().numpy()[0], gref, tol, "dJ/ddelta")
    ew = assert_grad_close(dw.cpu().numpy(), wref, tol, "dJ/dw")
    print("grad errors (L2, max)", eg, ew)


def test_backward_batch_autograd(mp3):
    """torch.autograd through Zeta3PCF on a batch of two fields equals the oracle gradient."""
    _say("autograd batch")
    n, box, lmax = 16, 160.0, 2
    edges = np.linspace(15.0, 55.0, 4)
    d = np.stack([random_field(n, 71), random_field(n, 72)])
    lam = np.random.default_rng(73).standard_normal((2, lmax + 1, 3, 3))
    plan = mp3.Plan(n, box, lmax, edges, precision="f64", batch=2)
    x = _dev(d, torch.float64).requires_grad_(True)
    z = mp3.Zeta3PCF.apply(x, plan)
    (z * _dev(lam, torch.float64)).sum().backward()
    op = E.Plan(n, box, lmax, edges)
    for j in range(2):
        ref = A.zeta_nodal_grad(op, d[j], lam[j])
        assert_grad_close(x.grad[j].cpu().numpy(), ref, 1e-10, f"dJ/ddelta mock {j}")


def test_weight_gradient_finite_difference_f64(mp3):
    """Central differences of J(w) along seeded unit directions on the float64 GPU form."""
    _say("fd weights")
    n, box, lmax = 16, 160.0, 2
    edges = np.linspace(15.0, 55.0, 4)
    pos, w = lognormal_catalogue(n, box, 3000, 8.0, 81, 82, 83, (0.5, 1.5))
    plan = mp3.Plan(n, box, lmax, edges, precision="f64")
    lam = np.random.default_rng(84).standard_normal((1, lmax + 1, 3, 3))
    lt = _dev(lam, torch.float64)
    pt = _dev(pos, torch.float32)
    w64 = w.astype(np.float64)

    def J(wv):
        wt = _dev(wv.astype(np.float32), torch.float32)
        return float((plan.zeta(plan.deposit(pt, wt)) * lt).sum())

    wt = _dev(w, torch.float32)
    _, dw = plan.zeta_backward(plan.deposit(pt, wt), lt, pt, wt)
    rng = np.random.default_rng(85)
    v = rng.standard_normal(w.shape)
    v /= np.linalg.norm(v)
    h = 1e-3
    # weights are float32 on the device: use the rounded perturbation actually applied
    wp = (w64 + h * v).astype(np.float32).astype(np.float64)
    wm = (w64 - h * v).astype(np.float32).astype(np.float64)
    fd = (J(wp) - J(wm))
    an = float(np.dot(dw.cpu().numpy(), wp - wm))
    assert abs(fd - an) < 1e-5 * abs(an)


def test_zeta_f32_matches_f64_form(mp3):
    """Float32 form against the float64 GPU form on a 128^3 log-normal mock (L = 8, 12 bins)."""
    wl = WORKLOADS["batch64_n128_l8"]
    _say("f32 vs f64", wl.name)
    pos, w = workload_catalogue(wl, 0)
    res = {}
    for prec in ("f32", "f64"):
        plan = mp3.Plan(wl.n, wl.box, wl.lmax, wl.edges, precision=prec)
        res[prec] = plan.zeta(plan.deposit(_dev(pos, torch.float32), _dev(w, torch.float32))).cpu().numpy()[0]
        del plan
        torch.cuda.empty_cache()
    assert_zeta_close(res["f32"], res["f64"], 1e-4)


def test_invalid_arguments_raise(mp3):
    _say("invalid args")
    plan = mp3.Plan(16, 100.0, 2, [10.0, 20.0, 30.0])
    d = torch.zeros((1, 16, 16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(mp3.Mp3Error):
        plan.multipole_fields(d, 3, 0)
    with pytest.raises(mp3.Mp3Error):
        plan.multipole_fields(d, 1, 2)
    pos = torch.zeros((4, 3), dtype=torch.float32, device="cuda")
    b2 = mp3.Plan(16, 100.0, 1, [10.0, 20.0], batch=2)
    with pytest.raises(ValueError):
        b2.deposit(pos, None, [0, 4, 4])       # empty second mock: the binding refuses it
    with pytest.raises(ValueError):
        b2.deposit(pos, None, [0, 2, 6])       # more particles than pos holds
    import ctypes
    from paper_2507_15209_amd import _lib
    # and so does the library itself
    off = np.array([0, 4, 4], dtype=np.int64)
    ws = b2._workspace(4)
    dd = torch.empty((2, 16, 16, 16), dtype=torch.float32, device="cuda")
    st = b2.lib.mp3_deposit(b2._h, ctypes.c_void_p(pos.data_ptr()), None,
                            off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.c_void_p(dd.data_ptr()),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert st == _lib.MP3_EINVAL
    z = torch.empty((1, 3, 2, 2), dtype=torch.float64, device="cuda")
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    st = plan.lib.mp3_zeta(plan._h, ctypes.c_void_p(d.data_ptr()), None, None, None, ctypes.c_void_p(z.data_ptr()),
                           ctypes.c_void_p(ws.data_ptr()), 16, None)
    assert st == _lib.MP3_EWORKSPACE
    pp = mp3.Plan(16, 100.0, 1, [10.0, 20.0], summation="particle")
    with pytest.raises(ValueError):
        pp.zeta(d)                                # catalogue missing
    with pytest.raises(ValueError):
        pp.zeta_backward(d, torch.zeros((1, 2, 1, 1), dtype=torch.float64, device="cuda"))   # catalogue missing
    dd = torch.zeros((1, 16, 16, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):                # dzeta of the wrong shape: the binding refuses it
        mp3.Plan(16, 100.0, 1, [10.0, 20.0], precision="f64").zeta_backward(dd, torch.zeros((1, 3, 1, 1),
                                                                              dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,lmax,nb,npart", [(16, 2, 3, 3000), (32, 4, 6, 20000), (64, 3, 5, 50000)])
def test_zeta_particle(mp3, prec, n, lmax, nb, npart):
    """Particle summation (primary on the catalogue, exact volume mean subtracted) against the oracle."""
    _say("particle", prec, n, lmax, nb, npart)
    box = 8.0 * n
    edges = np.linspace(0.06 * box, 0.35 * box, nb + 1)
    pos, w = lognormal_catalogue(n, box, npart, 0.04 * box, 90 + n, 91 + n, 92 + n, (0.5, 1.5))
    plan = mp3.Plan(n, box, lmax, edges, precision=prec, summation="particle")
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    delta = plan.deposit(pt, wt)
    z = plan.zeta(delta, pt, wt).cpu().numpy()[0]
    ref = E.zeta_particle(E.Plan(n, box, lmax, edges), pos, w)
    e = assert_zeta_close(z, ref, TOL[prec])
    print("per-l errors", e)
    assert np.abs(z - z.transpose(0, 2, 1)).max() <= 1e-12 * np.abs(z).max()


def test_zeta_particle_batch_uneven(mp3):
    """Two catalogues of different size in one particle-form call (float32, 40 bins: vector-ALU contraction)."""
    _say("particle batch")
    n, box, lmax = 32, 400.0, 2
    edges = np.linspace(20.0, 140.0, 41)
    cats = [lognormal_catalogue(n, box, npart, 10.0, 300 + j, 310 + j) for j, npart in enumerate((7000, 2500))]
    pos = np.concatenate([c[0] for c in cats])
    w = np.concatenate([c[1] for c in cats])
    off = np.cumsum([0] + [len(c[1]) for c in cats])
    plan = mp3.Plan(n, box, lmax, edges, precision="f32", batch=2, summation="particle")
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    delta = plan.deposit(pt, wt, off)
    z = plan.zeta(delta, pt, wt, off).cpu().numpy()
    op = E.Plan(n, box, lmax, edges)
    for j, (p_, w_) in enumerate(cats):
        assert_zeta_close(z[j], E.zeta_particle(op, p_, w_), 1e-4)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,lmax,nb", [(16, 2, 3), (32, 3, 5)])
def test_zeta_gamma_random_field(mp3, prec, n, lmax, nb):
    """Grid summation with connection coefficients against the oracle's Delta-stencil form."""
    _say("gamma", prec, n, lmax, nb)
    box = 8.0 * n
    edges = np.linspace(0.06 * box, 0.35 * box, nb + 1)
    delta = random_field(n, 50 + n)
    plan = mp3.Plan(n, box, lmax, edges, precision=prec, summation="gamma")
    rd = torch.float64 if prec == "f64" else torch.float32
    z = plan.zeta(_dev(delta[None], rd)).cpu().numpy()[0]
    ref = E.zeta_gamma_quadrature(E.Plan(n, box, lmax, edges), delta)
    e = assert_zeta_close(z, ref, TOL[prec])
    print("per-l errors", e)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_zeta_gamma_small_workload(mp3, prec):
    """Box 250, 32^3, L = 4, 6 bins, 2000-particle mock: the grid-Gamma form of the small workload."""
    wl = WORKLOADS["box250_n32_l4"]
    _say("gamma workload", prec)
    pos, w = workload_catalogue(wl)
    plan = mp3.Plan(wl.n, wl.box, wl.lmax, wl.edges, precision=prec, summation="gamma")
    delta = plan.deposit(_dev(pos, torch.float32), _dev(w, torch.float32))
    z = plan.zeta(delta).cpu().numpy()[0]
    dref = basis.density_contrast(basis.deposit(pos, w, wl.n, wl.box), float(len(w)))
    ref = E.zeta_gamma_quadrature(E.Plan(wl.n, wl.box, wl.lmax, wl.edges), dref)
    e = assert_zeta_close(z, ref, TOL[prec])
    print("per-l errors", e)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,lmax,nb,npart", [(16, 2, 3, 3000), (32, 3, 5, 20000)])
def test_backward_particle(mp3, prec, n, lmax, nb, npart):
    """Particle-form gradient (dJ/ddelta at fixed primary weights, dJ/dw) against the oracle's."""
    _say("backward particle", prec, n, lmax, nb, npart)
    box = 8.0 * n
    edges = np.linspace(0.06 * box, 0.35 * box, nb + 1)
    pos, w = lognormal_catalogue(n, box, npart, 0.04 * box, 190 + n, 191 + n, 192 + n, (0.5, 1.5))
    lam = np.random.default_rng(193 + n).standard_normal((1, lmax + 1, nb, nb))
    plan = mp3.Plan(n, box, lmax, edges, precision=prec, summation="particle")
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    delta = plan.deposit(pt, wt)
    g, dw = plan.zeta_backward(delta, _dev(lam, torch.float64), pt, wt)
    g, dw = g.cpu().numpy()[0], dw.cpu().numpy()
    gref, dwref = A.zeta_particle_grad(E.Plan(n, box, lmax, edges), pos, w, lam[0])
    eg = assert_grad_close(g, gref, TOL[prec], "dJ/ddelta")
    ew = assert_grad_close(dw, dwref, TOL[prec], "dJ/dw")
    print("grad errors (L2, max)", eg, ew)


def test_backward_particle_batch_autograd(mp3):
    """Two uneven catalogues, particle form, float32, through zeta_from_catalogue's autograd."""
    _say("backward particle batch")
    n, box, lmax = 32, 320.0, 2
    edges = np.linspace(20.0, 100.0, 5)
    cats = [lognormal_catalogue(n, box, npart, 12.0, 400 + j, 410 + j, 420 + j, (0.5, 1.5))
            for j, npart in enumerate((9000, 4000))]
    pos = np.concatenate([c[0] for c in cats])
    w = np.concatenate([c[1] for c in cats])
    off = np.cumsum([0] + [len(c[1]) for c in cats])
    lam = np.random.default_rng(430).standard_normal((2, lmax + 1, 4, 4))
    plan = mp3.Plan(n, box, lmax, edges, precision="f32", batch=2, summation="particle")
    pt = _dev(pos, torch.float32)
    wt = _dev(w, torch.float32).requires_grad_(True)
    z = mp3.zeta_from_catalogue(plan, pt, wt, off)
    (z * _dev(lam, torch.float64)).sum().backward()
    dw = wt.grad.cpu().numpy()
    op = E.Plan(n, box, lmax, edges)
    for j, (p_, w_) in enumerate(cats):
        _, dwref = A.zeta_particle_grad(op, p_, w_, lam[j])
        assert_grad_close(dw[off[j]:off[j + 1]], dwref, 1e-4, f"dJ/dw mock {j}")


# BF16-split contraction inputs: each product carries a relative error of about
# 2^-16 instead of 2^-24, random over the summed products; the float32 bar
# still holds (measured per-l errors 2e-7 .. 6e-6 on these cases)
TOL_BF16X3 = 1e-4


@pytest.mark.parametrize("summation,n,lmax,nb", [("nodal", 32, 4, 6), ("nodal", 32, 3, 20), ("gamma", 16, 2, 3),
                                                  ("gamma", 32, 3, 20), ("particle", 32, 3, 5)])
def test_zeta_bf16x3(mp3, summation, n, lmax, nb):
    """float32 fields with BF16-split inputs to the matrix-core contraction, against the oracle."""
    _say("bf16x3", summation, n, lmax, nb)
    box = 8.0 * n
    edges = np.linspace(0.06 * box, 0.35 * box, nb + 1)
    op = E.Plan(n, box, lmax, edges)
    out = {}
    for prec in ("bf16x3", "f32"):
        plan = mp3.Plan(n, box, lmax, edges, precision=prec, summation=summation)
        if summation == "particle":
            pos, w = lognormal_catalogue(n, box, 20000, 0.04 * box, 500 + n, 501 + n, 502 + n, (0.5, 1.5))
            pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
            out[prec] = plan.zeta(plan.deposit(pt, wt), pt, wt).cpu().numpy()[0]
        else:
            delta = random_field(n, 510 + n + nb)
            out[prec] = plan.zeta(_dev(delta[None], torch.float32)).cpu().numpy()[0]
    if summation == "particle":
        ref = E.zeta_particle(op, pos, w)
    elif summation == "gamma":
        ref = E.zeta_gamma(op, delta)
    else:
        ref = E.zeta_nodal(op, delta)
    e16 = assert_zeta_close(out["bf16x3"], ref, TOL_BF16X3)
    e32 = assert_zeta_close(out["f32"], ref, 1e-4)
    print("per-l errors bf16x3", e16, "f32", e32)
    z = out["bf16x3"]
    assert np.abs(z - z.transpose(0, 2, 1)).max() <= 1e-12 * np.abs(z).max()


@pytest.mark.parametrize("summation", ["nodal", "particle", "gamma"])
def test_zeta_20_bins_matrix_cores(mp3, summation):
    """17..20 bins take the 4x4-block matrix-core contraction (nodal z pass, gather and grid-Gamma)."""
    _say("20 bins", summation)
    n, box, lmax, nb = (128, 1024.0, 2, 20) if summation != "gamma" else (32, 256.0, 2, 18)
    edges = np.linspace(0.05 * box, 0.3 * box, nb + 1)
    op = E.Plan(n, box, lmax, edges)
    plan = mp3.Plan(n, box, lmax, edges, precision="f32", summation=summation)
    if summation == "particle":
        pos, w = lognormal_catalogue(n, box, 30000, 0.03 * box, 600, 601, 602, (0.5, 1.5))
        pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
        z = plan.zeta(plan.deposit(pt, wt), pt, wt).cpu().numpy()[0]
        ref = E.zeta_particle(op, pos, w)
    else:
        delta = random_field(n, 603)
        z = plan.zeta(_dev(delta[None], torch.float32)).cpu().numpy()[0]
        ref = E.zeta_gamma(op, delta) if summation == "gamma" else E.zeta_nodal(op, delta)
    e = assert_zeta_close(z, ref, 1e-4)
    print("per-l errors", e)
    assert np.abs(z - z.transpose(0, 2, 1)).max() <= 1e-12 * np.abs(z).max()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,lmax,nb", [(16, 2, 3), (16, 3, 6), (32, 2, 4)])
def test_backward_gamma(mp3, prec, n, lmax, nb):
    """Grid-Gamma gradient (dJ/ddelta and dJ/dw through the deposit) against the oracle's."""
    _say("backward gamma", prec, n, lmax, nb)
    box = 8.0 * n
    edges = np.linspace(0.06 * box, 0.35 * box, nb + 1)
    pos, w = lognormal_catalogue(n, box, 6000, 0.04 * box, 700 + n, 701 + n, 702 + n, (0.5, 1.5))
    lam = np.random.default_rng(703 + n + nb).standard_normal((1, lmax + 1, nb, nb))
    plan = mp3.Plan(n, box, lmax, edges, precision=prec, summation="gamma")
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    delta = plan.deposit(pt, wt)
    g, dw = plan.zeta_backward(delta, _dev(lam, torch.float64), pt, wt)
    g, dw = g.cpu().numpy()[0], dw.cpu().numpy()
    dref = basis.density_contrast(basis.deposit(pos, w, n, box), float(np.sum(w.astype(np.float64))))
    gref = A.zeta_gamma_grad(E.Plan(n, box, lmax, edges), dref, lam[0])
    dwref = A.deposit_weight_grad(pos, w, n, box, gref)
    eg = assert_grad_close(g, gref, TOL[prec], "dJ/ddelta")
    ew = assert_grad_close(dw, dwref, TOL[prec], "dJ/dw")
    print("grad errors (L2, max)", eg, ew)


def test_backward_gamma_20_bins_autograd(mp3):
    """20 bins (the largest float32 adjoint tile) through the autograd wrapper of the catalogue."""
    _say("backward gamma 20 bins")
    n, box, lmax, nb = 16, 160.0, 1, 20
    edges = np.linspace(10.0, 60.0, nb + 1)
    pos, w = lognormal_catalogue(n, box, 4000, 6.0, 710, 711, 712, (0.5, 1.5))
    lam = np.random.default_rng(713).standard_normal((1, lmax + 1, nb, nb))
    plan = mp3.Plan(n, box, lmax, edges, precision="f32", summation="gamma")
    pt = _dev(pos, torch.float32)
    wt = _dev(w, torch.float32).requires_grad_(True)
    z = mp3.zeta_from_catalogue(plan, pt, wt)
    (z * _dev(lam, torch.float64)).sum().backward()
    dref = basis.density_contrast(basis.deposit(pos, w, n, box), float(np.sum(w.astype(np.float64))))
    gref = A.zeta_gamma_grad(E.Plan(n, box, lmax, edges), dref, lam[0])
    dwref = A.deposit_weight_grad(pos, w, n, box, gref)
    assert_grad_close(wt.grad.cpu().numpy(), dwref, 1e-4, "dJ/dw")


def test_extreme_orders_and_bins(mp3):
    """The largest multipole order (L = 20) and the largest bin count (64, vector-ALU contraction and adjoint)."""
    _say("extremes")
    n, box = 16, 160.0
    delta = random_field(n, 800)
    # L = 20, 2 bins, float64
    edges = np.array([20.0, 40.0, 60.0])
    plan = mp3.Plan(n, box, 20, edges, precision="f64")
    z = plan.zeta(_dev(delta[None], torch.float64)).cpu().numpy()[0]
    assert_zeta_close(z, E.zeta_nodal(E.Plan(n, box, 20, edges), delta), 1e-10)
    # 64 bins, L = 1, float32 forward and gradient
    edges = np.linspace(5.0, 70.0, 65)
    op = E.Plan(n, box, 1, edges)
    plan = mp3.Plan(n, box, 1, edges, precision="f32")
    d = _dev(delta[None], torch.float32)
    z = plan.zeta(d).cpu().numpy()[0]
    assert_zeta_close(z, E.zeta_nodal(op, delta), 1e-4)
    lam = np.random.default_rng(801).standard_normal((1, 2, 64, 64))
    g, _ = plan.zeta_backward(d, _dev(lam, torch.float64))
    gref = A.zeta_nodal_grad(op, delta, lam[0])
    assert_grad_close(g.cpu().numpy()[0], gref, 1e-4, "dJ/ddelta, 64 bins")


@pytest.mark.parametrize("summation", ["nodal", "gamma", "particle"])
def test_degenerate_inputs(mp3, summation):
    """A zero contrast gives zeta = 0 and a zero gradient; a one-particle catalogue deposits exactly."""
    _say("degenerate", summation)
    n, box, lmax = 16, 160.0, 2
    edges = np.linspace(15.0, 55.0, 4)
    plan = mp3.Plan(n, box, lmax, edges, precision="f64", summation=summation)
    lam = _dev(np.ones((1, lmax + 1, 3, 3)), torch.float64)
    # one particle at a node: delta = B3 stencil * n^3 - 1, exactly
    pos = np.array([[50.0, 70.0, 90.0]], dtype=np.float32)
    pt = _dev(pos, torch.float32)
    d = plan.deposit(pt)
    ref = basis.density_contrast(basis.deposit(pos, None, n, box), 1.0)
    assert np.abs(d.cpu().numpy()[0] - ref).max() <= 1e-12 * np.abs(ref).max()
    if summation == "particle":
        # a lone particle at a node: by the blob's cubic symmetry F_l(u) = 0 for l = 1, 2,
        # so zeta_{l>0} is minus the volume mean alone
        z = plan.zeta(d, pt).cpu().numpy()[0]
        assert_zeta_close(z, E.zeta_particle(E.Plan(n, box, lmax, edges), pos, None), 1e-10)
        return
    zero = torch.zeros((1, n, n, n), dtype=torch.float64, device="cuda")
    z = plan.zeta(zero).cpu().numpy()
    assert np.all(z == 0.0)
    g, _ = plan.zeta_backward(zero, lam)
    assert torch.count_nonzero(g).item() == 0


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,lmax,nb", [(16, 2, 3), (32, 3, 5), (32, 3, 20), (32, 2, 24), (16, 2, 32)])
def test_value_and_grad_nodal(mp3, prec, n, lmax, nb):
    """One-sweep value and gradient: zeta, dJ/ddelta and dJ/dw against the oracle and the two separate calls."""
    _say("value and grad", prec, n, lmax, nb)
    box = 10.0 * n
    edges = np.linspace(0.08 * box, 0.35 * box, nb + 1)
    pos, w = lognormal_catalogue(n, box, 6000, 0.05 * box, 81 + nb, 82 + nb, 83 + nb, (0.5, 1.5))
    lam = np.random.default_rng(84 + nb).standard_normal((lmax + 1, nb, nb))
    plan = mp3.Plan(n, box, lmax, edges, precision=prec)
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    delta = plan.deposit(pt, wt)
    lt = _dev(lam[None], torch.float64)
    z, dd, dw = plan.zeta_value_and_grad(delta, lt, pt, wt)
    z2 = plan.zeta(delta)
    dd2, dw2 = plan.zeta_backward(delta, lt, pt, wt)
    dref = basis.density_contrast(basis.deposit(pos, w, n, box), float(np.sum(w.astype(np.float64))))
    op = E.Plan(n, box, lmax, edges)
    zref = E.zeta_nodal(op, dref)
    gref = A.zeta_nodal_grad(op, dref, lam)
    wref = A.deposit_weight_grad(pos, w, n, box, gref)
    tol = TOL[prec]
    assert_zeta_close(z.cpu().numpy()[0], zref, tol)
    eg = assert_grad_close(dd.cpu().numpy()[0], gref, tol, "dJ/ddelta")
    ew = assert_grad_close(dw.cpu().numpy(), wref, tol, "dJ/dw")
    print("grad errors (L2, max)", eg, ew)
    # against the separate calls: rounding-order differences only
    agree = 1e-12 if prec == "f64" else 2e-5
    assert_zeta_close(z.cpu().numpy()[0], z2.cpu().numpy()[0], agree)
    g1, g2 = dd.cpu().numpy(), dd2.cpu().numpy()
    assert np.abs(g1 - g2).max() <= agree * np.abs(g2).max()
    zz = z.cpu().numpy()[0]
    assert np.abs(zz - zz.transpose(0, 2, 1)).max() <= 1e-12 * np.abs(zz).max()


def test_value_and_grad_batch_and_other_forms(mp3):
    """A batch of uneven mocks (float32, 12 bins), and the forms that run the two calls in turn (identical results)."""
    _say("value and grad batch")
    n, box, lmax, batch = 32, 250.0, 3, 3
    edges = np.linspace(20.0, 90.0, 13)
    sizes = [int(s) for s in batch_sizes(batch, 91, 2000, 8000)]
    cats = [lognormal_catalogue(n, box, s, 12.0, 92 + j, 95 + j, 98 + j, (0.5, 1.5)) for j, s in enumerate(sizes)]
    pos = np.concatenate([c[0] for c in cats])
    w = np.concatenate([c[1] for c in cats])
    off = np.concatenate([[0], np.cumsum(sizes)])
    lam = np.random.default_rng(101).standard_normal((batch, lmax + 1, 12, 12))
    pt, wt, lt = _dev(pos, torch.float32), _dev(w, torch.float32), _dev(lam, torch.float64)
    plan = mp3.Plan(n, box, lmax, edges, precision="f32", batch=batch)
    delta = plan.deposit(pt, wt, off)
    z, dd, dw = plan.zeta_value_and_grad(delta, lt, pt, wt, off)
    op = E.Plan(n, box, lmax, edges)
    for j, (p, ww) in enumerate(cats):
        dref = basis.density_contrast(basis.deposit(p, ww, n, box), float(np.sum(ww.astype(np.float64))))
        assert_zeta_close(z.cpu().numpy()[j], E.zeta_nodal(op, dref), 1e-4)
        gref = A.zeta_nodal_grad(op, dref, lam[j])
        wref = A.deposit_weight_grad(p, ww, n, box, gref)
        assert_grad_close(dd.cpu().numpy()[j], gref, 1e-4, f"dJ/ddelta mock {j}")
        assert_grad_close(dw.cpu().numpy()[off[j]:off[j + 1]], wref, 1e-4, f"dJ/dw mock {j}")
    for summation, prec in (("particle", "f64"), ("gamma", "f64"), ("nodal", "bf16x3")):
        _say("value and grad, two calls:", summation, prec)
        n2, box2, lmax2 = 16, 160.0, 2
        edges2 = np.linspace(15.0, 55.0, 4)
        p2, w2 = lognormal_catalogue(n2, box2, 3000, 8.0, 111, 112, 113, (0.5, 1.5))
        pt2, wt2 = _dev(p2, torch.float32), _dev(w2, torch.float32)
        lam2 = _dev(np.random.default_rng(114).standard_normal((1, lmax2 + 1, 3, 3)), torch.float64)
        plan2 = mp3.Plan(n2, box2, lmax2, edges2, precision=prec, summation=summation)
        d2 = plan2.deposit(pt2, wt2)
        cat = (pt2, wt2) if summation == "particle" else ()
        z1, g1, w1 = plan2.zeta_value_and_grad(d2, lam2, pt2, wt2)
        z0 = plan2.zeta(d2, *cat)
        g0, w0 = plan2.zeta_backward(d2, lam2, pt2, wt2)
        # the same two calls run; the grid-Gamma adjoint folds tiles with atomics (summation order varies)
        agree = 1e-12 if prec == "f64" else 2e-5
        assert_zeta_close(z1.cpu().numpy()[0], z0.cpu().numpy()[0], agree)
        for a1, a0 in ((g1, g0), (w1, w0)):
            a1, a0 = a1.cpu().numpy(), a0.cpu().numpy()
            assert np.abs(a1 - a0).max() <= agree * np.abs(a0).max()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_value_and_grad_particle(mp3, prec):
    """Particle form in one sweep: zeta, dJ/ddelta and dJ/dw against the oracle."""
    _say("value and grad particle", prec)
    n, lmax, nb, npart = 32, 3, 5, 20000
    box = 8.0 * n
    edges = np.linspace(0.06 * box, 0.35 * box, nb + 1)
    pos, w = lognormal_catalogue(n, box, npart, 0.04 * box, 121, 122, 123, (0.5, 1.5))
    lam = np.random.default_rng(124).standard_normal((1, lmax + 1, nb, nb))
    plan = mp3.Plan(n, box, lmax, edges, precision=prec, summation="particle")
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    delta = plan.deposit(pt, wt)
    z, g, dw = plan.zeta_value_and_grad(delta, _dev(lam, torch.float64), pt, wt)
    op = E.Plan(n, box, lmax, edges)
    assert_zeta_close(z.cpu().numpy()[0], E.zeta_particle(op, pos, w), TOL[prec])
    gref, dwref = A.zeta_particle_grad(op, pos, w, lam[0])
    eg = assert_grad_close(g.cpu().numpy()[0], gref, TOL[prec], "dJ/ddelta")
    ew = assert_grad_close(dw.cpu().numpy(), dwref, TOL[prec], "dJ/dw")
    print("grad errors (L2, max)", eg, ew)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nb", [3, 18])
def test_value_and_grad_gamma(mp3, prec, nb):
    """Grid-Gamma form in one sweep (the adjoint kernel also contracts): zeta and dJ/ddelta against the oracle."""
    _say("value and grad gamma", prec, nb)
    n, box, lmax = 16, 160.0, 2
    edges = np.linspace(15.0, 55.0, nb + 1)
    delta = random_field(n, 131 + nb)
    lam = np.random.default_rng(132 + nb).standard_normal((lmax + 1, nb, nb))
    plan = mp3.Plan(n, box, lmax, edges, precision=prec, summation="gamma")
    dd = _dev(delta[None], torch.float64 if prec == "f64" else torch.float32)
    z, g, _ = plan.zeta_value_and_grad(dd, _dev(lam[None], torch.float64))
    op = E.Plan(n, box, lmax, edges)
    assert_zeta_close(z.cpu().numpy()[0], E.zeta_gamma(op, delta), TOL[prec])
    gref = A.zeta_gamma_grad(op, delta, lam)
    eg = assert_grad_close(g.cpu().numpy()[0], gref, TOL[prec], "dJ/ddelta")
    print("grad error (L2, max)", eg)
    zz = z.cpu().numpy()[0]
    assert np.abs(zz - zz.transpose(0, 2, 1)).max() <= 1e-12 * np.abs(zz).max()


@pytest.mark.parametrize("nb", [10, 15, 20])
def test_particle_gradient_bin_chunks(mp3, nb):
    """Particle-form gradients where the adjoint scatter takes its bins in chunks.

    float32: 10 bins in one 10-bin workgroup chunk, 15 bins in two 8-bin
    chunks, 20 bins in two 10-bin chunks; float64: 4-bin chunks (3, 4, 5 of
    them).  Both the separate backward and the one-sweep value and gradient,
    for dJ/ddelta and dJ/dw, against the oracle (L2 and element-wise)."""
    n, lmax, npart = 32, 1, 20000
    box = 8.0 * n
    edges = np.linspace(0.06 * box, 0.35 * box, nb + 1)
    pos, w = lognormal_catalogue(n, box, npart, 0.04 * box, 1300 + nb, 1301 + nb, 1302 + nb, (0.5, 1.5))
    lam = np.random.default_rng(1303 + nb).standard_normal((1, lmax + 1, nb, nb))
    op = E.Plan(n, box, lmax, edges)
    _say("particle gradient chunks: oracle", nb)
    zref = E.zeta_particle(op, pos, w)
    gref, dwref = A.zeta_particle_grad(op, pos, w, lam[0])
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    for prec in ("f32", "f64"):
        _say("particle gradient chunks: GPU", prec, nb)
        plan = mp3.Plan(n, box, lmax, edges, precision=prec, summation="particle")
        delta = plan.deposit(pt, wt)
        lt = _dev(lam, torch.float64)
        g0, dw0 = plan.zeta_backward(delta, lt, pt, wt)
        z1, g1, dw1 = plan.zeta_value_and_grad(delta, lt, pt, wt)
        assert_zeta_close(z1.cpu().numpy()[0], zref, TOL[prec])
        for call, g, dw in (("backward", g0, dw0), ("value_and_grad", g1, dw1)):
            eg = assert_grad_close(g.cpu().numpy()[0], gref, TOL[prec], f"{prec} {call} dJ/ddelta")
            ew = assert_grad_close(dw.cpu().numpy(), dwref, TOL[prec], f"{prec} {call} dJ/dw")
            print(prec, call, "grad errors (L2, max)", eg, ew)


@pytest.mark.parametrize("prec,nb", [("f64", 20), ("f64", 12), ("f32", 24), ("f32", 30)])
def test_gamma_bin_chunks(mp3, prec, nb):
    """Grid-Gamma plans whose tiles do not hold every bin: the contraction by pairs of bin chunks
    (float64 above 14 bins, float32 above 28) and the adjoint by bin chunks through the grid mix of
    the fields (float64 above 9 bins, float32 above 20): zeta, dJ/ddelta and dJ/dw, separate calls
    and one sweep, against the oracle (30 bins: zeta only, the oracle's gradient being slow there)."""
    _say("gamma bin chunks", prec, nb)
    n, box, lmax = 16, 160.0, 1
    edges = np.linspace(12.0, 60.0, nb + 1)
    pos, w = lognormal_catalogue(n, box, 5000, 6.0, 1601, 1602, 1603, (0.5, 1.5))
    lam = np.random.default_rng(1604 + nb).standard_normal((1, lmax + 1, nb, nb))
    plan = mp3.Plan(n, box, lmax, edges, precision=prec, summation="gamma")
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    delta = plan.deposit(pt, wt)
    lt = _dev(lam, torch.float64)
    z0 = plan.zeta(delta).cpu().numpy()[0]
    dref = basis.density_contrast(basis.deposit(pos, w, n, box), float(np.sum(w.astype(np.float64))))
    op = E.Plan(n, box, lmax, edges)
    zref = E.zeta_gamma(op, dref)
    if nb == 30:
        assert_zeta_close(z0, zref, TOL[prec])
        return
    g0, dw0 = plan.zeta_backward(delta, lt, pt, wt)
    z1, g1, dw1 = plan.zeta_value_and_grad(delta, lt, pt, wt)
    gref = A.zeta_gamma_grad(op, dref, lam[0])
    wref = A.deposit_weight_grad(pos, w, n, box, gref)
    for z, g, dw in ((z0, g0, dw0), (z1.cpu().numpy()[0], g1, dw1)):
        e = assert_zeta_close(z, zref, TOL[prec])
        eg = assert_grad_close(g.cpu().numpy()[0], gref, TOL[prec], "dJ/ddelta")
        ew = assert_grad_close(dw.cpu().numpy(), wref, TOL[prec], "dJ/dw")
        print("per-l", e, "grad (L2, max)", eg, ew)
        assert np.abs(z - z.transpose(0, 2, 1)).max() <= 1e-12 * np.abs(z).max()
