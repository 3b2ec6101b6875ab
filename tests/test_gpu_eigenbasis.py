"""GPU: the nodal and particle gradients run in the eigenbasis of each symmetrised cotangent
(radial tables rotated per (l, mock), diagonal adjoint sources, the value rotated back).  These
cases stress the eigen-decomposition: equal eigenvalues (a multiple of the identity, nothing to
rotate), a single off-diagonal entry given on one side only (symmetrised to a rank-2 indefinite
matrix), an all-zero cotangent, and different cotangents per mock of a batch.  Bars as in the
parity tests: 1e-10 (float64) / 1e-4 (float32) against the oracle, which takes the cotangent as
given (no rotation)."""
import numpy as np
import pytest

from mockgen import lognormal_catalogue, batch_sizes
from oracle import basis
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


def _cotangent(kind, lmax, nb, seed):
    lam = np.zeros((lmax + 1, nb, nb))
    if kind == "identity":
        for l in range(lmax + 1):
            lam[l] = (2.5 - 0.5 * l) * np.eye(nb)
    elif kind == "single":
        lam[1, 0, nb - 1] = 1.0                      # symmetrised: 0.5 at (0, nb-1) and (nb-1, 0)
    elif kind == "mixed":
        rng = np.random.default_rng(seed)
        lam = rng.standard_normal((lmax + 1, nb, nb))
        lam[0] = np.diag(rng.standard_normal(nb))     # already diagonal
        lam[lmax] = 0.0                               # nothing for the last multipole
    return lam


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["identity", "single", "mixed"])
def test_nodal_degenerate_cotangents(mp3, prec, kind):
    """One sweep and the separate backward against the oracle for cotangents with repeated or zero eigenvalues."""
    _say("nodal cotangent", kind, prec)
    n, lmax, nb = 32, 3, 7
    box = 10.0 * n
    edges = np.linspace(0.08 * box, 0.35 * box, nb + 1)
    pos, w = lognormal_catalogue(n, box, 6000, 0.05 * box, 301, 302, 303, (0.5, 1.5))
    lam = _cotangent(kind, lmax, nb, 304)
    plan = mp3.Plan(n, box, lmax, edges, precision=prec)
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    delta = plan.deposit(pt, wt)
    lt = _dev(lam[None], torch.float64)
    z, dd, dw = plan.zeta_value_and_grad(delta, lt, pt, wt)
    dd2, dw2 = plan.zeta_backward(delta, lt, pt, wt)
    dref = basis.density_contrast(basis.deposit(pos, w, n, box), float(np.sum(w.astype(np.float64))))
    op = E.Plan(n, box, lmax, edges)
    zz = z.cpu().numpy()[0]
    assert_zeta_close(zz, E.zeta_nodal(op, dref), TOL[prec])
    assert np.abs(zz - zz.transpose(0, 2, 1)).max() <= 1e-12 * np.abs(zz).max()
    gref = A.zeta_nodal_grad(op, dref, lam)
    wref = A.deposit_weight_grad(pos, w, n, box, gref)
    for g, gw in ((dd, dw), (dd2, dw2)):
        assert_grad_close(g.cpu().numpy()[0], gref, TOL[prec], "dJ/ddelta")
        assert_grad_close(gw.cpu().numpy(), wref, TOL[prec], "dJ/dw")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_zero_cotangent(mp3, prec):
    """dzeta = 0: the gradients are exactly zero and the one sweep still returns zeta."""
    _say("zero cotangent", prec)
    n, lmax, nb = 16, 2, 4
    box = 160.0
    edges = np.linspace(15.0, 55.0, nb + 1)
    pos, w = lognormal_catalogue(n, box, 3000, 8.0, 311, 312, 313, (0.5, 1.5))
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    lt = _dev(np.zeros((1, lmax + 1, nb, nb)), torch.float64)
    for summation in ("nodal", "particle"):
        plan = mp3.Plan(n, box, lmax, edges, precision=prec, summation=summation)
        delta = plan.deposit(pt, wt)
        z, dd, dw = plan.zeta_value_and_grad(delta, lt, pt, wt)
        zp = plan.zeta(delta, pt, wt).cpu().numpy()[0]
        assert_zeta_close(z.cpu().numpy()[0], zp, 1e-12 if prec == "f64" else 2e-5)
        # the particle form's volume-mean term does not depend on the cotangent either
        assert np.abs(dd.cpu().numpy()).max() == 0.0, summation
        assert np.abs(dw.cpu().numpy()).max() == 0.0, summation


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_per_mock_cotangents_batch(mp3, prec):
    """A batch of two mocks with different cotangents (one random, one diagonal): each mock's
    fields come from its own rotated tables."""
    _say("per-mock cotangents", prec)
    n, box, lmax, nb, batch = 32, 250.0, 2, 6, 2
    edges = np.linspace(20.0, 90.0, nb + 1)
    sizes = [int(s) for s in batch_sizes(batch, 321, 2000, 6000)]
    cats = [lognormal_catalogue(n, box, s, 12.0, 322 + j, 324 + j, 326 + j, (0.5, 1.5)) for j, s in enumerate(sizes)]
    pos = np.concatenate([c[0] for c in cats])
    w = np.concatenate([c[1] for c in cats])
    rng = np.random.default_rng(328)
    lam = np.stack([rng.standard_normal((lmax + 1, nb, nb)),
                    np.stack([np.diag(rng.standard_normal(nb)) for _ in range(lmax + 1)])])
    plan = mp3.Plan(n, box, lmax, edges, precision=prec, batch=batch)
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    np_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    delta = plan.deposit(pt, wt, np_off)
    z, dd, _ = plan.zeta_value_and_grad(delta, _dev(lam, torch.float64), pt, wt, np_off)
    op = E.Plan(n, box, lmax, edges)
    for j in range(batch):
        pj, wj = cats[j]
        dref = basis.density_contrast(basis.deposit(pj, wj, n, box), float(np.sum(wj.astype(np.float64))))
        assert_zeta_close(z.cpu().numpy()[j], E.zeta_nodal(op, dref), TOL[prec])
        assert_grad_close(dd.cpu().numpy()[j], A.zeta_nodal_grad(op, dref, lam[j]), TOL[prec], f"dJ/ddelta mock {j}")


@pytest.mark.parametrize("kind", ["identity", "single"])
def test_particle_degenerate_cotangents(mp3, kind):
    """Particle form at 20 bins (three particles per wave in the gather) in float32: one sweep
    and the separate backward against the oracle."""
    _say("particle cotangent", kind)
    n, lmax, nb, npart = 32, 2, 20, 20000
    box = 8.0 * n
    edges = np.linspace(0.06 * box, 0.35 * box, nb + 1)
    pos, w = lognormal_catalogue(n, box, npart, 0.04 * box, 331, 332, 333, (0.5, 1.5))
    lam = _cotangent(kind, lmax, nb, 334)
    plan = mp3.Plan(n, box, lmax, edges, precision="f32", summation="particle")
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    delta = plan.deposit(pt, wt)
    lt = _dev(lam[None], torch.float64)
    z, g, dw = plan.zeta_value_and_grad(delta, lt, pt, wt)
    g2, dw2 = plan.zeta_backward(delta, lt, pt, wt)
    op = E.Plan(n, box, lmax, edges)
    assert_zeta_close(z.cpu().numpy()[0], E.zeta_particle(op, pos, w), TOL["f32"])
    gref, dwref = A.zeta_particle_grad(op, pos, w, lam)
    for gg, ww in ((g, dw), (g2, dw2)):
        assert_grad_close(gg.cpu().numpy()[0], gref, TOL["f32"], "dJ/ddelta")
        assert_grad_close(ww.cpu().numpy(), dwref, TOL["f32"], "dJ/dw")
