"""GPU: the launch-shape knobs and the autotuner leave the results unchanged.

Every knob value is checked against the float64 oracle (deposit 1e-13,
zeta 1e-10 relative per multipole) or, for the backward, against the
default knobs' output of the same float64 path at 1e-12.
"""
import numpy as np
import pytest

from mockgen import random_field, lognormal_catalogue, batch_sizes
from oracle import basis
from oracle import estimator as E
from tests._common import assert_zeta_close, assert_grad_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("n", [16, 32, 64])
@pytest.mark.parametrize("tile", [4, 8, 16])
@pytest.mark.parametrize("wgs", [64, 2048])
def test_deposit_tiles(mp3, n, tile, wgs):
    _say("deposit tile", n, tile, wgs)
    box = 8.0 * n
    pos, w = lognormal_catalogue(n, box, 30000, 2.0, 2001 + n, 2002, 2003, (0.5, 1.5))
    plan = mp3.Plan(n, box, 1, [10.0, 20.0], precision="f64")
    plan.tune_set("deposit_tile", tile)
    plan.tune_set("deposit_wgs", wgs)
    d = plan.deposit(_dev(pos, torch.float32), _dev(w, torch.float32)).cpu().numpy()[0]
    ref = basis.density_contrast(basis.deposit(pos, w, n, box), float(np.sum(w.astype(np.float64))))
    assert np.abs(d - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("tile", [4, 16])
def test_deposit_tiles_batch_uneven(mp3, tile):
    _say("deposit tile batch", tile)
    n, box, batch = 32, 250.0, 5
    sizes = [int(s) for s in batch_sizes(batch, 77, 300, 9000)]
    cats = [lognormal_catalogue(n, box, s, 3.0, 3001 + j, 3101 + j, 3201 + j, (0.5, 1.5)) for j, s in enumerate(sizes)]
    pos = np.concatenate([c[0] for c in cats])
    w = np.concatenate([c[1] for c in cats])
    off = np.concatenate([[0], np.cumsum(sizes)])
    plan = mp3.Plan(n, box, 1, [10.0, 20.0], precision="f64", batch=batch)
    plan.tune_set("deposit_tile", tile)
    d = plan.deposit(_dev(pos, torch.float32), _dev(w, torch.float32), off).cpu().numpy()
    for j, (p, ww) in enumerate(cats):
        ref = basis.density_contrast(basis.deposit(p, ww, n, box), float(np.sum(ww.astype(np.float64))))
        assert np.abs(d[j] - ref).max() <= 1e-13 * np.abs(ref).max(), j


@pytest.mark.parametrize("knob,value", [("zpass_wgs", 64), ("zpass_wgs", 16384), ("fft_x_plan", 1)])
def test_knobs_keep_nodal_zeta_and_gradient(mp3, knob, value):
    _say("nodal knob", knob, value)
    n, box, lmax = 32, 320.0, 4
    edges = np.linspace(30.0, 110.0, 7)
    delta = random_field(n, 4001)
    dd = _dev(delta[None], torch.float64)
    lam = _dev(np.random.default_rng(4002).standard_normal((1, lmax + 1, 6, 6)), torch.float64)
    base = mp3.Plan(n, box, lmax, edges, precision="f64")
    g0, _ = base.zeta_backward(dd, lam)
    plan = mp3.Plan(n, box, lmax, edges, precision="f64")
    plan.tune_set(knob, value)
    assert plan.tune_get(knob) == value
    z = plan.zeta(dd).cpu().numpy()[0]
    ref = E.zeta_nodal(E.Plan(n, box, lmax, edges), delta)
    assert_zeta_close(z, ref, 1e-10)
    g1, _ = plan.zeta_backward(dd, lam)
    g0, g1 = g0.cpu().numpy(), g1.cpu().numpy()
    assert np.abs(g1 - g0).max() <= 1e-12 * np.abs(g0).max()


@pytest.mark.parametrize("summation", ["gamma", "particle"])
@pytest.mark.parametrize("value", [64, 16384])
def test_contract_workgroups_keep_zeta(mp3, summation, value):
    _say("contract knob", summation, value)
    n, box, lmax = 16, 160.0, 3
    edges = np.linspace(15.0, 55.0, 5)
    oplan = E.Plan(n, box, lmax, edges)
    plan = mp3.Plan(n, box, lmax, edges, precision="f64", summation=summation)
    plan.tune_set("contract_wgs", value)
    if summation == "gamma":
        delta = random_field(n, 5001)
        z = plan.zeta(_dev(delta[None], torch.float64)).cpu().numpy()[0]
        ref = E.zeta_gamma(oplan, delta)
    else:
        pos, w = lognormal_catalogue(n, box, 5000, 2.0, 5002, 5003, 5004, (0.5, 1.5))
        pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
        delta = plan.deposit(pt, wt)
        z = plan.zeta(delta, pt, wt).cpu().numpy()[0]
        ref = E.zeta_particle(oplan, pos, w)
    assert_zeta_close(z, ref, 1e-10)


def test_tune_set_rejects_out_of_range(mp3):
    _say("tune invalid")
    plan = mp3.Plan(16, 160.0, 1, [10.0, 20.0])
    for knob, bad in [("zpass_wgs", 10), ("zpass_wgs", 1 << 20), ("contract_wgs", 0), ("fft_x_plan", 2),
                      ("deposit_tile", 5), ("deposit_tile", 32), ("deposit_wgs", 63), ("fused_waves", -1),
                      ("fused_waves", 9), ("item_group", -1), ("item_group", 1025),
                      ("gamma_adjoint", 2), ("gamma_adjoint", -1)]:
        before = plan.tune_get(knob)
        with pytest.raises(mp3.Mp3Error):
            plan.tune_set(knob, bad)
        assert plan.tune_get(knob) == before


def test_autotune_caches_and_keeps_results(mp3, tmp_path):
    _say("autotune")
    from paper_2507_15209_amd import autotune as at
    n, box, lmax = 32, 320.0, 3
    edges = np.linspace(30.0, 110.0, 5)
    pos, w = lognormal_catalogue(n, box, 20000, 3.0, 6001, 6002, 6003, (0.5, 1.5))
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    cache = str(tmp_path / "tuning.json")
    plan = mp3.Plan(n, box, lmax, edges, precision="f64")
    delta = plan.deposit(pt, wt)
    knobs = at.autotune(plan, delta, pt, wt, cache=cache, reps=1)
    assert set(knobs) == set(at.CANDIDATES)
    for k, v in knobs.items():
        assert v in at.CANDIDATES[k]
    other = mp3.Plan(n, box, lmax, edges, precision="f64")
    assert at.load_tuning(other, cache)
    assert other.tuning() == knobs
    d2 = other.deposit(pt, wt)
    z = other.zeta(d2).cpu().numpy()[0]
    ref_delta = basis.density_contrast(basis.deposit(pos, w, n, box), float(np.sum(w.astype(np.float64))))
    assert np.abs(d2.cpu().numpy()[0] - ref_delta).max() <= 1e-13 * np.abs(ref_delta).max()
    assert_zeta_close(z, E.zeta_nodal(E.Plan(n, box, lmax, edges), ref_delta), 1e-10)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,waves", [(32, 1), (32, 4), (32, 8), (128, 2), (128, 4), (128, 6), (128, 8)])
def test_fused_waves_keep_value_and_gradient(mp3, prec, n, waves):
    """Every waves-per-workgroup setting of the one-sweep z pass: zeta against the oracle (n = 32)
    and zeta, dJ/ddelta, dJ/dw against the default setting (all n; 1e-12 / 2e-5)."""
    _say("fused waves", prec, n, waves)
    box, lmax, nb = 10.0 * n, 2, 20
    edges = np.linspace(0.08 * box, 0.35 * box, nb + 1)
    pos, w = lognormal_catalogue(n, box, 20000, 0.05 * box, 7001, 7002, 7003, (0.5, 1.5))
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    lam = _dev(np.random.default_rng(7004).standard_normal((1, lmax + 1, nb, nb)), torch.float64)
    base = mp3.Plan(n, box, lmax, edges, precision=prec)
    d = base.deposit(pt, wt)
    z0, g0, w0 = base.zeta_value_and_grad(d, lam, pt, wt)
    plan = mp3.Plan(n, box, lmax, edges, precision=prec)
    plan.tune_set("fused_waves", waves)
    z1, g1, w1 = plan.zeta_value_and_grad(d, lam, pt, wt)
    agree = 1e-12 if prec == "f64" else 2e-5
    assert_zeta_close(z1.cpu().numpy()[0], z0.cpu().numpy()[0], agree)
    for a1, a0 in ((g1, g0), (w1, w0)):
        a1, a0 = a1.cpu().numpy(), a0.cpu().numpy()
        assert np.abs(a1 - a0).max() <= agree * np.abs(a0).max()
    if n == 32:
        dref = basis.density_contrast(basis.deposit(pos, w, n, box), float(np.sum(w.astype(np.float64))))
        assert_zeta_close(z1.cpu().numpy()[0], E.zeta_nodal(E.Plan(n, box, lmax, edges), dref),
                          1e-10 if prec == "f64" else 1e-4)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("group", [1, 2, 5, 7, 1024])
def test_item_group_keeps_value_and_gradient(mp3, prec, group):
    """Items per launch of the nodal adjoint passes on a batch of two uneven catalogues (L = 4, 15
    items, so groups of 2, 5, 7 leave a ragged last group): the one sweep and the backward alone
    against the oracle's zeta and dJ/ddelta per mock, and against one item per launch (1e-12 / 2e-5)."""
    from oracle import adjoint as A
    _say("item group", prec, group)
    n, box, lmax, nb = 32, 320.0, 4, 6
    edges = np.linspace(30.0, 110.0, nb + 1)
    cats = [lognormal_catalogue(n, box, npart, 16.0, 7101 + j, 7111 + j, 7121 + j, (0.5, 1.5))
            for j, npart in enumerate((9000, 4000))]
    pos = np.concatenate([c[0] for c in cats])
    w = np.concatenate([c[1] for c in cats])
    off = np.array([0, 9000, 13000], dtype=np.int64)
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    lam = np.random.default_rng(7131).standard_normal((2, lmax + 1, nb, nb))
    lt = _dev(lam, torch.float64)

    def run(g):
        plan = mp3.Plan(n, box, lmax, edges, precision=prec, batch=2)
        plan.tune_set("item_group", g)
        d = plan.deposit(pt, wt, off)
        z, dd, dw = plan.zeta_value_and_grad(d, lt, pt, wt, off)
        dd2, dw2 = plan.zeta_backward(d, lt, pt, wt, off)
        return d, [t.cpu().numpy() for t in (z, dd, dw, dd2, dw2)]

    d, got = run(group)
    _, one = run(1)
    agree = 1e-12 if prec == "f64" else 2e-5
    assert_zeta_close(got[0], one[0], agree)
    for a1, a0 in zip(got[1:], one[1:]):
        assert np.abs(a1 - a0).max() <= agree * np.abs(a0).max()
    op = E.Plan(n, box, lmax, edges)
    dn = d.cpu().numpy()
    for j in range(2):
        assert_zeta_close(got[0][j], E.zeta_nodal(op, dn[j]), 1e-10 if prec == "f64" else 1e-4)
        ref = A.zeta_nodal_grad(op, dn[j], lam[j])
        for k in (1, 3):
            assert_grad_close(got[k][j], ref, 1e-10 if prec == "f64" else 1e-4, f"dJ/ddelta mock {j}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nb", [3, 20])
def test_gamma_adjoint_kernels_agree(mp3, prec, nb):
    """The B-spline grid-Gamma gradient by the shift stencil (default) and by the transposed node
    quadrature: the same dJ/ddelta (1e-12 / 2e-5) and the oracle's (1e-10 / 1e-4), forward value too."""
    from oracle import adjoint as A
    from tests._common import assert_grad_close
    _say("gamma adjoint kernels", prec, nb)
    n, box, lmax = 16, 160.0, 2
    edges = np.linspace(15.0, 55.0, nb + 1)
    delta = random_field(n, 261 + nb)
    lam = np.random.default_rng(262 + nb).standard_normal((lmax + 1, nb, nb))
    dd = _dev(delta[None], torch.float64 if prec == "f64" else torch.float32)
    lt = _dev(lam[None], torch.float64)
    out = []
    for k in (0, 1):
        plan = mp3.Plan(n, box, lmax, edges, precision=prec, summation="gamma")
        plan.tune_set("gamma_adjoint", k)
        z, g, _ = plan.zeta_value_and_grad(dd, lt)
        out.append((z.cpu().numpy()[0], g.cpu().numpy()[0]))
    agree = 1e-12 if prec == "f64" else 2e-5
    assert_zeta_close(out[0][0], out[1][0], agree)
    assert np.abs(out[0][1] - out[1][1]).max() <= agree * np.abs(out[1][1]).max()
    op = E.Plan(n, box, lmax, edges)
    assert_grad_close(out[0][1], A.zeta_gamma_grad(op, delta, lam), 1e-10 if prec == "f64" else 1e-4, "dJ/ddelta")
