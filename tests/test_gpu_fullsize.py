"""GPU parity at the full workload sizes, in the launch configuration the bench times.

At these sizes the float64 oracle takes minutes to tens of minutes, so its
sampled results are stored by tests/golden/make_fullsize.py (oracle and
mockgen only) in tests/golden/fullsize_*.json.  Each test compares
  * the stored oracle sample (a few (l, bin) sub-blocks of zeta, the density
    contrast and the gradients at seeded nodes or particles): float64 GPU form
    at 1e-10 and float32 at 1e-4, per multipole for zeta (A17 reading) and
    relative to the largest magnitude for the samples, and
  * every multipole of the float32 path against the float64 GPU form (a
    property that holds at any size) at 1e-4 per multipole (the grid-Gamma
    test compares its float32 and BF16-split forms instead).
Progress lines name the case before each step.
"""
import json
import os
import time

import numpy as np
import pytest

from mockgen import WORKLOADS, workload_catalogue
from tests._common import ROOT, assert_zeta_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(ROOT, "tests", "golden")


def _say(*a):
    print("[fullsize]", time.strftime("%H:%M:%S"), *a, flush=True)


def _golden(name):
    path = os.path.join(GOLDEN, f"fullsize_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"oracle sample missing: python tests/golden/make_fullsize.py {name}")
    return json.load(open(path))


@pytest.fixture(scope="module")
def mp3():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_15209_amd as m
    return m


def _dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _sub(z, ls, bins):
    return np.asarray(z)[np.ix_(ls, bins, bins)]


def _samples_close(got, ref, scale, tol):
    err = np.abs(np.asarray(got, np.float64) - np.asarray(ref, np.float64)).max() / scale
    assert err <= tol, err
    return err


def _embed_lam(g, wl, batch=1, per_mock=None):
    lam = np.zeros((batch, wl.lmax + 1, wl.nbins, wl.nbins))
    for j in range(batch):
        src = g["lam"] if per_mock is None else per_mock[j]
        for li, l in enumerate(g["ls"]):
            lam[j, l][np.ix_(g["bins"], g["bins"])] = np.asarray(src[li])
    return lam


def test_nodal_256_forward_and_gradient(mp3):
    """box 2000, 256^3, L = 10, 20 bins, 8e6 particles: the bench's workload and launch shapes.

    Per precision: the separate calls (zeta, then zeta_backward) and the
    one-sweep value and gradient with dJ/dw (the bench's timed step, whose z
    pass contracts 64 z columns per wave) against the oracle's sample, and the
    one sweep against the two calls on every entry and every node."""
    g = _golden("nodal_256")
    wl = WORKLOADS[g["workload"]]
    ls, bins, nodes = g["ls"], g["bins"], np.asarray(g["nodes"])
    parts = np.asarray(g["particles"]) if "particles" in g else None
    _say("nodal 256: mock")
    pos, w = workload_catalogue(wl)
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    lam = _dev(_embed_lam(g, wl), torch.float64)
    res = {}
    for prec in ("f32", "f64"):
        _say("nodal 256: GPU two calls", prec)
        plan = mp3.Plan(wl.n, wl.box, wl.lmax, wl.edges, precision=prec)
        d = plan.deposit(pt, wt)
        z = plan.zeta(d).cpu().numpy()[0]
        gr, _ = plan.zeta_backward(d, lam)
        gr = gr.cpu().numpy()[0].ravel()
        _say("nodal 256: GPU one sweep", prec)
        z1, g1, dw1 = plan.zeta_value_and_grad(d, lam, pt, wt)
        z1, g1, dw1 = z1.cpu().numpy()[0], g1.cpu().numpy()[0].ravel(), dw1.cpu().numpy()
        agree = 1e-12 if prec == "f64" else 2e-5
        e = assert_zeta_close(z1, z, agree)
        _say("one sweep vs two calls, zeta per l", np.array2string(e, precision=2))
        eg = np.abs(g1 - gr).max() / np.abs(gr).max()
        _say("one sweep vs two calls, max |d grad| / max |grad|", eg)
        assert eg <= agree, eg
        res[prec] = dict(delta=d.cpu().numpy()[0].ravel()[nodes], z=z, g=gr[nodes], z1=z1, g1=g1[nodes],
                         dw1=dw1[parts] if parts is not None else None)
        del plan, d
        torch.cuda.empty_cache()
    for key in ("z", "z1"):
        e = assert_zeta_close(res["f32"][key], res["f64"][key], 1e-4)
        _say("f32 vs f64 per l", key, np.array2string(e, precision=2))
    z64 = res["f64"]["z1"]
    assert np.abs(z64 - z64.transpose(0, 2, 1)).max() <= 1e-12 * np.abs(z64).max()
    for prec, tol in (("f64", 1e-10), ("f32", 1e-4)):
        r = res[prec]
        _samples_close(r["delta"], g["delta"], g["delta_max"], 1e-12 if prec == "f64" else 1e-6)
        for zk, gk in (("z", "g"), ("z1", "g1")):
            e = assert_zeta_close(_sub(r[zk], ls, bins), g["zeta"], tol)
            eg = _samples_close(r[gk], g["grad"], g["grad_max"], tol)
            _say(prec, zk, "vs oracle sample: zeta per l", np.array2string(e, precision=2), "grad", eg)
        if parts is not None:
            ew = _samples_close(r["dw1"], g["dw"], g["dw_max"], tol)
            _say(prec, "one sweep dJ/dw vs oracle sample", ew)


def test_nodal_onesweep_128(mp3):
    """128^3, L = 1, 20 bins: the one-sweep z pass with its contraction spread over two waves per
    pencil, float32 and float64, against every oracle zeta entry and the gradients at 4096 nodes
    and particles."""
    g = _golden("onesweep_128")
    n, box, lmax, edges = g["n"], g["box"], g["lmax"], np.asarray(g["edges"])
    npart, smooth, s1, s2, s3 = g["mock"]
    from mockgen import lognormal_catalogue
    pos, w = lognormal_catalogue(n, box, int(npart), smooth, int(s1), int(s2), int(s3), (0.5, 1.5))
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    lam = _dev(np.asarray(g["lam"])[None], torch.float64)
    nodes, parts = np.asarray(g["nodes"]), np.asarray(g["particles"])
    for prec, tol in (("f64", 1e-10), ("f32", 1e-4)):
        _say("one sweep 128: GPU", prec)
        plan = mp3.Plan(n, box, lmax, edges, precision=prec)
        d = plan.deposit(pt, wt)
        z, gr, dw = plan.zeta_value_and_grad(d, lam, pt, wt)
        e = assert_zeta_close(z.cpu().numpy()[0], g["zeta"], tol)
        eg = _samples_close(gr.cpu().numpy()[0].ravel()[nodes], g["grad"], g["grad_max"], tol)
        ew = _samples_close(dw.cpu().numpy()[parts], g["dw"], g["dw_max"], tol)
        _say(prec, "zeta per l", np.array2string(e, precision=2), "grad", eg, "dw", ew)


def test_particle_128_gradient(mp3):
    """box 1000, 128^3, L = 10, 15 bins, 1e6 particles, particle form: dJ/ddelta at the oracle's
    sampled nodes and dJ/dw at its sampled particles, for the backward and the one sweep
    (float32: two-chunk scatter at 15 bins; float64: one gather for both)."""
    g = _golden("particle_128_grad")
    wl = WORKLOADS[g["workload"]]
    nodes, parts = np.asarray(g["nodes"]), np.asarray(g["particles"])
    _say("particle 128 gradient: mock")
    pos, w = workload_catalogue(wl)
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    lam = _dev(_embed_lam(g, wl), torch.float64)
    for prec, tol in (("f64", 1e-10), ("f32", 1e-4)):
        plan = mp3.Plan(wl.n, wl.box, wl.lmax, wl.edges, precision=prec, summation="particle")
        d = plan.deposit(pt, wt)
        calls = [("value_and_grad", lambda: plan.zeta_value_and_grad(d, lam, pt, wt)[1:])]
        if prec == "f32":
            calls.append(("backward", lambda: plan.zeta_backward(d, lam, pt, wt)))
        for call, fn in calls:
            _say("particle 128 gradient: GPU", prec, call)
            gr, dw = fn()
            eg = _samples_close(gr.cpu().numpy()[0].ravel()[nodes], g["grad"], g["grad_max"], tol)
            ew = _samples_close(dw.cpu().numpy()[parts], g["dw"], g["dw_max"], tol)
            _say(prec, call, "grad", eg, "dw", ew)
        del plan, d
        torch.cuda.empty_cache()


@pytest.mark.parametrize("name", ["particle_512", "particle_128"])
def test_particle_fullsize(mp3, name):
    """512^3 / 5e7 weighted particles (the target workload) and 128^3 / 1e6 particles, particle summation."""
    g = _golden(name)
    wl = WORKLOADS[g["workload"]]
    ls, bins, nodes = g["ls"], g["bins"], np.asarray(g["nodes"])
    _say(name, "mock")
    pos, w = workload_catalogue(wl)
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    res = {}
    for prec in ("f32", "f64"):
        _say(name, "GPU", prec)
        plan = mp3.Plan(wl.n, wl.box, wl.lmax, wl.edges, precision=prec, summation="particle")
        d = plan.deposit(pt, wt)
        res[prec] = (d.cpu().numpy()[0].ravel()[nodes], plan.zeta(d, pt, wt).cpu().numpy()[0])
        del plan, d
        torch.cuda.empty_cache()
    e = assert_zeta_close(res["f32"][1], res["f64"][1], 1e-4)
    _say("f32 vs f64 per l", np.array2string(e, precision=2))
    for prec, tol in (("f64", 1e-10), ("f32", 1e-4)):
        dsm, z = res[prec]
        _samples_close(dsm, g["delta"], g["delta_max"], 1e-12 if prec == "f64" else 1e-6)
        assert_zeta_close(_sub(z, ls, bins), g["zeta"], tol)


def test_gamma_256(mp3):
    """box 2000, 256^3, L = 10, 20 bins, 8e6 particles, grid summation with connection coefficients.

    The float64 form of this kernel holds 20 bins of a 7^3-coefficient tile in
    LDS only up to 14 bins, so here float32 and the BF16-split inputs are
    checked against the oracle's sample, and against each other on every l.
    """
    g = _golden("gamma_256")
    wl = WORKLOADS[g["workload"]]
    ls, bins = g["ls"], g["bins"]
    _say("gamma 256: mock")
    pos, w = workload_catalogue(wl)
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    out = {}
    for prec in ("f32", "bf16x3"):
        _say("gamma 256: GPU", prec)
        plan = mp3.Plan(wl.n, wl.box, wl.lmax, wl.edges, precision=prec, summation="gamma")
        out[prec] = plan.zeta(plan.deposit(pt, wt)).cpu().numpy()[0]
        del plan
        torch.cuda.empty_cache()
    for prec in ("f32", "bf16x3"):
        e = assert_zeta_close(_sub(out[prec], ls, bins), g["zeta"], 1e-4)
        _say(prec, "vs oracle sample per l", np.array2string(e, precision=2))
    e = assert_zeta_close(out["bf16x3"], out["f32"], 1e-4)
    _say("bf16x3 vs f32 per l", np.array2string(e, precision=2))
    z = out["f32"]
    assert np.abs(z - z.transpose(0, 2, 1)).max() <= 1e-12 * np.abs(z).max()


def test_gamma_256_gradient(mp3):
    """box 2000, 256^3, L = 10, 20 bins: the grid-Gamma adjoint (float32) at the oracle's sampled nodes."""
    g = _golden("gamma_256_grad")
    wl = WORKLOADS[g["workload"]]
    nodes = np.asarray(g["nodes"])
    _say("gamma 256 gradient: mock")
    pos, w = workload_catalogue(wl)
    pt, wt = _dev(pos, torch.float32), _dev(w, torch.float32)
    # only l = 0 enters J, so a plan with lmax = 0 has the same gradient (and 1/66 of the work)
    assert g["ls"] == [0]
    lam = np.zeros((1, 1, wl.nbins, wl.nbins))
    lam[0, 0][np.ix_(g["bins"], g["bins"])] = np.asarray(g["lam"][0])
    lam = _dev(lam, torch.float64)
    _say("gamma 256 gradient: GPU f32")
    plan = mp3.Plan(wl.n, wl.box, 0, wl.edges, precision="f32", summation="gamma")
    gr, _ = plan.zeta_backward(plan.deposit(pt, wt), lam)
    e = _samples_close(gr.cpu().numpy()[0].ravel()[nodes], g["grad"], g["grad_max"], 1e-4)
    _say("gamma 256 gradient: max sampled error / max |grad|", e)


def test_batch64_forward_and_weight_gradient(mp3):
    """64 mocks of 2e5..1e6 particles, 128^3, L = 8, 12 bins, float32, one call per step."""
    g = _golden("batch64")
    wl = WORKLOADS[g["workload"]]
    ls, bins, sizes = g["ls"], g["bins"], g["sizes"]
    _say("batch64: mocks")
    cats = [workload_catalogue(wl, j, sizes[j]) for j in range(64)]
    off = np.concatenate([[0], np.cumsum(sizes)])
    pt = _dev(np.concatenate([c[0] for c in cats]), torch.float32)
    wt = _dev(np.concatenate([c[1] for c in cats]), torch.float32)
    zero = [[[0.0] * len(bins)] * len(bins)] * len(ls)
    per_mock = [g["mocks"][str(j)]["lam"] if str(j) in g["mocks"] else zero for j in range(64)]
    lam = _dev(_embed_lam(g, wl, 64, per_mock), torch.float64)
    _say("batch64: GPU f32 forward + backward")
    plan = mp3.Plan(wl.n, wl.box, wl.lmax, wl.edges, precision="f32", batch=64)
    delta = plan.deposit(pt, wt, off)
    z = plan.zeta(delta).cpu().numpy()
    _, dw = plan.zeta_backward(delta, lam, pt, wt, off)
    dw = dw.cpu().numpy()
    for key, ref in g["mocks"].items():
        j = int(key)
        assert_zeta_close(_sub(z[j], ls, bins), ref["zeta"], 1e-4)
        got = dw[off[j]:off[j + 1]][np.asarray(ref["particles"])]
        _samples_close(got, ref["dw"], ref["dw_max"], 1e-4)
