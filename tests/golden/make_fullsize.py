"""Write the float64 oracle's sampled results for the full-size workloads.

    python tests/golden/make_fullsize.py [case ...]

Each case draws its seeded mock with ``mockgen``, evaluates the requested
(l, bin) sub-blocks of zeta (and gradient samples) with ``oracle`` only, and
writes tests/golden/fullsize_<case>.json.  The GPU tests of
tests/test_gpu_fullsize.py compare against these files; the oracle at these
sizes takes minutes to tens of minutes on a few cores, which is why the values
are stored rather than recomputed on every run.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from mockgen import WORKLOADS, workload_catalogue, batch_sizes, lognormal_catalogue  # noqa: E402
from oracle import basis  # noqa: E402
from oracle import estimator as E  # noqa: E402
from oracle import adjoint as A  # noqa: E402

NODE_SAMPLES = 256


def say(*a):
    print(time.strftime("%H:%M:%S"), *a, flush=True)


def contrast(pos, w, n, box):
    return basis.density_contrast(basis.deposit(pos, w, n, box), float(np.sum(np.asarray(w, np.float64))))


def node_sample(n, seed):
    return np.random.default_rng(seed).integers(0, n ** 3, NODE_SAMPLES)


def nodal_lam(nl, nb, seed):
    """lam[l index][b1][b2] for the sampled multipoles and bins (the tests draw the same)."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.standard_normal((nb, nb)) for _ in range(nl)])


def case_nodal_256():
    wl = WORKLOADS["box2000_n256_l10"]
    ls, bins = [0, 3, 10], [0, 9, 19]
    pos, w = workload_catalogue(wl)
    say("nodal_256 deposit")
    delta = contrast(pos, w, wl.n, wl.box)
    idx = node_sample(wl.n, 8102)
    op = E.Plan(wl.n, wl.box, wl.lmax, wl.edges)
    say("nodal_256 zeta")
    z = E.zeta_nodal(op, delta, ls=ls, bins=bins)
    say("nodal_256 gradient")
    lam = nodal_lam(len(ls), len(bins), 8101)
    g = A.zeta_nodal_grad(op, delta, lam, ls=ls, bins=bins)
    say("nodal_256 weight gradient")
    dw = A.deposit_weight_grad(pos, w, wl.n, wl.box, g)
    pidx = np.random.default_rng(8109).integers(0, len(w), NODE_SAMPLES)
    return dict(workload=wl.name, ls=ls, bins=bins, zeta=z.tolist(), lam=lam.tolist(), nodes=idx.tolist(),
                delta=delta.ravel()[idx].tolist(), delta_max=float(np.abs(delta).max()),
                grad=g.ravel()[idx].tolist(), grad_max=float(np.abs(g).max()),
                particles=pidx.tolist(), dw=dw[pidx].tolist(), dw_max=float(np.abs(dw).max()))


def case_particle(name, ls, bins):
    wl = WORKLOADS[name]
    pos, w = workload_catalogue(wl)
    say(name, "deposit")
    delta = contrast(pos, w, wl.n, wl.box)
    idx = node_sample(wl.n, 8103)
    say(name, "zeta")
    z = E.zeta_particle(E.Plan(wl.n, wl.box, wl.lmax, wl.edges), pos, w, ls=ls, bins=bins)
    return dict(workload=wl.name, ls=ls, bins=bins, zeta=z.tolist(), nodes=idx.tolist(),
                delta=delta.ravel()[idx].tolist(), delta_max=float(np.abs(delta).max()))


def case_particle_grad(name, ls, bins):
    """Gradient samples of the particle form: dJ/ddelta at seeded nodes, dJ/dw at seeded particles."""
    wl = WORKLOADS[name]
    pos, w = workload_catalogue(wl)
    idx = node_sample(wl.n, 8106)
    pidx = np.random.default_rng(8107).integers(0, len(w), NODE_SAMPLES)
    lam = nodal_lam(len(ls), len(bins), 8108)
    say(name, "particle gradient")
    g, dw = A.zeta_particle_grad(E.Plan(wl.n, wl.box, wl.lmax, wl.edges), pos, w, lam, ls=ls, bins=bins)
    return dict(workload=wl.name, ls=ls, bins=bins, lam=lam.tolist(), nodes=idx.tolist(),
                grad=g.ravel()[idx].tolist(), grad_max=float(np.abs(g).max()),
                particles=pidx.tolist(), dw=dw[pidx].tolist(), dw_max=float(np.abs(dw).max()))


def case_onesweep_128():
    """128^3, L = 1, 20 bins, nodal form: every zeta entry, the gradient at seeded nodes and particles.

    The one-sweep z pass contracts 64 z columns per wave, so 128 points per
    pencil spread the contraction over several waves."""
    n, box, lmax = 128, 1280.0, 1
    edges = np.linspace(0.08 * box, 0.35 * box, 21)
    pos, w = lognormal_catalogue(n, box, 60000, 0.05 * box, 901, 902, 903, (0.5, 1.5))
    say("onesweep_128 deposit")
    delta = contrast(pos, w, n, box)
    op = E.Plan(n, box, lmax, edges)
    say("onesweep_128 zeta")
    z = E.zeta_nodal(op, delta)
    lam = np.random.default_rng(904).standard_normal((lmax + 1, 20, 20))
    say("onesweep_128 gradient")
    g = A.zeta_nodal_grad(op, delta, lam)
    dw = A.deposit_weight_grad(pos, w, n, box, g)
    idx = np.random.default_rng(905).integers(0, n ** 3, 4096)
    pidx = np.random.default_rng(906).integers(0, len(w), 4096)
    return dict(n=n, box=box, lmax=lmax, edges=edges.tolist(), mock=[60000, 0.05 * box, 901, 902, 903],
                zeta=z.tolist(), lam=lam.tolist(), nodes=idx.tolist(), grad=g.ravel()[idx].tolist(),
                grad_max=float(np.abs(g).max()), particles=pidx.tolist(), dw=dw[pidx].tolist(),
                dw_max=float(np.abs(dw).max()))


def case_gamma_256():
    wl = WORKLOADS["box2000_n256_l10"]
    ls, bins = [0], [0, 19]
    pos, w = workload_catalogue(wl)
    say("gamma_256 deposit")
    delta = contrast(pos, w, wl.n, wl.box)
    say("gamma_256 zeta")
    z = E.zeta_gamma(E.Plan(wl.n, wl.box, wl.lmax, wl.edges), delta, ls=ls, bins=bins)
    return dict(workload=wl.name, ls=ls, bins=bins, zeta=z.tolist())


def case_gamma_256_grad():
    wl = WORKLOADS["box2000_n256_l10"]
    ls, bins = [0], [0, 19]
    pos, w = workload_catalogue(wl)
    say("gamma_256_grad deposit")
    delta = contrast(pos, w, wl.n, wl.box)
    idx = node_sample(wl.n, 8104)
    lam = nodal_lam(len(ls), len(bins), 8105)
    say("gamma_256_grad gradient")
    g = A.zeta_gamma_grad(E.Plan(wl.n, wl.box, wl.lmax, wl.edges), delta, lam, ls=ls, bins=bins)
    return dict(workload=wl.name, ls=ls, bins=bins, lam=lam.tolist(), nodes=idx.tolist(),
                grad=g.ravel()[idx].tolist(), grad_max=float(np.abs(g).max()))


def case_batch64():
    wl = WORKLOADS["batch64_n128_l8"]
    ls, bins = [0, 8], [0, 11]
    sizes = [int(s) for s in batch_sizes(64)]
    op = E.Plan(wl.n, wl.box, wl.lmax, wl.edges)
    out = dict(workload=wl.name, ls=ls, bins=bins, sizes=sizes, mocks={})
    for j in (0, 37, 63):
        say("batch64 mock", j)
        pos, w = workload_catalogue(wl, j, sizes[j])
        delta = contrast(pos, w, wl.n, wl.box)
        z = E.zeta_nodal(op, delta, ls=ls, bins=bins)
        lam = nodal_lam(len(ls), len(bins), 8201 + j)
        g = A.zeta_nodal_grad(op, delta, lam, ls=ls, bins=bins)
        dw = A.deposit_weight_grad(pos, w, wl.n, wl.box, g)
        pidx = np.random.default_rng(8300 + j).integers(0, sizes[j], NODE_SAMPLES)
        out["mocks"][str(j)] = dict(zeta=z.tolist(), lam=lam.tolist(), particles=pidx.tolist(),
                                    dw=dw[pidx].tolist(), dw_max=float(np.abs(dw).max()))
    return out


CASES = {
    "nodal_256": case_nodal_256,
    "particle_512": lambda: case_particle("box3000_n512_l10", [0], [0, 19]),
    "particle_128": lambda: case_particle("box1000_n128_l10", [0, 2, 10], [0, 7, 14]),
    "particle_128_grad": lambda: case_particle_grad("box1000_n128_l10", [0, 2, 10], [0, 7, 14]),
    "onesweep_128": case_onesweep_128,
    "gamma_256": case_gamma_256,
    "gamma_256_grad": case_gamma_256_grad,
    "batch64": case_batch64,
}


def main(names):
    for name in names or list(CASES):
        t0 = time.time()
        say("case", name)
        data = CASES[name]()
        data["oracle_seconds"] = round(time.time() - t0, 1)
        path = os.path.join(HERE, f"fullsize_{name}.json")
        with open(path, "w") as f:
            json.dump(data, f)
        say("wrote", path, f"{data['oracle_seconds']} s")


if __name__ == "__main__":
    main(sys.argv[1:])
