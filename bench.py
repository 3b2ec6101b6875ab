"""Throughput of the in-situ multipole 3PCF path on one MI355X.

One step = the whole path over one catalogue: deposit (B-spline scatter and
contrast), forward DFT, the (l, m >= 0) loop of windowed inverse transforms
with the nodal contraction (zeta_l for all l <= L and all bin pairs), and the
hand-written adjoint (fields recomputed, adjoint transforms, gradient with
respect to the grid and to every particle weight).

Metric: zeta_l evaluations per second, one evaluation unit being one
(grid cell, (l, m) with |m| <= l, radial bin): N^3 (L+1)^2 N_r units per step
and mock, forward + adjoint.  Inputs are resident on the GPU before timing.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "zeta_l evals/s (N_g·(L+1)^2·Nr per s) fwd+adjoint, 256^3 L=10, vs FP64 form"
HBM_PEAK_GBS = 8000.0
PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_traffic.txt")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pass_bytes(name, n, nb, batch, real_bytes, summation="nodal", np_total=0):
    """Algorithmic HBM bytes of one launch of a pass (each element read or written once)."""
    n3 = float(n) ** 3 * batch
    c = 2 * real_bytes
    rec = 4 + 12 * real_bytes + 8           # per particle: packed cell, 12 tap weights, order index, weight
    if name == "gather" and np_total:
        return nb * n3 * c + np_total * rec                                # fields once, particle records
    if name == "scatter" and np_total:
        return np_total * (nb * c + rec) + nb * n3 * c                     # sources + records in, fields out
    if name == "z_store":
        return 2.0 * nb * n3 * c                                           # nb fields in, bin-interleaved out
    if name == "z_adjoint" and summation != "nodal":
        return 2.0 * nb * n3 * c                                           # plain adjoint z transform in place
    return {
        "filter": n3 * c + nb * n3 * c,                                    # dhat in, nb fields out
        "x": 2.0 * nb * n3 * c,                                            # nb fields in and out
        "z_nodal": nb * n3 * c + n3 * real_bytes,                          # nb fields + delta in
        "z_adjoint": 2.0 * nb * n3 * c + n3 * real_bytes + 2 * n3 * real_bytes,  # fields in/out, delta, direct rmw
        "z_fused": 2.0 * nb * n3 * c + n3 * real_bytes + 2 * n3 * real_bytes,    # as z_adjoint (partials are KB)
        "adjoint": nb * n3 * c + 2.0 * n3 * c,                             # nb sources in, G rmw
    }.get(name)


def read_pmc(kernel_tag):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if it matches the source."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    digest = _source_digest()
    for line in open(PMC_SUMMARY):
        p = line.split()
        if len(p) >= 4 and p[0] == "traffic" and p[1] == kernel_tag and p[2] == digest:
            return float(p[3])
    return None


COPY_BYTES = 1 << 30


def pmc_probe(wl, precision, lmax=None):
    """One step of the path and a plain 1 GiB device copy, for hardware-counter runs.

    The copy reads and writes COPY_BYTES each; what FETCH_SIZE / WRITE_SIZE
    report for it calibrates the counters against known traffic.  The plan
    takes the workload's summation form; lmax (default the workload's) can be
    lowered to keep a counter run of a large workload short."""
    import torch
    import paper_2507_15209_amd as mp3
    from mockgen import workload_catalogue
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copy done")
    pos, w = workload_catalogue(wl)
    pt, wt = torch.as_tensor(pos, device=dev), torch.as_tensor(w, device=dev)
    lmax = wl.lmax if lmax is None else lmax
    lam = torch.as_tensor(np.random.default_rng(11).standard_normal((1, lmax + 1, wl.nbins, wl.nbins)), device=dev)
    plan = mp3.Plan(wl.n, wl.box, lmax, wl.edges, precision=precision, summation=wl.form, device=dev)
    from paper_2507_15209_amd import autotune as at
    at.load_tuning(plan)                           # the knobs the bench runs with, when cached
    delta = plan.deposit(pt, wt)
    plan.zeta_value_and_grad(delta, lam, pt, wt)
    torch.cuda.synchronize()
    log("one-sweep value and gradient done")
    plan.zeta(delta, pt, wt)
    torch.cuda.synchronize()
    log("forward done")
    plan.zeta_backward(delta, lam, pt, wt)
    torch.cuda.synchronize()
    log("backward done")


def copy_probe(nbytes=2684354560, reps=5):
    """Best time of a plain device-to-device copy of nbytes (the fields of one (l, m) at
    256^3, 20 bins, float32): the streaming bandwidth a pass that reads and writes every
    byte once can reach on this card."""
    import torch
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    best = None
    for _ in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    print(json.dumps({"copy_bytes": nbytes, "best_ms": best, "tb_per_s": 2.0 * nbytes / best / 1e9}))


def _csv_rows(root, suffix):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(root, "**", "*" + suffix), recursive=True)):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _source_digest():
    import hashlib
    src = open(os.path.join(ROOT, "paper_2507_15209_amd", "csrc", "kernels.hip"), "rb").read()
    src += open(os.path.join(ROOT, "paper_2507_15209_amd", "csrc", "fft_core.hpp"), "rb").read()
    return hashlib.sha256(src).hexdigest()[:16]


# kernels whose traffic is summarised: pass name -> kernel-name test
PMC_KERNELS = {"x": lambda k: "k_fft_strided" in k, "filter": lambda k: "k_filter_y" in k,
               "z_nodal": lambda k: "k_zpass_nodal" in k,
               "z_adjoint": lambda k: "k_zpass_adjoint" in k and "false, false, false>" in k,
               "z_fused": lambda k: "k_zpass_adjoint" in k and ", true," in k.split(">")[0],
               "adjoint": lambda k: "k_adjoint_y" in k}


def pmc_summarize(fetch_dir, write_dir, wl, precision):
    """Per-launch HBM bytes of the path's kernels from two rocprofv3 --pmc runs of --pmc-probe."""
    n, nb = wl.n, wl.nbins
    real_bytes = 4 if precision == "f32" else 8
    out = [f"# HBM traffic per launch from rocprofv3 counters, workload {wl.name} ({precision})",
           f"# source digest {_source_digest()} (kernels.hip + fft_core.hpp); a changed kernel voids these lines",
           "# columns: traffic <pass> <digest> <bytes per launch> | fetch_bytes write_bytes algorithmic_bytes launches"]
    per = {}
    for cname, root in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _csv_rows(root, "counter_collection.csv") if r.get("Counter_Name") == cname]
        if not rows:
            raise SystemExit(f"no {cname} rows under {root}")
        copy = [float(r["Counter_Value"]) for r in rows if "copy" in r["Kernel_Name"].lower()]
        if not copy:
            names = sorted({r["Kernel_Name"][:80] for r in rows})
            raise SystemExit(f"no copy kernel among the {cname} rows: {names}")
        big = sorted(v for v in copy if v >= 0.5 * max(copy))
        kib = big[len(big) // 2]
        factor = kib * 1024.0 / COPY_BYTES
        out.append(f"# {cname}: plain 1 GiB device copy counts {kib:.0f} KiB -> factor {factor:.4f} "
                   f"(counter bytes per true byte)")
        for tag, match in PMC_KERNELS.items():
            sel = [r for r in rows if match(r["Kernel_Name"])]
            if tag == "x" and sel:
                # the x pass transforms all bins in one launch: the largest grid of the strided kernel
                gmax = max(int(r.get("Grid_Size") or 0) for r in sel)
                sel = [r for r in sel if int(r.get("Grid_Size") or 0) == gmax]
            vals = [float(r["Counter_Value"]) for r in sel]
            if vals:
                per.setdefault(tag, {})[cname] = (sum(vals) / len(vals) * 1024.0 / factor, len(vals))
    dig = _source_digest()
    for tag, d in per.items():
        if "FETCH_SIZE" in d and "WRITE_SIZE" in d:
            f, cnt = d["FETCH_SIZE"]
            w_, _ = d["WRITE_SIZE"]
            alg = pass_bytes(tag, n, nb, 1, real_bytes)
            out.append(f"traffic {tag} {dig} {f + w_:.6g} | {f:.6g} {w_:.6g} {alg:.6g} {cnt}")
    print("\n".join(out))


def pmc_table(root):
    """Markdown table of per-dispatch counter averages by kernel from rocprofv3 --pmc runs under root."""
    rows = _csv_rows(root, "counter_collection.csv")
    agg = {}
    for r in rows:
        name = r["Kernel_Name"].split("(")[0].replace("void ", "")
        d = agg.setdefault(name, {})
        v = d.setdefault(r["Counter_Name"], [0.0, 0])
        v[0] += float(r["Counter_Value"])
        v[1] += 1
    counters = sorted({c for d in agg.values() for c in d})
    print("| kernel | " + " | ".join(counters) + " |")
    print("|---" * (len(counters) + 1) + "|")
    for name in sorted(agg):
        cells = []
        for c in counters:
            v = agg[name].get(c)
            cells.append(f"{v[0] / v[1]:.4g}" if v else "")
        print(f"| `{name[:70]}` | " + " | ".join(cells) + " |")


def stats_summarize(root, top=20):
    """Markdown table of a rocprofv3 --kernel-trace --stats run (kernel_stats.csv)."""
    rows = _csv_rows(root, "kernel_stats.csv")
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print("| kernel | calls | total ms | avg ms | min ms | max ms | % |")
    print("|---|---|---|---|---|---|---|")
    for r in rows[:top]:
        name = r["Name"]
        name = name if len(name) < 90 else name[:87] + "..."
        print(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['AverageNs']) / 1e6:.4f} "
              f"| {float(r['MinNs']) / 1e6:.4f} | {float(r['MaxNs']) / 1e6:.4f} | {float(r['Percentage']):.2f} |")


# secondary measurements: (workload, summation, precision, with adjoint, plan options)
TRIPLE_SPHERE = {"binning": "thin", "smoothing": 8.0}
FORMS = {
    "gamma_256_f32": ("box2000_n256_l10", "gamma", "f32", False, {}),
    "gamma_256_bf16x3": ("box2000_n256_l10", "gamma", "bf16x3", False, {}),
    "gamma_256_f32_adj": ("box2000_n256_l10", "gamma", "f32", True, {}),
    "particle_512_f32": ("box3000_n512_l10", "particle", "f32", True, {}),
    "particle_512_f64": ("box3000_n512_l10", "particle", "f64", True, {}),
    "batch64_f32": ("batch64_n128_l8", "nodal", "f32", True, {}),
    # the paper's triple-sphere binning: thin shells, top-hat R = 8 on every vertex
    "nodal_256_thin_tophat_f32": ("box2000_n256_l10", "nodal", "f32", True, TRIPLE_SPHERE),
    # the paper's Daubechies-4 basis: nodal one sweep, and the grid summation with its connection coefficients
    "nodal_256_d4_f32": ("box2000_n256_l10", "nodal", "f32", True, {"basis": "d4"}),
    "gamma_256_d4_f32_adj": ("box2000_n256_l10", "gamma", "f32", True, {"basis": "d4"}),
    # the remaining configurations (not run by default)
    "gamma_32_f64": ("box250_n32_l4", "gamma", "f64", True, {}),
    "nodal_32_f64": ("box250_n32_l4", "nodal", "f64", True, {}),
    "particle_128_f32": ("box1000_n128_l10", "particle", "f32", True, {}),
    "particle_128_f64": ("box1000_n128_l10", "particle", "f64", True, {}),
}
DEFAULT_FORMS = ("gamma_256_f32", "gamma_256_bf16x3", "gamma_256_f32_adj", "particle_512_f32", "particle_512_f64",
                 "batch64_f32", "nodal_256_thin_tophat_f32", "nodal_256_d4_f32", "gamma_256_d4_f32_adj")


def measure_form(name, steps=1):
    """Throughput of one form on its workload: deposit + zeta (+ the one-sweep gradient with dJ/dw).

    The first step runs with per-pass HIP-event timing (it also warms up); the
    timed steps run without it.  The form's dominant pass gets a roofline
    entry when its algorithmic bytes are known."""
    import torch
    import paper_2507_15209_amd as mp3
    from mockgen import WORKLOADS, workload_catalogue
    from mockgen import batch_sizes
    wname, summation, precision, backward, opts = FORMS[name]
    wl = WORKLOADS[wname]
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    if wname.startswith("batch"):
        sizes = [int(x) for x in batch_sizes()]
        cats = [workload_catalogue(wl, j, sizes[j]) for j in range(len(sizes))]
        pos = np.concatenate([c[0] for c in cats])
        w = np.concatenate([c[1] for c in cats])
        off = np.concatenate([[0], np.cumsum(sizes)])
        del cats
    else:
        pos, w = workload_catalogue(wl)
        off = None
    batch = 1 if off is None else len(off) - 1
    log(f"{name}: mock drawn in {time.perf_counter() - t0:.1f} s")
    pt, wt = torch.as_tensor(pos, device=dev), torch.as_tensor(w, device=dev)
    np_total = len(w)
    del pos, w
    lam = torch.as_tensor(np.random.default_rng(12).standard_normal((batch, wl.lmax + 1, wl.nbins, wl.nbins)),
                          device=dev)
    plan = mp3.Plan(wl.n, wl.box, wl.lmax, wl.edges, precision=precision, device=dev, summation=summation,
                    batch=batch, **opts)
    from paper_2507_15209_amd import autotune as at
    at.load_tuning(plan)                           # shipped knobs for this configuration, if any
    cat = (pt, wt, off) if summation == "particle" else ()

    def step():
        delta = plan.deposit(pt, wt, off)
        if backward:
            plan.zeta_value_and_grad(delta, lam, pt, wt, off)
        else:
            plan.zeta(delta, *cat)

    plan.profile(True)
    step()
    torch.cuda.synchronize()
    prof = {k: v for k, v in plan.profile_read().items() if v[1] > 0}
    plan.profile(False)
    t1 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t1) / steps
    log(f"{name}: {dt * 1e3:.1f} ms per step")
    del plan, pt, wt
    torch.cuda.empty_cache()
    units = float(wl.n) ** 3 * (wl.lmax + 1) ** 2 * wl.nbins * batch
    out = {"workload": wl.name, "summation": summation, "precision": precision, "batch": batch, "options": opts,
           "pass": "deposit + forward" + (" + adjoint with dJ/dw (one sweep)" if backward else ""),
           "value": units / dt, "unit": "zeta_l evals/s", "ms_per_step": dt * 1e3, "steps": steps,
           "passes_ms": {k: {"total_ms": v[0], "launches": v[1]} for k, v in prof.items()}}
    real_bytes = 8 if precision == "f64" else 4
    # the dominant pass by total time; HBM roofline from its algorithmic bytes where they are defined
    per_step = {k: v for k, v in prof.items() if k not in ("deposit", "dft")}
    if per_step:
        dom = max(per_step, key=lambda k: per_step[k][0])
        avg = per_step[dom][0] / per_step[dom][1]
        ab = pass_bytes(dom, wl.n, wl.nbins, batch, real_bytes, summation, np_total)
        if ab:
            ach = ab / (avg * 1e-3) / 1e9
            out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": ach / HBM_PEAK_GBS, "avg_launch_ms": avg, "algorithmic_bytes_per_launch": ab,
                               "traffic": None}
        else:
            out["roofline"] = {"kernel": dom, "avg_launch_ms": avg, "frac": None,
                               "note": "no HBM-byte model for this pass (matrix-core or gather bound)"}
    return out


_ORACLE_DELTA = None


def _oracle_item(args):
    """One oracle work item: forward and gradient of zeta_l over its bins (float64)."""
    wl_name, l, bins = args
    from mockgen import WORKLOADS
    from oracle import estimator as E
    from oracle import adjoint as A
    wl = WORKLOADS[wl_name]
    t0 = time.process_time()
    plan = E.Plan(wl.n, wl.box, wl.lmax, wl.edges)
    lam = np.random.default_rng(7 + l).standard_normal((1, len(bins), len(bins)))
    E.zeta_nodal(plan, _ORACLE_DELTA, ls=[l], bins=bins)
    A.zeta_nodal_grad(plan, _ORACLE_DELTA, lam, ls=[l], bins=bins)
    return float(wl.n) ** 3 * (2 * l + 1) * len(bins), time.process_time() - t0


def cpu_baseline(wl, pos, w):
    """The float64 oracle on a bounded sample of the same workload, on every host core.

    The oracle deposits the full catalogue once; then one worker process per
    core (fork, before anything touches the GPU) evaluates the forward and the
    gradient of zeta_0 for its own radial bin, the work items of a step dealt
    out over the cores.  Throughput = units of all items / wall time of
    the whole sample (deposit included)."""
    import multiprocessing as mp
    from oracle import basis
    global _ORACLE_DELTA
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    workers = max(1, min(cores, 16, wl.nbins))
    t0 = time.perf_counter()
    c0 = time.process_time()
    eps = basis.deposit(pos, w, wl.n, wl.box)
    _ORACLE_DELTA = basis.density_contrast(eps, float(np.sum(w.astype(np.float64))))
    c_dep = time.process_time() - c0
    items = [(wl.name, 0, [j]) for j in range(workers)]
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_item, items)
    dt = time.perf_counter() - t0
    units = sum(r[0] for r in res)
    cpu_s = c_dep + sum(r[1] for r in res)
    _ORACLE_DELTA = None
    return {"value": units / dt, "unit": "zeta_l evals/s", "cores": workers, "kind": "oracle",
            "host_cores": cores,
            "sample": f"deposit of the full catalogue, then forward and gradient of zeta_0 for one radial bin per "
                      f"worker ({workers} worker processes, bins 0..{workers - 1}): {units:.3g} units in "
                      f"{dt:.1f} s wall, {cpu_s:.0f} s CPU (numpy float64)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="box2000_n256_l10")
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--two-call-steps", type=int, default=3,
                    help="also time the step as zeta() then zeta_backward() (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default knobs (else: cached knobs, or a tuning run on a cache miss)")
    ap.add_argument("--tune-cache", default=None,
                    help="tuning cache file to read and write (default: the per-user cache, then the packaged one)")
    ap.add_argument("--forms", default=",".join(DEFAULT_FORMS),
                    help="secondary measurements after the headline (comma list of %s, all, or none)" % ", ".join(FORMS))
    ap.add_argument("--pmc-probe", action="store_true", help="one step plus a 1 GiB copy, for counter runs")
    ap.add_argument("--probe-lmax", type=int, default=None, help="multipole order of the --pmc-probe plan")
    ap.add_argument("--copy-probe", action="store_true", help="time a plain 2.5 GiB device copy (streaming ceiling)")
    ap.add_argument("--pmc-summarize", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the per-launch traffic summary of two rocprofv3 --pmc runs of --pmc-probe")
    ap.add_argument("--stats-summarize", metavar="DIR", help="print a table of a rocprofv3 --stats run")
    ap.add_argument("--pmc-table", metavar="DIR", help="print per-kernel averages of rocprofv3 --pmc runs")
    args = ap.parse_args()
    if args.stats_summarize:
        stats_summarize(args.stats_summarize)
        return
    if args.pmc_table:
        pmc_table(args.pmc_table)
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.pmc_summarize:
        from mockgen import WORKLOADS
        pmc_summarize(args.pmc_summarize[0], args.pmc_summarize[1], WORKLOADS[args.workload], args.precision)
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the multi-GPU path is a design "
              "note only, see DESIGN.md", file=sys.stderr)
        sys.exit(2)

    from mockgen import WORKLOADS, workload_catalogue
    wl = WORKLOADS[args.workload]
    if args.pmc_probe:
        pmc_probe(wl, args.precision, args.probe_lmax)
        return

    log("workload", wl.name, "n", wl.n, "L", wl.lmax, "bins", wl.nbins, "particles", wl.n_particles)
    t0 = time.perf_counter()
    pos, w = workload_catalogue(wl)
    log(f"mock drawn in {time.perf_counter() - t0:.1f} s")

    # the CPU oracle first: its worker processes fork before anything touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        cpu = cpu_baseline(wl, pos, w)
        log("cpu baseline:", cpu["sample"])

    import torch
    import paper_2507_15209_amd as mp3
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    pt = torch.as_tensor(pos, device=dev)
    wt = torch.as_tensor(w, device=dev)
    lam = torch.as_tensor(np.random.default_rng(11).standard_normal((1, wl.lmax + 1, wl.nbins, wl.nbins)),
                          device=dev)
    units = float(wl.n) ** 3 * (wl.lmax + 1) ** 2 * wl.nbins
    tunings = {}

    def tune(plan, precision):
        """Cached knobs for this configuration, or a descent over the knobs on the one-sweep call."""
        if args.no_autotune:
            return
        from paper_2507_15209_amd import autotune as at
        t0 = time.perf_counter()
        d0 = plan.deposit(pt, wt)
        try:
            at.autotune(plan, d0, pt, wt, dzeta=lam, backward=True, reps=1, log=log, cache=args.tune_cache)
        except OSError as e:                      # tuning cache not writable: keep the tuned knobs anyway
            log("tuning cache not written:", e)
        tunings[precision] = plan.tuning()
        log(f"{precision} knobs {tunings[precision]} ({time.perf_counter() - t0:.1f} s)")

    def run(precision, steps, warmup, profile, one_sweep=True):
        t0 = time.perf_counter()
        plan = mp3.Plan(wl.n, wl.box, wl.lmax, wl.edges, precision=precision, device=dev)
        log(f"{precision} plan built in {time.perf_counter() - t0:.1f} s")
        tune(plan, precision)

        def step():
            delta = plan.deposit(pt, wt)
            if one_sweep:
                # zeta and the gradient of J = <lam, zeta> (lam fixed before the forward)
                plan.zeta_value_and_grad(delta, lam, pt, wt)
            else:
                plan.zeta(delta)
                plan.zeta_backward(delta, lam, pt, wt)

        for i in range(warmup):
            step()
            torch.cuda.synchronize()
            log(f"{precision} warmup step {i + 1}/{warmup} done")
        if profile:
            plan.profile(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(steps):
            step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        log(f"{precision}: {steps} steps in {dt:.3f} s")
        prof = plan.profile_read() if profile else None
        if profile:
            plan.profile(False)
        del plan
        torch.cuda.empty_cache()
        return dt / steps, prof

    # the headline: timed with per-pass profiling off
    t_step, _ = run(args.precision, args.steps, args.warmup, False)
    value = units / t_step
    # per-pass times (HIP events around every launch on the library's stream), a separate run
    prof_steps = max(1, min(3, args.steps))
    t_prof, prof = run(args.precision, prof_steps, 1, True)
    real_bytes = 4 if args.precision == "f32" else 8
    passes = {k: v for k, v in prof.items() if v[1] > 0}
    dom = max((k for k in passes if pass_bytes(k, wl.n, wl.nbins, 1, real_bytes) is not None),
              key=lambda k: passes[k][0])
    ms_tot, cnt = passes[dom]
    avg_ms = ms_tot / cnt
    # (l, m) items per launch of the pass on average (1 unless the plan groups items)
    per_item = {"filter": 1, "x": 2, "z_fused": 1, "adjoint": 1}.get(dom, 1)
    items = (wl.lmax + 1) * (wl.lmax + 2) // 2
    ipl = per_item * items * prof_steps / cnt
    abytes = pass_bytes(dom, wl.n, wl.nbins, 1, real_bytes) * ipl
    achieved = abytes / (avg_ms * 1e-3) / 1e9
    log("per-pass totals (ms, launches):", {k: (round(v[0], 2), v[1]) for k, v in passes.items()})
    # every pass with a byte model, for comparison with the dominant one
    per_pass = {}
    for k, (mt, c) in passes.items():
        b = pass_bytes(k, wl.n, wl.nbins, 1, real_bytes)
        if b is None:
            continue
        ipk = {"filter": 1, "x": 2, "z_fused": 1, "adjoint": 1}.get(k, 1) * items * prof_steps / c
        ach_k = b * ipk / (mt / c * 1e-3) / 1e9
        per_pass[k] = {"avg_launch_ms": mt / c, "achieved": ach_k, "frac": ach_k / HBM_PEAK_GBS}
    traffic = read_pmc(dom)

    two_calls = None
    if args.two_call_steps > 0:
        t2, prof2 = run(args.precision, args.two_call_steps, 1, True, one_sweep=False)
        two_calls = {"value": units / t2, "ms_per_step": t2 * 1e3, "steps": args.two_call_steps,
                     "pass": "zeta then zeta_backward (the fields of each (l, m) computed twice)",
                     "passes_ms": {k: {"total_ms": v[0] / args.two_call_steps, "launches": v[1] // args.two_call_steps}
                                   for k, v in prof2.items() if v[1] > 0}}

    fp64 = None
    if args.precision == "f32" and args.fp64_steps > 0:
        t64, _ = run("f64", args.fp64_steps, 1, False)
        fp64 = {"value": units / t64, "ms_per_step": t64 * 1e3, "ratio_f32_over_f64": t64 / t_step}

    forms = {}
    names = list(FORMS) if args.forms == "all" else [f for f in args.forms.split(",") if f and f != "none"]
    for name in names:
        forms[name] = measure_form(name)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "zeta_l evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic seeded log-normal mock (stand-in for the N-body snapshot)",
        "config": {"workload": wl.name, "form": "nodal grid summation, forward + adjoint incl. deposit and dJ/dw "
                   "(one sweep: zeta_value_and_grad)",
                   "grid": wl.n, "box": wl.box, "lmax": wl.lmax, "nbins": wl.nbins,
                   "n_particles": wl.n_particles, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": abytes, "items_per_launch": ipl,
                     "passes": per_pass},
        "passes_ms": {k: {"total_ms": v[0] / prof_steps, "launches": v[1] // prof_steps} for k, v in passes.items()},
        "profiled_ms_per_step": t_prof * 1e3,
        "two_calls": two_calls,
        "fp64_form": fp64,
        "forms": forms,
        "cpu_baseline": cpu,
        "tuning": tunings,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
