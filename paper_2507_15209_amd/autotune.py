"""Autotuner of the plan's launch-shape knobs.

The knobs (``mp3_tune_knob`` in include/mp3.h) change how the work is cut
into workgroups and which radix plan the strided x pass uses, never the
arithmetic.  The tuner times the plan's own calls on the device with events
on the current stream, descends one knob at a time over a short candidate
list, keeps the fastest value, and stores the winners in a JSON cache keyed
by (device, n, nbins, lmax, form, precision, batch) so that a later plan of
the same configuration starts from them.
"""
from __future__ import annotations

import json
import os
import tempfile

import torch

from . import _lib

__all__ = ["CANDIDATES", "cache_key", "cache_path", "load_tuning", "save_tuning", "autotune"]

CANDIDATES = {
    "deposit_tile": (4, 8, 16),
    "deposit_wgs": (256, 512, 1024, 2048, 4096, 8192),
    "fft_x_plan": (0, 1),
    "zpass_wgs": (1024, 2048, 4096, 8192, 16384),
    "contract_wgs": (1024, 2048, 4096, 8192, 16384),
    "fused_waves": (0, 4, 8),
    "item_group": (0, 1, 2, 4),
    "gamma_adjoint": (0, 1),
}


# knobs measured on this package's target device, shipped with it (read when no
# other cache is named); entries are keyed by device name and configuration
PACKAGED_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def cache_path(path: str | None = None) -> str:
    """The cache to use: ``path``, else $MP3_TUNE_CACHE, else the per-user cache."""
    if path:
        return path
    env = os.environ.get("MP3_TUNE_CACHE")
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "mp3", "tuning.json")


def _device_tag(device) -> str:
    """Architecture and compute-unit count (stable across driver name strings)."""
    if not torch.cuda.is_available():
        return "nodevice"
    prop = torch.cuda.get_device_properties(device)
    arch = str(getattr(prop, "gcnArchName", "") or torch.cuda.get_device_name(device)).split(":")[0]
    return f"{arch}/cu{prop.multi_processor_count}"


def cache_key(plan) -> str:
    name = _device_tag(plan.device)
    return (f"{name}|n={plan.n}|nbins={plan.nbins}|lmax={plan.lmax}|{plan.summation}|{plan.precision}"
            f"|batch={plan.batch}|basis={getattr(plan, 'basis', 'b3')}")


def _read(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def load_tuning(plan, path: str | None = None) -> bool:
    """Apply cached knobs to the plan (the named or per-user cache, then the packaged one);
    False if neither has an entry for it."""
    entry = _read(cache_path(path)).get(cache_key(plan))
    if not isinstance(entry, dict) and not path:
        entry = _read(PACKAGED_CACHE).get(cache_key(plan))
    if not isinstance(entry, dict):
        return False
    for k, v in entry.get("knobs", {}).items():
        if k in _lib.TUNE_KNOBS:
            plan.tune_set(k, int(v))
    return True


def save_tuning(plan, timings: dict | None = None, path: str | None = None) -> str:
    """Write the plan's current knobs (and the measured times) into the cache."""
    path = cache_path(path)
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    data = _read(path)
    data[cache_key(plan)] = {"knobs": plan.tuning(), "ms": timings or {}}
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(path) or ".", suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return path


def _time_ms(fn, reps: int) -> float:
    """Best of ``reps`` timed calls after one untimed call, events on the current stream."""
    fn()
    best = float("inf")
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def _descend(plan, knob: str, fn, reps: int, log) -> float:
    best_v, best_t = plan.tune_get(knob), float("inf")
    for v in CANDIDATES[knob]:
        plan.tune_set(knob, v)
        t = _time_ms(fn, reps)
        if log:
            log(f"autotune {knob}={v}: {t:.3f} ms")
        if t < best_t:
            best_v, best_t = v, t
    plan.tune_set(knob, best_v)
    return best_t


def autotune(plan, delta, pos=None, w=None, np_off=None, dzeta=None, backward: bool = True,
             reps: int = 2, cache: str | None = None, force: bool = False, log=None, rounds: int = 2) -> dict:
    """Tune ``plan`` on representative inputs and return its knobs.

    delta: a density contrast of the plan's shape (the forward's input).
    pos, w, np_off: a catalogue; needed by the particle form and for the
    deposit knobs (skipped without it).  dzeta: the gradient's seed (random
    if None).  With ``backward`` the timed call is the one-sweep value and
    gradient (the path the benchmark times), else the forward alone.  With a
    cache entry for this configuration and ``force`` False the cached knobs
    are applied and nothing is timed.  The path's knobs are descended one at a
    time, the one with the largest effect first, over ``rounds`` passes (the
    knobs interact: the best persistent-grid size depends on the waves per
    workgroup).
    """
    if not force and load_tuning(plan, cache):
        return plan.tuning()
    with torch.cuda.device(plan.device):
        times = {}
        if pos is not None:
            dep = lambda: plan.deposit(pos, w, np_off)
            for k in ("deposit_tile", "deposit_wgs"):
                times[k] = _descend(plan, k, dep, reps, log)
        cat = (pos, w, np_off) if plan.summation == "particle" else (None, None, None)
        do_bwd = backward and (plan.summation != "particle" or pos is not None)
        if do_bwd and dzeta is None:
            g = torch.Generator(device=plan.device).manual_seed(0)
            dzeta = torch.randn((plan.batch, plan.lmax + 1, plan.nbins, plan.nbins), dtype=torch.float64,
                                device=plan.device, generator=g)

        def path():
            if do_bwd:
                plan.zeta_value_and_grad(delta, dzeta, *cat)
            else:
                plan.zeta(delta, *cat)

        knobs = []
        if do_bwd and plan.summation == "nodal":
            # item_group is left at its default (as many items per launch as fit 1 GiB of fields),
            # the best or within noise of it wherever it was measured
            knobs.append("fused_waves")
        knobs += ["fft_x_plan", "zpass_wgs"]
        if plan.summation != "nodal":
            knobs.append("contract_wgs")
        if do_bwd and plan.summation == "gamma" and getattr(plan, "basis", "b3") == "b3":
            knobs.append("gamma_adjoint")
        for _ in range(max(1, rounds)):
            for k in knobs:
                times[k] = _descend(plan, k, path, reps, log)
    save_tuning(plan, times, cache)
    return plan.tuning()
