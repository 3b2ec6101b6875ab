"""Shared helpers for the GPU parity tests (tolerances, library loading)."""
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def ensure_library():
    """Build libmp3.so if it is not there (tests load what is built)."""
    from paper_2507_15209_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return build.LIB


def per_l_errors(got, ref):
    """Per-multipole relative error (Frobenius), with an absolute floor for small moments.

    For l with ||zeta_l|| >= 1e-2 max_l' ||zeta_l'|| the error is ||d zeta_l|| / ||zeta_l||;
    otherwise it is max|d zeta_l| / (1e-2 max_l' ||zeta_l'||).  Returns an array over l.
    """
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    norms = np.array([np.linalg.norm(r) for r in ref])
    top = norms.max()
    errs = []
    for g, r, nr in zip(got, ref, norms):
        if nr >= 1e-2 * top:
            errs.append(np.linalg.norm(g - r) / nr)
        else:
            errs.append(np.abs(g - r).max() / (1e-2 * top))
    return np.array(errs)


def assert_zeta_close(got, ref, tol):
    e = per_l_errors(got, ref)
    assert np.all(e <= tol), f"per-l errors {e} exceed {tol}"
    return e


def grad_errors(got, ref):
    """(relative L2 error, max |got - ref| / max |ref|) of a gradient array."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    l2 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    mx = np.abs(got - ref).max() / np.abs(ref).max()
    return l2, mx


def assert_grad_close(got, ref, tol, what="gradient"):
    """Both the relative L2 error and the element-wise error (relative to max |ref|) within tol."""
    l2, mx = grad_errors(got, ref)
    assert l2 <= tol and mx <= tol, f"{what}: relative L2 {l2:.3e}, max element {mx:.3e} (tol {tol:g})"
    return l2, mx
