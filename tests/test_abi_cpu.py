"""The C-ABI library loads, exports every declared symbol and rejects bad arguments on the host."""
import ctypes
import os
import re

import numpy as np
import pytest

from tests._common import ROOT, ensure_library


def _declared():
    src = open(os.path.join(ROOT, "include", "mp3.h")).read()
    # function declarations: a return type at the start of the line, then the name
    return sorted(set(re.findall(r"^(?:int|size_t|const char\*)\s+(mp3_\w+)\s*\(", src, re.M)))


def test_header_declares_expected_entry_points():
    names = _declared()
    for f in ("mp3_plan_create", "mp3_deposit", "mp3_multipole_fields", "mp3_zeta", "mp3_zeta_backward"):
        assert f in names


def test_library_exports_every_declared_symbol():
    path = ensure_library()
    lib = ctypes.CDLL(path)
    for name in _declared():
        assert hasattr(lib, name), name
    from paper_2507_15209_amd import _lib
    assert set(_lib.EXPORTS) == set(_declared())


def _desc(**kw):
    from paper_2507_15209_amd import _lib
    edges = np.asarray(kw.pop("edges", np.linspace(10.0, 60.0, 7)), dtype=np.float64)
    d = dict(n=32, box=250.0, lmax=4, nbins=edges.size - 1, precision=0, summation=0, batch=1, basis=0, kflags=0,
             binning=0, smoothing=0.0)
    d.update(kw)
    desc = _lib.PlanDesc(d["n"], d["box"], d["lmax"], d["nbins"],
                         edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), d["precision"], d["summation"],
                         d["batch"], d["basis"], d["kflags"], d["binning"], d["smoothing"])
    return desc, edges


@pytest.mark.parametrize("kw,code", [
    (dict(n=48), -4), (dict(n=1024), -4), (dict(box=0.0), -1), (dict(box=float("nan")), -6),
    (dict(box=float("inf")), -6), (dict(lmax=-1), -1), (dict(lmax=21), -1), (dict(nbins=0), -1),
    (dict(nbins=65), -1), (dict(edges=[10.0, 5.0, 20.0]), -1), (dict(edges=[-1.0, 5.0]), -1),
    (dict(edges=[1.0, float("nan")]), -6), (dict(precision=3), -1), (dict(summation=3), -4), (dict(batch=0), -1),
    (dict(basis=2), -1), (dict(basis=1, summation=1, precision=2), -4), (dict(kflags=4), -1), (dict(binning=2), -1), (dict(smoothing=-1.0), -1),
    (dict(smoothing=float("nan")), -6),
])
def test_plan_create_rejects_bad_descriptions(kw, code):
    ensure_library()
    from paper_2507_15209_amd import _lib
    lib = _lib.load()
    desc, _ = _desc(**kw)
    h = ctypes.c_void_p()
    assert lib.mp3_plan_create(ctypes.byref(desc), ctypes.byref(h)) == code
    assert h.value is None
    assert len(lib.mp3_last_error()) > 0


def test_null_arguments_are_rejected():
    ensure_library()
    from paper_2507_15209_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.mp3_plan_create(None, ctypes.byref(h)) == _lib.MP3_EINVAL
    assert lib.mp3_zeta(None, None, None, None, None, None, None, 0, None) == _lib.MP3_EINVAL
    sz = ctypes.c_size_t()
    assert lib.mp3_workspace_size(None, 0, ctypes.byref(sz)) == _lib.MP3_EINVAL
    assert lib.mp3_plan_destroy(None) == _lib.MP3_OK
    assert lib.mp3_status_string(-5) == b"MP3_EWORKSPACE"


def test_tuning_knobs_reject_null_plan_and_bad_knobs():
    ensure_library()
    from paper_2507_15209_amd import _lib
    lib = _lib.load()
    v = ctypes.c_int32(-7)
    assert lib.mp3_tune_set(None, 0, 4096) == _lib.MP3_EINVAL
    assert lib.mp3_tune_get(None, 0, ctypes.byref(v)) == _lib.MP3_EINVAL
    assert v.value == -7
    assert len(_lib.TUNE_KNOBS) == 8
