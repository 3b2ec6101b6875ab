"""The allocation-free value-and-gradient entry point against the workspace one, through the C ABI.

Two calls in a row on one plan, the second with a smaller catalogue (fewer
particles), each compared with mp3_zeta_value_and_grad on the same inputs:
zeta per multipole, dJ/ddelta and dJ/dw within the float64 (1e-10) and
float32 (1e-4) bars.
"""
import ctypes

import numpy as np
import pytest

from mockgen import lognormal_catalogue
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


def _vp(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


@pytest.mark.parametrize("prec,summation", [("f64", "nodal"), ("f32", "nodal"), ("f32", "particle")])
def test_static_matches_workspace_entry(mp3, prec, summation):
    from paper_2507_15209_amd import _lib
    lib = _lib.load()
    assert lib.mp3_static_scratch_bytes() == 64 << 20
    n, box, lmax, nb = 32, 320.0, 3, 6
    edges = np.linspace(20.0, 110.0, nb + 1)
    tol = 1e-10 if prec == "f64" else 1e-4
    plan = mp3.Plan(n, box, lmax, edges, precision=prec, summation=summation)
    rd = plan.real_dtype
    for call, npart in enumerate((20000, 5000)):
        _say("static scratch", prec, summation, "call", call, "particles", npart)
        pos, w = lognormal_catalogue(n, box, npart, 12.0, 1500 + call, 1510 + call, 1520 + call, (0.5, 1.5))
        pt = torch.as_tensor(pos, device="cuda")
        wt = torch.as_tensor(w, device="cuda")
        delta = plan.deposit(pt, wt)
        lam = torch.as_tensor(np.random.default_rng(1530 + call).standard_normal((1, lmax + 1, nb, nb)),
                              device="cuda")
        z0, g0, dw0 = plan.zeta_value_and_grad(delta, lam, pt, wt)
        z1 = torch.empty_like(z0)
        g1 = torch.empty_like(delta)
        dw1 = torch.empty(npart, dtype=rd, device="cuda")
        off = np.array([0, npart], dtype=np.int64)
        st = lib.mp3_zeta_value_and_grad_static(plan._h, _vp(delta), _vp(lam), _vp(z1), _vp(g1), _vp(pt), _vp(wt),
                                                off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _vp(dw1),
                                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        _lib.check(st, "mp3_zeta_value_and_grad_static")
        torch.cuda.synchronize()
        assert_zeta_close(z1.cpu().numpy()[0], z0.cpu().numpy()[0], tol)
        assert_grad_close(g1.cpu().numpy(), g0.cpu().numpy(), tol, "dJ/ddelta")
        assert_grad_close(dw1.cpu().numpy(), dw0.cpu().numpy(), tol, "dJ/dw")


def test_static_rejects_oversized_calls(mp3):
    """A plan whose workspace exceeds the static scratch is refused before any launch."""
    from paper_2507_15209_amd import _lib
    lib = _lib.load()
    plan = mp3.Plan(128, 1000.0, 1, np.linspace(20.0, 140.0, 21), precision="f32")
    assert plan.workspace_bytes(0) > lib.mp3_static_scratch_bytes()
    d = torch.zeros((1, 128, 128, 128), dtype=torch.float32, device="cuda")
    lam = torch.zeros((1, 2, 20, 20), dtype=torch.float64, device="cuda")
    z = torch.empty((1, 2, 20, 20), dtype=torch.float64, device="cuda")
    g = torch.empty_like(d)
    st = lib.mp3_zeta_value_and_grad_static(plan._h, _vp(d), _vp(lam), _vp(z), _vp(g), None, None, None, None,
                                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.MP3_EWORKSPACE
    assert b"static scratch" in lib.mp3_last_error()
