"""MI355X in-situ multipole 3PCF: Python binding of the HIP library.

Every step of the estimator runs in the gfx950 kernels of ``libmp3.so``; this
module only marshals torch device tensors (memory and the current stream) into
the C ABI of ``include/mp3.h``.  There is no CPU fallback: without the built
library or without a GPU the calls raise.

    plan = Plan(n=256, box=2000.0, lmax=10, edges=np.linspace(20, 200, 21))
    delta = plan.deposit(pos, w)                # [batch, n, n, n]
    zeta = plan.zeta(delta)                     # [batch, lmax+1, nbins, nbins] float64
    ddelta, dw = plan.zeta_backward(delta, dzeta, pos, w)
    zeta, ddelta, dw = plan.zeta_value_and_grad(delta, dzeta, pos, w)   # both in one sweep
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib

__all__ = ["Plan", "Zeta3PCF", "zeta_from_catalogue", "Mp3Error"]

Mp3Error = _lib.Mp3Error


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """A configuration of the estimator: grid, box, multipole order, radial bins.

    precision "f32": fields, FFTs and window in float32 (tables generated in
    float64, reductions in float64); "f64": the plain float64 form; "bf16x3":
    "f32" with BF16-split inputs to the matrix-core contractions.
    summation "nodal": grid summation on the nodes; "gamma": grid summation
    with the B-spline connection coefficients; "particle": primary vertex on
    the catalogue (zeta() then needs pos, w, np_off).
    binning "shell": r^2-weighted average of j_l over each bin; "thin": the
    thin shell at each bin's mid radius.  smoothing: radius of the spherical
    top-hat window on every vertex (0 = none).  phi_hat: multiply the
    secondary windows by the scaling function's power spectrum.
    check_finite: validate inputs on the device (calls then block).
    basis "b3": centred cubic B-spline; "d4": Daubechies-4 scaling function
    (nodal and particle summation).
    """

    PRECISIONS = {"f32": _lib.MP3_F32, "f64": _lib.MP3_F64, "bf16x3": _lib.MP3_F32_BF16X3}
    SUMMATIONS = {"nodal": _lib.MP3_SUM_NODAL, "gamma": _lib.MP3_SUM_GRID_GAMMA, "particle": _lib.MP3_SUM_PARTICLE}

    BINNINGS = {"shell": _lib.MP3_BIN_SHELL_AVERAGE, "thin": _lib.MP3_BIN_THIN_SHELL}
    BASES = {"b3": _lib.MP3_BASIS_BSPLINE3, "d4": _lib.MP3_BASIS_DAUBECHIES4}

    def __init__(self, n: int, box: float, lmax: int, edges, precision: str = "f32", batch: int = 1,
                 device=None, summation: str = "nodal", binning: str = "shell", smoothing: float = 0.0,
                 phi_hat: bool = False, check_finite: bool = False, basis: str = "b3"):
        self.lib = _lib.load()
        self.n, self.box, self.lmax, self.batch = int(n), float(box), int(lmax), int(batch)
        self.edges = np.ascontiguousarray(edges, dtype=np.float64)
        self.nbins = self.edges.size - 1
        if precision not in self.PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(self.PRECISIONS)}")
        self.precision = precision
        if summation not in self.SUMMATIONS:
            raise ValueError(f"summation must be one of {sorted(self.SUMMATIONS)}")
        self.summation = summation
        if binning not in self.BINNINGS:
            raise ValueError(f"binning must be one of {sorted(self.BINNINGS)}")
        self.binning, self.smoothing = binning, float(smoothing)
        if basis not in self.BASES:
            raise ValueError(f"basis must be one of {sorted(self.BASES)}")
        self.basis = basis
        kflags = (_lib.MP3_KF_PHI_HAT if phi_hat else 0) | (_lib.MP3_KF_CHECK_FINITE if check_finite else 0)
        self.real_dtype = torch.float64 if precision == "f64" else torch.float32
        self.complex_dtype = torch.complex128 if precision == "f64" else torch.complex64
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        desc = _lib.PlanDesc(self.n, self.box, self.lmax, self.nbins,
                             self.edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             self.PRECISIONS[precision],
                             self.SUMMATIONS[summation], self.batch, self.BASES[basis], kflags,
                             self.BINNINGS[binning], self.smoothing)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self.lib.mp3_plan_create(ctypes.byref(desc), ctypes.byref(handle)), "mp3_plan_create")
        self._h = handle
        self._ws = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.mp3_plan_destroy(h)
            self._h = None

    # -- workspace -------------------------------------------------------
    def workspace_bytes(self, np_total: int = 0) -> int:
        out = ctypes.c_size_t()
        _lib.check(self.lib.mp3_workspace_size(self._h, int(np_total), ctypes.byref(out)), "mp3_workspace_size")
        return out.value

    def _workspace(self, np_total: int = 0):
        need = self.workspace_bytes(np_total)
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def _offsets(self, np_off, np_total):
        if np_off is None:
            if self.batch != 1:
                raise ValueError("np_off is required when batch > 1")
            np_off = [0, np_total]
        off = np.ascontiguousarray(np_off, dtype=np.int64)
        if off.ndim != 1 or off.size != self.batch + 1:
            raise ValueError("np_off must have batch + 1 entries")
        # the library reads np_off[batch] particles from pos / w and writes as many dw
        if off[0] != 0 or off[-1] != np_total or np.any(np.diff(off) <= 0):
            raise ValueError(f"np_off must start at 0, increase strictly and end at the number of particles "
                             f"({np_total}); got {off.tolist()}")
        return off

    def _real(self, x, name):
        if x.device != self.device or x.dtype != self.real_dtype or not x.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.real_dtype} tensor on {self.device}")
        if x.numel() != self.batch * self.n ** 3:
            raise ValueError(f"{name} must hold batch * n^3 values")
        return x

    def _catalogue(self, pos, w):
        if pos.device != self.device or pos.dtype != torch.float32 or not pos.is_contiguous() or pos.dim() != 2 \
                or pos.shape[1] != 3:
            raise ValueError("pos must be a contiguous float32 [np, 3] tensor on the plan's device")
        if w is not None and (w.device != self.device or w.dtype != torch.float32 or not w.is_contiguous()
                              or w.numel() != pos.shape[0]):
            raise ValueError("w must be a contiguous float32 [np] tensor on the plan's device")

    # -- per-pass timing (HIP events around every pass launch) ---------------
    def profile(self, enable: bool = True):
        _lib.check(self.lib.mp3_profile(self._h, 1 if enable else 0), "mp3_profile")

    def profile_read(self):
        """{pass name: (total ms, launches)} since the last profile() call."""
        out = {}
        for i, name in enumerate(_lib.PASSES):
            ms, cnt = ctypes.c_double(), ctypes.c_int64()
            _lib.check(self.lib.mp3_profile_read(self._h, i, ctypes.byref(ms), ctypes.byref(cnt)), "mp3_profile_read")
            out[name] = (ms.value, cnt.value)
        return out

    # -- launch-shape knobs -------------------------------------------------
    def tune_set(self, knob: str, value: int):
        _lib.check(self.lib.mp3_tune_set(self._h, _lib.TUNE_KNOBS.index(knob), int(value)), "mp3_tune_set")

    def tune_get(self, knob: str) -> int:
        v = ctypes.c_int32()
        _lib.check(self.lib.mp3_tune_get(self._h, _lib.TUNE_KNOBS.index(knob), ctypes.byref(v)), "mp3_tune_get")
        return v.value

    def tuning(self) -> dict:
        """All knobs as {name: value}."""
        return {k: self.tune_get(k) for k in _lib.TUNE_KNOBS}

    # -- entry points ------------------------------------------------------
    def deposit(self, pos, w=None, np_off=None):
        self._catalogue(pos, w)
        off = self._offsets(np_off, pos.shape[0])
        delta = torch.empty((self.batch, self.n, self.n, self.n), dtype=self.real_dtype, device=self.device)
        ws = self._workspace(pos.shape[0])
        st = self.lib.mp3_deposit(self._h, _ptr(pos), _ptr(w), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  _ptr(delta), _ptr(ws), ws.numel(), _stream(self.device))
        _lib.check(st, "mp3_deposit")
        return delta

    def multipole_fields(self, delta, l: int, m: int):
        self._real(delta, "delta")
        out = torch.empty((self.batch, self.nbins, self.n, self.n, self.n), dtype=self.complex_dtype,
                          device=self.device)
        ws = self._workspace()
        st = self.lib.mp3_multipole_fields(self._h, _ptr(delta), int(l), int(m), _ptr(out), _ptr(ws), ws.numel(),
                                           _stream(self.device))
        _lib.check(st, "mp3_multipole_fields")
        return out

    def zeta(self, delta, pos=None, w=None, np_off=None):
        """zeta_l [batch, lmax+1, nbins, nbins] float64; the particle form needs the catalogue."""
        self._real(delta, "delta")
        offp = None
        np_total = 0
        if self.summation == "particle":
            if pos is None:
                raise ValueError("particle summation needs pos (and w, np_off)")
            self._catalogue(pos, w)
            np_total = pos.shape[0]
            off = self._offsets(np_off, np_total)
            offp = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        z = torch.empty((self.batch, self.lmax + 1, self.nbins, self.nbins), dtype=torch.float64, device=self.device)
        ws = self._workspace(np_total)
        st = self.lib.mp3_zeta(self._h, _ptr(delta), _ptr(pos if offp is not None else None),
                               _ptr(w if offp is not None else None), offp, _ptr(z), _ptr(ws), ws.numel(),
                               _stream(self.device))
        _lib.check(st, "mp3_zeta")
        return z

    def zeta_backward(self, delta, dzeta, pos=None, w=None, np_off=None):
        """Returns (dJ/ddelta, dJ/dw or None) for J = sum dzeta * zeta (nodal and particle forms)."""
        self._real(delta, "delta")
        dzeta = dzeta.to(device=self.device, dtype=torch.float64).contiguous()
        if dzeta.numel() != self.batch * (self.lmax + 1) * self.nbins ** 2:
            raise ValueError("dzeta must have shape [batch, lmax+1, nbins, nbins]")
        ddelta = torch.empty_like(delta)
        dw = None
        offp = None
        np_total = 0
        if self.summation == "particle" and pos is None:
            raise ValueError("the particle form's backward needs pos (and w, np_off)")
        if pos is not None:
            self._catalogue(pos, w)
            np_total = pos.shape[0]
            off = self._offsets(np_off, np_total)
            offp = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            dw = torch.empty(np_total, dtype=self.real_dtype, device=self.device)
        ws = self._workspace(np_total)
        st = self.lib.mp3_zeta_backward(self._h, _ptr(delta), _ptr(dzeta), _ptr(ddelta), _ptr(pos), _ptr(w), offp,
                                        _ptr(dw), _ptr(ws), ws.numel(), _stream(self.device))
        _lib.check(st, "mp3_zeta_backward")
        return ddelta, dw

    def zeta_value_and_grad(self, delta, dzeta, pos=None, w=None, np_off=None):
        """Returns (zeta, dJ/ddelta, dJ/dw or None) for J = sum dzeta * zeta in one sweep.

        Same results as zeta() followed by zeta_backward(); every form except
        BF16-split plans (and nodal plans above 32 bins) computes each (l, m)'s
        fields once for both."""
        self._real(delta, "delta")
        dzeta = dzeta.to(device=self.device, dtype=torch.float64).contiguous()
        if dzeta.numel() != self.batch * (self.lmax + 1) * self.nbins ** 2:
            raise ValueError("dzeta must have shape [batch, lmax+1, nbins, nbins]")
        if self.summation == "particle" and pos is None:
            raise ValueError("the particle form needs pos (and w, np_off)")
        z = torch.empty((self.batch, self.lmax + 1, self.nbins, self.nbins), dtype=torch.float64, device=self.device)
        ddelta = torch.empty_like(delta)
        dw = None
        offp = None
        np_total = 0
        if pos is not None:
            self._catalogue(pos, w)
            np_total = pos.shape[0]
            off = self._offsets(np_off, np_total)
            offp = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            dw = torch.empty(np_total, dtype=self.real_dtype, device=self.device)
        ws = self._workspace(np_total)
        st = self.lib.mp3_zeta_value_and_grad(self._h, _ptr(delta), _ptr(dzeta), _ptr(z), _ptr(ddelta), _ptr(pos),
                                              _ptr(w), offp, _ptr(dw), _ptr(ws), ws.numel(), _stream(self.device))
        _lib.check(st, "mp3_zeta_value_and_grad")
        return z, ddelta, dw


    def xi(self, delta, radii):
        """Two-point function xi(r) [batch, len(radii)] float64 of delta by the same windows."""
        self._real(delta, "delta")
        r = np.ascontiguousarray(radii, dtype=np.float64).ravel()
        out = torch.empty((self.batch, r.size), dtype=torch.float64, device=self.device)
        ws = self._workspace()
        st = self.lib.mp3_xi(self._h, _ptr(delta), r.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(r.size),
                             _ptr(out), _ptr(ws), ws.numel(), _stream(self.device))
        _lib.check(st, "mp3_xi")
        return out

    def xi_multipoles(self, delta, radii, ell_max: int):
        """Line-of-sight (z) multipoles of xi, [batch, ell_max+1, len(radii)] float64."""
        self._real(delta, "delta")
        r = np.ascontiguousarray(radii, dtype=np.float64).ravel()
        out = torch.empty((self.batch, int(ell_max) + 1, r.size), dtype=torch.float64, device=self.device)
        ws = self._workspace()
        st = self.lib.mp3_xi_multipoles(self._h, _ptr(delta), r.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        int(r.size), int(ell_max), _ptr(out), _ptr(ws), ws.numel(),
                                        _stream(self.device))
        _lib.check(st, "mp3_xi_multipoles")
        return out

    def ss_fields(self, delta_d, delta_r):
        """(f, r) = (delta_D - delta_R, 1 + delta_R): the fields of D - R and R (edge-corrected estimator)."""
        self._real(delta_d, "delta_d")
        self._real(delta_r, "delta_r")
        f, r = torch.empty_like(delta_d), torch.empty_like(delta_d)
        _lib.check(self.lib.mp3_ss_fields(self._h, _ptr(delta_d), _ptr(delta_r), _ptr(f), _ptr(r),
                                          _stream(self.device)), "mp3_ss_fields")
        return f, r

    def ss_multipoles(self, zeta_n, zeta_r, lt=None, nquad: int = 64):
        """Multipoles [batch, lt+1, nbins, nbins] of (D - R)^3 / R^3 from those of f and r."""
        zn = zeta_n.to(device=self.device, dtype=torch.float64).contiguous()
        zr = zeta_r.to(device=self.device, dtype=torch.float64).contiguous()
        lt = self.lmax if lt is None else int(lt)
        out = torch.empty((self.batch, lt + 1, self.nbins, self.nbins), dtype=torch.float64, device=self.device)
        ws = self._workspace()
        st = self.lib.mp3_ss_multipoles(self._h, _ptr(zn), _ptr(zr), lt, int(nquad), _ptr(out), _ptr(ws), ws.numel(),
                                        _stream(self.device))
        _lib.check(st, "mp3_ss_multipoles")
        return out

    def reduced_3pcf(self, zeta, mu, lt=None, delta=None):
        """(zeta(r_b1, r_b2, theta), Q or None), each [batch, nbins, nbins, len(mu)] float64.

        zeta(theta) = sum_{l <= lt} zeta_l P_l(mu); Q needs delta (for xi)."""
        zeta = zeta.to(device=self.device, dtype=torch.float64).contiguous()
        if zeta.numel() != self.batch * (self.lmax + 1) * self.nbins ** 2:
            raise ValueError("zeta must have shape [batch, lmax+1, nbins, nbins]")
        mu = np.ascontiguousarray(mu, dtype=np.float64).ravel()
        lt = self.lmax if lt is None else int(lt)
        zt = torch.empty((self.batch, self.nbins, self.nbins, mu.size), dtype=torch.float64, device=self.device)
        q = None
        if delta is not None:
            self._real(delta, "delta")
            q = torch.empty_like(zt)
        ws = self._workspace()
        st = self.lib.mp3_reduced_3pcf(self._h, _ptr(delta), _ptr(zeta), lt,
                                       mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(mu.size), _ptr(zt),
                                       _ptr(q), _ptr(ws), ws.numel(), _stream(self.device))
        _lib.check(st, "mp3_reduced_3pcf")
        return zt, q


class Zeta3PCF(torch.autograd.Function):
    """zeta = Zeta3PCF.apply(delta, plan); backward gives dJ/ddelta from the hand-written adjoint."""

    @staticmethod
    def forward(ctx, delta, plan):
        ctx.plan = plan
        ctx.save_for_backward(delta)
        return plan.zeta(delta.contiguous())

    @staticmethod
    def backward(ctx, gz):
        (delta,) = ctx.saved_tensors
        ddelta, _ = ctx.plan.zeta_backward(delta.contiguous(), gz)
        return ddelta, None


class _CatalogueZeta(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w, pos, plan, np_off):
        delta = plan.deposit(pos, w, np_off)
        ctx.plan, ctx.np_off = plan, np_off
        ctx.save_for_backward(w, pos, delta)
        if plan.summation == "particle":
            return plan.zeta(delta, pos, w, np_off)
        return plan.zeta(delta)

    @staticmethod
    def backward(ctx, gz):
        w, pos, delta = ctx.saved_tensors
        _, dw = ctx.plan.zeta_backward(delta, gz, pos, w, ctx.np_off)
        return dw, None, None, None


def zeta_from_catalogue(plan: Plan, pos, w, np_off=None):
    """zeta of a catalogue, differentiable with respect to the particle weights."""
    return _CatalogueZeta.apply(w, pos, plan, np_off)
