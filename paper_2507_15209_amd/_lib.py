"""ctypes binding of libmp3.so (the C ABI of include/mp3.h); marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmp3.so")

MP3_OK = 0
MP3_EINVAL = -1
MP3_ENOMEM = -2
MP3_EHIP = -3
MP3_EUNSUPPORTED = -4
MP3_EWORKSPACE = -5
MP3_ENONFINITE = -6
MP3_F32 = 0
MP3_F64 = 1
MP3_F32_BF16X3 = 2
MP3_SUM_NODAL = 0
MP3_SUM_PARTICLE = 2
MP3_SUM_GRID_GAMMA = 1
MP3_BASIS_BSPLINE3 = 0
MP3_BASIS_DAUBECHIES4 = 1
MP3_BIN_SHELL_AVERAGE = 0
MP3_BIN_THIN_SHELL = 1
MP3_KF_PHI_HAT = 1
MP3_KF_CHECK_FINITE = 2
# launch-shape knobs (enum mp3_tune_knob)
TUNE_KNOBS = ("zpass_wgs", "contract_wgs", "fft_x_plan", "deposit_tile", "deposit_wgs", "fused_waves",
              "item_group", "gamma_adjoint")

# every entry point of include/mp3.h
EXPORTS = (
    "mp3_plan_create", "mp3_plan_destroy", "mp3_workspace_size", "mp3_deposit",
    "mp3_multipole_fields", "mp3_zeta", "mp3_zeta_backward", "mp3_plan_info",
    "mp3_status_string", "mp3_last_error", "mp3_profile", "mp3_profile_read",
    "mp3_tune_set", "mp3_tune_get", "mp3_zeta_value_and_grad", "mp3_xi", "mp3_xi_multipoles", "mp3_reduced_3pcf",
    "mp3_ss_fields", "mp3_ss_multipoles",
    "mp3_sph_bessel", "mp3_window_table", "mp3_zeta_value_and_grad_static", "mp3_static_scratch_bytes",
    "mp3_basis_tables",
)
PASSES = ("dft", "filter", "x", "z_nodal", "z_adjoint", "adjoint", "deposit", "z_store", "gather", "gamma",
          "scatter", "z_fused")


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("box", ctypes.c_double),
        ("lmax", ctypes.c_int32),
        ("nbins", ctypes.c_int32),
        ("edges", ctypes.POINTER(ctypes.c_double)),
        ("precision", ctypes.c_int32),
        ("summation", ctypes.c_int32),
        ("batch", ctypes.c_int32),
        ("basis", ctypes.c_int32),
        ("kflags", ctypes.c_uint32),
        ("binning", ctypes.c_int32),
        ("smoothing", ctypes.c_double),
    ]


class Mp3Error(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {_status_name(status)}: {detail}")


_lib = None


def _status_name(s: int) -> str:
    if _lib is None:
        return str(s)
    return _lib.mp3_status_string(s).decode()


def load(path: str | None = None) -> ctypes.CDLL:
    """Load libmp3.so; raises if it has not been built (there is no fallback path).

    MP3_LIBRARY may name another build of the same library (A/B timing)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("MP3_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it first (python -m paper_2507_15209_amd.build)")
    lib = ctypes.CDLL(path)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.mp3_plan_create.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(vp)]
    lib.mp3_plan_destroy.argtypes = [vp]
    lib.mp3_workspace_size.argtypes = [vp, i64, ctypes.POINTER(sz)]
    lib.mp3_deposit.argtypes = [vp, vp, vp, ctypes.POINTER(i64), vp, vp, sz, vp]
    lib.mp3_multipole_fields.argtypes = [vp, vp, i32, i32, vp, vp, sz, vp]
    lib.mp3_zeta.argtypes = [vp, vp, vp, vp, ctypes.POINTER(i64), vp, vp, sz, vp]
    lib.mp3_zeta_backward.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(i64), vp, vp, sz, vp]
    lib.mp3_zeta_value_and_grad.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(i64), vp, vp, sz, vp]
    lib.mp3_plan_info.argtypes = [vp] + [ctypes.POINTER(i32)] * 5
    lib.mp3_profile.argtypes = [vp, ctypes.c_int]
    lib.mp3_profile_read.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.mp3_tune_set.argtypes = [vp, ctypes.c_int, i32]
    lib.mp3_tune_get.argtypes = [vp, ctypes.c_int, ctypes.POINTER(i32)]
    lib.mp3_xi.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), i32, vp, vp, sz, vp]
    lib.mp3_xi_multipoles.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), i32, i32, vp, vp, sz, vp]
    lib.mp3_ss_fields.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.mp3_ss_multipoles.argtypes = [vp, vp, vp, i32, i32, vp, vp, sz, vp]
    lib.mp3_reduced_3pcf.argtypes = [vp, vp, vp, i32, ctypes.POINTER(ctypes.c_double), i32, vp, vp, vp, sz, vp]
    lib.mp3_sph_bessel.argtypes = [i32, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    lib.mp3_window_table.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(ctypes.c_double), sz]
    lib.mp3_basis_tables.argtypes = [i32, i32, ctypes.POINTER(ctypes.c_double), sz, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.mp3_zeta_value_and_grad_static.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(i64), vp, vp]
    lib.mp3_static_scratch_bytes.argtypes = []
    lib.mp3_status_string.argtypes = [ctypes.c_int]
    lib.mp3_status_string.restype = ctypes.c_char_p
    lib.mp3_last_error.argtypes = []
    lib.mp3_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("mp3_status_string", "mp3_last_error", "mp3_static_scratch_bytes"):
            getattr(lib, name).restype = ctypes.c_int
    lib.mp3_static_scratch_bytes.restype = sz
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != MP3_OK:
        raise Mp3Error(status, where, _lib.mp3_last_error().decode())
