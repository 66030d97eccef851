"""ctypes declarations of the C ABI in include/nslct.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnslct.so")

NSLCT_C64 = 0
NSLCT_C128 = 1

ERRORS = {
    -1: "NSLCT_E_ARG", -2: "NSLCT_E_NOT_SYMPLECTIC", -3: "NSLCT_E_NO_DECOMPOSITION",
    -4: "NSLCT_E_SIZE", -5: "NSLCT_E_HIP", -6: "NSLCT_E_UNSUPPORTED",
}


class NslctError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("type_override", ctypes.c_int),
                ("symplectic_tol", ctypes.c_double), ("det_min", ctypes.c_double)]


class Stages(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int), ("mats", (ctypes.c_double * 3) * 4),
                ("h", ctypes.c_double * 3), ("gauge_objective", ctypes.c_double),
                ("symplectic_residual", ctypes.c_double), ("dx", ctypes.c_double),
                ("dy", ctypes.c_double), ("dwx", ctypes.c_double), ("dwy", ctypes.c_double),
                ("phase_q", ctypes.c_int)]


def _load():
    # The HIP runtime must be the one torch already loaded (same SONAME), so
    # torch is imported first when it is installed.
    try:
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover - torch is part of the image
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1707_03688_amd/build.py")
    return ctypes.CDLL(LIB_PATH)


_L = _load()
P = ctypes.c_void_p
I = ctypes.c_int
D = ctypes.c_double

SIGNATURES = {
    "nslct_opts_default": (None, [ctypes.POINTER(Opts)]),
    "nslct_plan": (I, [ctypes.POINTER(D), I, I, D, D, ctypes.POINTER(P)]),
    "nslct_plan_ex": (I, [ctypes.POINTER(D), I, I, D, D, ctypes.POINTER(Opts), ctypes.POINTER(P)]),
    "nslct_plan_lie": (I, [ctypes.POINTER(D), ctypes.POINTER(D), I, I, D, D, ctypes.POINTER(Opts),
                           ctypes.POINTER(P)]),
    "nslct_plan_from_stages": (I, [ctypes.POINTER(Stages), I, I, ctypes.POINTER(Opts), ctypes.POINTER(P)]),
    "nslct_plan_get_stages": (I, [P, ctypes.POINTER(Stages)]),
    "nslct_plan_box_check": (I, [P, D, ctypes.POINTER(I)]),
    "nslct_plan_destroy": (None, [P]),
    "nslct_forward": (I, [P, P, P, P]),
    "nslct_inverse": (I, [P, P, P, P]),
    "nslct_forward_many": (I, [P, I, P, P, P]),
    "nslct_inverse_many": (I, [P, I, P, P, P]),
    "nslct_launch_pass": (I, [P, I, I, I, P, P, P]),
    "nslct_plan_passes": (I, [P, ctypes.POINTER(I)]),
    "nslct_plan_prepare": (I, [P]),
    "nslct_device_copy": (I, [P, P, ctypes.c_size_t, P]),
    "nslct_batch_create": (I, [ctypes.POINTER(P), I, ctypes.POINTER(P)]),
    "nslct_batch_info": (I, [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(I), ctypes.POINTER(D)]),
    "nslct_batch_set_grid": (I, [P, I]),
    "nslct_batch_group": (I, [P, I, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]),
    "nslct_batch_set_group": (I, [P, I, I, I, I, I]),
    "nslct_forward_batched": (I, [P, P, P, P]),
    "nslct_inverse_batched": (I, [P, P, P, P]),
    "nslct_batch_run": (I, [P, I, I, P, P, P]),
    "nslct_batch_destroy": (None, [P]),
    "nslct_backward": (I, [P, I, P, P, P, P, P, P]),
    "nslct_backward_theta": (I, [P, I, P, P, P, ctypes.POINTER(D), P]),
    "nslct_backward_theta_noalloc": (I, [P, I, P, P, P, ctypes.POINTER(D), P]),
    "nslct_plan_theta_jacobian": (I, [P, ctypes.POINTER(D)]),
    "nslct_plan_stage_gradient": (I, [P, ctypes.POINTER(D), ctypes.POINTER(D)]),
    "nslct_lie_point": (I, [ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D)]),
    "nslct_plan_jacobian": (I, [ctypes.POINTER(D), ctypes.POINTER(D), I, I, D, D, ctypes.POINTER(Opts), D,
                                ctypes.POINTER(D)]),
    "nslct_last_error": (ctypes.c_char_p, []),
    "nslct_strerror": (ctypes.c_char_p, [I]),
    "nslct_version": (ctypes.c_char_p, []),
}


class _Lib:
    def __init__(self, handle):
        self._handle = handle
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
            setattr(self, name, fn)

    def opts(self) -> Opts:
        o = Opts()
        self.nslct_opts_default(ctypes.byref(o))
        return o


lib = _Lib(_L)


def check(rc: int) -> int:
    if rc != 0:
        msg = lib.nslct_last_error().decode(errors="replace")
        raise NslctError(rc, msg)
    return rc
