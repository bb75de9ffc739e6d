"""ctypes declarations of ``libyee.so`` (the C ABI in ``include/yee.h``).

Argument marshalling only: every step of the update runs in the HIP
library.  If the library is missing or fails to load this module raises; there
is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libyee.so")

YEE_OK = 0
STATUS_NAMES = {0: "YEE_OK", -1: "YEE_EINVAL", -2: "YEE_ENOMEM", -3: "YEE_EHIP", -4: "YEE_ESTATE",
                -5: "YEE_ENUMERIC", -6: "YEE_EAGAIN", -7: "YEE_EOVERFLOW"}
PRECISIONS = {"f64": 0, "f32": 1, "f16": 2}
FLAG_NONFINITE = 1     # YEE_FLAG_NONFINITE
FLAG_OVERFLOW = 2      # YEE_FLAG_OVERFLOW
WAVEFORMS = {"gauss_deriv": 0, "mod_gauss": 1}

# Every symbol include/yee.h declares (checked by the CPU test suite).
EXPORTED = (
    "yee_last_error", "yee_api_version", "yee_create", "yee_destroy", "yee_time_step",
    "yee_set_materials", "yee_upload_materials", "yee_add_pec_plane", "yee_set_pec_mask", "yee_add_source",
    "yee_add_probe", "yee_set_dft_freqs", "yee_footprint", "yee_bind_workspace", "yee_reset",
    "yee_set_field", "yee_step", "yee_steps_done", "yee_read_field", "yee_read_series",
    "yee_read_dft", "yee_status_flags", "yee_state_bytes", "yee_save_state", "yee_load_state", "yee_sparams", "yee_set_launch", "yee_set_time_blocking", "yee_launch_info",
    "yee_debug_layout", "yee_debug_set_write_counts",
    "yee_batch_footprint", "yee_batch_create", "yee_batch_set_precision", "yee_batch_destroy",
    "yee_batch_bind_workspace", "yee_batch_admit", "yee_batch_run", "yee_batch_poll", "yee_batch_release",
    "yee_batch_info", "yee_adjoint_create", "yee_adjoint_destroy", "yee_adjoint_footprint",
    "yee_adjoint_bind_workspace", "yee_adjoint_forward", "yee_adjoint_backward", "yee_adjoint_set_history",
)


class GridDesc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
        ("courant", C.c_double),
        ("precision", C.c_int32),
        ("cpml_cells", C.c_int32 * 3),
        ("cpml_m", C.c_double),
        ("cpml_sigma_max", C.c_double),
        ("cpml_kappa_max", C.c_double),
        ("cpml_alpha_max", C.c_double),
        ("fp16_exp", C.c_int32 * 6),
        ("series_len", C.c_int32),
    ]


class SourceDesc(C.Structure):
    _fields_ = [
        ("component", C.c_int32), ("i", C.c_int32), ("j", C.c_int32), ("k", C.c_int32),
        ("waveform", C.c_int32),
        ("amp", C.c_double), ("t0", C.c_double), ("tau", C.c_double), ("f0", C.c_double),
    ]


class YeeError(RuntimeError):
    def __init__(self, status, fn, msg):
        super().__init__(f"{fn} -> {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libyee.so (after torch, so one HIP runtime serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  -- loads the HIP runtime libyee.so links against
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D, VP = C.POINTER, C.c_int32, C.c_int64, C.c_double, C.c_void_p
    sig = {
        "yee_last_error": (C.c_char_p, []),
        "yee_api_version": (I32, []),
        "yee_create": (I32, [P(GridDesc), P(VP)]),
        "yee_destroy": (None, [VP]),
        "yee_time_step": (I32, [VP, P(D)]),
        "yee_set_materials": (I32, [VP, I32, I32, I32, P(I32), P(I32), P(I32), P(D), P(D)]),
        "yee_upload_materials": (I32, [VP, VP]),
        "yee_add_pec_plane": (I32, [VP, I32, P(C.c_uint8)]),
        "yee_set_pec_mask": (I32, [VP, P(C.c_uint8)]),
        "yee_add_source": (I32, [VP, P(SourceDesc)]),
        "yee_add_probe": (I32, [VP, I32, I32, I32, I32, P(I32)]),
        "yee_set_dft_freqs": (I32, [VP, P(D), I32]),
        "yee_footprint": (I32, [VP, P(I64)]),
        "yee_bind_workspace": (I32, [VP, VP, I64]),
        "yee_reset": (I32, [VP, VP]),
        "yee_set_field": (I32, [VP, I32, P(D), VP]),
        "yee_step": (I32, [VP, I64, VP]),
        "yee_steps_done": (I32, [VP, P(I64)]),
        "yee_read_field": (I32, [VP, I32, P(D), VP]),
        "yee_read_series": (I32, [VP, I64, I64, P(D), VP]),
        "yee_read_dft": (I32, [VP, P(D), P(D), VP]),
        "yee_status_flags": (I32, [VP, P(C.c_uint32), VP]),
        "yee_state_bytes": (I32, [VP, P(I64)]),
        "yee_save_state": (I32, [VP, VP, I64, VP]),
        "yee_load_state": (I32, [VP, VP, I64, VP]),
        "yee_sparams": (I32, [I32, I32, P(D), P(D), P(D), P(D), I32, P(I32), P(I32), P(D),
                              P(D), P(D), P(D), P(D), P(D), P(D)]),
        "yee_set_launch": (I32, [VP, I32, I32, I32]),
        "yee_set_time_blocking": (I32, [VP, I32, I32, I32]),
        "yee_launch_info": (I32, [VP, P(I32), P(I32), P(I32), P(I32)]),
        "yee_debug_layout": (I32, [VP, P(I64), P(I32)]),
        "yee_debug_set_write_counts": (I32, [VP, VP, I64]),
        "yee_batch_footprint": (I32, [I32, P(I64)]),
        "yee_batch_create": (I32, [I32, I64, I32, P(VP)]),
        "yee_batch_set_precision": (I32, [VP, I32]),
        "yee_batch_destroy": (None, [VP]),
        "yee_batch_bind_workspace": (I32, [VP, VP, I64]),
        "yee_batch_admit": (I32, [VP, VP, I64, P(I32)]),
        "yee_batch_run": (I32, [VP, VP]),
        "yee_batch_poll": (I32, [VP, P(I32), I32, P(I32)]),
        "yee_batch_release": (I32, [VP, I32]),
        "yee_batch_info": (I32, [VP, P(I32), P(I64)]),
        "yee_adjoint_create": (I32, [VP, I64, I32, P(I32), P(VP)]),
        "yee_adjoint_destroy": (None, [VP]),
        "yee_adjoint_set_history": (I32, [VP, I32]),
        "yee_adjoint_footprint": (I32, [VP, P(I64)]),
        "yee_adjoint_bind_workspace": (I32, [VP, VP, I64]),
        "yee_adjoint_forward": (I32, [VP, P(D), VP]),
        "yee_adjoint_backward": (I32, [VP, VP, VP]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status, fn):
    if status != YEE_OK:
        msg = load().yee_last_error().decode(errors="replace")
        raise YeeError(status, fn, msg)

