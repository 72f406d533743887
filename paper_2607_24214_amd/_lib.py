"""ctypes declarations of libqsa.so (the C ABI of include/qsa.h).

Argument marshalling only.  torch is imported first so that the HIP runtime
it loads is the one libqsa.so binds to (both resolve libamdhip64.so.7).
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the process-wide HIP runtime first)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqsa.so")

QSA_MAX_SPECIES = 4
QSA_STATIC_MAX_CTX = 64
QSA_FP64, QSA_FP32 = 0, 1
QSA_OK = 0

FIELD_IDS = {"psi": 0, "Ex": 1, "Ey": 2, "Ez": 3, "Bx": 4, "By": 5, "Bz": 6,
             "dxpsi": 7, "dypsi": 8, "src_S": 9, "src_Jx": 10, "src_Jy": 11, "src_Jz": 12}

STATUS = {0: "QSA_OK", -1: "QSA_E_INVALID", -2: "QSA_E_NOMEM", -3: "QSA_E_DEVICE",
          -4: "QSA_E_BREAKDOWN", -5: "QSA_E_NONFINITE", -6: "QSA_E_STATE"}

EXPORTS = ("qsa_workspace_bytes", "qsa_create", "qsa_load_plasma", "qsa_load_beam", "qsa_load_beam_range",
           "qsa_read_beam", "qsa_slice_sweep", "qsa_beam_step", "qsa_fields", "qsa_sync",
           "qsa_destroy", "qsa_status_string", "qsa_last_error", "qsa_timing_begin",
           "qsa_timing_end", "qsa_set_option", "qsa_get_option", "qsa_autotune", "qsa_adjoint_sweep",
           "qsa_field_moments", "qsa_beam_moments", "qsa_linear_model",
           "qsa_batch_workspace_bytes",
           "qsa_batch_create",
           "qsa_batch_sweep", "qsa_batch_step", "qsa_batch_sync", "qsa_batch_destroy",
           "qsa_batch_sweep_static", "qsa_load_plasma_weights", "qsa_load_ions", "qsa_dirichlet_solve")

KERNEL_CLASSES = {"push_pred": 0, "push_final": 1, "dep_S": 2, "dep_J": 3, "row_r2c": 4,
                  "col": 5, "row_c2r": 6, "beam_deposit": 7, "beam_push": 8}


class QSASpecies(C.Structure):
    _fields_ = [("Z", C.c_int32), ("pad_", C.c_int32), ("M", C.c_double)]


class QSAParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nxi", C.c_int32), ("precision", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double), ("dxi", C.c_double), ("dt", C.c_double),
        ("n_corr", C.c_int32), ("n_species", C.c_int32), ("kappa2", C.c_double),
        ("n_plasma", C.c_int64), ("plasma_w", C.c_double),
        ("species", QSASpecies * QSA_MAX_SPECIES),
        ("beam_capacity", C.c_int64 * QSA_MAX_SPECIES),
        ("pipeline", C.c_int32), ("adjoint_steps", C.c_int32), ("ckpt_every", C.c_int32),
        ("no_field_pack", C.c_int32), ("plasma_weights", C.c_int32),
        ("lean_pipeline", C.c_int32), ("b0z", C.c_double),
        ("ion_m", C.c_double), ("ion_z", C.c_int32), ("pad2_", C.c_int32),
    ]


class QSAError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libqsa.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2607_24214_amd.build` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, dp, i32, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64
    L.qsa_workspace_bytes.argtypes = [C.POINTER(QSAParams)]
    L.qsa_workspace_bytes.restype = C.c_size_t
    L.qsa_create.argtypes = [C.POINTER(QSAParams), vp, C.c_size_t, vp, C.POINTER(vp)]
    L.qsa_load_plasma.argtypes = [vp, vp, vp, vp, vp, i64, i32]
    L.qsa_load_plasma_weights.argtypes = [vp, vp, i64, i32]
    L.qsa_load_ions.argtypes = [vp, vp, i64, i32]
    L.qsa_dirichlet_solve.argtypes = [i32, i32, i32, i32, C.c_double, C.c_double, C.c_double, vp, vp, vp]
    L.qsa_load_beam.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, i64, i32]
    L.qsa_load_beam_range.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp, vp, vp, i64, i32]
    L.qsa_read_beam.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, i64, C.POINTER(i64), i32]
    L.qsa_slice_sweep.argtypes = [vp]
    L.qsa_beam_step.argtypes = [vp, i32]
    L.qsa_fields.argtypes = [vp, i32, i32, i32, vp, C.c_size_t, i32]
    L.qsa_field_moments.argtypes = [vp, i32, vp, C.c_size_t, i32]
    L.qsa_beam_moments.argtypes = [vp, i32, i32, vp, C.c_size_t, i32]
    L.qsa_linear_model.argtypes = [i32, i32, C.c_double, C.c_double, vp, i32, vp, i32, dp, vp, vp, vp]
    L.qsa_sync.argtypes = [vp]
    L.qsa_destroy.argtypes = [vp]
    L.qsa_timing_begin.argtypes = [vp, i32]
    L.qsa_timing_end.argtypes = [vp, dp, C.POINTER(i64)]
    L.qsa_set_option.argtypes = [vp, i32, i64]
    L.qsa_get_option.argtypes = [vp, i32, C.POINTER(i64)]
    L.qsa_autotune.argtypes = [vp, dp]
    L.qsa_adjoint_sweep.argtypes = [vp, i32, i32, dp, C.POINTER(C.POINTER(i32)), dp, dp]
    L.qsa_batch_workspace_bytes.argtypes = [i32]
    L.qsa_batch_workspace_bytes.restype = C.c_size_t
    L.qsa_batch_create.argtypes = [C.POINTER(vp), i32, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.qsa_batch_sweep.argtypes = [vp]
    L.qsa_batch_step.argtypes = [vp, i32]
    L.qsa_batch_sync.argtypes = [vp]
    L.qsa_batch_destroy.argtypes = [vp]
    L.qsa_batch_sweep_static.argtypes = [C.POINTER(vp), i32, vp]
    L.qsa_status_string.argtypes = [i32]
    L.qsa_status_string.restype = C.c_char_p
    L.qsa_last_error.argtypes = [vp]
    L.qsa_last_error.restype = C.c_char_p
    for name in ("qsa_create", "qsa_load_plasma", "qsa_load_beam", "qsa_load_beam_range", "qsa_read_beam",
                 "qsa_slice_sweep", "qsa_beam_step", "qsa_fields", "qsa_sync", "qsa_destroy",
                 "qsa_timing_begin", "qsa_timing_end", "qsa_set_option", "qsa_get_option", "qsa_autotune",
                 "qsa_adjoint_sweep", "qsa_batch_create",
                 "qsa_batch_sweep", "qsa_batch_step", "qsa_batch_sync", "qsa_batch_destroy",
                 "qsa_batch_sweep_static", "qsa_load_plasma_weights", "qsa_load_ions", "qsa_dirichlet_solve"):
        getattr(L, name).restype = i32
    _lib = L
    return L
