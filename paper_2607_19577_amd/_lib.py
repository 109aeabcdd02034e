"""ctypes loader for ``libqst.so`` (the C ABI of include/qst.h).

Marshalling only: every step of the hot path runs in the HIP library.  If the
library has not been built the import of this module still succeeds, but the
first use raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqst.so")

# Enums of include/qst.h
QST_OK = 0
STATUS_NAMES = {
    0: "QST_OK", 1: "QST_ERR_INVALID_ARG", 2: "QST_ERR_SHAPE", 3: "QST_ERR_ALIGN", 4: "QST_ERR_UNSUPPORTED",
    5: "QST_ERR_DEVICE", 6: "QST_ERR_OOM", 7: "QST_ERR_NUMERIC", 8: "QST_ERR_CAPTURE",
}
LOSS_CE, LOSS_LS, LOSS_NONE = 0, 1, 2
(PATH_AUTO, PATH_BUTTERFLY_F32, PATH_BUTTERFLY_F64, PATH_PLAIN_F32, PATH_TILE_F16, PATH_TILE_BF16,
 PATH_BUTTERFLY_BF16) = range(7)

# Entry points declared in include/qst.h (checked against the header by the tests).
EXPORTS = (
    "qst_create", "qst_destroy", "qst_set_stream", "qst_status_string", "qst_last_error", "qst_plan",
    "qst_forward", "qst_backward", "qst_backward_static", "qst_atom_trial", "qst_reweight_simplex", "qst_refactor", "qst_solve",
    "qst_state_error", "qst_build_info", "qst_profile_enable", "qst_profile_read", "qst_plan_choice",
)


class QstInstance(ctypes.Structure):
    _fields_ = [
        ("n_qubits", ctypes.c_int32),
        ("rank", ctypes.c_int32),
        ("n_settings", ctypes.c_int32),
        ("settings_per_batch", ctypes.c_int32),
        ("atoms", ctypes.c_void_p),
        ("weights", ctypes.c_void_p),
        ("settings", ctypes.c_void_p),
        ("freqs", ctypes.c_void_p),
        ("probs_base", ctypes.c_void_p),
        ("unitaries", ctypes.c_void_p),
        ("freqs_rowptr", ctypes.c_void_p),
        ("freqs_index", ctypes.c_void_p),
        ("freqs_nnz", ctypes.c_int64),
        ("n_unitaries", ctypes.c_int32),
    ]


class QstSolveParams(ctypes.Structure):
    _fields_ = [
        ("max_slots", ctypes.c_int32),
        ("t_alpha", ctypes.c_int32),
        ("t_ref", ctypes.c_int32),
        ("n_grid", ctypes.c_int32),
        ("rank_max", ctypes.c_int32),
        ("n_lanczos", ctypes.c_int32),
        ("stop_window", ctypes.c_int32),
        ("loss_kind", ctypes.c_int32),
        ("stop_delta", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("tau_acc", ctypes.c_double),
        ("oracle_budget", ctypes.c_int64),
    ]


class QstChoice(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("settings_per_batch", ctypes.c_int32),
        ("tile_bits_fwd", ctypes.c_int32),
        ("tile_bits_adj", ctypes.c_int32),
        ("values_per_thread_log2", ctypes.c_int32),
        ("w_row_bits", ctypes.c_int32),
        ("x_row_bits", ctypes.c_int32),
        ("tuned", ctypes.c_int32),
        ("best_ms", ctypes.c_double),
        ("default_ms", ctypes.c_double),
    ]


class QSTError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")


_lib = None


def load() -> ctypes.CDLL:
    """Load ``libqst.so`` (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    P = ctypes.POINTER
    lib.qst_create.argtypes = [ctypes.c_int, vp, P(vp)]
    lib.qst_destroy.argtypes = [vp]
    lib.qst_set_stream.argtypes = [vp, vp]
    lib.qst_status_string.argtypes = [ctypes.c_int]
    lib.qst_status_string.restype = ctypes.c_char_p
    lib.qst_last_error.argtypes = [vp]
    lib.qst_last_error.restype = ctypes.c_char_p
    lib.qst_build_info.argtypes = []
    lib.qst_build_info.restype = ctypes.c_char_p
    lib.qst_plan.argtypes = [vp, P(QstInstance), ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.qst_forward.argtypes = [vp, P(QstInstance), ctypes.c_int, P(vp), vp, ctypes.c_int, dbl, ctypes.c_int]
    lib.qst_backward.argtypes = [vp, P(QstInstance), ctypes.c_int, P(vp), P(vp), P(vp), vp, ctypes.c_int, dbl,
                                 ctypes.c_int, ctypes.c_int]
    lib.qst_backward_static.argtypes = lib.qst_backward.argtypes
    lib.qst_atom_trial.argtypes = [vp, P(QstInstance), ctypes.c_int, vp, vp, vp, vp, ctypes.c_int, dbl,
                                   ctypes.c_int]
    lib.qst_reweight_simplex.argtypes = [vp, vp, vp, ctypes.c_int, dbl, dbl, vp, vp, vp]
    lib.qst_refactor.argtypes = [vp, P(QstInstance), ctypes.c_int, dbl, dbl, dbl, dbl, ctypes.c_int, ctypes.c_int,
                                 vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int]
    lib.qst_solve.argtypes = [vp, P(QstInstance), P(QstSolveParams), vp, ctypes.c_int, vp, vp, P(i32), vp, vp,
                              ctypes.c_int]
    lib.qst_state_error.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int, vp, vp, ctypes.c_int, P(dbl), ctypes.c_int]
    lib.qst_plan_choice.argtypes = [vp, P(QstInstance), ctypes.c_int, ctypes.c_int, P(QstChoice)]
    lib.qst_profile_enable.argtypes = [vp, ctypes.c_int]
    lib.qst_profile_read.argtypes = [vp, ctypes.c_int, P(ctypes.c_int64), P(dbl), ctypes.c_int]
    for name in EXPORTS:
        if name not in ("qst_status_string", "qst_last_error", "qst_build_info"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(status: int, handle=None) -> None:
    if status != QST_OK:
        lib = load()
        msg = lib.qst_last_error(handle).decode() if handle else lib.qst_status_string(status).decode()
        raise QSTError(status, msg or lib.qst_status_string(status).decode())
