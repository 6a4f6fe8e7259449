"""ctypes declarations of libposetx.so (the C ABI in include/posetx.h).

Argument marshalling only: every step of the transforms runs in the library.
Importing this module fails loudly if the library has not been built.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libposetx.so")

PX_I64, PX_F32, PX_F64 = 0, 1, 2
PX_BUILD_HOST_ONLY = 0x1
PX_BUILD_NO_ADJOINT = 0x2
PX_BUILD_LEVELS_MIRSKY = 0x4
PX_BUILD_SPARSE_NIV = 0x8
PX_BUILD_MIN_CHAINS = 0x10
PX_LAYOUT_NODES, PX_LAYOUT_ROWS = 0, 1

STATUS = {0: "PX_OK", 1: "PX_EINVAL", 2: "PX_ECYCLE", 3: "PX_ECHAIN", 4: "PX_ENOMEM", 5: "PX_EHIP",
          6: "PX_EUNSUPPORTED", 7: "PX_ENONFINITE", 8: "PX_ENOTCONV"}

EXPORTS = [
    "px_poset_build", "px_poset_free", "px_poset_info", "px_poset_chains", "px_poset_niv",
    "px_poset_levels", "px_reserve", "px_zeta", "px_zeta_adjoint", "px_mobius", "px_mobius_adjoint",
    "px_batch_build", "px_batch_free", "px_batch_reserve", "px_batch_rows", "px_zeta_batched",
    "px_zeta_adjoint_batched", "px_last_error", "px_version", "px_profile", "px_profile_read",
    "px_profile_phase_name", "px_autotune", "px_batch_autotune", "px_poset_niv_csr", "px_poset_rows",
    "px_poset_save", "px_poset_load", "px_zeta_noalloc", "px_poset_set_layout",
    "px_batch_set_layout", "px_batch_row_order",
]


class PosetxError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{where}: {self.name}: {msg}")


class Info(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "n", "k", "edges", "nnz_niv", "nnz_niv_up", "max_chain", "levels_down", "levels_up",
        "mirsky_levels", "udep_levels", "device_bytes", "walk_runs", "walk_events", "walk_snapshots", "walk_T",
        "walk_emax", "walk_rows_distinct", "walk_row_loads")] + [
        ("chains_planted", ctypes.c_int32), ("device", ctypes.c_int32)] + [
        (name, ctypes.c_double) for name in ("t_validate", "t_chains", "t_niv", "t_levels", "t_upload")] + [
        ("niv_sparse", ctypes.c_int32), ("niv_device_rounds", ctypes.c_int32),
        ("run_chunks", ctypes.c_int64), ("run_events", ctypes.c_int64), ("path_cover", ctypes.c_int64),
        ("layout", ctypes.c_int64), ("scan_flat", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class TuneReport(ctypes.Structure):
    _fields_ = [("walk_T", ctypes.c_int32), ("walk_emax", ctypes.c_int32), ("rhs_tile", ctypes.c_int32),
                ("ms_best", ctypes.c_double), ("ms_default", ctypes.c_double), ("from_cache", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class RefineReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("nonfinite", ctypes.c_int32), ("residual", ctypes.c_double),
                ("correction", ctypes.c_double)]

    def as_dict(self):
        return {"iterations": self.iterations, "nonfinite": bool(self.nonfinite), "residual": self.residual,
                "correction": self.correction}


def _declare(lib):
    P = ctypes.c_void_p
    i64, i32, u32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_uint32, ctypes.c_double
    sig = {
        "px_poset_build": [i64, P, P, P, P, u32, i32, ctypes.POINTER(P)],
        "px_poset_free": [P],
        "px_poset_info": [P, ctypes.POINTER(Info)],
        "px_poset_chains": [P, P, P],
        "px_poset_niv": [P, i32, P],
        "px_poset_niv_csr": [P, i32, P, P],
        "px_poset_rows": [P, P],
        "px_poset_set_layout": [P, u32],
        "px_batch_set_layout": [P, u32],
        "px_batch_row_order": [P, P],
        "px_poset_save": [P, ctypes.c_char_p],
        "px_poset_load": [ctypes.c_char_p, u32, i32, ctypes.POINTER(P)],
        "px_poset_levels": [P, i32, P],
        "px_reserve": [P, i32, i64],
        "px_zeta": [P, i32, P, i64, P, i64, i64, P],
        "px_zeta_adjoint": [P, i32, P, i64, P, i64, i64, P],
        "px_zeta_noalloc": [P, i32, P, i64, P, i64, i64, P],
        "px_mobius": [P, i32, P, i64, P, i64, i64, i32, f64, P, ctypes.POINTER(RefineReport)],
        "px_mobius_adjoint": [P, i32, P, i64, P, i64, i64, i32, f64, P, ctypes.POINTER(RefineReport)],
        "px_batch_build": [i32, P, ctypes.POINTER(P)],
        "px_batch_free": [P],
        "px_batch_reserve": [P, i32, i64],
        "px_batch_rows": [P, ctypes.POINTER(i64)],
        "px_zeta_batched": [P, i32, P, i64, P, i64, i64, P],
        "px_zeta_adjoint_batched": [P, i32, P, i64, P, i64, i64, P],
        "px_profile": [i32],
        "px_autotune": [P, i32, i64, ctypes.POINTER(TuneReport)],
        "px_batch_autotune": [P, i32, i64, ctypes.POINTER(TuneReport)],
        "px_profile_read": [P, P, i32],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.px_last_error.restype = ctypes.c_char_p
    lib.px_last_error.argtypes = []
    lib.px_version.restype = ctypes.c_char_p
    lib.px_version.argtypes = []
    lib.px_profile_phase_name.restype = ctypes.c_char_p
    lib.px_profile_phase_name.argtypes = [i32]
    return lib


_LIB = None


def lib():
    """The loaded library; raises ImportError if it is not built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2211_13706_amd.build`")
        _LIB = _declare(ctypes.CDLL(LIB_PATH))
    return _LIB


def check(status: int, where: str):
    if status != 0:
        raise PosetxError(status, where, lib().px_last_error().decode())
