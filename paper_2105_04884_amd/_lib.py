"""ctypes declarations of librbl's C-ABI (include/rbl.h).

Argument marshalling only: every computation happens in the HIP kernels of
librbl.so.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbl.so")

RBL_OK = 0
RBL_W_SKIN = 1
RBL_E_ARG = -1
RBL_E_BOX = -2
RBL_E_STATE = -3
RBL_E_CAPACITY = -4
RBL_E_NONFINITE = -5
RBL_E_HIP = -6
RBL_E_NOMEM = -7

STATUS_NAMES = {
    0: "RBL_OK", 1: "RBL_W_SKIN", -1: "RBL_E_ARG", -2: "RBL_E_BOX", -3: "RBL_E_STATE",
    -4: "RBL_E_CAPACITY", -5: "RBL_E_NONFINITE", -6: "RBL_E_HIP", -7: "RBL_E_NOMEM",
}

PREC_FP64, PREC_MIXED = 0, 1
PAIR_LJ, PAIR_LJ_ERFC = 0, 1
LIST_CORE, LIST_SHELL, LIST_FULL = 1, 2, 4
SHELL_LIST, SHELL_STENCIL, SHELL_PAPER = 0, 1, 2
MAX_P = 128

KIND_FORCE_RBL, KIND_FORCE_FULL, KIND_BUILD, KIND_BIN, KIND_INTEGRATE, KIND_REDUCE, KIND_PREDRAW = range(7)


class Config(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("n_replicas", C.c_int32),
        ("precision", C.c_int32),
        ("pair", C.c_int32),
        ("lists", C.c_int32),
        ("skin", C.c_double),
        ("alpha", C.c_double),
        ("shift", C.c_int32),
        ("momentum_fix", C.c_int32),
        ("predraw", C.c_int32),
        ("graphs", C.c_int32),
        ("lanes", C.c_int32),
        ("persistent", C.c_int32),
        ("capacity_factor", C.c_double),
        ("replica_offsets", C.POINTER(C.c_int64)),
        ("charges", C.c_void_p),
        ("shell_source", C.c_int32),
        ("rebuild_check", C.c_int32),
        ("core_filter", C.c_int32),
        ("n_types", C.c_int32),
        ("types", C.POINTER(C.c_int32)),
        ("pair_coeffs", C.POINTER(C.c_double)),
    ]


_lib = None
_names = [
    "rbl_config_init", "rbl_create", "rbl_destroy", "rbl_build", "rbl_forces", "rbl_forces_noalloc",
    "rbl_full_forces",
    "rbl_step", "rbl_continue", "rbl_last_run", "rbl_row_counts", "rbl_export_lists", "rbl_export_batches", "rbl_export_drawn_batches",
    "rbl_export_binning",
    "rbl_sync", "rbl_set_profiling", "rbl_kernel_stats", "rbl_info", "rbl_tuning", "rbl_launch_modes",
    "rbl_core_filter",
    "rbl_set_thermostat", "rbl_unwrap", "rbl_msd", "rbl_rdf", "rbl_thermo",
    "rbl_last_error",
    "rbl_version",
]


class LibraryMissing(RuntimeError):
    pass


def load(path: str = LIB_PATH):
    """Loads librbl.so and declares its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise LibraryMissing(
            f"{path} is not built; run __graft_entry__.build() (hipcc --offload-arch=gfx950)")
    lib = C.CDLL(path)
    vp, i64, i32, u64, d = C.c_void_p, C.c_int64, C.c_int, C.c_uint64, C.c_double
    p64 = C.POINTER(C.c_int64)
    p32 = C.POINTER(C.c_int32)
    pd = C.POINTER(C.c_double)
    sig = {
        "rbl_config_init": (None, [C.POINTER(Config), i64]),
        "rbl_create": (i32, [C.POINTER(Config), vp, C.POINTER(vp)]),
        "rbl_destroy": (i32, [vp]),
        "rbl_build": (i32, [vp, vp, pd, d, d]),
        "rbl_forces": (i32, [vp, i32, u64, u64, vp, vp, vp]),
        "rbl_forces_noalloc": (i32, [vp, i32, u64, u64, vp, vp, vp]),
        "rbl_full_forces": (i32, [vp, vp, vp, vp]),
        "rbl_step": (i32, [vp, vp, vp, vp, i64, d, i32, u64, i64, i32, i32, vp]),
        "rbl_continue": (i32, [vp, vp, vp, vp, i64, vp]),
        "rbl_last_run": (i32, [vp, p32, p64, p32, p64, p64]),
        "rbl_row_counts": (i32, [vp, i64, p64, p64]),
        "rbl_export_lists": (i32, [vp, i64, p64, p64, p32, p64, p32, p64, p32]),
        "rbl_export_batches": (i32, [vp, i32, u64, u64, i64, p64, p32, p32]),
        "rbl_export_drawn_batches": (i32, [vp, i64, p64, p32, p32, p32, p32, p64]),
        "rbl_export_binning": (i32, [vp, p32, p64, p32]),
        "rbl_sync": (i32, [vp]),
        "rbl_set_profiling": (i32, [vp, i32]),
        "rbl_kernel_stats": (i32, [vp, i32, p64, pd]),
        "rbl_info": (i32, [vp, p64, p32, p32, p32]),
        "rbl_tuning": (i32, [vp, p32, p32, pd]),
        "rbl_core_filter": (i32, [vp, p32, pd, pd]),
        "rbl_launch_modes": (i32, [vp, p32, p32, pd]),
        "rbl_set_thermostat": (i32, [vp, d, pd]),
        "rbl_unwrap": (i32, [vp, vp, vp]),
        "rbl_msd": (i32, [vp, vp, vp, vp]),
        "rbl_rdf": (i32, [vp, vp, d, i32, vp]),
        "rbl_thermo": (i32, [vp, vp, vp, pd]),
        "rbl_last_error": (C.c_char_p, []),
        "rbl_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_names():
    return list(_names)
