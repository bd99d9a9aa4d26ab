"""ctypes declarations of liblfem.so (the C ABI in include/lfem.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LFEM_LIBRARY", os.path.join(HERE, "liblfem.so"))

LFEM_OK = 0
LFEM_EINVAL = 1
LFEM_ENOMEM = 2
LFEM_EHIP = 3
LFEM_ERANGE = 4
LFEM_EDEGENERATE = 5
LFEM_EUNSUPPORTED = 6

LFEM_SURFACE = 0
LFEM_BULK = 1

LFEM_M = 1
LFEM_A = 2
LFEM_MC = 4

LFEM_SCATTER_AUTO = 0
LFEM_SCATTER_BLOCKED = 1
LFEM_SCATTER_STAGED = 2
LFEM_SCATTER_ATOMIC = 3
LFEM_TUNE_ALLOW_ATOMIC = 1
LFEM_TUNE_NO_CACHE = 2

STATUS_NAMES = {0: "LFEM_OK", 1: "LFEM_EINVAL", 2: "LFEM_ENOMEM", 3: "LFEM_EHIP",
                4: "LFEM_ERANGE", 5: "LFEM_EDEGENERATE", 6: "LFEM_EUNSUPPORTED"}

# every symbol include/lfem.h declares
EXPORTS = [
    "lfem_mesh_create", "lfem_mesh_set_coords", "lfem_pattern_build", "lfem_pattern_get",
    "lfem_pattern_info",
    "lfem_assemble", "lfem_assemble_mass", "lfem_assemble_stiffness", "lfem_assemble_weighted",
    "lfem_pattern_autotune", "lfem_pattern_autotune_ex", "lfem_tune_cache_clear", "lfem_pattern_schedule", "lfem_batch_create", "lfem_batch_create_ex", "lfem_assemble_batch", "lfem_shape_grad",
    "lfem_shape_grad_noalloc", "lfem_energy", "lfem_assemble_load", "lfem_assemble_kll", "lfem_spmv", "lfem_dziuk_system", "lfem_kll_system", "lfem_reference_table", "lfem_status_get", "lfem_status_reset", "lfem_last_error", "lfem_version", "lfem_set_debug",
    "lfem_mesh_destroy", "lfem_pattern_destroy", "lfem_batch_destroy",
]


class PatternInfo(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("nnz", C.c_int64), ("max_row", C.c_int32),
                ("blocks", C.c_int32), ("block_cap", C.c_int32), ("max_block_rows", C.c_int32),
                ("max_block_elems", C.c_int32), ("max_colors", C.c_int32), ("halo", C.c_double),
                ("scatter", C.c_int32), ("slot_bytes", C.c_int32)]


class LfemError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load():
    """Load liblfem.so once; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"liblfem.so not found at {LIB_PATH}: run "
                          "`python -c 'import __graft_entry__ as g; g.build()'` first")
    L = C.CDLL(LIB_PATH)
    vp, i64, ci, cu, dbl = C.c_void_p, C.c_int64, C.c_int, C.c_uint, C.c_double
    vpp = C.POINTER(C.c_void_p)
    L.lfem_mesh_create.argtypes = [ci, ci, ci, i64, vp, i64, vp, ci, vp, vpp]
    L.lfem_mesh_set_coords.argtypes = [vp, vp]
    L.lfem_pattern_build.argtypes = [vp, vp, vpp]
    L.lfem_pattern_get.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), vpp, vpp]
    L.lfem_pattern_info.argtypes = [vp, C.POINTER(PatternInfo)]
    L.lfem_assemble.argtypes = [vp, vp, cu, vp, vp, vp, vp, vp, ci, vp]
    L.lfem_assemble_mass.argtypes = [vp, vp, vp, vp]
    L.lfem_assemble_stiffness.argtypes = [vp, vp, vp, vp, vp]
    L.lfem_assemble_weighted.argtypes = [vp, vp, vp, vp, vp]
    L.lfem_pattern_autotune.argtypes = [vp, vp, cu, vp, C.POINTER(ci)]
    L.lfem_pattern_autotune_ex.argtypes = [vp, vp, cu, cu, vp, C.POINTER(ci), C.POINTER(ci)]
    L.lfem_tune_cache_clear.argtypes = []
    L.lfem_tune_cache_clear.restype = None
    L.lfem_pattern_schedule.argtypes = [vp, vp, ci, ci, vp]
    L.lfem_batch_create.argtypes = [ci, vpp, vpp, cu, ci, vp, vpp]
    L.lfem_batch_create_ex.argtypes = [ci, vpp, vpp, cu, vpp, vpp, ci, vp, vpp]
    L.lfem_assemble_batch.argtypes = [vp, vpp, vp]
    L.lfem_shape_grad.argtypes = [vp, vp, vp, dbl, vp, vp, dbl, vp, vp]
    L.lfem_shape_grad_noalloc.argtypes = [vp, vp, vp, dbl, vp, vp, dbl, vp, vp]
    L.lfem_energy.argtypes = [vp, vp, vp, dbl, vp, vp, dbl, vp, vp]
    L.lfem_assemble_load.argtypes = [vp, vp, vp, vp]
    L.lfem_assemble_kll.argtypes = [vp, vp, vp, vp, vp]
    L.lfem_spmv.argtypes = [vp, vp, vp, dbl, vp, ci, vp]
    L.lfem_dziuk_system.argtypes = [vp, vp, dbl, vp, vp, vp, vp, vp, vp]
    L.lfem_kll_system.argtypes = [vp, vp, dbl, dbl, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.lfem_reference_table.argtypes = [ci, ci, ci, C.POINTER(ci), C.POINTER(ci), vp, vp, vp, vp]
    L.lfem_status_get.argtypes = [vp, C.POINTER(i64)]
    L.lfem_status_reset.argtypes = [vp, vp]
    L.lfem_last_error.argtypes = []
    L.lfem_last_error.restype = C.c_char_p
    L.lfem_version.argtypes = []
    L.lfem_set_debug.argtypes = [ci]
    L.lfem_version.restype = C.c_char_p
    for name in ("lfem_mesh_destroy", "lfem_pattern_destroy", "lfem_batch_destroy"):
        getattr(L, name).argtypes = [vp]
        getattr(L, name).restype = None
    for name in EXPORTS:
        fn = getattr(L, name)
        if name not in ("lfem_last_error", "lfem_version", "lfem_mesh_destroy",
                        "lfem_pattern_destroy", "lfem_batch_destroy", "lfem_tune_cache_clear"):
            fn.restype = ci
    _lib = L
    return L


def check(status: int, where: str):
    if status != LFEM_OK:
        msg = load().lfem_last_error().decode(errors="replace")
        raise LfemError(status, where, msg)
