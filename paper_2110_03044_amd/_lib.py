"""ctypes loader of libfluxlim.so (the HIP library).  Marshals arguments only.

There is no fallback: if the library is not built, importing the package's operators raises.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfluxlim.so")

FL_OK = 0
STATUS = {0: "FL_OK", -1: "FL_E_INVALID", -2: "FL_E_TOPOLOGY", -3: "FL_E_UNSUPPORTED",
          -4: "FL_E_NOMEM", -5: "FL_E_HIP", -6: "FL_E_NONFINITE",
          -7: "FL_E_NODEVICE"}

FL_MESH_REORDER = 1
FL_MESH_FACE_PATH = 2
FL_MESH_REORDER_BFS = 4
FL_PATH_FACE_CELL = 1
FL_PATH_FUSED = 2


class FluxLimError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        self.status = status
        super().__init__(f"{func} failed with {STATUS.get(status, status)}: {msg}")


class MeshInfo(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int64), ("n_faces", ctypes.c_int64),
                ("max_degree", ctypes.c_int32), ("pairs", ctypes.c_int32),
                ("path", ctypes.c_int32), ("device", ctypes.c_int32),
                ("reordered", ctypes.c_int32), ("uniform_area", ctypes.c_int32),
                ("uniform_volume", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
                ("tile_cells", ctypes.c_int32), ("max_halo", ctypes.c_int32),
                ("halo_total", ctypes.c_int64), ("general", ctypes.c_int32),
                ("max_side", ctypes.c_int32), ("aligned", ctypes.c_int32),
                ("dist_weighted", ctypes.c_int32), ("n_boundary", ctypes.c_int64),
                ("compact", ctypes.c_int32), ("max_rated", ctypes.c_int32),
                ("max_nexts", ctypes.c_int32), ("side_entries", ctypes.c_int32),
                ("halo_nexts", ctypes.c_int64)]


class AlgebraicInfo(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64 * 5), ("width", ctypes.c_int32 * 5),
                ("device_bytes", ctypes.c_int64)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_D = ctypes.c_double
_S = ctypes.c_int32
_SZ = ctypes.c_size_t

# name -> (restype, argtypes); every symbol of include/fluxlim.h
SIGNATURES = {
    "fl_mesh_validate": (_S, [_I64, _I64, _P, _P]),
    "fl_mesh_create": (_S, [_I64, _I64, _P, _P, _P, _P, _I, ctypes.c_uint32, _P]),
    "fl_mesh_destroy": (_S, [_P]),
    "fl_mesh_info": (_S, [_P, _P]),
    "fl_mesh_create_dist": (_S, [_I64, _I64, _P, _P, _P, _P, _P, _I, ctypes.c_uint32, _P]),
    "fl_mesh_set_inflow": (_S, [_P, _P, _I]),
    "fl_mesh_permutation": (_S, [_P, _P, _P]),
    "fl_mesh_export_tables": (_S, [_P, _P, _P, _P]),
    "fl_permute_cells": (_S, [_P, _I, _I, _P, _P, _P]),
    "fl_permute_faces": (_S, [_P, _I, _P, _P, _P]),
    "fl_apply_workspace_bytes": (_SZ, [_P, _I]),
    "fl_convect_apply": (_S, [_P, _I, _I, _P, _P, _P, _P, _P]),
    "fl_rk_workspace_bytes": (_SZ, [_P, _I, _I]),
    "fl_rk_step": (_S, [_P, _I, _I, _D, _I, _P, _P, _P, _P]),
    "fl_rk_steps": (_S, [_P, _I, _I, _D, _I, _I64, _P, _P, _P, _P]),
    "fl_rk_steps_scaled": (_S, [_P, _I, _I, _D, _I, _I64, _P, _P, _P, _P, _P]),
    "fl_adjoint_workspace_bytes": (_SZ, [_P, _I]),
    "fl_convect_adjoint": (_S, [_P, _I, _I, _P, _P, _P, _P, _P, _P, _P]),
    "fl_rk_adjoint_workspace_bytes": (_SZ, [_P, _I, _I]),
    "fl_rk_step_adjoint": (_S, [_P, _I, _I, _D, _I, _P, _P, _P, _P, _P, _P]),
    "fl_rk_step_store": (_S, [_P, _I, _I, _D, _I, _P, _P, _P, _P, _P]),
    "fl_rk_steps_store": (_S, [_P, _I, _I, _D, _I, _I64, _P, _P, _P, _P, _P]),
    "fl_rk_steps_noalloc": (_S, [_P, _I, _I, _D, _I, _I64, _P, _P, _P]),
    "fl_adjoint_rates_bytes": (_SZ, [_P]),
    "fl_adjoint_rates": (_S, [_P, _P, _P, _P]),
    "fl_adjoint_uacc_bytes": (_SZ, [_P]),
    "fl_rk_steps_adjoint_workspace_bytes": (_SZ, [_P, _I, _I]),
    "fl_rk_steps_adjoint": (_S, [_P, _I, _I, _D, _I, _I64, _P, _P, _P, _P, _P, _P]),
    "fl_adjoint_uacc_scatter": (_S, [_P, _P, _P, _P]),
    "fl_batch_create": (_S, [_I, _P, _P, _P, _P, _I, _P, _P, _I, _I, _P]),
    "fl_batch_step": (_S, [_P, _I, _P]),
    "fl_batch_step_unbatched": (_S, [_P, _I, _P]),
    "fl_batch_tile": (_S, [_P, _P]),
    "fl_batch_lds": (_S, [_P, _P]),
    "fl_batch_tuned_from_cache": (_S, [_P, _P]),
    "fl_batch_destroy": (_S, [_P]),
    "fl_algebraic_create": (_S, [_P, _P]),
    "fl_algebraic_destroy": (_S, [_P]),
    "fl_algebraic_info": (_S, [_P, _P]),
    "fl_algebraic_export": (_S, [_P, _I, _P, _P]),
    "fl_algebraic_workspace_bytes": (_SZ, [_P]),
    "fl_algebraic_face_values": (_S, [_P, _I, _P, _P, _P, _P, _P]),
    "fl_algebraic_rk_steps": (_S, [_P, _I, _I, _D, _I64, _P, _P, _P, _P]),
    "fl_set_option": (_S, [_I, _I]),
    "fl_status_str": (ctypes.c_char_p, [_S]),
    "fl_last_error": (ctypes.c_char_p, []),
    "fl_debug_select": (_S, [_P, _P, _P, _P]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -m paper_2110_03044_amd._build` "
                "(the HIP library is required: there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int, func: str):
    if status != FL_OK:
        msg = lib().fl_last_error()
        raise FluxLimError(status, func, msg.decode() if msg else "")


def call(name: str, *args):
    st = getattr(lib(), name)(*args)
    check(st, name)
    return st
