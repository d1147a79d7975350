"""ctypes declarations of the gmmsp C ABI (include/gmmsp.h).

Argument marshalling only: every step of the method runs in libgmmsp.so.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_int32, c_int64, c_size_t, c_uint32, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmmsp.so")

GMMSP_OK = 0
GMMSP_E_INVAL = -1
GMMSP_E_SIZE = -2
GMMSP_E_HIP = -3
GMMSP_E_NOMEM = -4
GMMSP_E_STATE = -5
THETA_ROW = 13
THETA_ROW3 = 15
THETA_ROW_FULL = 21
THETA_ROW_GRAY = 8
THETA_ROWS = {0: THETA_ROW, 1: THETA_ROW3, 2: THETA_ROW_FULL, 3: THETA_ROW_GRAY}
LL_CAP = 4096
CONN_STATIC_BYTES = 96 << 20   # GMMSP_CONN_STATIC_BYTES
TUNE_CANDIDATES = 12           # GMMSP_TUNE_CANDIDATES


class GmmspParams(ctypes.Structure):
    _fields_ = [("W", c_int32), ("H", c_int32), ("K", c_int32), ("vx", c_int32),
                ("vy", c_int32), ("eps_s", c_double), ("eps_c", c_double),
                ("lam", c_double), ("cov_mode", c_int32), ("n_min", c_double)]


class GmmspGridInfo(ctypes.Structure):
    _fields_ = [("vx", c_int32), ("vy", c_int32), ("nx", c_int32), ("ny", c_int32),
                ("K", c_int32), ("ncx", c_int32), ("ncy", c_int32)]


class GmmspError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gmmsp error {code}: {msg}")
        self.code = code


_SIGS = {
    "gmmsp_grid": (c_int, [POINTER(GmmspParams), POINTER(GmmspGridInfo)]),
    "gmmsp_workspace_bytes": (c_int, [c_int32, POINTER(GmmspParams), POINTER(c_size_t)]),
    "gmmsp_create": (c_int, [c_int32, POINTER(GmmspParams), c_void_p, c_size_t, c_void_p,
                             POINTER(c_void_p)]),
    "gmmsp_destroy": (c_int, [c_void_p]),
    "gmmsp_batch_info": (c_int, [c_void_p, POINTER(c_int32), POINTER(c_int64), POINTER(c_int64)]),
    "gmmsp_image_grid": (c_int, [c_void_p, c_int32, POINTER(GmmspGridInfo)]),
    "gmmsp_init_seeds": (c_int, [c_void_p, c_void_p, c_void_p]),
    "gmmsp_set_params_dev": (c_int, [c_void_p, c_void_p, c_void_p]),
    "gmmsp_set_params": (c_int, [c_void_p, c_void_p, c_void_p]),
    "gmmsp_get_params": (c_int, [c_void_p, c_void_p, c_void_p]),
    "gmmsp_em_iterate": (c_int, [c_void_p, c_void_p, c_int32, c_double, c_void_p, c_void_p]),
    "gmmsp_ll_history": (c_int, [c_void_p, c_int32, c_void_p, c_int32, POINTER(c_int32),
                                 c_void_p]),
    "gmmsp_label": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "gmmsp_export_responsibilities": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "gmmsp_export_candidates": (c_int, [c_void_p, c_void_p, c_void_p]),
    "gmmsp_set_schedule": (c_int, [c_void_p, c_int32]),
    "gmmsp_get_schedule": (c_int, [c_void_p, POINTER(c_int32)]),
    "gmmsp_set_estep_kernel": (c_int, [c_void_p, c_int32]),
    "gmmsp_get_estep_kernel": (c_int, [c_void_p, POINTER(c_int32)]),
    "gmmsp_set_slot_rows": (c_int, [c_void_p, c_int32]),
    "gmmsp_get_slot_rows": (c_int, [c_void_p, POINTER(c_int32)]),
    "gmmsp_autotune": (c_int, [c_void_p, c_void_p, c_int32, c_void_p, POINTER(c_int32), c_void_p]),
    "gmmsp_set_gather_lanes": (c_int, [c_void_p, c_int32]),
    "gmmsp_get_gather_lanes": (c_int, [c_void_p, POINTER(c_int32)]),
    "gmmsp_autotune_gather": (c_int, [c_void_p, c_void_p, c_int32, c_void_p, POINTER(c_int32),
                                      c_void_p]),
    "gmmsp_set_graph_passes": (c_int, [c_void_p, c_int32]),
    "gmmsp_set_persistent": (c_int, [c_void_p, c_int32]),
    "gmmsp_get_persistent": (c_int, [c_void_p, POINTER(c_int32)]),
    "gmmsp_autotune_persistent": (c_int, [c_void_p, c_void_p, c_int32, c_void_p,
                                          POINTER(c_int32), c_void_p]),
    "gmmsp_profile_enable": (c_int, [c_void_p, c_int32]),
    "gmmsp_profile_read": (c_int, [c_void_p, POINTER(c_double), POINTER(c_int32), POINTER(c_int64),
                                   POINTER(c_int64), c_int32]),
    "gmmsp_ws_workspace_bytes": (c_int, [c_void_p, POINTER(c_size_t)]),
    "gmmsp_ws_attach": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "gmmsp_ws_features": (c_int, [c_void_p, c_void_p, c_void_p]),
    "gmmsp_ws_forward": (c_int, [c_void_p, c_void_p, c_int32, c_int32, c_void_p]),
    "gmmsp_ws_apply": (c_int, [c_void_p, c_void_p, c_uint32, c_void_p]),
    "gmmsp_ws_apply_guarded": (c_int, [c_void_p, c_void_p, c_uint32, c_void_p, c_void_p]),
    "gmmsp_ws_targets": (c_int, [c_void_p, c_void_p, c_void_p]),
    "gmmsp_ws_train_step": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_float,
                                    c_int32, c_int32, c_void_p, c_void_p]),
    "gmmsp_ws_read": (c_int, [c_void_p, c_int32, c_void_p, c_size_t, c_void_p]),
    "gmmsp_ws_write": (c_int, [c_void_p, c_int32, c_void_p, c_size_t, c_void_p]),
    "gmmsp_conn_workspace_bytes": (c_int, [c_void_p, POINTER(c_size_t)]),
    "gmmsp_srgb8_to_lab": (c_int, [c_void_p, c_int64, c_void_p, c_void_p]),
    "gmmsp_metrics_workspace_bytes": (c_int, [c_void_p, c_void_p, c_void_p, POINTER(c_size_t)]),
    "gmmsp_metrics": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                              c_size_t, c_void_p, c_void_p, c_void_p]),
    "gmmsp_connectivity": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                   c_int32, c_void_p, c_void_p]),
    "gmmsp_connectivity_static": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                                          c_void_p, c_void_p]),
    "gmmsp_last_error": (c_char_p, []),
}

WS_NPARAM = 26026
WS_ALL_OUTPUTS = 0x3FF
# outputs that move the spatial parameters: mu_x, mu_y, S_xx, S_yy
WS_SPATIAL_OUTPUTS = 0b0001100011
# warm-start workspace buffers: index -> (dtype, channels per superpixel)
WS_BUFFERS = {
    "feat": (0, "float32", 16), "x0": (1, "bf16", 16), "y1": (2, "bf16", 32),
    "y2": (3, "bf16", 32), "y3": (4, "bf16", 32), "out": (5, "float32", 16),
    "tgt": (6, "float32", 16), "g4": (7, "bf16", 16), "g3": (8, "bf16", 32),
    "g2": (9, "bf16", 32), "g1": (10, "bf16", 32), "grad": (11, "float32", None),
}

_lib = None


def lib():
    """Load libgmmsp.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def check(rc: int):
    if rc != GMMSP_OK:
        raise GmmspError(rc, lib().gmmsp_last_error().decode())
    return rc
