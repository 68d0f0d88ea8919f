"""ctypes declarations of the C ABI in ``include/wavestep.h``.

Argument marshalling only: every step of the method runs in the HIP kernels of
``libwavestep.so``.  Importing this module does not touch the GPU; loading the
library fails loudly when it has not been built.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwavestep.so")

WS_OK, WS_EINVAL, WS_ESTATE, WS_EHIP, WS_ENOMEM = 0, -1, -2, -3, -4
WS_F64, WS_F32 = 0, 1
WS_LIM_MC, WS_LIM_NONE, WS_LIM_VANLEER = 0, 1, 2
WS_TRANSVERSE_CORR = 0x100
WS_BC_NONE, WS_BC_EXTRAP, WS_BC_PERIODIC = 0, 1, 2
WS_TILE_DIRECT, WS_TILE_MARCH, WS_TILE_PACKED = 0, 1, 2

#: every symbol the header declares
EXPORTS = (
    "ws_layout", "ws_init_patches", "ws_set_tiling", "ws_get_tiling", "ws_upload_patch", "ws_download_patch",
    "ws_fill_ghosts", "ws_step_level", "ws_step_level_per_patch", "ws_set_dt", "ws_step_auto",
    "ws_capture_steps", "ws_graph_launch", "ws_read_dt_cfl", "ws_read_patch_cfl",
    "ws_conservation_sums", "ws_mask_bytes", "ws_patch_layout", "ws_step_record_masks",
    "ws_adjoint_step", "ws_gather", "ws_add_at", "ws_time_step_kernel", "ws_current_pool",
    "ws_attach_medium", "ws_upload_medium", "ws_link_layout", "ws_link_level",
    "ws_cf_layout", "ws_cf_init", "ws_cf_step", "ws_cf_nest", "ws_cf_fill_fine_ghosts",
    "ws_cf_destroy", "ws_noalloc_scratch_bytes", "ws_step_level_noalloc",
    "ws_destroy", "ws_last_error",
)


class PatchDesc(ctypes.Structure):
    _fields_ = [
        ("mx", ctypes.c_int32), ("my", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("instance", ctypes.c_int32), ("bc", ctypes.c_int32),
    ]


class Material(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("K", ctypes.c_double)]


class FinePlace(ctypes.Structure):
    _fields_ = [("coarse_patch", ctypes.c_int32), ("ci0", ctypes.c_int32),
                ("cj0", ctypes.c_int32)]


class WaveStepError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"wavestep error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load ``libwavestep.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it first (python -m paper_1808_02638_amd.build_lib "
            "or __graft_entry__.build()); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "ws_layout": [P(PatchDesc), i32, i32, i32, P(i64), P(i64)],
        "ws_init_patches": [P(vp), P(PatchDesc), i32, P(Material), i32, i32, i32, i32,
                            vp, vp, i64, vp, i64, vp],
        "ws_set_tiling": [vp, P(i32), P(i32), P(i32), i32],
        "ws_get_tiling": [vp, P(i32), P(i32), P(i32), P(i32), P(i32)],
        "ws_upload_patch": [vp, i32, vp],
        "ws_download_patch": [vp, i32, vp],
        "ws_fill_ghosts": [vp],
        "ws_step_level": [vp, dbl, P(dbl)],
        "ws_step_level_per_patch": [vp, dbl, P(dbl)],
        "ws_set_dt": [vp, P(dbl)],
        "ws_step_auto": [vp, dbl],
        "ws_capture_steps": [vp, i32, dbl],
        "ws_graph_launch": [vp],
        "ws_read_dt_cfl": [vp, P(dbl), P(dbl), P(dbl)],
        "ws_read_patch_cfl": [vp, P(dbl)],
        "ws_conservation_sums": [vp, P(dbl)],
        "ws_mask_bytes": [vp, P(i64)],
        "ws_patch_layout": [vp, i32, P(i64), P(i64), P(i64)],
        "ws_step_record_masks": [vp, dbl, vp, P(dbl)],
        "ws_adjoint_step": [vp, dbl, vp, vp, vp],
        "ws_gather": [vp, vp, i32, i32, i32, vp, vp],
        "ws_add_at": [vp, vp, i32, i32, i32, vp, vp],
        "ws_time_step_kernel": [vp, i32, i32, P(dbl)],
        "ws_current_pool": [vp, P(i32)],
        "ws_attach_medium": [vp, vp, i64],
        "ws_upload_medium": [vp, i32, P(dbl), P(dbl)],
        "ws_link_layout": [vp, P(i64)],
        "ws_link_level": [vp, P(i32), i32, i32, i32, vp, i64],
        "ws_cf_layout": [vp, i32, P(i64)],
        "ws_cf_init": [P(vp), vp, vp, i32, P(FinePlace), vp, i64],
        "ws_cf_step": [vp, dbl],
        "ws_cf_nest": [vp, vp],
        "ws_cf_fill_fine_ghosts": [vp, dbl],
        "ws_cf_destroy": [vp],
        "ws_step_level_noalloc": [P(PatchDesc), i32, P(Material), i32, i32, i32, vp, vp, i64,
                                  dbl, P(dbl), vp],
        "ws_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.ws_noalloc_scratch_bytes.argtypes = []
    L.ws_noalloc_scratch_bytes.restype = ctypes.c_int64
    L.ws_last_error.argtypes = []
    L.ws_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(rc):
    if rc != WS_OK:
        raise WaveStepError(rc, lib().ws_last_error().decode(errors="replace"))
    return rc
