"""ctypes binding of libtsdfs.so (argument marshalling only).

The library is built in-tree by ``paper_2311_17878_amd.build``; it is loaded
from the package directory and built only when no library is present.
"""
from __future__ import annotations

import ctypes
import os

from . import build as _build

c_int32, c_int64, c_float, c_size_t, c_void_p = (ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                                                ctypes.c_size_t, ctypes.c_void_p)
P = c_void_p

TSDFS_OK, TSDFS_EINVAL, TSDFS_ECAPACITY, TSDFS_EHIP, TSDFS_EUNSUPPORTED = 0, -1, -2, -3, -4
HIT, NO_FAR, MISS, INVALID = 0, 1, 2, 3
FP32, BF16, BF16X6 = 0, 1, 2


class TsdfsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tsdfs error {code}: {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("n", c_int32 * 3), ("lo", c_float * 3), ("h", c_float), ("d_t", c_float),
                ("d_s", c_float), ("nb_radius", c_int32), ("m_consec", c_int32)]


class FieldDesc(ctypes.Structure):
    _fields_ = [("width", c_int32), ("n_hidden", c_int32), ("pe_freqs", c_int32),
                ("skip_at", c_int32), ("n_feat", c_int32), ("col_hidden", c_int32),
                ("beta", c_float), ("center", c_float * 3), ("scale", c_float)]


# name -> argtypes (restype int unless listed in _RESTYPE)
SIGNATURES = {
    "tsdfs_last_error": [],
    "tsdfs_state_bytes": [P, P],
    "tsdf_reset": [P, P, P],
    "tsdf_integrate": [P, P, P, P, P, c_int64, P, P],
    "tsdf_finalize": [P, P, P, P, P],
    "tsdf_ray_bounds": [P, P, P, P, c_int64, c_float, P, P, P, P, P, P, P],
    "tsdf_ray_range": [P, P, P, c_int64, P, P, P],
    "place_samples_ws_bytes": [c_int64, P],
    "place_samples": [P, P, P, P, c_int64, c_int32, c_int32, c_int32, c_int32, P, P, P, P, P,
                      c_int64, P, P, P, c_size_t, P],
    "place_samples_noalloc": [P, P, P, P, c_int64, c_int32, c_int32, c_int32, c_int32, P, P, P, P,
                              P, c_int64, P, P, P],
    "hs_coarse": [P, P, c_int64, c_int32, P, P, P],
    "hs_upsample": [P, P, P, c_int64, c_int32, c_int32, c_float, P, P, P, P, P],
    "tsdf_bound_stats": [P, P, P, P, P, P, c_int64, P, P],
    "tsdfs_field_params": [P, P, P, P],
    "tsdfs_field_repack": [P, P],
    "adam_step": [P, P, P, P, c_int64, c_float, c_float, c_float, c_float, c_int32, P],
    "tsdf_frontier_ws_bytes": [P, P],
    "tsdf_frontier": [P, P, P, c_int64, P, P, P, P, P, c_size_t, P],
    "tsdf_sparse_meta_bytes": [P, P],
    "tsdf_sparse_reset": [P, P, P],
    "tsdf_sparse_mark": [P, P, P, P, P, c_int64, P],
    "tsdf_sparse_alloc_ws_bytes": [P, P],
    "tsdf_sparse_alloc": [P, P, P, P, c_size_t, P],
    "tsdf_sparse_pool_bytes": [c_int64, P],
    "tsdf_sparse_pool_reset": [c_int64, P, P],
    "tsdf_sparse_accumulate": [P, P, P, c_int64, P, P, P, c_int64, P, P],
    "tsdf_sparse_finalize": [P, P, P, c_int64, P, P, P],
    "select_rays_ws_bytes": [c_int64, P],
    "select_rays": [P, c_int64, c_float, P, P, P, c_size_t, P],
    "gather_rays": [P, P, c_int64, P, P, P, P, P],
    "scatter_rays": [P, P, c_int64, P, P, P, P, P, P, P, P, P],
    "place_fine_samples_ws_bytes": [c_int64, P],
    "place_fine_samples": [P, P, P, P, P, c_int64, c_int32, c_float, P, P, P, P, c_int64, P, P,
                           c_size_t, P],
    "tsdfs_field_create": [P, P, P, P],
    "tsdfs_field_destroy": [P],
    "sdf_mlp_fwd_ws_bytes": [P, P],
    "sdf_mlp_fwd": [P, P, P, P, P, c_int64, P, c_int32, P, P, P, P, c_size_t, P],
    "composite": [P, c_int64, P, P, P, P, P, P, c_float, P, P, P, P, P, P],
    "composite_bwd": [P, c_int64, P, P, P, P, P, P, c_float, P, P, P, P, P, P, P, P],
    "rgb_loss": [P, P, c_int64, P, P, P],
    "sdf_mlp_bwd_ws_bytes": [P, c_int64, P],
    "sdf_mlp_bwd": [P, P, P, P, P, c_int64, P, c_int64, c_float, P, P, P, c_int32, P, P, P, P,
                    c_size_t, P],
}
_RESTYPE = {"tsdfs_last_error": ctypes.c_char_p}

_lib = None


def lib_path():
    return _build.LIB


def load():
    """Load the HIP library (build it first only if it does not exist)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        for name, args in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = _RESTYPE.get(name, ctypes.c_int)
        _lib = L
    return _lib


def check(rc):
    if rc != TSDFS_OK:
        msg = load().tsdfs_last_error()
        raise TsdfsError(rc, msg.decode() if msg else "")
    return rc
