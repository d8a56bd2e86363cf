"""ctypes declarations of the C ABI in include/conegauss.h (argument marshalling only).

The shared library is loaded from this package's directory; if it is missing the
import of the renderer raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libconegauss.so")

CG_OK = 0
STATUS_NAMES = {0: "CG_OK", -1: "CG_ERR_INVALID_ARG", -2: "CG_ERR_UNSUPPORTED", -3: "CG_ERR_OUT_OF_MEMORY",
                -4: "CG_ERR_HIP", -5: "CG_ERR_STATE", -6: "CG_ERR_TIMEOUT"}


class CgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class CgCamera(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("full_w", C.c_int32), ("full_h", C.c_int32),
        ("crop_x0", C.c_int32), ("crop_y0", C.c_int32), ("crop_w", C.c_int32), ("crop_h", C.c_int32),
        ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
        ("k", C.c_float * 4), ("R_c2w", C.c_float * 9), ("origin", C.c_float * 3),
        ("theta_max", C.c_float),
    ]


class CgGaussians(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("color_mode", C.c_int32),
        ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
        ("opacity_logits", C.c_void_p), ("color", C.c_void_p), ("rho2", C.c_void_p),
    ]


class CgOpts(C.Structure):
    _fields_ = [
        ("filter_mode", C.c_int32), ("use_floor", C.c_int32), ("composition", C.c_int32),
        ("alpha_min", C.c_float), ("alpha_max", C.c_float), ("T_min", C.c_float), ("t_near", C.c_float),
        ("bg", C.c_float * 3), ("footprint_scale", C.c_float), ("count_pairs", C.c_int32),
        ("order_mode", C.c_int32), ("backbone", C.c_int32),
    ]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class CgAllocator(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN)]


class CgStats(C.Structure):
    _fields_ = [("n_pairs", C.c_int64), ("n_tiles", C.c_int64), ("n_pixels", C.c_int64),
                ("n_gaussian_views", C.c_int64), ("sort_bits", C.c_int32), ("n_segments", C.c_int32),
                ("n_evaluated", C.c_int64), ("n_full", C.c_int64), ("n_contrib", C.c_int64),
                ("n_order_overflow", C.c_int64), ("max_tile_pairs", C.c_int64)]


# Every symbol the header declares, with its ctypes signature.
_vp = C.c_void_p
SIGNATURES = {
    "cg_version": (C.c_int, []),
    "cg_last_error": (C.c_char_p, []),
    "cg_default_opts": (None, [_vp]),
    "cg_render_forward": (C.c_int, [_vp, _vp, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cg_render_forward_noalloc": (C.c_int, [_vp, _vp, C.c_int32, _vp, _vp, _vp, _vp]),
    "cg_render_backward": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cg_fwd_state_release": (None, [_vp]),
    "cg_bwd_replay_mismatches": (C.c_int64, [_vp]),
    "cg_camera_unproject": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp]),
    "cg_bake_rho2": (C.c_int, [_vp, _vp, C.c_int32, C.c_float, _vp, _vp]),
    "cg_profile_num_stages": (C.c_int, []),
    "cg_profile_stage_name": (C.c_char_p, [C.c_int]),
    "cg_profile_enable": (None, [C.c_int]),
    "cg_profile_enable_stages": (None, [C.c_uint32]),
    "cg_set_tile_split": (None, [C.c_int64, C.c_int64, C.c_int64]),
    "cg_debug_set_scratch_guards": (None, [C.c_int32]),
    "cg_debug_guard_violations": (C.c_int64, []),
    "cg_profile_collect": (C.c_int, []),
    "cg_profile_read": (None, [_vp, _vp]),
    "cg_profile_valu_probe": (C.c_int, [C.c_int32, C.c_int32, _vp, _vp]),
    "cg_release_cached_memory": (C.c_int, []),
}

_LIB = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run python -m paper_2609_13397_amd.build_lib or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def check(status: int):
    if status != CG_OK:
        msg = lib().cg_last_error()
        raise CgError(status, msg.decode() if msg else "")


def byref(s) -> C.c_void_p:
    return C.cast(C.pointer(s), C.c_void_p)
