"""ctypes binding of liboctgs.so (the C ABI in include/octgs.h).

Argument marshalling only: every step of the render path runs in the HIP
library.  PyTorch provides device memory and the current stream.  Importing
this module does not touch the GPU; `lib()` raises if the library is not
built.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboctgs.so")

OCTGS_OK, OCTGS_EINVAL, OCTGS_ENOSPC, OCTGS_EHIP, OCTGS_EUNSUPPORTED = 0, -1, -2, -3, -4
OCTGS_FP32, OCTGS_BF16 = 0, 1
OCTGS_RASTER_STAGES = 5
OCTGS_RASTER_BWD_STAGES = 2
OCTGS_SELECT_NOALLOC_MAX_ANCHORS = 1 << 23
OCTGS_RASTER_TRAIN = 1
OCTGS_RASTER_TILE_ORDER = 2
OCTGS_STATUS_PAIR_OVERFLOW, OCTGS_STATUS_SYNC_ERROR, OCTGS_STATUS_TRUNCATED = 1, 2, 4
RASTER_STAGE_NAMES = ("project", "depth_sort", "emit", "tile_sort", "composite")

_p = ctypes.c_void_p
_f = ctypes.c_float
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


class Camera(ctypes.Structure):
    _fields_ = [("R", _f * 9), ("C", _f * 3), ("fx", _f), ("fy", _f), ("cx", _f), ("cy", _f),
                ("width", _i32), ("height", _i32), ("z_near", _f), ("lod_scale2", _f),
                ("lod_blend", _i32)]


class Anchors(ctypes.Structure):
    _fields_ = [("n", _i64), ("k", _i32), ("feat_dim", _i32), ("n_levels", _i32),
                ("d_max", _f), ("pos", _p), ("level", _p), ("lod_bias", _p), ("feat", _p),
                ("feat_bf16", _p), ("offsets", _p), ("offset_scale", _p), ("base_scale", _p),
                ("thr2", _p), ("bound_r", _p)]


class Mlp(ctypes.Structure):
    _fields_ = [("width", _i32), ("w1", _p * 3), ("b1", _p * 3), ("w2", _p * 3), ("b2", _p * 3)]


class Gaussians(ctypes.Structure):
    _fields_ = [("capacity", _i64), ("data", _p), ("count", _p), ("status", _p)]


class RasterParams(ctypes.Structure):
    _fields_ = [("alpha_max", _f), ("alpha_min", _f), ("t_min", _f), ("dilation", _f),
                ("jac_clamp", _f), ("bg", _f * 3), ("flags", ctypes.c_uint32)]


class AnchorGrads(ctypes.Structure):
    _fields_ = [("pos", _p), ("feat", _p), ("offsets", _p), ("offset_scale", _p),
                ("base_scale", _p)]


class MlpGrads(ctypes.Structure):
    _fields_ = [("w1", _p * 3), ("b1", _p * 3), ("w2", _p * 3), ("b2", _p * 3)]


class SkipNet(ctypes.Structure):
    _fields_ = [("w1", _p), ("b1", _p), ("w2", _p), ("b2", _p), ("w3", _p), ("b3", _p)]


class Explicit(ctypes.Structure):
    _fields_ = [("sh_degree", _i32), ("mean", _p), ("log_scale", _p), ("rot", _p),
                ("opacity", _p), ("sh", _p), ("sh_bf16", _p)]


class ExplicitGrads(ctypes.Structure):
    _fields_ = [("mean", _p), ("log_scale", _p), ("rot", _p), ("opacity", _p), ("sh", _p)]


class DensifyStats(ctypes.Structure):
    _fields_ = [("grad_sum", _p), ("grad_count", _p), ("opacity_sum", _p), ("view_count", _p)]


class DensifyParams(ctypes.Structure):
    _fields_ = [("tau_g", _f), ("beta", _f), ("epsilon", _f), ("tau_opacity", _f), ("tau_v", _f),
                ("n_views", _i32)]


class RasterStats(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_uint32), ("n_visible", ctypes.c_uint32),
                ("n_pairs", ctypes.c_uint32), ("pair_overflow", ctypes.c_uint32),
                ("sync_error", ctypes.c_uint32), ("n_candidates", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 10)]


# (name, restype, argtypes); kept in the order of include/octgs.h
SIGNATURES = [
    ("octgs_prepare_anchors", _i32, [ctypes.POINTER(Anchors), _p, _p, _p, _p]),
    ("octgs_select_workspace_bytes", ctypes.c_size_t, [_i64]),
    ("octgs_select_lod", _i32, [ctypes.POINTER(Anchors), ctypes.POINTER(Camera),
                                ctypes.POINTER(RasterParams), _p, _p, _p, ctypes.c_size_t, _p]),
    ("octgs_select_lod_noalloc", _i32, [ctypes.POINTER(Anchors), ctypes.POINTER(Camera),
                                        ctypes.POINTER(RasterParams), _p, _p, _p]),
    ("octgs_decode_workspace_bytes", ctypes.c_size_t, [_i32]),
    ("octgs_decode", _i32, [ctypes.POINTER(Anchors), ctypes.POINTER(Mlp), ctypes.POINTER(Camera),
                            _p, _p, _i32, ctypes.POINTER(Gaussians), _p, ctypes.c_size_t, _p]),
    ("octgs_raster_workspace_bytes", ctypes.c_size_t, [_i64, _i64, _i32, _i32]),
    ("octgs_rasterize_fwd", _i32, [ctypes.POINTER(Gaussians), ctypes.POINTER(Camera),
                                   ctypes.POINTER(RasterParams), _i64, _p, _p, _p, _p, _p,
                                   ctypes.c_size_t, _p, _p]),
    ("octgs_rasterize_bwd", _i32, [ctypes.POINTER(Gaussians), ctypes.POINTER(Camera),
                                   ctypes.POINTER(RasterParams), _i64, _p, _p, _p, _p, _p,
                                   ctypes.c_size_t, _p, _p]),
    ("octgs_decode_bwd_workspace_bytes", ctypes.c_size_t, [_i64, _i32, _i32]),
    ("octgs_decode_bwd", _i32, [ctypes.POINTER(Anchors), ctypes.POINTER(Mlp),
                                ctypes.POINTER(Camera), _p, _p, _p, _i64,
                                ctypes.POINTER(AnchorGrads), ctypes.POINTER(MlpGrads), _p,
                                ctypes.c_size_t, _p]),
    ("octgs_decode_bwd_rows", _i32, [ctypes.POINTER(Anchors), ctypes.POINTER(Mlp),
                                     ctypes.POINTER(Camera), _p, _p, _p, _i64, _p,
                                     ctypes.c_size_t, _p]),
    ("octgs_decode_bwd_apply", _i32, [ctypes.POINTER(Anchors), ctypes.POINTER(Mlp), _p, _p, _i64,
                                      ctypes.POINTER(AnchorGrads), ctypes.POINTER(MlpGrads), _p,
                                      ctypes.c_size_t, _p]),
    ("octgs_l1_loss_grad", _i32, [_p, _p, _i64, _f, _p, _p, _p]),
    ("octgs_photometric_workspace_bytes", ctypes.c_size_t, [_i64, _i32, _i32]),
    ("octgs_photometric_loss_grad", _i32, [_p, _p, _i64, _i32, _i32, _f, _f, _p, _p, _p,
                                           ctypes.c_size_t, _p]),
    ("octgs_volume_loss_grad", _i32, [ctypes.POINTER(Gaussians), _f, _p, _p, _p]),
    ("octgs_adam_step", _i32, [_p, _p, _p, _p, _i64, _f, _f, _f, _f, _i32, _p]),
    ("octgs_adam_step_many", _i32, [_i32, _p, _p, _p, _p, _p, _f, _f, _f, _f, _i32, _p]),
    ("octgs_anchor_weights", _i32, [_p, _p, _i32, _i64, _p, _p]),
    ("octgs_skip_features", _i32, [ctypes.POINTER(Anchors), ctypes.POINTER(Camera), _p, _p, _i64,
                                   _p, _p]),
    ("octgs_skip_predict_workspace_bytes", ctypes.c_size_t, [_i64]),
    ("octgs_skip_predict", _i32, [ctypes.POINTER(Anchors), ctypes.POINTER(Camera),
                                  ctypes.POINTER(SkipNet), _f, _p, _p, _i64, _p, _p, _p, _p,
                                  ctypes.c_size_t, _p]),
    ("octgs_skip_train_workspace_bytes", ctypes.c_size_t, [_i32]),
    ("octgs_skip_train_grad", _i32, [ctypes.POINTER(SkipNet), _p, _p, _p, _i32, ctypes.c_uint64,
                                     _f, ctypes.POINTER(SkipNet), _p, _p, ctypes.c_size_t, _p]),
    ("octgs_prepare_explicit", _i32, [ctypes.POINTER(Anchors), ctypes.POINTER(Explicit), _p, _p,
                                      _p, _p]),
    ("octgs_decode_explicit", _i32, [ctypes.POINTER(Anchors), ctypes.POINTER(Explicit),
                                     ctypes.POINTER(Camera), _p, _p, _i32,
                                     ctypes.POINTER(Gaussians), _p]),
    ("octgs_decode_explicit_bwd", _i32, [ctypes.POINTER(Anchors), ctypes.POINTER(Explicit),
                                         ctypes.POINTER(Camera), _p, _p, _p, _i64,
                                         ctypes.POINTER(ExplicitGrads), _p]),
    ("octgs_densify_accumulate", _i32, [ctypes.POINTER(Gaussians), ctypes.POINTER(Camera), _i64,
                                        _p, ctypes.c_size_t, _p, _p, _i32,
                                        ctypes.POINTER(DensifyStats), _p]),
    ("octgs_densify_decide", _i32, [ctypes.POINTER(Anchors), ctypes.POINTER(DensifyStats),
                                    ctypes.POINTER(DensifyParams), _p, _p, _p, _p, _p]),
    ("octgs_raster_views", _i32, [_p, _i64, _i64, _i32, _i32, ctypes.POINTER(_p),
                                  ctypes.POINTER(_p), ctypes.POINTER(_p), ctypes.POINTER(_p)]),
    ("octgs_strerror", ctypes.c_char_p, [_i32]),
    ("octgs_version", _i32, []),
]

_lib = None


class OctgsError(RuntimeError):
    pass


def lib():
    """Load liboctgs.so; raises (never falls back) if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OctgsError(f"{LIB_PATH} is not built; run paper_2403_17898_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int, what: str):
    if status != OCTGS_OK:
        msg = lib().octgs_strerror(status).decode()
        raise OctgsError(f"{what} failed: {msg} ({status})")
