"""ctypes declarations of the C-ABI in include/nnvisr.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
import re

from ctypes import POINTER, c_char_p, c_float, c_int32, c_int64, c_size_t, c_uint32, c_uint64, c_void_p

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libnnvisr.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "nnvisr.h")

NV_OK, NV_E_INVALID, NV_E_UNSUPPORTED, NV_E_NOMEM, NV_E_DEVICE, NV_E_BUSY = range(6)
NV_FP32, NV_FP16, NV_BF16, NV_FP8_E4M3 = range(4)
NV_FLAG_INTERP, NV_FLAG_EXTRA, NV_FLAG_DOUBLE = 1, 2, 4
NV_FLAG_HEAD_FP32 = 8
NV_FLAG_FP8_FUSION = 16
NV_STATIC_SCRATCH_BYTES = 64 << 20
NV_MATRIX_BT709, NV_MATRIX_BT601, NV_MATRIX_BT2020 = 0, 1, 2
NV_RANGE_LIMITED, NV_RANGE_FULL = 0, 1
NV_SITING_LEFT, NV_SITING_CENTER = 0, 1
MATRIX_CODES = {709: NV_MATRIX_BT709, 601: NV_MATRIX_BT601, 2020: NV_MATRIX_BT2020}
STATUS_NAMES = {0: "NV_OK", 1: "NV_E_INVALID", 2: "NV_E_UNSUPPORTED", 3: "NV_E_NOMEM",
                4: "NV_E_DEVICE", 5: "NV_E_BUSY"}


class NvFormat(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("bits", c_int32), ("chroma", c_int32),
                ("matrix", c_int32), ("range", c_int32), ("chroma_loc", c_int32)]


class NvPlanes(ctypes.Structure):
    _fields_ = [("data", c_void_p * 3), ("pitch_bytes", c_int64 * 3)]


class NvNetConfig(ctypes.Structure):
    _fields_ = [("channels", c_int32), ("res_blocks", c_int32), ("offset_groups", c_int32),
                ("scale", c_int32), ("align", c_int32), ("flags", c_uint32), ("precision", c_int32),
                ("matrix", c_int32), ("range", c_int32), ("scale_v", c_int32), ("levels", c_int32)]


class NvSceneParams(ctypes.Structure):
    _fields_ = [("mad_thresh_8bit", c_int32), ("hist_frac_num", c_int32),
                ("hist_frac_den", c_int32), ("enable", c_int32)]


class NvBatchReq(ctypes.Structure):
    _fields_ = [("stream", c_void_p), ("n_frames", c_int32), ("frames", POINTER(NvPlanes)),
                ("external_cut", POINTER(c_int32)), ("out", POINTER(NvPlanes)),
                ("n_out", POINTER(c_int32)), ("end_of_clip", c_int32)]


PF = POINTER(c_float)
_SIGS = {
    "nv_context_create": (c_int32, [c_int32, POINTER(NvNetConfig), PF, c_size_t, POINTER(c_void_p)]),
    "nv_context_destroy": (c_int32, [c_void_p]),
    "nv_last_error": (c_char_p, []),
    "nv_weight_count": (c_size_t, [POINTER(NvNetConfig)]),
    "nv_unpack": (c_int32, [POINTER(NvFormat), POINTER(NvPlanes), c_void_p, c_int32, c_int32, c_void_p]),
    "nv_pack": (c_int32, [POINTER(NvFormat), c_void_p, c_int32, c_int32, POINTER(NvPlanes), c_void_p]),
    "nv_scene_metric": (c_int32, [POINTER(NvFormat), POINTER(NvPlanes), POINTER(NvPlanes), c_void_p,
                                  POINTER(NvSceneParams), c_int32, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p]),
    "nv_feature_elem_bytes": (c_int32, [c_void_p]),
    "nv_feature_bytes": (c_size_t, [c_void_p, c_int32, c_int32]),
    "nv_extract": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_void_p]),
    "nv_fuse": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                          c_void_p, c_uint32, POINTER(c_void_p), c_void_p, c_void_p, c_void_p]),
    "nv_enhance_group": (c_int32, [c_void_p, POINTER(NvFormat), POINTER(NvPlanes), POINTER(NvPlanes),
                                   c_void_p]),
    "nv_enhance_group_static": (c_int32, [c_void_p, POINTER(NvFormat), POINTER(NvPlanes), POINTER(NvPlanes),
                                          c_void_p]),
    "nv_clip_open": (c_int32, [c_void_p, POINTER(NvFormat), POINTER(NvSceneParams), c_int32, c_int32,
                               POINTER(c_void_p)]),
    "nv_clip_push": (c_int32, [c_void_p, POINTER(NvPlanes), c_int32, POINTER(NvPlanes), c_int32, POINTER(c_int32),
                               c_void_p]),
    "nv_clip_end": (c_int32, [c_void_p, POINTER(NvPlanes), c_int32, POINTER(c_int32), c_void_p]),
    "nv_clip_trace": (c_int32, [c_void_p, POINTER(c_int32), c_int32, POINTER(c_int32)]),
    "nv_clip_close": (c_int32, [c_void_p]),
    "nv_stream_open": (c_int32, [c_void_p, POINTER(NvFormat), POINTER(NvSceneParams), POINTER(c_void_p)]),
    "nv_stream_push": (c_int32, [c_void_p, POINTER(NvPlanes), c_int32, POINTER(NvPlanes),
                                 POINTER(c_int32), c_void_p]),
    "nv_stream_end": (c_int32, [c_void_p, POINTER(NvPlanes), POINTER(c_int32), c_void_p]),
    "nv_stream_close": (c_int32, [c_void_p]),
    "nv_stream_cuts": (c_int32, [c_void_p, POINTER(c_uint32), c_int32, c_void_p]),
    "nv_stream_footprint": (c_int32, [c_void_p, POINTER(NvFormat), POINTER(c_size_t)]),
    "nv_stream_reset": (c_int32, [c_void_p]),
    "nv_profile_enable": (c_int32, [c_void_p, c_int32]),
    "nv_profile_read": (c_int32, [c_void_p, POINTER(c_int64), POINTER(ctypes.c_double)]),
    "nv_profile_kind_name": (c_char_p, [c_int32]),
    "nv_enhance_batch": (c_int32, [c_void_p, POINTER(NvBatchReq), c_int32, c_void_p]),
    "nv_batch_graph": (c_int32, [c_void_p, c_int32]),
    "nv_batch_footprint": (c_int32, [c_void_p, POINTER(c_size_t)]),
    "nv_batch_bytes_per_px": (c_int32, [c_void_p, POINTER(c_size_t), POINTER(c_size_t)]),
    "nv_autotune": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, ctypes.c_char_p, c_size_t]),
    "nv_calibrate": (c_int32, [c_void_p, POINTER(NvFormat), POINTER(NvPlanes), c_int32, c_void_p]),
    "nv_fp8_scales": (c_int32, [c_void_p, PF, c_int32, c_int32, c_void_p]),
}
NV_K_COUNT = 13

_lib = None


def header_functions(path: str = HEADER):
    """Names of the functions include/nnvisr.h declares."""
    with open(path) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nv_[a-z0-9_]+)\s*\(", text)))


def load(path: str = LIB_PATH):
    """Load the library once.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2308_03121_amd.build")
    lib = ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class NvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int):
    if status != NV_OK:
        raise NvError(status, load().nv_last_error().decode(errors="replace"))
