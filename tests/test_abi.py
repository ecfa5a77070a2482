"""Host-only checks of the C-ABI library: it loads, exports every declared symbol, and
rejects invalid arguments before touching the device."""
import ctypes
import os

import numpy as np
import pytest

import paper_2308_03121_amd as pkg
from paper_2308_03121_amd import _abi


@pytest.fixture(scope="module")
def lib():
    return _abi.load()


def test_library_exports_every_header_function(lib):
    names = pkg.header_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    assert set(_abi._SIGS) == set(pkg.header_functions())


def test_weight_count_matches_generator(lib):
    import synth
    for cfg in (synth.NET_C1, synth.NET_C2, synth.NET_C4):
        c = _abi.NvNetConfig(cfg.channels, cfg.res_blocks, cfg.offset_groups, 2, 8, 7, 0)
        assert lib.nv_weight_count(ctypes.byref(c)) == synth.gen_weights(cfg).size
    assert lib.nv_weight_count(None) == 0


def _fmt(w=64, h=64, bits=8, chroma=420):
    return _abi.NvFormat(w, h, bits, chroma)


def _planes(ptr=0x1000, pitches=(64, 32, 32)):
    p = _abi.NvPlanes()
    for i in range(3):
        p.data[i] = ptr
        p.pitch_bytes[i] = pitches[i]
    return p


@pytest.mark.parametrize("fmt,planes,why", [
    (_fmt(bits=9), _planes(), "bits"),
    (_fmt(chroma=422), _planes(), "chroma"),
    (_fmt(w=63), _planes(), "even"),
    (_fmt(w=0), _planes(), "size"),
    (_fmt(), _planes(pitches=(63, 32, 32)), "pitch"),
    (_fmt(), _planes(ptr=0), "NULL"),
    (_fmt(bits=10), _planes(ptr=0x1001, pitches=(128, 64, 64)), "aligned"),
])
def test_unpack_rejects_bad_arguments(lib, fmt, planes, why):
    st = lib.nv_unpack(ctypes.byref(fmt), ctypes.byref(planes), ctypes.c_void_p(0x2000), 64, 64, None)
    assert st == _abi.NV_E_INVALID
    assert why.lower() in lib.nv_last_error().decode().lower()


def test_unpack_rejects_small_padding(lib):
    st = lib.nv_unpack(ctypes.byref(_fmt()), ctypes.byref(_planes()), ctypes.c_void_p(0x2000), 56, 64, None)
    assert st == _abi.NV_E_INVALID


def test_scene_rejects_external_flag(lib):
    z = ctypes.c_void_p(0x3000)
    st = lib.nv_scene_metric(ctypes.byref(_fmt()), None, ctypes.byref(_planes()), None, None, 2,
                             z, z, z, z, None)
    assert st == _abi.NV_E_INVALID


def test_context_rejects_bad_config(lib):
    h = ctypes.c_void_p()
    w = np.zeros(10, np.float32)
    wp = w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    for cfg, code in [((48, 2, 8, 2, 8, 7, 0), _abi.NV_E_INVALID),
                      ((96, 2, 8, 2, 8, 7, 0), _abi.NV_E_UNSUPPORTED),
                      ((64, 2, 7, 2, 8, 7, 0), _abi.NV_E_INVALID),
                      ((64, 2, 1, 2, 8, 7, 0), _abi.NV_E_INVALID),
                      ((64, 2, 8, 3, 8, 7, 0), _abi.NV_E_UNSUPPORTED),
                      ((64, 2, 8, 2, 8, 1, 0), _abi.NV_E_UNSUPPORTED),
                      ((64, 2, 8, 2, 8, 7, 9), _abi.NV_E_INVALID),
                      ((32, 2, 8, 2, 8, 7, 3), _abi.NV_E_UNSUPPORTED),    # FP8 needs C = 64
                      ((64, 2, 8, 2, 8, 7 | 16, 1), _abi.NV_E_INVALID),   # FP8 fusion without FP8
                      ((64, 2, 8, 2, 8, 7 | 32, 3), _abi.NV_E_UNSUPPORTED)]:
        c = _abi.NvNetConfig(*cfg)
        assert lib.nv_context_create(0, ctypes.byref(c), wp, 10, ctypes.byref(h)) == code, cfg
        assert not h.value
    c = _abi.NvNetConfig(32, 2, 8, 2, 8, 7, 0)
    assert lib.nv_context_create(0, ctypes.byref(c), wp, 10, ctypes.byref(h)) == _abi.NV_E_INVALID
    assert "needs" in lib.nv_last_error().decode()


def test_fp8_entry_points_reject_null(lib):
    f = ctypes.c_float()
    assert lib.nv_calibrate(None, None, None, 2, None) == _abi.NV_E_INVALID
    assert lib.nv_fp8_scales(None, ctypes.byref(f), 1, 0, None) == _abi.NV_E_INVALID


def test_null_handles_are_rejected(lib):
    n = ctypes.c_int32()
    assert lib.nv_stream_push(None, None, -1, None, ctypes.byref(n), None) == _abi.NV_E_INVALID
    assert lib.nv_extract(None, None, 8, 8, None, None) == _abi.NV_E_INVALID
    assert lib.nv_context_destroy(None) == _abi.NV_OK
    assert lib.nv_stream_close(None) == _abi.NV_OK


def test_missing_library_fails_loudly(tmp_path):
    saved = _abi._lib
    try:
        _abi._lib = None
        with pytest.raises(RuntimeError, match="missing"):
            _abi.load(str(tmp_path / "nope.so"))
    finally:
        _abi._lib = saved
