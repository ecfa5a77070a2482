"""Thin Python layer over the C-ABI: torch tensors provide device memory and the HIP
stream, the library does every step of the path.  No computation happens here."""
from __future__ import annotations

import ctypes
from ctypes import byref, c_int32, c_size_t, c_uint32, c_void_p

import numpy as np
import torch

from . import _abi
from ._abi import NvFormat, NvNetConfig, NvPlanes, NvSceneParams, check

PRECISIONS = {"fp32": _abi.NV_FP32, "fp16": _abi.NV_FP16, "bf16": _abi.NV_BF16,
              "fp8": _abi.NV_FP8_E4M3}


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t: torch.Tensor | None):
    return None if t is None else c_void_p(t.data_ptr())


def fmt_struct(width: int, height: int, bits: int, chroma: int, matrix: int = 709, full: bool = False,
               centre: bool = False) -> NvFormat:
    """Frame format; matrix 709 / 601 / 2020, full range, centre chroma siting (4:2:0)."""
    return NvFormat(width, height, bits, chroma, _abi.MATRIX_CODES[matrix],
                    _abi.NV_RANGE_FULL if full else _abi.NV_RANGE_LIMITED,
                    _abi.NV_SITING_CENTER if centre else _abi.NV_SITING_LEFT)


def chroma_shape(width, height, chroma):
    return (height // 2, width // 2) if chroma == 420 else (height, width)


def planes_struct(Y: torch.Tensor, U: torch.Tensor, V: torch.Tensor) -> NvPlanes:
    p = NvPlanes()
    for i, t in enumerate((Y, U, V)):
        if t.dim() != 2 or t.stride(1) != 1:
            raise ValueError("planes must be 2-D with unit column stride")
        p.data[i] = t.data_ptr()
        p.pitch_bytes[i] = t.stride(0) * t.element_size()
    return p


def alloc_frame(width, height, bits, chroma, device="cuda"):
    dt = torch.uint8 if bits == 8 else torch.int16
    hc, wc = chroma_shape(width, height, chroma)
    return (torch.empty((height, width), dtype=dt, device=device),
            torch.empty((hc, wc), dtype=dt, device=device),
            torch.empty((hc, wc), dtype=dt, device=device))


def to_device_frame(Y: np.ndarray, U: np.ndarray, V: np.ndarray, device="cuda"):
    """numpy uint8/uint16 planes -> device tensors (uint16 travels as int16 bits)."""
    def conv(a):
        a = np.ascontiguousarray(a)
        if a.dtype == np.uint16:
            a = a.view(np.int16)
        return torch.from_numpy(a).to(device)
    return conv(Y), conv(U), conv(V)


def frame_to_numpy(planes, bits):
    out = []
    for t in planes:
        a = t.cpu().numpy()
        if bits == 10:
            a = a.view(np.uint16)
        out.append(a)
    return tuple(out)


def scene_params(mad=24, num=1, den=4, enable=True) -> NvSceneParams:
    return NvSceneParams(mad, num, den, 1 if enable else 0)


def unpack(fmt: NvFormat, planes, hp: int, wp: int, stream=None) -> torch.Tensor:
    lib = _abi.load()
    rgb = torch.empty((3, hp, wp), dtype=torch.float32, device=planes[0].device)
    p = planes_struct(*planes)
    check(lib.nv_unpack(byref(fmt), byref(p), _ptr(rgb), hp, wp, c_void_p(_stream(stream))))
    return rgb


def pack(fmt: NvFormat, rgb: torch.Tensor, out=None, stream=None):
    lib = _abi.load()
    if rgb.dtype != torch.float32 or not rgb.is_contiguous() or rgb.dim() != 3:
        raise ValueError("rgb must be a contiguous float32 [3, H, W] tensor")
    if out is None:
        out = alloc_frame(fmt.width, fmt.height, fmt.bits, fmt.chroma, rgb.device)
    p = planes_struct(*out)
    check(lib.nv_pack(byref(fmt), _ptr(rgb), rgb.shape[1], rgb.shape[2], byref(p),
                      c_void_p(_stream(stream))))
    return out


def scene_metric(fmt: NvFormat, prev, cur, hist_prev: torch.Tensor | None, params=None,
                 external_cut: int = -1, stream=None):
    """Returns device tensors (sad u64 as int64[1], hist int32[64], hd int32[1], cut int32[1])."""
    lib = _abi.load()
    dev = cur[0].device
    sad = torch.zeros(1, dtype=torch.int64, device=dev)
    hist = torch.zeros(64, dtype=torch.int32, device=dev)
    hd = torch.zeros(1, dtype=torch.int32, device=dev)
    cut = torch.zeros(1, dtype=torch.int32, device=dev)
    pc = planes_struct(*cur)
    pp = planes_struct(*prev) if prev is not None else None
    check(lib.nv_scene_metric(byref(fmt), byref(pp) if pp is not None else None, byref(pc),
                              _ptr(hist_prev), byref(params) if params is not None else None,
                              external_cut, _ptr(sad), _ptr(hist), _ptr(hd), _ptr(cut),
                              c_void_p(_stream(stream))))
    return sad, hist, hd, cut


class Context:
    """A network context: repacked weights and workspace on one device."""

    def __init__(self, channels: int, res_blocks: int, offset_groups: int, weights: np.ndarray,
                 precision: str = "fp32", device: int = 0, head_fp32: bool = False,
                 fp8_fusion: bool = False, matrix: int = 709, full: bool = False, scale: int = 2,
                 scale_v: int = 0, interp: bool = True, double: bool = True, levels: int = 1):
        lib = _abi.load()
        # the task: scale factors (columns, rows; 0 = the same) and the network flags (Double
        # frame is a flag of interpolating networks only; a per-frame network has none)
        flags = 0
        if interp:
            flags = _abi.NV_FLAG_INTERP | _abi.NV_FLAG_EXTRA | (_abi.NV_FLAG_DOUBLE if double else 0)
        if head_fp32:
            flags |= _abi.NV_FLAG_HEAD_FP32
        if fp8_fusion:
            flags |= _abi.NV_FLAG_FP8_FUSION
        self.fp8_fusion = fp8_fusion
        # matrix / full: the colourspace the weights were trained for
        self.cfg = NvNetConfig(channels, res_blocks, offset_groups, scale, 8, flags, PRECISIONS[precision],
                               _abi.MATRIX_CODES[matrix], _abi.NV_RANGE_FULL if full else _abi.NV_RANGE_LIMITED,
                               scale_v, levels)
        self.levels = levels
        self.scale_h, self.scale_v = scale, scale_v or scale
        self.interp, self.double = interp, interp and double
        self.colourspace = (matrix, bool(full))
        w = np.ascontiguousarray(weights, dtype=np.float32)
        self._h = c_void_p()
        check(lib.nv_context_create(device, byref(self.cfg),
                                    w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w.size,
                                    byref(self._h)))
        self.channels = channels
        self.offset_groups = offset_groups
        self.device = torch.device("cuda", device)
        self.precision = precision
        self.res_blocks = res_blocks
        self.feat_dtype = {4: torch.float32, 2: torch.bfloat16 if precision == "bf16" else torch.float16}[
            lib.nv_feature_elem_bytes(self._h)]
        self.ldo = 16 * ((27 * offset_groups + 15) // 16)

    @staticmethod
    def weight_count(channels, res_blocks, offset_groups) -> int:
        cfg = NvNetConfig(channels, res_blocks, offset_groups, 2, 8, 7, 0, 0, 0)
        return int(_abi.load().nv_weight_count(byref(cfg)))

    def close(self):
        if self._h:
            _abi.load().nv_context_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def extract(self, rgb: torch.Tensor, stream=None) -> torch.Tensor:
        """Level 1 of the frame's features, [hp][wp][C]; with a pyramid the tensor's storage
        holds every level (see pyramid_levels)."""
        _c, hp, wp = rgb.shape
        lib = _abi.load()
        n = int(lib.nv_feature_bytes(self._h, hp, wp)) // lib.nv_feature_elem_bytes(self._h)
        store = torch.empty(n, dtype=self.feat_dtype, device=rgb.device)
        check(lib.nv_extract(self._h, _ptr(rgb), hp, wp, _ptr(store), c_void_p(_stream(stream))))
        return store[:hp * wp * self.channels].view(hp, wp, self.channels)

    def pyramid_levels(self, feat: torch.Tensor) -> list:
        """Views [level 1, level 2, ...] of the features extract() returned (NHWC each)."""
        hp, wp, C = feat.shape
        store = feat.untyped_storage()
        flat = torch.empty(0, dtype=feat.dtype, device=feat.device).set_(store, feat.storage_offset(),
                                                                        (store.nbytes() // feat.element_size(),))
        out, off = [], 0
        for lv in range(1, self.levels + 1):
            h, w = hp >> (lv - 1), wp >> (lv - 1)
            out.append(flat[off:off + h * w * C].view(h, w, C))
            off += h * w * C
        return out

    def fuse(self, rgb_a, rgb_b, feat_a, feat_b, out_mask=7, sel: torch.Tensor | None = None,
             want_offsets=False, want_fmid=False, stream=None):
        _c, hp, wp = rgb_a.shape
        dev = rgb_a.device
        hr = [torch.empty((3, 2 * hp, 2 * wp), dtype=torch.float32, device=dev)
              if out_mask & (1 << t) else None for t in range(3)]
        arr = (c_void_p * 3)(*[t.data_ptr() if t is not None else None for t in hr])
        offs = torch.empty((hp, wp, self.ldo), dtype=torch.float32, device=dev) if want_offsets else None
        fmid = torch.empty((hp, wp, self.channels), dtype=self.feat_dtype, device=dev) if want_fmid else None
        check(_abi.load().nv_fuse(self._h, _ptr(rgb_a), _ptr(rgb_b), _ptr(feat_a), _ptr(feat_b), hp, wp,
                                  _ptr(sel), out_mask, arr, _ptr(offs), _ptr(fmid),
                                  c_void_p(_stream(stream))))
        return hr, offs, fmid

    def enhance_group(self, fmt: NvFormat, frame_a, frame_b, outs=None, stream=None):
        """Two device frames in, three output frames (t = 0, 1/2, 1) at twice the size."""
        if outs is None:
            outs = [alloc_frame(self.scale_h * fmt.width, self.scale_v * fmt.height, fmt.bits, fmt.chroma,
                                frame_a[0].device)
                    for _ in range(3)]
        pin = (NvPlanes * 2)(planes_struct(*frame_a), planes_struct(*frame_b))
        pout = (NvPlanes * 3)(*[planes_struct(*o) for o in outs])
        check(_abi.load().nv_enhance_group(self._h, byref(fmt), pin, pout, c_void_p(_stream(stream))))
        return outs

    def enhance_group_static(self, fmt: NvFormat, frame_a, frame_b, outs=None, stream=None):
        """enhance_group through the allocation-free entry point (nv_enhance_group_static):
        the library's temporaries live in its static per-device scratch."""
        if outs is None:
            outs = [alloc_frame(self.scale_h * fmt.width, self.scale_v * fmt.height, fmt.bits, fmt.chroma,
                                frame_a[0].device)
                    for _ in range(3)]
        pin = (NvPlanes * 2)(planes_struct(*frame_a), planes_struct(*frame_b))
        pout = (NvPlanes * 3)(*[planes_struct(*o) for o in outs])
        check(_abi.load().nv_enhance_group_static(self._h, byref(fmt), pin, pout, c_void_p(_stream(stream))))
        return outs

    def stream_footprint(self, fmt: NvFormat) -> int:
        n = c_size_t()
        check(_abi.load().nv_stream_footprint(self._h, byref(fmt), byref(n)))
        return int(n.value)

    def open_stream(self, fmt: NvFormat, params: NvSceneParams | None = None) -> "Stream":
        return Stream(self, fmt, params)

    def enhance_batch(self, requests, stream=None):
        """requests: list of (Stream, [device frames], external cuts or None, end_of_clip).
        Returns, per request, the list of output frames written (emission order)."""
        lib = _abi.load()
        n = len(requests)
        reqs = (_abi.NvBatchReq * max(n, 1))()
        keep, outs_all = [], []
        for i, (st, frames, ext, end) in enumerate(requests):
            k = len(frames)
            n_emit = k - (1 if st.n_pushed == 0 else 0) + (1 if end else 0)
            outs = [alloc_frame(2 * st.fmt.width, 2 * st.fmt.height, st.fmt.bits, st.fmt.chroma, self.device)
                    for _ in range(2 * n_emit)]
            fr = (NvPlanes * k)(*[planes_struct(*f) for f in frames])
            op = (NvPlanes * max(1, len(outs)))(*[planes_struct(*o) for o in outs])
            ec = (c_int32 * k)(*ext) if ext is not None else None
            cnt = c_int32()
            keep += [fr, op, ec, cnt]
            reqs[i].stream = st._h
            reqs[i].n_frames = k
            reqs[i].frames = ctypes.cast(fr, ctypes.POINTER(NvPlanes))
            reqs[i].external_cut = ctypes.cast(ec, ctypes.POINTER(c_int32)) if ec is not None else None
            reqs[i].out = ctypes.cast(op, ctypes.POINTER(NvPlanes))
            reqs[i].n_out = ctypes.pointer(cnt)
            reqs[i].end_of_clip = 1 if end else 0
            outs_all.append((outs, cnt))
        check(lib.nv_enhance_batch(self._h, reqs, n, c_void_p(_stream(stream))))
        for i, (st, frames, _e, _end) in enumerate(requests):
            st.n_pushed += len(frames)
        return [outs[:cnt.value] for outs, cnt in outs_all]

    def batch_graph(self, on: bool):
        check(_abi.load().nv_batch_graph(self._h, 1 if on else 0))

    def batch_bytes_per_px(self) -> tuple:
        """(bytes per group, bytes per frame) per padded LR pixel of the batch pools."""
        g, f = c_size_t(), c_size_t()
        check(_abi.load().nv_batch_bytes_per_px(self._h, byref(g), byref(f)))
        return int(g.value), int(f.value)

    def batch_footprint(self) -> int:
        n = c_size_t()
        check(_abi.load().nv_batch_footprint(self._h, byref(n)))
        return int(n.value)

    def autotune(self, hp: int, wp: int, stream=None) -> str:
        buf = ctypes.create_string_buffer(1024)
        check(_abi.load().nv_autotune(self._h, hp, wp, c_void_p(_stream(stream)), buf, 1024))
        return buf.value.decode()

    def calibrate(self, fmt: NvFormat, frames, stream=None):
        """FP8 contexts: set the static activation scales from consecutive groups of
        the given device frames."""
        arr = (NvPlanes * len(frames))(*[planes_struct(*f) for f in frames])
        check(_abi.load().nv_calibrate(self._h, byref(fmt), arr, len(frames), c_void_p(_stream(stream))))

    def fp8_scales(self, amax=None, stream=None) -> np.ndarray:
        """FP8 contexts: read the per-layer input maxima, or set them when amax is given."""
        n = 2 * self.res_blocks + (2 if self.fp8_fusion else 0)
        buf = (ctypes.c_float * n)(*(amax if amax is not None else [0.0] * n))
        check(_abi.load().nv_fp8_scales(self._h, buf, n, 0 if amax is None else 1, c_void_p(_stream(stream))))
        return np.array(buf[:], dtype=np.float32)

    def profile(self, on: bool):
        check(_abi.load().nv_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> dict:
        """{kind name: (launches, total device ms)} since profiling was enabled."""
        lib = _abi.load()
        n = _abi.NV_K_COUNT
        launches = (ctypes.c_int64 * n)()
        ms = (ctypes.c_double * n)()
        check(lib.nv_profile_read(self._h, launches, ms))
        return {lib.nv_profile_kind_name(k).decode(): (int(launches[k]), float(ms[k])) for k in range(n)}


class Stream:
    """Clip-level streaming: push frames, get two output frames per group."""

    def __init__(self, ctx: Context, fmt: NvFormat, params: NvSceneParams | None = None):
        self.ctx = ctx
        self.fmt = fmt
        self._h = c_void_p()
        check(_abi.load().nv_stream_open(ctx._h, byref(fmt), byref(params) if params is not None else None,
                                         byref(self._h)))
        self.n_pushed = 0

    def _outs(self, outs):
        if outs is None:
            outs = [alloc_frame(self.ctx.scale_h * self.fmt.width, self.ctx.scale_v * self.fmt.height, self.fmt.bits,
                                self.fmt.chroma, self.ctx.device) for _ in range(2)]
        return outs, (NvPlanes * 2)(*[planes_struct(*o) for o in outs])

    def push(self, frame, external_cut: int = -1, outs=None, stream=None):
        outs, pout = self._outs(outs)
        n = c_int32()
        check(_abi.load().nv_stream_push(self._h, byref(planes_struct(*frame)), external_cut, pout,
                                         byref(n), c_void_p(_stream(stream))))
        self.n_pushed += 1
        return outs[:n.value]

    def end(self, outs=None, stream=None):
        outs, pout = self._outs(outs)
        n = c_int32()
        check(_abi.load().nv_stream_end(self._h, pout, byref(n), c_void_p(_stream(stream))))
        return outs[:n.value]

    def reset(self):
        check(_abi.load().nv_stream_reset(self._h))
        self.n_pushed = 0

    def cuts(self, stream=None):
        n = self.n_pushed
        buf = (c_uint32 * max(n, 1))()
        check(_abi.load().nv_stream_cuts(self._h, buf, n, c_void_p(_stream(stream))))
        return [int(buf[i]) for i in range(n)]

    def close(self):
        if self._h:
            _abi.load().nv_stream_close(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Clip:
    """A clip grouped for a network consuming n frames per run, in batches of b groups over
    the Fig. 1 frame store (nv_clip_*).  push() returns the output frames emitted by it."""

    def __init__(self, ctx: Context, fmt: NvFormat, n: int, b: int, params: NvSceneParams | None = None):
        self.ctx, self.fmt, self.n, self.b = ctx, fmt, n, b
        self._h = c_void_p()
        check(_abi.load().nv_clip_open(ctx._h, byref(fmt), byref(params) if params is not None else None, n, b,
                                       byref(self._h)))

    def _room(self):
        cap = 2 * self.n * self.b
        outs = [alloc_frame(2 * self.fmt.width, 2 * self.fmt.height, self.fmt.bits, self.fmt.chroma,
                            self.ctx.device) for _ in range(cap)]
        return outs, (NvPlanes * cap)(*[planes_struct(*o) for o in outs]), cap

    def push(self, frame, external_cut: int = -1, stream=None):
        outs, pout, cap = self._room()
        n = c_int32()
        check(_abi.load().nv_clip_push(self._h, byref(planes_struct(*frame)), external_cut, pout, cap, byref(n),
                                       c_void_p(_stream(stream))))
        return outs[:n.value]

    def end(self, stream=None):
        outs, pout, cap = self._room()
        n = c_int32()
        check(_abi.load().nv_clip_end(self._h, pout, cap, byref(n), c_void_p(_stream(stream))))
        return outs[:n.value]

    def trace(self):
        """[(kind, [group inputs], [frame at each store position])] per batch run so far."""
        lib = _abi.load()
        ln = c_int32()
        check(lib.nv_clip_trace(self._h, None, 0, byref(ln)))
        buf = (c_int32 * max(ln.value, 1))()
        check(lib.nv_clip_trace(self._h, buf, ln.value, byref(ln)))
        vals, out, i, P = list(buf)[:ln.value], [], 0, self.n * self.b + self.b
        while i < len(vals):
            kind, g = vals[i], vals[i + 1]
            i += 2
            groups = [vals[i + j * (self.n + 1):i + (j + 1) * (self.n + 1)] for j in range(g)]
            i += g * (self.n + 1)
            out.append((kind, groups, vals[i:i + P]))
            i += P
        return out

    def close(self):
        if self._h:
            _abi.load().nv_clip_close(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
