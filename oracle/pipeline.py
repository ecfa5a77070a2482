"""The frame-group enhancement path end to end in FP64 (test infrastructure only).

Per frame: unpack + pad, scene metric, extract.  Per group [a, b] (section 3.3
grouping with n = 1 and the Interpolation, Extra-frame and Double-frame flags
of section 3.1): fusion into HR frames at t = 0 and t = 1/2 (t = 1 too for a
lone group), crop to twice the input size, requantise to the input's format.
``colour`` (a dict of ``pixel`` keyword arguments: matrix, full, centre) is the
clip's colourspace, used by both pixel-format stages; None is the default reading.

The task (section 3.2, end-user usage; flags of section 3.1) is given by ``scale``
(rows, columns) and the flags: ``interp`` (Interpolation with Extra frame: groups
[a, b] as above) and ``double`` (Double frame: the group also emits frame a enhanced;
without it frame a passes through unchanged, which needs scale (1, 1)).  Without
``interp`` every frame is enhanced alone: one output per input frame.  ``levels`` is the
number of feature-pyramid levels (section 3.1: the extract stage's output; cascaded
alignment over them, see oracle.network); it needs ``interp``.
"""
from __future__ import annotations

import numpy as np

from . import network, pixel, scene


def weights_dict(blob, layout):
    """{name: (w OIHW float64, b float64)} from a flat float32 blob and its layout list."""
    out, off = {}, 0
    for name, cout, cin, _gain in layout:
        n = cout * cin * 9
        w = np.asarray(blob[off:off + n], dtype=np.float64).reshape(cout, cin, 3, 3)
        off += n
        b = np.asarray(blob[off:off + cout], dtype=np.float64)
        off += cout
        out[name] = (w, b)
    if off != len(blob):
        raise ValueError("blob size does not match the layout")
    return out


def frame_rgb(Y, U, V, bits, chroma, align=8, colour=None):
    return pixel.pad(pixel.unpack(Y, U, V, bits, chroma, **(colour or {})), align)


def _features(rgb, W, res_blocks, levels):
    f = network.extract(rgb, W, res_blocks)
    return f if levels == 1 else network.pyramid(f, W, levels)


def enhance_group(fa_planes, fb_planes, bits, chroma, W, res_blocks, groups,
                  times=(0.0, 0.5, 1.0), align=8, keep=False, colour=None, scale=(2, 2), levels=1):
    """One frame group.  fb_planes=None means the duplicated group [a, a].

    Returns {"codes": {t: (Y, Cb, Cr)}, "hr": {t: cropped float HR RGB}} plus the
    intermediates when keep=True.
    """
    h, w = fa_planes[0].shape
    rgb_a = frame_rgb(*fa_planes, bits, chroma, align, colour)
    fa = _features(rgb_a, W, res_blocks, levels)
    if fb_planes is None:
        rgb_b, fb = rgb_a, fa
    else:
        rgb_b = frame_rgb(*fb_planes, bits, chroma, align, colour)
        fb = _features(rgb_b, W, res_blocks, levels)
    res = network.fuse(rgb_a, rgb_b, fa, fb, W, groups, times=times, keep=keep, scale=scale)
    out = {"codes": {}, "hr": {}}
    for t in times:
        hr = res[t][:, :scale[0] * h, :scale[1] * w]
        out["hr"][t] = hr
        out["codes"][t] = pixel.pack(hr, bits, chroma, **(colour or {}))
    if keep:
        out.update(rgb_a=rgb_a, rgb_b=rgb_b, fa=fa, fb=fb, offsets=res["offsets"],
                   mask=res["mask"], fmid=res["fmid"], levels=res.get("levels"))
    return out


def enhance_clip(frames, bits, chroma, W, res_blocks, groups, params=scene.SceneParams(),
                 external=None, align=8, colour=None, scale=(2, 2), interp=True, double=True, levels=1):
    """A whole clip in stream order.  frames: list of (Y, U, V).

    Returns (cuts, outputs) where outputs is the list of emitted frames (2N with
    interp, N without), each {"group": (a, b), "t": t, "codes": (Y, Cb, Cr), "hr": float
    RGB or None for a frame passed through}.
    """
    cuts = scene.detect_cuts([f[0] for f in frames], bits, params, external)
    h, w = frames[0][0].shape
    sv, sh = scale
    pk = lambda x: pixel.pack(x, bits, chroma, **(colour or {}))   # noqa: E731
    rgb_cache, feat_cache = {}, {}

    if levels > 1 and not interp:
        raise ValueError("a feature pyramid needs an interpolating network")

    def feat(i):
        if i not in feat_cache:
            rgb_cache[i] = frame_rgb(*frames[i], bits, chroma, align, colour)
            feat_cache[i] = _features(rgb_cache[i], W, res_blocks, levels)
        return rgb_cache[i], feat_cache[i]

    outputs = []
    if not interp:
        for t in range(len(frames)):
            rgb, f = feat(t)
            hr = network.reconstruct(f, network.upsample_bilinear(rgb, sv, sh), W, scale)[:, :sv * h, :sh * w]
            outputs.append({"group": (t, t), "t": 0.0, "hr": hr, "codes": pk(hr)})
            for old in [k for k in feat_cache if k < t]:
                del feat_cache[old], rgb_cache[old]
        return cuts, outputs
    if not double and scale != (1, 1):
        raise ValueError("input frames pass through only at scale (1, 1)")
    for a, b in scene.groups_n1(cuts):
        rgb_a, fa = feat(a)
        rgb_b, fb = feat(b)
        res = network.fuse(rgb_a, rgb_b, fa, fb, W, groups, times=(0.0, 0.5), scale=scale)
        for t in (0.0, 0.5):
            if t == 0.0 and not double:
                outputs.append({"group": (a, b), "t": t, "hr": None, "codes": tuple(np.asarray(p) for p in frames[a])})
                continue
            hr = res[t][:, :sv * h, :sh * w]
            outputs.append({"group": (a, b), "t": t, "hr": hr, "codes": pk(hr)})
        for old in [k for k in feat_cache if k < a]:
            del feat_cache[old], rgb_cache[old]
    return cuts, outputs


def psnr_float(ref: np.ndarray, test: np.ndarray) -> float:
    """PSNR of clamped RGB, peak 1.0."""
    d = np.clip(np.asarray(ref, np.float64), 0, 1) - np.clip(np.asarray(test, np.float64), 0, 1)
    mse = float(np.mean(d * d))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


def psnr_codes(ref_planes, test_planes, bits: int) -> float:
    """PSNR over the pooled Y, Cb, Cr samples, peak 2^bits - 1."""
    se, n = 0.0, 0
    for r, t in zip(ref_planes, test_planes):
        d = np.asarray(r, np.float64) - np.asarray(t, np.float64)
        se += float(np.sum(d * d))
        n += d.size
    if se == 0:
        return float("inf")
    peak = float((1 << bits) - 1)
    return 10.0 * np.log10(peak * peak / (se / n))
