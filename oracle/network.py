"""The generic frame-group enhancement network in FP64 (test infrastructure only).

The paper accepts any network that splits into an extract stage, run once per
frame and producing a feature pyramid (one level here), and a fusion stage that
mixes the features of a frame group into output frames (section 3.1, "Network
Integration").  It singles out modulated deformable convolution (DCNv2) with
torchvision's offset/mask conventions as the operator it had to supply itself
(same section, the DCN paragraph).  This module fixes one seeded instance:

  extract : x = LReLU(conv(rgb; 3->C));  R times  x = x + conv(LReLU(conv(x)))
  offsets : o = LReLU(conv(cat(Fa, Fb); 2C->C));  raw = conv(o; C->27G)
            offsets = raw[:18G] (per group g, tap k: dy at 2(9g+k), dx at 2(9g+k)+1)
            mask    = sigmoid(raw[18G:])  (per group g, tap k at 9g+k)
  align   : Fmid = LReLU(DCN(cat(Fa, Fb), offsets, mask; 2C->C))   (aligned once, as in YOGO)
  output t: U = LReLU(pixel_shuffle_(sv,sh)(conv(G_t; C->sv sh C))),  HR_t = conv(U; C->3) + base_t
            G_0 = Fa, G_1/2 = Fmid, G_1 = Fb;  base_0 = up(rgb_a), base_1 = up(rgb_b),
            base_1/2 = (base_0 + base_1) / 2, up = bilinear x sv rows, x sh columns

With a feature pyramid of L levels (the extract stage's output as section 3.1 defines
it; L = 1 is the network above), level 1 is the trunk's output and each further level
halves both dimensions:

  pyramid : F^1 = extract(rgb);  F^l = LReLU(conv(avgpool2(F^(l-1)); C->C))  for l = 2..L
  cascade : from l = L down to 1, with the level's own offset head and DCN weights,
            offsets^l = head offsets^l + 2 up2(offsets^(l+1))   (coarse motion in fine pixels)
            mask^l    = the head's mask^l
            A^l       = LReLU(DCN(cat(Fa^l, Fb^l), offsets^l, mask^l)) + up2(A^(l+1))
            Fmid = A^1
  (the terms with l + 1 are absent at l = L; up2 is the x2 bilinear resize below)

The scale (sv, sh) is the task's (section 3.2, end-user usage): (2, 2) space-time
super-resolution, (1, 1) denoising or interpolation at the input size, (2, 1)
deinterlacing (rows doubled).  A factor of 1 leaves that axis alone.

All convs are 3x3, stride 1, zero padding 1, with bias; LReLU slope 0.1.
Arrays are channel-first (C, H, W), float64.
"""
from __future__ import annotations

import numpy as np

SLOPE = 0.1


def lrelu(x: np.ndarray) -> np.ndarray:
    return np.where(x >= 0.0, x, SLOPE * x)


def sigmoid(x: np.ndarray) -> np.ndarray:
    return 1.0 / (1.0 + np.exp(-x))


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """out[o, y, x] = b[o] + sum_{c, ky, kx} w[o, c, ky, kx] * xz[c, y + ky - 1, x + kx - 1],
    xz = x extended by zeros.  Written as a sum over the nine taps of a channel
    contraction (one matrix product per tap)."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    cin, h, wd = x.shape
    cout = w.shape[0]
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    out = np.repeat(np.asarray(b, dtype=np.float64)[:, None], h * wd, axis=1)
    for ky in range(3):
        for kx in range(3):
            tap = np.ascontiguousarray(xp[:, ky:ky + h, kx:kx + wd]).reshape(cin, h * wd)
            out += w[:, :, ky, kx] @ tap
    return out.reshape(cout, h, wd)


def pixel_shuffle(x: np.ndarray, r: int = 2, rw: int | None = None) -> np.ndarray:
    """out[c, r*h + i, rw*w + j] = in[r*rw*c + rw*i + j, h, w] (rows by r, columns by rw,
    rw = r unless given)."""
    rw = r if rw is None else rw
    cr, h, w = x.shape
    c = cr // (r * rw)
    return x.reshape(c, r, rw, h, w).transpose(0, 3, 1, 4, 2).reshape(c, h * r, w * rw)


def bilinear_zero(x: np.ndarray, py: np.ndarray, px: np.ndarray) -> np.ndarray:
    """Bilinear sample of every channel of x (C, H, W) at real positions (py, px),
    with x taken as zero outside the map: sum over the four integer neighbours n of
    (1 - |py - y_n|)(1 - |px - x_n|) x(y_n, x_n)."""
    _c, h, w = x.shape
    y0 = np.floor(py)
    x0 = np.floor(px)
    ly = py - y0
    lx = px - x0
    out = np.zeros((x.shape[0],) + py.shape)
    for dy in (0, 1):
        wy = ly if dy else 1.0 - ly
        yy = y0.astype(np.int64) + dy
        for dx in (0, 1):
            wx = lx if dx else 1.0 - lx
            xx = x0.astype(np.int64) + dx
            inside = (yy >= 0) & (yy < h) & (xx >= 0) & (xx < w)
            vals = x[:, np.clip(yy, 0, h - 1), np.clip(xx, 0, w - 1)]
            out += vals * (wy * wx * inside)
    return out


def deform_conv3x3(x, offsets, mask, w, b, groups: int) -> np.ndarray:
    """Modulated deformable 3x3 conv (DCNv2), stride 1, padding 1.

    out[o, p] = b[o] + sum_{c, k} w[o, c, k] * m_{g(c),k}(p) * xt_c(p + p_k + d_{g(c),k}(p))
    with g(c) = c // (Cin / groups), p_k = (ky - 1, kx - 1), k = 3 ky + kx, and xt the
    zero-extended bilinear interpolation of x.
    """
    x = np.asarray(x, dtype=np.float64)
    cin, h, wd = x.shape
    cg = cin // groups
    cout = w.shape[0]
    ys, xs = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(wd, dtype=np.float64),
                         indexing="ij")
    out = np.repeat(np.asarray(b, dtype=np.float64)[:, None], h * wd, axis=1)
    for g in range(groups):
        xg = x[g * cg:(g + 1) * cg]
        for ky in range(3):
            for kx in range(3):
                k = 3 * ky + kx
                dy = offsets[2 * (9 * g + k)]
                dx = offsets[2 * (9 * g + k) + 1]
                m = mask[9 * g + k]
                val = bilinear_zero(xg, ys + (ky - 1) + dy, xs + (kx - 1) + dx) * m
                out += np.asarray(w[:, g * cg:(g + 1) * cg, ky, kx], dtype=np.float64) \
                    @ val.reshape(cg, h * wd)
    return out.reshape(cout, h, wd)


def upsample_bilinear(x: np.ndarray, sv: int = 2, sh: int = 2) -> np.ndarray:
    """Bilinear resize by sv rows and sh columns (each 1 or 2): a factor of 1 keeps the
    axis, a factor of 2 is upsample2_bilinear's rule along it."""
    out = np.asarray(x, dtype=np.float64)
    if sv == 2:
        out = upsample2_bilinear(out, axes=(1,))
    if sh == 2:
        out = upsample2_bilinear(out, axes=(2,))
    return out


def upsample2_bilinear(x: np.ndarray, axes=(1, 2)) -> np.ndarray:
    """x2 bilinear resize with half-pixel centres and clamped edges: output row 2i
    takes 3/4 x_i + 1/4 x_{i-1}, row 2i+1 takes 3/4 x_i + 1/4 x_{i+1}; same for columns."""
    def along(a, axis):
        n = a.shape[axis]
        prev = np.take(a, np.clip(np.arange(n) - 1, 0, n - 1), axis=axis)
        nxt = np.take(a, np.clip(np.arange(n) + 1, 0, n - 1), axis=axis)
        even = 0.75 * a + 0.25 * prev
        odd = 0.75 * a + 0.25 * nxt
        out = np.stack([even, odd], axis=axis + 1)
        shp = list(a.shape)
        shp[axis] = 2 * n
        return out.reshape(shp)
    out = np.asarray(x, dtype=np.float64)
    for ax in axes:
        out = along(out, ax)
    return out


def avgpool2(x: np.ndarray) -> np.ndarray:
    """Mean of each 2x2 block: out[c, i, j] = (x[c, 2i, 2j] + x[c, 2i, 2j+1] + x[c, 2i+1, 2j]
    + x[c, 2i+1, 2j+1]) / 4 (even dimensions)."""
    x = np.asarray(x, dtype=np.float64)
    c, h, w = x.shape
    if h % 2 or w % 2:
        raise ValueError("avgpool2 needs even dimensions")
    return x.reshape(c, h // 2, 2, w // 2, 2).mean(axis=(2, 4))


def _wb(W, name):
    w, b = W[name]
    return np.asarray(w, dtype=np.float64), np.asarray(b, dtype=np.float64)


def extract(rgb: np.ndarray, W: dict, res_blocks: int) -> np.ndarray:
    x = lrelu(conv3x3(rgb, *_wb(W, "conv_in")))
    for r in range(res_blocks):
        t = lrelu(conv3x3(x, *_wb(W, f"block{r}.a")))
        x = x + conv3x3(t, *_wb(W, f"block{r}.b"))
    return x


def level_suffix(level: int) -> str:
    """Weight-name suffix of a pyramid level's fusion layers ("" for level 1)."""
    return "" if level == 1 else f".l{level}"


def pyramid(f1: np.ndarray, W: dict, levels: int) -> list:
    """[F^1, ..., F^L] from the trunk's output F^1."""
    out = [np.asarray(f1, dtype=np.float64)]
    for lv in range(2, levels + 1):
        out.append(lrelu(conv3x3(avgpool2(out[-1]), *_wb(W, f"down{lv}"))))
    return out


def offset_head(fa: np.ndarray, fb: np.ndarray, W: dict, groups: int, level: int = 1):
    sfx = level_suffix(level)
    o = lrelu(conv3x3(np.concatenate([fa, fb]), *_wb(W, "off1" + sfx)))
    raw = conv3x3(o, *_wb(W, "off2" + sfx))
    return raw[:18 * groups], sigmoid(raw[18 * groups:27 * groups])


def align(fa, fb, offsets, mask, W: dict, groups: int, level: int = 1) -> np.ndarray:
    return lrelu(deform_conv3x3(np.concatenate([fa, fb]), offsets, mask,
                                *_wb(W, "dcn" + level_suffix(level)), groups=groups))


def align_pyramid(pa: list, pb: list, W: dict, groups: int):
    """Cascaded alignment over two pyramids, coarsest level first.  Returns (Fmid, per-level
    list of (offsets, mask, A) from level 1 up)."""
    levels = len(pa)
    offs_c = feat_c = None
    per = []
    for lv in range(levels, 0, -1):
        offs, mask = offset_head(pa[lv - 1], pb[lv - 1], W, groups, lv)
        if offs_c is not None:
            offs = offs + 2.0 * upsample2_bilinear(offs_c)
        a = align(pa[lv - 1], pb[lv - 1], offs, mask, W, groups, lv)
        if feat_c is not None:
            a = a + upsample2_bilinear(feat_c)
        per.append((offs, mask, a))
        offs_c, feat_c = offs, a
    return feat_c, per[::-1]


def reconstruct(feat: np.ndarray, base: np.ndarray, W: dict, scale=(2, 2)) -> np.ndarray:
    u = lrelu(pixel_shuffle(conv3x3(feat, *_wb(W, "up")), scale[0], scale[1]))
    return conv3x3(u, *_wb(W, "hr")) + base


def fuse(rgb_a, rgb_b, fa, fb, W: dict, groups: int, times=(0.0, 0.5, 1.0), keep=False, scale=(2, 2)):
    """Fusion stage of one group [a, b]: output RGB for each requested time t.  fa / fb are
    the frames' features, or their pyramids (lists, level 1 first)."""
    res = {}
    base0 = upsample_bilinear(rgb_a, *scale)
    base1 = base0 if rgb_b is rgb_a else upsample_bilinear(rgb_b, *scale)
    if isinstance(fa, list):
        pa, pb = fa, fb
        fa, fb = pa[0], pb[0]
    else:
        pa = pb = None
    if 0.5 in times or keep:
        if pa is None:
            offs, mask = offset_head(fa, fb, W, groups)
            fmid = align(fa, fb, offs, mask, W, groups)
        else:
            fmid, per = align_pyramid(pa, pb, W, groups)
            offs, mask = per[0][0], per[0][1]
            if keep:
                res["levels"] = per
        if keep:
            res["offsets"], res["mask"], res["fmid"] = offs, mask, fmid
    for t in times:
        if t == 0.0:
            res[t] = reconstruct(fa, base0, W, scale)
        elif t == 1.0:
            res[t] = reconstruct(fb, base1, W, scale)
        elif t == 0.5:
            res[t] = reconstruct(fmid, 0.5 * (base0 + base1), W, scale)
        else:
            raise ValueError("times must be 0, 0.5 or 1")
    return res
