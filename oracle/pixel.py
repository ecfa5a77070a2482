"""Pixel-format stages in FP64 (test infrastructure only, see ``oracle/__init__``).

The paper lets a network take or produce RGB or Y'CbCr 4:2:0 and requires
colourspace awareness (section 3.1, "Network Integration", the paragraphs on
pixel formats and colourspace).  It fixes no matrix, range, siting or filter;
this module takes ITU-R BT.709 limited range with non-linear R'G'B', left
(MPEG-2 type 0) chroma siting, bilinear chroma upsampling, a [1,2,1]x[1,1]
chroma downsampling filter, replicate edges, alignment padding by edge
replication and round-half-up requantisation.
"""
from __future__ import annotations

import numpy as np

# ITU-R BT.709 luma coefficients; the derived ones are computed, not rounded constants.
KR = 0.2126
KB = 0.0722
KG = 1.0 - KR - KB


def code_scale(bits: int) -> float:
    return float(1 << (bits - 8))


def decode(plane: np.ndarray, bits: int) -> np.ndarray:
    """Code value = stored sample with the unused container bits masked off."""
    return (plane.astype(np.int64) & ((1 << bits) - 1)).astype(np.float64)


def upsample_chroma_420(c: np.ndarray) -> np.ndarray:
    """Left-sited 4:2:0 -> 4:4:4 bilinear upsampling with replicated edges.

    Chroma sample (i, j) sits at luma column 2j and halfway between luma rows
    2i and 2i+1.  Hence luma row 2i takes 3/4 c_i + 1/4 c_{i-1}, row 2i+1
    takes 3/4 c_i + 1/4 c_{i+1}; luma column 2j takes c_j and column 2j+1
    the mean of c_j and c_{j+1}.
    """
    c = np.asarray(c, dtype=np.float64)
    hc, wc = c.shape
    above = np.concatenate([c[:1], c[:-1]], axis=0)
    below = np.concatenate([c[1:], c[-1:]], axis=0)
    v = np.empty((2 * hc, wc))
    v[0::2] = 0.75 * c + 0.25 * above
    v[1::2] = 0.75 * c + 0.25 * below
    right = np.concatenate([v[:, 1:], v[:, -1:]], axis=1)
    out = np.empty((2 * hc, 2 * wc))
    out[:, 0::2] = v
    out[:, 1::2] = 0.5 * (v + right)
    return out


def ycbcr_to_rgb(y: np.ndarray, cb: np.ndarray, cr: np.ndarray, bits: int) -> np.ndarray:
    """Limited-range BT.709 codes (4:4:4) -> non-linear R'G'B' in nominal [0, 1], unclamped."""
    s = code_scale(bits)
    yn = (y - 16.0 * s) / (219.0 * s)
    cbn = (cb - 128.0 * s) / (224.0 * s)
    crn = (cr - 128.0 * s) / (224.0 * s)
    r = yn + 2.0 * (1.0 - KR) * crn
    b = yn + 2.0 * (1.0 - KB) * cbn
    g = (yn - KR * r - KB * b) / KG
    return np.stack([r, g, b])


def unpack(Y: np.ndarray, U: np.ndarray, V: np.ndarray, bits: int, chroma: int) -> np.ndarray:
    """Stored planes -> planar RGB (3, H, W) float64."""
    y = decode(Y, bits)
    cb = decode(U, bits)
    cr = decode(V, bits)
    if chroma == 420:
        cb = upsample_chroma_420(cb)
        cr = upsample_chroma_420(cr)
    elif chroma != 444:
        raise ValueError("chroma must be 420 or 444")
    return ycbcr_to_rgb(y, cb, cr, bits)


def padded_size(h: int, w: int, align: int = 8):
    return (-(-h // align)) * align, (-(-w // align)) * align


def pad(rgb: np.ndarray, align: int = 8) -> np.ndarray:
    """Replicate the last row / column so both sizes become multiples of ``align``."""
    _c, h, w = rgb.shape
    hp, wp = padded_size(h, w, align)
    return np.pad(rgb, ((0, 0), (0, hp - h), (0, wp - w)), mode="edge")


def rgb_to_ycbcr_float(rgb: np.ndarray):
    """R'G'B' -> (Y', Cb', Cr') in nominal units, after clamping R'G'B' to [0, 1]."""
    r, g, b = np.clip(np.asarray(rgb, dtype=np.float64), 0.0, 1.0)
    yn = KR * r + KG * g + KB * b
    cbn = (b - yn) / (2.0 * (1.0 - KB))
    crn = (r - yn) / (2.0 * (1.0 - KR))
    return yn, cbn, crn


def downsample_chroma_420(c: np.ndarray) -> np.ndarray:
    """4:4:4 -> left-sited 4:2:0: weights (1/4, 1/2, 1/4) over columns 2j-1..2j+1,
    times 1/2 over rows 2i and 2i+1, replicating edge samples."""
    c = np.asarray(c, dtype=np.float64)
    h, w = c.shape
    left = np.concatenate([c[:, :1], c[:, :-1]], axis=1)
    right = np.concatenate([c[:, 1:], c[:, -1:]], axis=1)
    horiz = 0.25 * left + 0.5 * c + 0.25 * right
    horiz = horiz[:, 0::2]
    return 0.5 * (horiz[0::2] + horiz[1::2])


def quantise(v: np.ndarray, bits: int):
    """code = clamp(floor(v + 1/2), 0, 2^bits - 1)."""
    return np.clip(np.floor(v + 0.5), 0, (1 << bits) - 1)


def pack_values(rgb: np.ndarray, bits: int, chroma: int):
    """Pre-rounding code-space values (luma, Cb, Cr) of the requantisation."""
    s = code_scale(bits)
    yn, cbn, crn = rgb_to_ycbcr_float(rgb)
    if chroma == 420:
        cbn = downsample_chroma_420(cbn)
        crn = downsample_chroma_420(crn)
    elif chroma != 444:
        raise ValueError("chroma must be 420 or 444")
    return (219.0 * yn + 16.0) * s, (224.0 * cbn + 128.0) * s, (224.0 * crn + 128.0) * s


def pack(rgb: np.ndarray, bits: int, chroma: int):
    """Planar RGB (3, H, W) -> integer code planes (Y, Cb, Cr) in the stored dtype."""
    dt = np.uint8 if bits == 8 else np.uint16
    return tuple(quantise(v, bits).astype(dt) for v in pack_values(rgb, bits, chroma))
