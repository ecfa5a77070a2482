"""Pixel-format stages in FP64 (test infrastructure only, see ``oracle/__init__``).

The paper lets a network take or produce RGB or Y'CbCr 4:2:0 and requires
colourspace awareness: the same code values mean different colours under different
colourspaces, and a network is trained per colourspace (section 3.1, "Network
Integration", the paragraphs on pixel formats and colourspace).  It fixes no matrix,
range, siting or filter.  The default reading is ITU-R BT.709 limited range with
non-linear R'G'B', left (MPEG-2 type 0) chroma siting, bilinear chroma upsampling, a
[1,2,1]x[1,1] chroma downsampling filter, replicate edges, alignment padding by edge
replication and round-half-up requantisation.  The variants are the BT.601 and BT.2020
(non-constant luminance) matrices, full range (ITU-T H.273 with the full-range flag:
Y = (2^b - 1) Y', C = (2^b - 1) C' + 2^(b-1)) and centre chroma siting (MPEG-1 / JPEG
type 1: a 4:2:0 chroma sample at the centre of its 2x2 luma block, bilinear
upsampling in both directions and a 2x2 box for downsampling).

Every function takes the colourspace as keyword arguments: ``matrix`` (601, 709,
2020), ``full`` (False: limited range) and, for 4:2:0, ``centre`` (False: left siting).
"""
from __future__ import annotations

import numpy as np

# Luma coefficients (Kr, Kb) of ITU-R BT.601, BT.709 and BT.2020 (non-constant
# luminance); Kg = 1 - Kr - Kb and every derived coefficient are computed, not rounded
# constants.
MATRICES = {601: (0.299, 0.114), 709: (0.2126, 0.0722), 2020: (0.2627, 0.0593)}
KR, KB = MATRICES[709]
KG = 1.0 - KR - KB


def coefficients(matrix: int = 709):
    """(Kr, Kg, Kb) of a matrix."""
    kr, kb = MATRICES[matrix]
    return kr, 1.0 - kr - kb, kb


def code_range(bits: int, full: bool = False):
    """(luma scale, luma offset, chroma scale, chroma offset) of the code values:
    Y = scale * Y' + offset with Y' in [0, 1], C = scale * C' + offset with C' in [-1/2, 1/2]."""
    if full:
        m = float((1 << bits) - 1)
        return m, 0.0, m, float(1 << (bits - 1))
    s = code_scale(bits)
    return 219.0 * s, 16.0 * s, 224.0 * s, 128.0 * s


def code_scale(bits: int) -> float:
    return float(1 << (bits - 8))


def decode(plane: np.ndarray, bits: int) -> np.ndarray:
    """Code value = stored sample with the unused container bits masked off."""
    return (plane.astype(np.int64) & ((1 << bits) - 1)).astype(np.float64)


def upsample_chroma_420(c: np.ndarray, centre: bool = False) -> np.ndarray:
    """4:2:0 -> 4:4:4 bilinear upsampling with replicated edges.

    Chroma sample (i, j) sits halfway between luma rows 2i and 2i+1, so luma row 2i
    takes 3/4 c_i + 1/4 c_{i-1} and row 2i+1 takes 3/4 c_i + 1/4 c_{i+1}.  Left siting:
    the sample sits at luma column 2j, so column 2j takes c_j and column 2j+1 the mean
    of c_j and c_{j+1}.  Centre siting: it sits halfway between columns 2j and 2j+1,
    so columns are weighted like rows (3/4 c_j + 1/4 c_{j-1}, 3/4 c_j + 1/4 c_{j+1}).
    """
    c = np.asarray(c, dtype=np.float64)
    hc, wc = c.shape
    above = np.concatenate([c[:1], c[:-1]], axis=0)
    below = np.concatenate([c[1:], c[-1:]], axis=0)
    v = np.empty((2 * hc, wc))
    v[0::2] = 0.75 * c + 0.25 * above
    v[1::2] = 0.75 * c + 0.25 * below
    left = np.concatenate([v[:, :1], v[:, :-1]], axis=1)
    right = np.concatenate([v[:, 1:], v[:, -1:]], axis=1)
    out = np.empty((2 * hc, 2 * wc))
    if centre:
        out[:, 0::2] = 0.75 * v + 0.25 * left
        out[:, 1::2] = 0.75 * v + 0.25 * right
    else:
        out[:, 0::2] = v
        out[:, 1::2] = 0.5 * (v + right)
    return out


def ycbcr_to_rgb(y: np.ndarray, cb: np.ndarray, cr: np.ndarray, bits: int, matrix: int = 709,
                 full: bool = False) -> np.ndarray:
    """Y'CbCr codes (4:4:4) -> non-linear R'G'B' in nominal [0, 1], unclamped: the codes
    are normalised by the range, then the matrix's luma and colour-difference
    definitions (Y' = Kr R + Kg G + Kb B, Cb' = (B - Y') / (2 (1 - Kb)),
    Cr' = (R - Y') / (2 (1 - Kr))) are solved for R, B, then G."""
    kr, kg, kb = coefficients(matrix)
    ys, yo, cs, co = code_range(bits, full)
    yn = (y - yo) / ys
    cbn = (cb - co) / cs
    crn = (cr - co) / cs
    r = yn + 2.0 * (1.0 - kr) * crn
    b = yn + 2.0 * (1.0 - kb) * cbn
    g = (yn - kr * r - kb * b) / kg
    return np.stack([r, g, b])


def unpack(Y: np.ndarray, U: np.ndarray, V: np.ndarray, bits: int, chroma: int, matrix: int = 709,
           full: bool = False, centre: bool = False) -> np.ndarray:
    """Stored planes -> planar RGB (3, H, W) float64."""
    y = decode(Y, bits)
    cb = decode(U, bits)
    cr = decode(V, bits)
    if chroma == 420:
        cb = upsample_chroma_420(cb, centre)
        cr = upsample_chroma_420(cr, centre)
    elif chroma != 444:
        raise ValueError("chroma must be 420 or 444")
    return ycbcr_to_rgb(y, cb, cr, bits, matrix, full)


def padded_size(h: int, w: int, align: int = 8):
    return (-(-h // align)) * align, (-(-w // align)) * align


def pad(rgb: np.ndarray, align: int = 8) -> np.ndarray:
    """Replicate the last row / column so both sizes become multiples of ``align``."""
    _c, h, w = rgb.shape
    hp, wp = padded_size(h, w, align)
    return np.pad(rgb, ((0, 0), (0, hp - h), (0, wp - w)), mode="edge")


def rgb_to_ycbcr_float(rgb: np.ndarray, matrix: int = 709):
    """R'G'B' -> (Y', Cb', Cr') in nominal units, after clamping R'G'B' to [0, 1]."""
    kr, kg, kb = coefficients(matrix)
    r, g, b = np.clip(np.asarray(rgb, dtype=np.float64), 0.0, 1.0)
    yn = kr * r + kg * g + kb * b
    cbn = (b - yn) / (2.0 * (1.0 - kb))
    crn = (r - yn) / (2.0 * (1.0 - kr))
    return yn, cbn, crn


def downsample_chroma_420(c: np.ndarray, centre: bool = False) -> np.ndarray:
    """4:4:4 -> 4:2:0, replicating edge samples.  Left siting: weights (1/4, 1/2, 1/4)
    over columns 2j-1..2j+1, times 1/2 over rows 2i and 2i+1.  Centre siting: the mean
    of the 2x2 luma block (columns 2j, 2j+1 times rows 2i, 2i+1)."""
    c = np.asarray(c, dtype=np.float64)
    if centre:
        return 0.25 * (c[0::2, 0::2] + c[0::2, 1::2] + c[1::2, 0::2] + c[1::2, 1::2])
    h, w = c.shape
    left = np.concatenate([c[:, :1], c[:, :-1]], axis=1)
    right = np.concatenate([c[:, 1:], c[:, -1:]], axis=1)
    horiz = 0.25 * left + 0.5 * c + 0.25 * right
    horiz = horiz[:, 0::2]
    return 0.5 * (horiz[0::2] + horiz[1::2])


def quantise(v: np.ndarray, bits: int):
    """code = clamp(floor(v + 1/2), 0, 2^bits - 1)."""
    return np.clip(np.floor(v + 0.5), 0, (1 << bits) - 1)


def pack_values(rgb: np.ndarray, bits: int, chroma: int, matrix: int = 709, full: bool = False,
                centre: bool = False):
    """Pre-rounding code-space values (luma, Cb, Cr) of the requantisation."""
    ys, yo, cs, co = code_range(bits, full)
    yn, cbn, crn = rgb_to_ycbcr_float(rgb, matrix)
    if chroma == 420:
        cbn = downsample_chroma_420(cbn, centre)
        crn = downsample_chroma_420(crn, centre)
    elif chroma != 444:
        raise ValueError("chroma must be 420 or 444")
    return ys * yn + yo, cs * cbn + co, cs * crn + co


def pack(rgb: np.ndarray, bits: int, chroma: int, matrix: int = 709, full: bool = False,
         centre: bool = False):
    """Planar RGB (3, H, W) -> integer code planes (Y, Cb, Cr) in the stored dtype."""
    dt = np.uint8 if bits == 8 else np.uint16
    return tuple(quantise(v, bits).astype(dt) for v in pack_values(rgb, bits, chroma, matrix, full, centre))
