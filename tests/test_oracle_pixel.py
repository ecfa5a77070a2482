"""Pins of the oracle's pixel-format stages against published values and closed forms."""
import json
import os

import numpy as np
import pytest

from oracle import pixel

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _bars():
    with open(os.path.join(GOLD, "bt709_colour_bars.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("bits", [8, 10])
def test_colour_bars_encode(bits):
    bars = _bars()
    codes = bars[f"codes_{bits}bit"]
    for name, rgb in bars["rgb"].items():
        img = np.array(rgb, dtype=np.float64).reshape(3, 1, 1)
        y, cb, cr = pixel.pack(img, bits, 444)
        assert [int(y[0, 0]), int(cb[0, 0]), int(cr[0, 0])] == codes[name], name


@pytest.mark.parametrize("bits", [8, 10])
def test_colour_bars_decode(bits):
    bars = _bars()
    s = 1 << (bits - 8)
    for name, code in bars[f"codes_{bits}bit"].items():
        p = [np.full((1, 1), c, dtype=np.uint16) for c in code]
        rgb = pixel.unpack(*p, bits, 444)[:, 0, 0]
        # a code carries at most half a step of error in each of Y', Cb', Cr'
        tol = 0.5 / (219 * s) + 2 * 0.5 / (224 * s) + 1e-12
        assert np.allclose(rgb, bars["rgb"][name], atol=tol), (name, rgb)


def test_matrix_neutral_and_primaries():
    # neutral chroma gives R' = G' = B' = Y'; a pure Cr step moves R' and G' only
    y = np.array([[16.0 + 219 * 0.3]])
    rgb = pixel.ycbcr_to_rgb(y, np.array([[128.0]]), np.array([[128.0]]), 8)
    assert np.allclose(rgb.ravel(), 0.3, atol=1e-15)
    d = pixel.ycbcr_to_rgb(y, np.array([[128.0]]), np.array([[128.0 + 22.4]]), 8).ravel() - 0.3
    assert d[2] == pytest.approx(0.0, abs=1e-15)
    assert d[0] == pytest.approx(2 * (1 - 0.2126) * 0.1, rel=1e-12)
    # luma of the result is unchanged by a chroma step (definition of the matrix)
    r, g, b = d + 0.3
    assert 0.2126 * r + 0.7152 * g + 0.0722 * b == pytest.approx(0.3, abs=1e-15)


def _all_444_triples(bits, sample=None, seed=0):
    if sample is None:
        v = np.arange(1 << bits)
        yy, uu, vv = np.meshgrid(v, v, v, indexing="ij")
        return yy.ravel(), uu.ravel(), vv.ravel()
    rng = np.random.default_rng(seed)
    return tuple(rng.integers(0, 1 << bits, sample) for _ in range(3))


@pytest.mark.parametrize("bits,sample", [(8, None), (10, 2_000_000)])
def test_roundtrip_in_gamut_444(bits, sample):
    """decode -> encode is the identity for every code triple whose R'G'B' is in [0, 1]^3
    (exhaustive at 8 bits, 2e6 random triples at 10 bits)."""
    Y, U, V = _all_444_triples(bits, sample)
    checked = 0
    for lo in range(0, Y.size, 1 << 21):
        y, u, v = (a[lo:lo + (1 << 21)].reshape(1, -1) for a in (Y, U, V))
        rgb = pixel.unpack(y, u, v, bits, 444)
        ok = np.all((rgb >= 0) & (rgb <= 1), axis=0)[0]
        if not ok.any():
            continue
        y2, u2, v2 = pixel.pack(rgb[:, :, ok], bits, 444)
        assert np.array_equal(y2[0], y[0, ok]) and np.array_equal(u2[0], u[0, ok]) \
            and np.array_equal(v2[0], v[0, ok])
        checked += int(ok.sum())
    assert checked > (1 << (3 * bits)) // 8 if sample is None else checked > sample // 8


def test_chroma_upsample_constant_and_affine():
    c = np.full((5, 7), 77.0)
    assert np.array_equal(pixel.upsample_chroma_420(c), np.full((10, 14), 77.0))
    # left siting: chroma column j sits on luma column 2j, chroma row i at luma row 2i + 1/2
    i, j = np.meshgrid(np.arange(6.0), np.arange(8.0), indexing="ij")
    c = 100.0 + 3.0 * j + 5.0 * i
    up = pixel.upsample_chroma_420(c)
    Y, X = np.meshgrid(np.arange(12.0), np.arange(16.0), indexing="ij")
    expect = 100.0 + 3.0 * X / 2.0 + 5.0 * (Y - 0.5) / 2.0
    inner = (slice(1, -1), slice(0, -1))     # replicated edges differ from the ramp
    assert np.array_equal(up[inner], expect[inner])


def test_chroma_downsample_constant_and_affine():
    assert np.array_equal(pixel.downsample_chroma_420(np.full((6, 8), 3.0)), np.full((3, 4), 3.0))
    Y, X = np.meshgrid(np.arange(8.0), np.arange(12.0), indexing="ij")
    C = 0.01 * X - 0.02 * Y
    d = pixel.downsample_chroma_420(C)
    i, j = np.meshgrid(np.arange(4.0), np.arange(6.0), indexing="ij")
    expect = 0.01 * (2 * j) - 0.02 * (2 * i + 0.5)
    assert np.allclose(d[:, 1:], expect[:, 1:], atol=1e-15)


def test_420_roundtrip_constant_chroma():
    rng = np.random.default_rng(3)
    Y = rng.integers(60, 200, (8, 12)).astype(np.uint8)
    U = np.full((4, 6), 120, np.uint8)
    V = np.full((4, 6), 135, np.uint8)
    rgb = pixel.unpack(Y, U, V, 8, 420)
    assert rgb.min() >= 0 and rgb.max() <= 1
    y2, u2, v2 = pixel.pack(rgb, 8, 420)
    assert np.array_equal(y2, Y) and np.array_equal(u2, U) and np.array_equal(v2, V)


def test_420_roundtrip_affine_chroma_interior():
    i, j = np.meshgrid(np.arange(6), np.arange(8), indexing="ij")
    U = (120 + 2 * j + i).astype(np.uint8)
    V = (130 - j + 2 * i).astype(np.uint8)
    Y = np.full((12, 16), 120, np.uint8)
    rgb = pixel.unpack(Y, U, V, 8, 420)
    assert rgb.min() >= 0 and rgb.max() <= 1
    _y2, u2, v2 = pixel.pack(rgb, 8, 420)
    assert np.array_equal(u2[1:-1, 1:-1], U[1:-1, 1:-1])
    assert np.array_equal(v2[1:-1, 1:-1], V[1:-1, 1:-1])


def test_10bit_container_masking():
    rng = np.random.default_rng(5)
    Y = rng.integers(64, 940, (4, 6)).astype(np.uint16)
    U = rng.integers(64, 960, (2, 3)).astype(np.uint16)
    V = rng.integers(64, 960, (2, 3)).astype(np.uint16)
    junk = lambda a: a | (rng.integers(0, 64, a.shape).astype(np.uint16) << 10)
    a = pixel.unpack(Y, U, V, 10, 420)
    b = pixel.unpack(junk(Y), junk(U), junk(V), 10, 420)
    assert np.array_equal(a, b)


def test_quantise_round_half_up_and_clamp():
    v = np.array([-3.0, 0.49999, 0.5, 1.5, 2.5, 254.4, 254.5, 300.0])
    assert pixel.quantise(v, 8).tolist() == [0, 0, 1, 2, 3, 254, 255, 255]
    assert pixel.quantise(np.array([1022.5, 5000.0]), 10).tolist() == [1023, 1023]


def test_pack_clamps_rgb_first():
    img = np.array([1.7, -0.3, 0.5]).reshape(3, 1, 1)
    clamped = np.array([1.0, 0.0, 0.5]).reshape(3, 1, 1)
    assert all(np.array_equal(a, b) for a, b in zip(pixel.pack(img, 8, 444),
                                                     pixel.pack(clamped, 8, 444)))


def test_pad_replicate_and_identity():
    x = np.arange(3 * 5 * 6, dtype=np.float64).reshape(3, 5, 6)
    p = pixel.pad(x, 8)
    assert p.shape == (3, 8, 8)
    assert np.array_equal(p[:, :5, :6], x)
    assert np.array_equal(p[:, 5:, :6], np.repeat(x[:, 4:5, :], 3, axis=1))
    assert np.array_equal(p[:, :5, 6:], np.repeat(x[:, :, 5:6], 2, axis=2))
    assert pixel.padded_size(540, 960) == (544, 960)
    y = np.ones((3, 16, 24))
    assert pixel.pad(y).shape == y.shape



# ---- colourspace variants: other matrices, full range, centre siting ----

def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_bt601_colour_bars_encode():
    bars = _gold("bt601_colour_bars.json")
    for name, rgb in bars["rgb"].items():
        img = np.array(rgb, dtype=np.float64).reshape(3, 1, 1)
        y, cb, cr = pixel.pack(img, 8, 444, matrix=601)
        assert [int(y[0, 0]), int(cb[0, 0]), int(cr[0, 0])] == bars["codes_8bit"][name], name


def test_jfif_full_range_encode_and_decode():
    gold = _gold("jfif_full_range.json")
    for name, rgb8 in gold["rgb8"].items():
        img = np.array(rgb8, dtype=np.float64).reshape(3, 1, 1) / 255.0
        y, cb, cr = pixel.pack(img, 8, 444, matrix=601, full=True)
        code = gold["codes_8bit"][name]
        assert [int(y[0, 0]), int(cb[0, 0]), int(cr[0, 0])] == code, name
        # decoding the codes returns the colour within the code's half-step, except where
        # the encoder clamped a colour-difference value (red Cr, blue Cb at +1/2 -> 255.5)
        p = [np.full((1, 1), c, dtype=np.uint16) for c in code]
        back = pixel.unpack(*p, 8, 444, matrix=601, full=True)[:, 0, 0]
        if name not in ("red", "blue", "magenta"):
            assert np.allclose(back, img.ravel(), atol=3 * 0.5 / 255 + 1e-12), (name, back)


@pytest.mark.parametrize("matrix,coeffs", [(601, (0.299, 0.587, 0.114)), (709, (0.2126, 0.7152, 0.0722)),
                                           (2020, (0.2627, 0.6780, 0.0593))])
def test_matrix_luma_of_primaries(matrix, coeffs):
    """Y' of the R, G, B primaries are the standards' published luma weights (BT.601-7
    2.5, BT.709-6 3.2, BT.2020-2 Table 4), which includes Kg = 1 - Kr - Kb."""
    for k in range(3):
        rgb = np.zeros((3, 1, 1))
        rgb[k] = 1.0
        yn, cbn, crn = pixel.rgb_to_ycbcr_float(rgb, matrix)
        assert yn[0, 0] == pytest.approx(coeffs[k], abs=1e-12)
    # the colour-difference signals reach exactly +1/2 at blue (Cb) and red (Cr)
    assert pixel.rgb_to_ycbcr_float(np.array([0.0, 0.0, 1.0]).reshape(3, 1, 1), matrix)[1][0, 0] == \
        pytest.approx(0.5, abs=1e-15)
    assert pixel.rgb_to_ycbcr_float(np.array([1.0, 0.0, 0.0]).reshape(3, 1, 1), matrix)[2][0, 0] == \
        pytest.approx(0.5, abs=1e-15)


@pytest.mark.parametrize("matrix", [601, 2020])
@pytest.mark.parametrize("full", [False, True])
def test_grey_is_neutral(matrix, full):
    """Equal R', G', B' give neutral chroma codes and Y' equal to the grey level."""
    bits = 10
    v = np.linspace(0, 1, 11).reshape(1, 1, 11)
    rgb = np.repeat(v, 3, axis=0)
    y, cb, cr = pixel.pack_values(rgb, bits, 444, matrix, full)
    ys, yo, cs, co = (1023.0, 0.0, 1023.0, 512.0) if full else (876.0, 64.0, 896.0, 512.0)
    assert np.allclose(cb, co, atol=1e-9) and np.allclose(cr, co, atol=1e-9)
    assert np.allclose(y, ys * v.ravel() + yo, atol=1e-9)


@pytest.mark.parametrize("matrix", [601, 709, 2020])
@pytest.mark.parametrize("full", [False, True])
def test_exhaustive_8bit_round_trip_variants(matrix, full):
    """Every 8-bit 4:4:4 code triple whose decoded R'G'B' is inside [0,1]^3 encodes back
    to itself, for each matrix and range."""
    y, u, v = _all_444_triples(8)
    rgb = pixel.unpack(y.reshape(1, -1), u.reshape(1, -1), v.reshape(1, -1), 8, 444, matrix, full)
    ok = np.all((rgb >= 0.0) & (rgb <= 1.0), axis=0)[0]
    assert ok.sum() > 1_000_000
    y2, u2, v2 = pixel.pack(rgb[:, :, ok], 8, 444, matrix, full)
    assert np.array_equal(y2[0], y[ok]) and np.array_equal(u2[0], u[ok]) and np.array_equal(v2[0], v[ok])


@pytest.mark.parametrize("centre", [False, True])
def test_chroma_upsample_equals_library_bilinear(centre):
    """The 4:2:0 upsampler is bilinear interpolation at the luma sample positions
    expressed in chroma coordinates with replicated edges: row (y - 1/2) / 2 for both
    sitings, column x / 2 (left) or (x - 1/2) / 2 (centre); scipy's order-1
    map_coordinates with mode 'nearest' computes the same."""
    from scipy import ndimage
    rng = np.random.default_rng(3)
    c = rng.uniform(16, 240, (7, 9))
    yy, xx = np.meshgrid(np.arange(14, dtype=np.float64), np.arange(18, dtype=np.float64), indexing="ij")
    cy = (yy - 0.5) / 2.0
    cx = (xx - 0.5) / 2.0 if centre else xx / 2.0
    ref = ndimage.map_coordinates(c, [cy, cx], order=1, mode="nearest")
    assert np.allclose(pixel.upsample_chroma_420(c, centre), ref, atol=1e-12)


def test_centre_siting_closed_forms():
    # constant chroma stays constant both ways
    assert np.array_equal(pixel.upsample_chroma_420(np.full((4, 5), 90.0), True), np.full((8, 10), 90.0))
    assert np.array_equal(pixel.downsample_chroma_420(np.full((8, 10), 90.0), True), np.full((4, 5), 90.0))
    # the box filter is the mean of each 2x2 luma block
    C = np.arange(48, dtype=np.float64).reshape(6, 8)
    d = pixel.downsample_chroma_420(C, True)
    assert d[1, 2] == np.mean(C[2:4, 4:6])
    # up then down reproduces affine chroma away from the edges: 3/4 c_j + 1/8 (c_{j-1} + c_{j+1}) = c_j
    ii, jj = np.meshgrid(np.arange(6, dtype=np.float64), np.arange(8, dtype=np.float64), indexing="ij")
    aff = 100.0 + 3.0 * ii - 2.0 * jj
    back = pixel.downsample_chroma_420(pixel.upsample_chroma_420(aff, True), True)
    assert np.allclose(back[1:-1, 1:-1], aff[1:-1, 1:-1], atol=1e-12)


@pytest.mark.parametrize("centre", [False, True])
def test_420_variant_round_trip_constant_chroma(centre):
    """A 4:2:0 frame with constant in-gamut chroma and any luma survives decode and
    encode in every matrix and range."""
    rng = np.random.default_rng(5)
    for matrix, full in [(601, True), (2020, False), (709, True)]:
        Y = rng.integers(90, 160, (8, 12)).astype(np.uint8)
        U = np.full((4, 6), 120, np.uint8)
        V = np.full((4, 6), 135, np.uint8)
        rgb = pixel.unpack(Y, U, V, 8, 420, matrix, full, centre)
        assert rgb.min() >= 0 and rgb.max() <= 1
        y2, u2, v2 = pixel.pack(rgb, 8, 420, matrix, full, centre)
        assert np.array_equal(y2, Y) and np.array_equal(u2, U) and np.array_equal(v2, V)
