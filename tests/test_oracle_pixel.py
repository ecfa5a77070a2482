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

