"""Exactness of the integer path on the device: Y'CbCr codes -> R'G'B' -> network -> codes.

With the output conv's weights and bias set to zero, the network's output is its base
image: at scale 1 the frame itself (the x1 denoise task of section 3.2, and frame a of an
interpolating group at t = 0).  The whole device path (unpack, pad, the network's
kernels, crop, pack) must then return the input codes bit for bit wherever the decode ->
encode round trip of the pixel formats (section 3.1) is exact in exact arithmetic:

  4:4:4, any code triple whose R'G'B' lies inside [0, 1]^3;
  4:2:0 with constant chroma;
  4:2:0 with chroma affine in position, away from the replicated edge rows / columns.

The inputs are built so that the oracle's round trip is the identity on them (asserted),
and the device output is compared with the input codes."""
import numpy as np
import pytest
import torch

import synth
from oracle import pixel
from tests._helpers import require_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    require_gpu()
    from paper_2308_03121_amd import binding
    return binding


def _identity_blob(cfg, seed):
    """Random weights everywhere except the output conv, which is all zero."""
    blob = synth.gen_weights(cfg, seed=seed)
    w, b = synth.unpack_weights(cfg, blob)["hr"]
    w[...] = 0.0
    b[...] = 0.0
    return blob


def _in_gamut_444(h, w, bits, seed):
    """Codes of random R'G'B' well inside the gamut (decoding them stays inside [0, 1])."""
    rng = np.random.default_rng(seed)
    rgb = rng.uniform(0.05, 0.95, (3, h, w))
    return pixel.pack(rgb, bits, 444)


def _const_420(h, w, bits, seed):
    rng = np.random.default_rng(seed)
    s = 1 << (bits - 8)
    dt = np.uint8 if bits == 8 else np.uint16
    Y = (rng.integers(60, 200, (h, w)) * s).astype(dt)
    U = np.full((h // 2, w // 2), 120 * s, dt)
    V = np.full((h // 2, w // 2), 135 * s, dt)
    return Y, U, V


def _affine_420(h, w, bits, seed):
    s = 1 << (bits - 8)
    dt = np.uint8 if bits == 8 else np.uint16
    i, j = np.meshgrid(np.arange(h // 2), np.arange(w // 2), indexing="ij")
    U = ((110 + (j % 20) + (i % 15)) * s).astype(dt)          # piecewise affine ramps
    V = ((130 - (j % 20) + (i % 15)) * s).astype(dt)
    Y = np.full((h, w), 120 * s, dt)
    return Y, U, V


def _affine_mask(h, w):
    """Chroma samples whose 3x3 chroma neighbourhood lies on one affine piece and inside
    the plane (the round trip reads one neighbour each way)."""
    i, j = np.meshgrid(np.arange(h // 2), np.arange(w // 2), indexing="ij")
    return (i >= 1) & (i <= h // 2 - 2) & (j >= 1) & (j <= w // 2 - 2) & \
        (j % 20 >= 1) & (j % 20 <= 18) & (i % 15 >= 1) & (i % 15 <= 13)


CASES = [("444-8", 72, 40, 8, 444, _in_gamut_444), ("444-10", 72, 40, 10, 444, _in_gamut_444),
         ("420-const-8", 72, 40, 8, 420, _const_420), ("420-const-10", 96, 56, 10, 420, _const_420),
         ("420-affine-8", 160, 96, 8, 420, _affine_420), ("420-affine-10", 160, 96, 10, 420, _affine_420)]


def _check(got, frame, name, h, w):
    if "affine" in name:
        assert np.array_equal(got[0], frame[0])
        m = _affine_mask(h, w)
        for g, f in zip(got[1:], frame[1:]):
            assert np.array_equal(g[m], f[m])
    else:
        for g, f in zip(got, frame):
            assert np.array_equal(g, f)


def _oracle_round_trip_is_identity(frame, name, bits, chroma, h, w):
    rgb = pixel.unpack(*frame, bits, chroma)
    assert rgb.min() >= 0 and rgb.max() <= 1
    _check(pixel.pack(rgb, bits, chroma), frame, name, h, w)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
@pytest.mark.parametrize("name,w,h,bits,chroma,gen", CASES, ids=[c[0] for c in CASES])
def test_identity_network_returns_input_codes(B, name, w, h, bits, chroma, gen, prec):
    say(f"integer path {name} {prec}")
    frames = [gen(h, w, bits, 31 + k) for k in range(3)]
    for f in frames:
        _oracle_round_trip_is_identity(f, name, bits, chroma, h, w)
    cfg = synth.NetConfig(32, 1, 8, scale=1, interp=False)
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, _identity_blob(cfg, 4), precision=prec,
                    scale=1, interp=False)
    st = ctx.open_stream(B.fmt_struct(w, h, bits, chroma))
    got = []
    for f in frames:
        got += st.push(B.to_device_frame(*f))
    got += st.end()
    torch.cuda.synchronize()
    assert len(got) == len(frames)
    for g, f in zip(got, frames):
        _check(B.frame_to_numpy(g, bits), f, name, h, w)
    st.close()
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_identity_interpolating_group_keeps_frame_a(B, prec):
    """Interpolation + denoise at scale 1: the t = 0 output of a group is frame a's base."""
    say(f"integer path interp group {prec}")
    h, w, bits = 40, 72, 10
    fa, fb = _in_gamut_444(h, w, bits, 5), _in_gamut_444(h, w, bits, 6)
    cfg = synth.NetConfig(32, 1, 8, scale=1)
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, _identity_blob(cfg, 7), precision=prec,
                    scale=1)
    outs = ctx.enhance_group(B.fmt_struct(w, h, bits, 444), B.to_device_frame(*fa), B.to_device_frame(*fb))
    torch.cuda.synchronize()
    for t, ref in ((0, fa), (2, fb)):
        for g, f in zip(B.frame_to_numpy(outs[t], bits), ref):
            assert np.array_equal(g, f)
    ctx.close()


def test_identity_network_full_size(B):
    """1920x1080 4:2:0, constant chroma, FP16, through the same stream path."""
    say("integer path 1080p")
    h, w, bits = 1080, 1920, 8
    frame = _const_420(h, w, bits, 9)
    cfg = synth.NetConfig(32, 1, 8, scale=1, interp=False)
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, _identity_blob(cfg, 4), precision="fp16",
                    scale=1, interp=False)
    st = ctx.open_stream(B.fmt_struct(w, h, bits, 420))
    got = st.push(B.to_device_frame(*frame)) + st.end()
    torch.cuda.synchronize()
    assert len(got) == 1
    for g, f in zip(B.frame_to_numpy(got[0], bits), frame):
        assert np.array_equal(g, f)
    st.close()
    ctx.close()
