"""Pins of the oracle's network operators: brute force, library routines, special cases."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F
from scipy.ndimage import map_coordinates

import synth
from oracle import network, pipeline


def _rng(seed=0):
    return np.random.default_rng(seed)


def test_conv3x3_brute_force():
    rng = _rng(1)
    x = rng.standard_normal((3, 5, 6))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = network.conv3x3(x, w, b)
    ref = np.zeros((4, 5, 6))
    for o in range(4):
        for yy in range(5):
            for xx in range(6):
                acc = b[o]
                for c in range(3):
                    for ky in range(3):
                        for kx in range(3):
                            sy, sx = yy + ky - 1, xx + kx - 1
                            if 0 <= sy < 5 and 0 <= sx < 6:
                                acc += w[o, c, ky, kx] * x[c, sy, sx]
                ref[o, yy, xx] = acc
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_conv3x3_matches_torch_f64():
    rng = _rng(2)
    x = rng.standard_normal((16, 19, 23))
    w = rng.standard_normal((24, 16, 3, 3))
    b = rng.standard_normal(24)
    ref = F.conv2d(torch.tensor(x)[None], torch.tensor(w), torch.tensor(b), padding=1)[0].numpy()
    assert np.allclose(network.conv3x3(x, w, b), ref, rtol=1e-12, atol=1e-12)


def test_pixel_shuffle_permutation():
    x = np.arange(8 * 3 * 5, dtype=np.float64).reshape(8, 3, 5)
    y = network.pixel_shuffle(x)
    assert y.shape == (2, 6, 10)
    assert np.array_equal(np.sort(y.ravel()), x.ravel())
    assert np.array_equal(y, F.pixel_shuffle(torch.tensor(x)[None], 2)[0].numpy())
    for c, i, j, h, w in [(0, 0, 0, 0, 0), (1, 1, 0, 2, 4), (0, 1, 1, 1, 3)]:
        assert y[c, 2 * h + i, 2 * w + j] == x[4 * c + 2 * i + j, h, w]
    inv = F.pixel_unshuffle(torch.tensor(y)[None], 2)[0].numpy()
    assert np.array_equal(inv, x)


def test_upsample2_matches_torch():
    rng = _rng(3)
    x = rng.standard_normal((3, 7, 9))
    ref = F.interpolate(torch.tensor(x)[None], scale_factor=2, mode="bilinear",
                        align_corners=False)[0].numpy()
    assert np.allclose(network.upsample2_bilinear(x), ref, rtol=0, atol=1e-14)


def test_bilinear_zero_matches_scipy():
    rng = _rng(4)
    x = rng.standard_normal((3, 6, 8))
    py = rng.uniform(-2.5, 7.5, (5, 7))
    px = rng.uniform(-2.5, 9.5, (5, 7))
    py[0, 0], px[0, 0] = 2.0, 3.0           # exact grid point
    py[0, 1], px[0, 1] = -1.0, 3.0          # on the zero border
    py[0, 2], px[0, 2] = 5.5, 7.25          # straddles the last row / column
    got = network.bilinear_zero(x, py, px)
    for c in range(3):
        ref = map_coordinates(x[c], [py, px], order=1, mode="grid-constant", cval=0.0)
        assert np.allclose(got[c], ref, atol=1e-13)
    assert got[0, 0, 0] == x[0, 2, 3]


def _dcn_inputs(cin=8, cout=5, h=6, w=7, groups=2, seed=5):
    rng = _rng(seed)
    x = rng.standard_normal((cin, h, w))
    wt = rng.standard_normal((cout, cin, 3, 3))
    b = rng.standard_normal(cout)
    return x, wt, b


def test_dcn_zero_offsets_unit_mask_is_conv():
    x, wt, b = _dcn_inputs()
    offs = np.zeros((36, 6, 7))
    mask = np.ones((18, 6, 7))
    got = network.deform_conv3x3(x, offs, mask, wt, b, groups=2)
    assert np.allclose(got, network.conv3x3(x, wt, b), rtol=1e-12, atol=1e-12)


def _shift_zero(x, dy, dx):
    out = np.zeros_like(x)
    _c, h, w = x.shape
    for yy in range(h):
        for xx in range(w):
            sy, sx = yy + dy, xx + dx
            if 0 <= sy < h and 0 <= sx < w:
                out[:, yy, xx] = x[:, sy, sx]
    return out


def test_dcn_integer_offsets_per_group_is_shifted_conv():
    """Group g's channels read x(p + p_k + d_g): equals a conv over maps shifted by d_g.
    Different shifts per group pin the group of each channel and the dy/dx order."""
    x, wt, b = _dcn_inputs(cin=8, groups=2)
    shifts = [(1, -2), (-1, 0)]
    offs = np.zeros((36, 6, 7))
    for g, (dy, dx) in enumerate(shifts):
        for k in range(9):
            offs[2 * (9 * g + k)] = dy
            offs[2 * (9 * g + k) + 1] = dx
    mask = np.ones((18, 6, 7))
    got = network.deform_conv3x3(x, offs, mask, wt, b, groups=2)
    # a deformed sample p + p_k + d can land outside the map: zero; a shifted conv of the
    # zero-shifted map differs only where p + p_k lands outside but p + p_k + d inside,
    # so build the reference by brute force from the definition with integer positions
    ref = np.zeros_like(got)
    for o in range(5):
        for yy in range(6):
            for xx in range(7):
                acc = b[o]
                for c in range(8):
                    dy, dx = shifts[c // 4]
                    for ky in range(3):
                        for kx in range(3):
                            sy, sx = yy + ky - 1 + dy, xx + kx - 1 + dx
                            if 0 <= sy < 6 and 0 <= sx < 7:
                                acc += wt[o, c, ky, kx] * x[c, sy, sx]
                ref[o, yy, xx] = acc
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)
    # away from the borders it equals the plain conv of the shifted map, group by group
    sh = np.concatenate([_shift_zero(x[:4], 1, -2), _shift_zero(x[4:], -1, 0)])
    plain = network.conv3x3(sh, wt, b)
    assert np.allclose(got[:, 2:4, 3:4], plain[:, 2:4, 3:4], atol=1e-12)


def test_dcn_mask_per_tap_and_group():
    """The mask of (group g, tap k) sits in channel 9g + k and scales that tap only."""
    x, wt, b = _dcn_inputs(cin=8, groups=2)
    offs = np.zeros((36, 6, 7))
    mask = np.zeros((18, 6, 7))
    mask[9 * 1 + 4] = 1.0                      # group 1, centre tap
    got = network.deform_conv3x3(x, offs, mask, wt, b, groups=2)
    ref = b[:, None, None] + np.einsum("oc,chw->ohw", wt[:, 4:, 1, 1], x[4:])
    assert np.allclose(got, ref, atol=1e-12)
    half = network.deform_conv3x3(x, offs, 0.5 * np.ones((18, 6, 7)), wt, b, groups=2)
    assert np.allclose(half - b[:, None, None],
                       0.5 * (network.conv3x3(x, wt, b) - b[:, None, None]), atol=1e-12)


def test_dcn_far_offsets_give_bias():
    x, wt, b = _dcn_inputs()
    offs = np.full((36, 6, 7), 50.0)
    got = network.deform_conv3x3(x, offs, np.ones((18, 6, 7)), wt, b, groups=2)
    assert np.allclose(got, b[:, None, None] * np.ones((1, 6, 7)), atol=0)


def test_dcn_fractional_offset_matches_scipy_sampler():
    x, wt, b = _dcn_inputs(cin=4, cout=3, groups=1, seed=9)
    rng = _rng(10)
    offs = rng.uniform(-1.7, 1.7, (18, 6, 7))
    mask = rng.uniform(0, 1, (9, 6, 7))
    got = network.deform_conv3x3(x, offs, mask, wt, b, groups=1)
    ref = np.repeat(b[:, None, None], 6, 1).repeat(7, 2).astype(np.float64)
    ys, xs = np.meshgrid(np.arange(6.0), np.arange(7.0), indexing="ij")
    for k in range(9):
        ky, kx = divmod(k, 3)
        py = ys + ky - 1 + offs[2 * k]
        px = xs + kx - 1 + offs[2 * k + 1]
        for c in range(4):
            s = map_coordinates(x[c], [py, px], order=1, mode="grid-constant", cval=0.0)
            ref += wt[:, c, ky, kx][:, None, None] * (mask[k] * s)[None]
    assert np.allclose(got, ref, atol=1e-12)


def test_lrelu_and_sigmoid():
    v = np.array([-2.0, -0.0, 0.0, 3.0])
    assert network.lrelu(v).tolist() == [-0.2, 0.0, 0.0, 3.0]
    assert np.allclose(network.sigmoid(np.array([0.0, 50.0, -50.0])), [0.5, 1.0, 0.0], atol=1e-20)


def _torch_fuse(rgb_a, rgb_b, W, R, G):
    """Independent float64 composition of torch ops (+ scipy sampler for the DCN)."""
    T = lambda a: torch.tensor(np.asarray(a, dtype=np.float64))
    conv = lambda x, n: F.conv2d(x, T(W[n][0]), T(W[n][1]), padding=1)
    lr = lambda x: F.leaky_relu(x, 0.1)

    def ext(rgb):
        x = lr(conv(T(rgb)[None], "conv_in"))
        for r in range(R):
            x = x + conv(lr(conv(x, f"block{r}.a")), f"block{r}.b")
        return x

    fa, fb = ext(rgb_a), ext(rgb_b)
    cat = torch.cat([fa, fb], 1)
    raw = conv(lr(conv(cat, "off1")), "off2")[0].numpy()
    offs, mask = raw[:18 * G], 1 / (1 + np.exp(-raw[18 * G:27 * G]))
    x = cat[0].numpy()
    cin, h, w = x.shape
    cg = cin // G
    wd, bd = W["dcn"]
    acc = np.repeat(np.asarray(bd, np.float64)[:, None, None], h, 1).repeat(w, 2)
    ys, xs = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64),
                         indexing="ij")
    for c in range(cin):
        g = c // cg
        for k in range(9):
            ky, kx = divmod(k, 3)
            s = map_coordinates(x[c], [ys + ky - 1 + offs[2 * (9 * g + k)],
                                       xs + kx - 1 + offs[2 * (9 * g + k) + 1]],
                                order=1, mode="grid-constant", cval=0.0)
            acc += np.asarray(wd[:, c, ky, kx], np.float64)[:, None, None] * (mask[9 * g + k] * s)
    fmid = lr(T(acc)[None])

    def rec(f, base):
        u = lr(F.pixel_shuffle(conv(f, "up"), 2))
        return (conv(u, "hr") + base)[0].numpy()

    up = lambda rgb: F.interpolate(T(rgb)[None], scale_factor=2, mode="bilinear",
                                   align_corners=False)
    b0, b1 = up(rgb_a), up(rgb_b)
    return {0.0: rec(fa, b0), 0.5: rec(fmid, 0.5 * (b0 + b1)), 1.0: rec(fb, b1)}


def test_network_composition_matches_torch_composition():
    cfg = synth.NetConfig(8, 1, 2)
    blob = synth.gen_weights(cfg, seed=11)
    W = pipeline.weights_dict(blob, synth.weight_layout(cfg))
    rng = _rng(12)
    rgb_a = rng.uniform(0, 1, (3, 8, 16))
    rgb_b = rng.uniform(0, 1, (3, 8, 16))
    fa = network.extract(rgb_a, W, 1)
    fb = network.extract(rgb_b, W, 1)
    got = network.fuse(rgb_a, rgb_b, fa, fb, W, 2)
    ref = _torch_fuse(rgb_a, rgb_b, W, 1, 2)
    for t in (0.0, 0.5, 1.0):
        assert np.max(np.abs(got[t] - ref[t])) <= 1e-10


def test_group_duplicate_frame_midpoint():
    """For a duplicated group [a, a] the interpolation base is the frame itself."""
    cfg = synth.NetConfig(8, 1, 2)
    W = pipeline.weights_dict(synth.gen_weights(cfg, seed=2), synth.weight_layout(cfg))
    rgb = _rng(13).uniform(0, 1, (3, 8, 8))
    f = network.extract(rgb, W, 1)
    r = network.fuse(rgb, rgb, f, f, W, 2, times=(0.0, 1.0))
    assert np.array_equal(r[0.0], r[1.0])


def test_weights_blob_layout():
    cfg = synth.NET_C1
    blob = synth.gen_weights(cfg)
    W = synth.unpack_weights(cfg, blob)
    assert W["off2"][0].shape == (27 * 8, 32, 3, 3)
    assert W["up"][0].shape == (128, 32, 3, 3)
    # He scale with the 0.1 extra gain on each block's second conv and on hr
    he = np.sqrt(2 / 1.01)
    assert np.std(W["up"][0]) == pytest.approx(he / np.sqrt(32 * 9), rel=0.05)
    assert np.std(W["block0.b"][0]) == pytest.approx(0.1 * he / np.sqrt(32 * 9), rel=0.1)
    assert blob.dtype == np.float32


@pytest.mark.parametrize("r,rw", [(1, 1), (2, 1), (1, 2), (2, 2)])
def test_pixel_shuffle_rectangular_is_the_index_map(r, rw):
    """Brute force over every index: out[c, r*h + i, rw*w + j] = in[r*rw*c + rw*i + j, h, w]."""
    c, h, w = 3, 2, 4
    x = np.arange(c * r * rw * h * w, dtype=np.float64).reshape(c * r * rw, h, w)
    out = network.pixel_shuffle(x, r, rw)
    assert out.shape == (c, r * h, rw * w)
    for cc in range(c):
        for hh in range(h):
            for ww in range(w):
                for i in range(r):
                    for j in range(rw):
                        assert out[cc, r * hh + i, rw * ww + j] == x[r * rw * cc + rw * i + j, hh, ww]


@pytest.mark.parametrize("sv,sh", [(1, 1), (2, 1), (1, 2), (2, 2)])
def test_upsample_bilinear_per_axis_equals_torch(sv, sh):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    x = rng.standard_normal((3, 5, 7))
    ref = torch.nn.functional.interpolate(torch.from_numpy(x)[None], scale_factor=(sv, sh), mode="bilinear",
                                          align_corners=False)[0].numpy()
    assert np.allclose(network.upsample_bilinear(x, sv, sh), ref, atol=1e-12)


# ---- feature pyramid and cascaded alignment ----

def _torch_dcn(x, offs, mask, wd, bd, G):
    """Modulated DCN from scipy's bilinear sampler (zero outside the map), in float64."""
    cin, h, w = x.shape
    cg = cin // G
    acc = np.repeat(np.asarray(bd, np.float64)[:, None, None], h, 1).repeat(w, 2)
    ys, xs = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64), indexing="ij")
    for c in range(cin):
        g = c // cg
        for k in range(9):
            ky, kx = divmod(k, 3)
            s = map_coordinates(x[c], [ys + ky - 1 + offs[2 * (9 * g + k)], xs + kx - 1 + offs[2 * (9 * g + k) + 1]],
                                order=1, mode="grid-constant", cval=0.0)
            acc += np.asarray(wd[:, c, ky, kx], np.float64)[:, None, None] * (mask[9 * g + k] * s)
    return acc


def test_avgpool2_matches_torch_and_affine_closed_form():
    x = _rng(30).standard_normal((5, 8, 12))
    ref = F.avg_pool2d(torch.tensor(x)[None], 2)[0].numpy()
    assert np.allclose(network.avgpool2(x), ref, rtol=0, atol=1e-14)
    i, j = np.meshgrid(np.arange(8.0), np.arange(12.0), indexing="ij")
    a = (3.0 + 0.5 * i - 0.25 * j)[None]
    ii, jj = np.meshgrid(np.arange(4.0), np.arange(6.0), indexing="ij")
    # the mean of an affine map over a 2x2 block is its value at the block's centre
    assert np.allclose(network.avgpool2(a)[0], 3.0 + 0.5 * (2 * ii + 0.5) - 0.25 * (2 * jj + 0.5), atol=1e-14)
    with pytest.raises(ValueError):
        network.avgpool2(np.zeros((1, 3, 4)))


def test_pyramid_levels_identity_down_conv_is_the_pool():
    cfg = synth.NetConfig(8, 1, 2, levels=3)
    W = pipeline.weights_dict(synth.gen_weights(cfg, seed=31), synth.weight_layout(cfg))
    for lv in (2, 3):
        w, b = W[f"down{lv}"]
        w[...] = 0.0
        b[...] = 0.0
        for c in range(8):
            w[c, c, 1, 1] = 1.0                   # centre tap only: the identity
    f1 = _rng(32).uniform(0, 1, (8, 16, 24))      # non-negative: LReLU is the identity
    p = network.pyramid(f1, W, 3)
    assert len(p) == 3 and p[1].shape == (8, 8, 12) and p[2].shape == (8, 4, 6)
    assert np.allclose(p[1], network.avgpool2(f1), atol=1e-14)
    assert np.allclose(p[2], network.avgpool2(network.avgpool2(f1)), atol=1e-14)
    assert len(network.pyramid(f1, W, 1)) == 1 and network.pyramid(f1, W, 1)[0] is not None


def test_pyramid_one_level_is_the_plain_fusion():
    cfg = synth.NetConfig(8, 1, 2)
    W = pipeline.weights_dict(synth.gen_weights(cfg, seed=33), synth.weight_layout(cfg))
    rng = _rng(34)
    rgb_a, rgb_b = rng.uniform(0, 1, (3, 8, 16)), rng.uniform(0, 1, (3, 8, 16))
    fa, fb = network.extract(rgb_a, W, 1), network.extract(rgb_b, W, 1)
    plain = network.fuse(rgb_a, rgb_b, fa, fb, W, 2, keep=True)
    pyr = network.fuse(rgb_a, rgb_b, [fa], [fb], W, 2, keep=True)
    for k in (0.0, 0.5, 1.0, "offsets", "mask", "fmid"):
        assert np.array_equal(plain[k], pyr[k])


def test_two_level_cascade_matches_torch_composition():
    """Pyramid and cascade rebuilt from torch ops (avg_pool2d, conv2d, interpolate) and
    scipy's sampler for the DCN, in float64."""
    C, G = 8, 2
    cfg = synth.NetConfig(C, 1, G, levels=2)
    W = pipeline.weights_dict(synth.gen_weights(cfg, seed=35), synth.weight_layout(cfg))
    rng = _rng(36)
    rgb_a, rgb_b = rng.uniform(0, 1, (3, 16, 24)), rng.uniform(0, 1, (3, 16, 24))
    pa = network.pyramid(network.extract(rgb_a, W, 1), W, 2)
    pb = network.pyramid(network.extract(rgb_b, W, 1), W, 2)
    got = network.fuse(rgb_a, rgb_b, pa, pb, W, G, keep=True)

    T = lambda a: torch.tensor(np.asarray(a, dtype=np.float64))  # noqa: E731
    conv = lambda x, n: F.conv2d(x, T(W[n][0]), T(W[n][1]), padding=1)  # noqa: E731
    lr = lambda x: F.leaky_relu(x, 0.1)  # noqa: E731
    up = lambda x: F.interpolate(x, scale_factor=2, mode="bilinear", align_corners=False)  # noqa: E731
    ta = [T(pa[0])[None]]
    tb = [T(pb[0])[None]]
    ta.append(lr(conv(F.avg_pool2d(ta[0], 2), "down2")))
    tb.append(lr(conv(F.avg_pool2d(tb[0], 2), "down2")))
    assert np.allclose(ta[1][0].numpy(), pa[1], atol=1e-12)

    def head(a, b, sfx):
        raw = conv(lr(conv(torch.cat([a, b], 1), "off1" + sfx)), "off2" + sfx)
        return raw[:, :18 * G], torch.sigmoid(raw[:, 18 * G:27 * G])

    o2, m2 = head(ta[1], tb[1], ".l2")
    a2 = lr(T(_torch_dcn(torch.cat([ta[1], tb[1]], 1)[0].numpy(), o2[0].numpy(), m2[0].numpy(), *W["dcn.l2"], G))[None])
    o1, m1 = head(ta[0], tb[0], "")
    o1 = o1 + 2.0 * up(o2)
    a1 = lr(T(_torch_dcn(torch.cat([ta[0], tb[0]], 1)[0].numpy(), o1[0].numpy(), m1[0].numpy(), *W["dcn"], G))[None])
    a1 = a1 + up(a2)
    assert np.max(np.abs(got["offsets"] - o1[0].numpy())) <= 1e-10
    assert np.max(np.abs(got["levels"][1][0] - o2[0].numpy())) <= 1e-10
    assert np.max(np.abs(got["fmid"] - a1[0].numpy())) <= 1e-10


def test_cascade_doubles_the_coarse_offsets():
    """A constant integer offset d at level 2 (zero weights, bias d, unit masks) and no
    offset of level 1's own give level 1 the offset 2d: its DCN equals the brute-force
    conv of the maps shifted by 2d; level 1's DCN zeroed leaves Fmid = up2(A^2)."""
    C, G = 4, 2
    cfg = synth.NetConfig(C, 0, G, levels=2)
    W = pipeline.weights_dict(synth.gen_weights(cfg, seed=37), synth.weight_layout(cfg))
    d = (1.0, -1.0)
    for sfx, bias in ((".l2", d), ("", (0.0, 0.0))):
        w, b = W["off2" + sfx]
        w[...] = 0.0
        b[:18 * G:2] = bias[0]
        b[1:18 * G:2] = bias[1]
        b[18 * G:] = 40.0                          # sigmoid(40) is 1 in float64
    rng = _rng(38)
    fa = [rng.standard_normal((C, 8, 12)), None]
    fb = [rng.standard_normal((C, 8, 12)), None]
    fa[1] = network.pyramid(fa[0], W, 2)[1]
    fb[1] = network.pyramid(fb[0], W, 2)[1]
    _fm, per = network.align_pyramid(fa, fb, W, G)
    offs1, mask1, a1 = per[0]
    assert np.all(offs1[0::2] == 2 * d[0]) and np.all(offs1[1::2] == 2 * d[1]) and np.all(mask1 == 1.0)
    x = np.concatenate([fa[0], fb[0]])
    wd, bd = W["dcn"]
    ref = np.zeros((C, 8, 12))
    for o in range(C):
        for yy in range(8):
            for xx in range(12):
                acc = bd[o]
                for c in range(2 * C):
                    for ky in range(3):
                        for kx in range(3):
                            sy, sx = yy + ky - 1 + 2, xx + kx - 1 - 2
                            if 0 <= sy < 8 and 0 <= sx < 12:
                                acc += wd[o, c, ky, kx] * x[c, sy, sx]
                ref[o, yy, xx] = acc
    assert np.allclose(a1, network.lrelu(ref) + network.upsample2_bilinear(per[1][2]), atol=1e-12)
    wd[...] = 0.0
    bd[...] = 0.0
    fm, per = network.align_pyramid(fa, fb, W, G)
    assert np.allclose(fm, network.upsample2_bilinear(per[1][2]), atol=1e-14)


def test_pyramid_weight_layout_names_and_order():
    cfg = synth.NetConfig(8, 1, 2, levels=3)
    names = [n for n, *_ in synth.weight_layout(cfg)]
    assert names == ["conv_in", "block0.a", "block0.b", "down2", "down3", "off1", "off2", "dcn",
                     "off1.l2", "off2.l2", "dcn.l2", "off1.l3", "off2.l3", "dcn.l3", "up", "hr"]
