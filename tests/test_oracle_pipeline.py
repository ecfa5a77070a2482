"""The oracle's end-to-end composition: shapes, stream order and group consistency."""
import numpy as np
import pytest

import synth
from oracle import network, pipeline, pixel, scene


def _weights(cfg, seed=1):
    return pipeline.weights_dict(synth.gen_weights(cfg, seed), synth.weight_layout(cfg))


def test_group_c1_shapes_and_ranges():
    clip = synth.gen_group_c1()
    cfg = synth.NET_C1
    out = pipeline.enhance_group(clip.frame(0), clip.frame(1), 8, 420, _weights(cfg),
                                 cfg.res_blocks, cfg.offset_groups, keep=True)
    for t in (0.0, 0.5, 1.0):
        y, u, v = out["codes"][t]
        assert y.shape == (128, 128) and u.shape == (64, 64) and v.shape == (64, 64)
        assert y.dtype == np.uint8
        assert out["hr"][t].shape == (3, 128, 128)
    assert out["offsets"].shape == (144, 64, 64) and out["mask"].shape == (72, 64, 64)
    assert 0 < out["mask"].min() and out["mask"].max() < 1


def test_clip_stream_order_matches_groups():
    cfg = synth.NetConfig(8, 1, 2)
    W = _weights(cfg, 3)
    clip = synth.gen_clip(32, 16, 6, seed=3, scene_starts=[3])
    frames = [clip.frame(t) for t in range(clip.n_frames)]
    cuts, outs = pipeline.enhance_clip(frames, 8, 420, W, 1, 2)
    assert cuts == [1, 0, 0, 1, 0, 0]
    assert len(outs) == 2 * clip.n_frames
    assert [o["group"] for o in outs[::2]] == scene.groups_n1(cuts)
    # each emitted frame equals the lone-group computation of its group
    for o in outs:
        a, b = o["group"]
        g = pipeline.enhance_group(frames[a], None if a == b else frames[b], 8, 420, W, 1, 2,
                                   times=(o["t"],))
        assert np.array_equal(g["hr"][o["t"]], o["hr"])
        assert all(np.array_equal(p, q) for p, q in zip(g["codes"][o["t"]], o["codes"]))


def test_crop_and_padding_geometry():
    """Sizes that are not multiples of 8 are padded by replication and cropped back."""
    cfg = synth.NetConfig(8, 1, 2)
    W = _weights(cfg, 4)
    clip = synth.gen_clip(22, 10, 1, seed=5, scene_starts=[])
    out = pipeline.enhance_group(clip.frame(0), None, 8, 420, W, 1, 2, times=(0.0,), keep=True)
    assert out["rgb_a"].shape == (3, 16, 24)
    assert out["hr"][0.0].shape == (3, 20, 44)
    full = network.fuse(out["rgb_a"], out["rgb_a"], out["fa"], out["fa"], W, 2, times=(0.0,))
    assert np.array_equal(full[0.0][:, :20, :44], out["hr"][0.0])
    rgb = pixel.unpack(*clip.frame(0), 8, 420)
    assert np.array_equal(out["rgb_a"][:, :10, :22], rgb)


def test_psnr_definitions():
    a = np.zeros((3, 4, 4))
    assert pipeline.psnr_float(a, a) == float("inf")
    b = a + 0.01
    assert abs(pipeline.psnr_float(a, b) - 40.0) < 1e-9
    p = (np.zeros((2, 2), np.uint8),) * 3
    q = (np.ones((2, 2), np.uint8),) * 3
    assert abs(pipeline.psnr_codes(p, q, 8) - 20 * np.log10(255.0)) < 1e-9


def _marker_blob(order):
    """A blob in which every weight encodes its own position and every bias a distinct
    negative marker: w[L][o][i][ky][kx] = 100000 L + 1000 o + 100 i + 10 ky + kx and
    b[L][o] = -(100000 L + 1000 o + 1.5), all exact in float32 for the sizes used."""
    parts = []
    for L, (_name, cout, cin) in enumerate(order):
        o, i, ky, kx = np.meshgrid(np.arange(cout), np.arange(cin), np.arange(3), np.arange(3), indexing="ij")
        parts.append((100000 * L + 1000 * o + 100 * i + 10 * ky + kx).astype(np.float32).ravel())
        parts.append(-(100000 * L + 1000 * np.arange(cout) + 1.5).astype(np.float32))
    return np.concatenate(parts)


def test_weights_dict_order_and_oihw_reshape():
    """Pins the blob reader every oracle network test builds its weights with.  The
    expected tensor order is the one the C-ABI header documents for the weight blob
    (conv_in, then block.a / block.b per residual block, off1, off2, dcn, up, hr), each
    conv OIHW followed by its bias; it is written out here, not taken from the
    generator, and every element is checked against its position marker, so a
    bias/weight swap, a wrong layer order or a transposed reshape of a square layer
    (block convs are C x C) fails."""
    C, R, G = 4, 2, 2
    order = [("conv_in", C, 3)]
    for r in range(R):
        order += [(f"block{r}.a", C, C), (f"block{r}.b", C, C)]
    order += [("off1", C, 2 * C), ("off2", 27 * G, C), ("dcn", C, 2 * C), ("up", 4 * C, C), ("hr", 3, C)]
    cfg = synth.NetConfig(C, R, G)
    assert [(n, co, ci) for n, co, ci, _g in synth.weight_layout(cfg)] == order
    blob = _marker_blob(order)
    assert blob.size == sum(co * ci * 9 + co for _n, co, ci in order)
    W = pipeline.weights_dict(blob, synth.weight_layout(cfg))
    assert list(W) == [n for n, _co, _ci in order]
    for L, (name, cout, cin) in enumerate(order):
        w, b = W[name]
        assert w.shape == (cout, cin, 3, 3) and b.shape == (cout,)
        assert w.dtype == np.float64 and b.dtype == np.float64
        for o in range(cout):
            assert b[o] == -(100000 * L + 1000 * o + 1.5)
            for i in range(cin):
                for ky in range(3):
                    for kx in range(3):
                        assert w[o, i, ky, kx] == 100000 * L + 1000 * o + 100 * i + 10 * ky + kx
    # the generator's own views into a real blob agree element for element
    real = synth.gen_weights(cfg, seed=9)
    Wr = pipeline.weights_dict(real, synth.weight_layout(cfg))
    for name, (w, b) in synth.unpack_weights(cfg, real).items():
        assert np.array_equal(Wr[name][0], w.astype(np.float64))
        assert np.array_equal(Wr[name][1], b.astype(np.float64))


def test_weights_dict_rejects_a_wrong_size():
    cfg = synth.NetConfig(4, 1, 2)
    blob = synth.gen_weights(cfg)
    with pytest.raises(ValueError):
        pipeline.weights_dict(blob[:-1], synth.weight_layout(cfg))
    with pytest.raises(ValueError):
        pipeline.weights_dict(np.concatenate([blob, [0.0]]), synth.weight_layout(cfg))


def test_task_modes_output_counts_and_pass_through():
    """Section 3.2 tasks: without Interpolation one output per input frame that depends
    on that frame alone; Interpolation without Double frame passes the input frames
    through unchanged between the interpolated ones (scale 1)."""
    import synth
    from oracle import pipeline
    clip = synth.gen_clip(24, 16, 4, seed=2, scene_starts=[2])
    frames = [clip.frame(t) for t in range(4)]
    for cfg in (synth.NetConfig(32, 1, 8, scale=1, interp=False), synth.NetConfig(32, 1, 8, scale=2, interp=False),
                synth.NetConfig(32, 1, 8, scale=1, scale_v=2, interp=False)):
        W = pipeline.weights_dict(synth.gen_weights(cfg, seed=3), synth.weight_layout(cfg))
        _c, out = pipeline.enhance_clip(frames, 8, 420, W, 1, 8, scale=(cfg.sv, cfg.sh), interp=False)
        assert len(out) == 4 and out[0]["codes"][0].shape == (16 * cfg.sv, 24 * cfg.sh)
        alt = list(frames)
        alt[1] = tuple(np.ascontiguousarray(p[::-1]) for p in frames[1])
        _c, out2 = pipeline.enhance_clip(alt, 8, 420, W, 1, 8, scale=(cfg.sv, cfg.sh), interp=False)
        for t in (0, 2, 3):
            assert all(np.array_equal(a, b) for a, b in zip(out[t]["codes"], out2[t]["codes"]))
    cfg = synth.NetConfig(32, 1, 8, scale=1, double=False)
    W = pipeline.weights_dict(synth.gen_weights(cfg, seed=3), synth.weight_layout(cfg))
    _c, out = pipeline.enhance_clip(frames, 8, 420, W, 1, 8, scale=(1, 1), double=False)
    assert len(out) == 8
    for t in range(4):
        assert out[2 * t]["hr"] is None
        assert all(np.array_equal(a, b) for a, b in zip(out[2 * t]["codes"], frames[t]))
        assert out[2 * t + 1]["codes"][0].shape == (16, 24)
