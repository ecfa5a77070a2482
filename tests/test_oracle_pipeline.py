"""The oracle's end-to-end composition: shapes, stream order and group consistency."""
import numpy as np

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
