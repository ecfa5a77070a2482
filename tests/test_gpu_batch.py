"""Batched execution (one persistent launch per stage over many streams, replayed from a
HIP graph) against per-stream calls and the oracle.

The batched kernels run the same per-pixel arithmetic in the same order as the
per-stream kernels (a tile's shape only changes which workgroup computes a pixel, not
the order of its K accumulation), so the bar is bit-identity with the per-stream
results, for every precision, with the graph on and off, and with autotuned tiles.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import pipeline
from tests._helpers import oracle_weights, require_gpu, say

pytestmark = pytest.mark.gpu

# (width, height, bits, chroma, scene starts) of the clips mixed in one batch
CLIPS = [(64, 48, 8, 420, [3]), (48, 32, 10, 444, []), (80, 40, 8, 444, [2, 4]), (40, 24, 10, 420, [1])]
N_FRAMES = 6


@pytest.fixture(scope="module")
def B():
    require_gpu()
    from paper_2308_03121_amd import binding
    return binding


def _clips():
    return [synth.gen_clip(w, h, N_FRAMES, bits=b, chroma=c, seed=20 + i, scene_starts=s)
            for i, (w, h, b, c, s) in enumerate(CLIPS)]


def _per_stream(B, ctx, clips, dev_frames):
    res = []
    for clip, frames in zip(clips, dev_frames):
        st = ctx.open_stream(B.fmt_struct(clip.width, clip.height, clip.bits, clip.chroma))
        outs = []
        for f in frames:
            outs += st.push(f)
        outs += st.end()
        torch.cuda.synchronize()
        res.append(([B.frame_to_numpy(o, clip.bits) for o in outs], st.cuts()))
        st.close()
    return res


def _batched(B, ctx, clips, dev_frames, chains):
    """Push every clip through one stream per clip in batch calls; chains[i] = list of
    request sizes per call (the last call ends the clip)."""
    streams = [ctx.open_stream(B.fmt_struct(c.width, c.height, c.bits, c.chroma)) for c in clips]
    pos = [0] * len(clips)
    outs = [[] for _ in clips]
    ncalls = max(len(ch) for ch in chains)
    for call in range(ncalls):
        reqs, idx = [], []
        for i, ch in enumerate(chains):
            if call >= len(ch):
                continue
            k = ch[call]
            frames = dev_frames[i][pos[i]:pos[i] + k]
            end = call == len(ch) - 1
            reqs.append((streams[i], frames, None, end))
            idx.append(i)
            pos[i] += k
        got = ctx.enhance_batch(reqs)
        for i, o in zip(idx, got):
            outs[i] += o
    torch.cuda.synchronize()
    res = [([B.frame_to_numpy(o, c.bits) for o in outs[i]], streams[i].cuts()) for i, c in enumerate(clips)]
    for s in streams:
        s.close()
    return res


def _same(a, b):
    assert len(a) == len(b)
    for (oa, ca), (ob, cb) in zip(a, b):
        assert ca == cb
        assert len(oa) == len(ob)
        for fa, fb in zip(oa, ob):
            for pa, pb in zip(fa, fb):
                assert np.array_equal(pa, pb)


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_batch_bit_identical_to_streams(B, prec):
    say(f"batch vs streams {prec}")
    cfg = synth.NetConfig(32, 1, 8)
    blob = synth.gen_weights(cfg, seed=4)
    clips = _clips()
    dev = [[B.to_device_frame(*c.frame(t)) for t in range(N_FRAMES)] for c in clips]
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision=prec)
    ref = _per_stream(B, ctx, clips, dev)
    assert [[t for t, c in enumerate(r[1]) if c] for r in ref] == [c.scene_starts for c in clips]
    chains = [[3, 3], [1, 2, 3], [6], [2, 2, 2]]
    _same(_batched(B, ctx, clips, dev, chains), ref)          # recorded graph
    _same(_batched(B, ctx, clips, dev, [[2, 4], [4, 2], [5, 1], [1, 5]]), ref)   # replayed graph
    ctx.batch_graph(False)
    _same(_batched(B, ctx, clips, dev, chains), ref)          # direct launches
    ctx.profile(True)                                         # direct launches, timed
    _same(_batched(B, ctx, clips, dev, [[6]] * 4), ref)
    prof = ctx.profile_read()
    ctx.profile(False)
    n = prof["unpack"][0]                                     # one launch per stage and batch
    assert n >= 1 and prof["scene"][0] == n and prof["pack"][0] == 2 * n and prof["dcn"][0] == n, prof
    assert prof["conv_block"][0] == 2 * cfg.res_blocks * n and prof["unpack"][1] > 0, prof
    ctx.close()


def test_batch_autotuned_tiles_keep_results(B):
    say("batch autotune")
    cfg = synth.NetConfig(64, 2, 8)
    blob = synth.gen_weights(cfg, seed=5)
    clips = _clips()[:2]
    dev = [[B.to_device_frame(*c.frame(t)) for t in range(N_FRAMES)] for c in clips]
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision="fp16")
    ref = _per_stream(B, ctx, clips, dev)
    rep = ctx.autotune(48, 64)
    print("  autotune:", rep, flush=True)
    assert "block" in rep and "dcn" in rep
    _same(_batched(B, ctx, clips, dev, [[3, 3], [2, 4]]), ref)
    ctx.close()


def test_batch_matches_oracle(B):
    say("batch vs oracle")
    cfg = synth.NetConfig(32, 1, 8)
    blob = synth.gen_weights(cfg, seed=6)
    clips = _clips()[1:3]
    dev = [[B.to_device_frame(*c.frame(t)) for t in range(N_FRAMES)] for c in clips]
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob)
    got = _batched(B, ctx, clips, dev, [[4, 2], [2, 4]])
    W = oracle_weights(cfg, blob)
    for clip, (outs, cuts) in zip(clips, got):
        frames = [clip.frame(t) for t in range(N_FRAMES)]
        ref_cuts, ref_out = pipeline.enhance_clip(frames, clip.bits, clip.chroma, W, cfg.res_blocks,
                                                  cfg.offset_groups)
        assert cuts == ref_cuts
        assert len(outs) == 2 * N_FRAMES
        for g, r in zip(outs, ref_out):
            d = max(int(np.abs(a.astype(np.int64) - b.astype(np.int64)).max()) for a, b in zip(g, r["codes"]))
            assert d <= 1 and pipeline.psnr_codes(r["codes"], g, clip.bits) >= 50.0
    ctx.close()


def test_batch_rejects_bad_requests(B):
    cfg = synth.NetConfig(32, 1, 8)
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, synth.gen_weights(cfg))
    clip = _clips()[0]
    st = ctx.open_stream(B.fmt_struct(clip.width, clip.height, clip.bits, clip.chroma))
    f = B.to_device_frame(*clip.frame(0))
    from paper_2308_03121_amd import NvError
    with pytest.raises(NvError):
        ctx.enhance_batch([(st, [f] * 17, None, False)])          # chain too long
    with pytest.raises(NvError):
        ctx.enhance_batch([(st, [f], None, False), (st, [f], None, False)])   # same stream twice
    assert st.n_pushed == 0
    out = ctx.enhance_batch([(st, [f], None, False)])
    assert out == [[]]
    st.close()
    ctx.close()


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_offset_head_tiles_bit_identical(B, prec, tmp_path, monkeypatch):
    """The split offset head's three tile shapes (forced through the tuner's cache file)
    accumulate every output in the same order: per-stream and batched results are
    bit-identical to the default shapes."""
    say(f"offset-head tiles {prec}")
    cfg = synth.NetConfig(64, 1, 8)
    blob = synth.gen_weights(cfg, seed=8)
    clips = _clips()
    dev = [[B.to_device_frame(*c.frame(t)) for t in range(N_FRAMES)] for c in clips]
    ref_ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision=prec)
    ref = _per_stream(B, ref_ctx, clips, dev)
    ref_ctx.close()
    code = {"fp16": 1, "bf16": 2}[prec]
    pb4, w2 = 4, 2 | (1 << 8)                        # rows per wave 4; two waves along the blocks
    for off1, off2 in [(pb4, pb4), (w2, w2), (pb4, w2)]:
        cache = tmp_path / f"tune_{off1}_{off2}.txt"
        cache.write_text(f"prec={code} C=64 R=1 size=64x48 | 2 2 2 {off1} {off2}\n")
        ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision=prec)
        monkeypatch.setenv("NNVISR_TUNE_CACHE", str(cache))
        rep = ctx.autotune(48, 64)
        monkeypatch.delenv("NNVISR_TUNE_CACHE")
        print("  tiles:", rep, flush=True)
        assert "from cache" in rep
        _same(_per_stream(B, ctx, clips, dev), ref)
        _same(_batched(B, ctx, clips, dev, [[3, 3], [1, 2, 3], [6], [2, 2, 2]]), ref)
        ctx.close()


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_fused_residual_blocks_bit_identical(B, prec, tmp_path, monkeypatch):
    """Residual blocks as one launch each (forced through the tuner's cache file) give
    the same bits as the two separate convs, per stream (R = 3: the odd count ends with
    a copy back) and batched (which keeps the separate convs)."""
    say(f"fused residual blocks {prec}")
    cfg = synth.NetConfig(64, 3, 8)
    blob = synth.gen_weights(cfg, seed=9)
    clips = _clips()
    dev = [[B.to_device_frame(*c.frame(t)) for t in range(N_FRAMES)] for c in clips]
    ref_ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision=prec)
    ref = _per_stream(B, ref_ctx, clips, dev)
    ref_ctx.close()
    code = {"fp16": 1, "bf16": 2}[prec]
    cache = tmp_path / "tune.txt"
    cache.write_text(f"prec={code} C=64 R=3 size=64x48 | 2 2 2 2 2 1\n")
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision=prec)
    monkeypatch.setenv("NNVISR_TUNE_CACHE", str(cache))
    rep = ctx.autotune(48, 64)
    monkeypatch.delenv("NNVISR_TUNE_CACHE")
    print("  tiles:", rep, flush=True)
    assert "from cache" in rep and "fused blocks" in rep
    _same(_per_stream(B, ctx, clips, dev), ref)
    _same(_batched(B, ctx, clips, dev, [[3, 3], [1, 2, 3], [6], [2, 2, 2]]), ref)
    ctx.close()


def test_m32_tiles_batch_bit_identical(B, tmp_path, monkeypatch):
    """With the 32x32x16 MFMA tiles (forced through the tuner's cache file) the batched
    launches give the same bits as the per-stream launches."""
    say("m32 tiles batch vs streams")
    cfg = synth.NetConfig(64, 1, 8)
    blob = synth.gen_weights(cfg, seed=10)
    clips = _clips()
    dev = [[B.to_device_frame(*c.frame(t)) for t in range(N_FRAMES)] for c in clips]
    cache = tmp_path / "tune.txt"
    cache.write_text(f"prec=1 C=64 R=1 size=64x48 | {2 | (1 << 13)} {4 | (1 << 13)} 1 2 2 0\n")
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision="fp16")
    monkeypatch.setenv("NNVISR_TUNE_CACHE", str(cache))
    rep = ctx.autotune(48, 64)
    monkeypatch.delenv("NNVISR_TUNE_CACHE")
    assert "from cache" in rep and "m32" in rep, rep
    ref = _per_stream(B, ctx, clips, dev)
    _same(_batched(B, ctx, clips, dev, [[3, 3], [1, 2, 3], [6], [2, 2, 2]]), ref)
    ctx.close()


@pytest.mark.skip(reason="the LDS-resident-weight conv tile stopped in the HIP runtime on its first launch "
                         "(kernel symbol not found) and no cause has been found in the code yet; the tile is "
                         "switched off in the library and kept off the GPU until one is shown")
@pytest.mark.parametrize("prec", ["fp16", "bf16", "fp8"])
def test_lds_weight_tiles_bit_identical(B, prec, tmp_path, monkeypatch):
    """The persistent conv form that keeps a 64-channel output group's weights in LDS
    (forced through the tuner's cache file) accumulates every output in the same order
    as the default tiles: per-stream and batched results are bit-identical."""
    say(f"LDS-weight conv tiles {prec}")
    cfg = synth.NetConfig(64, 1, 8)
    blob = synth.gen_weights(cfg, seed=7)
    clips = _clips()
    dev = [[B.to_device_frame(*c.frame(t)) for t in range(N_FRAMES)] for c in clips]

    def context():
        ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision=prec)
        if prec == "fp8":
            c0 = clips[0]
            ctx.calibrate(B.fmt_struct(c0.width, c0.height, c0.bits, c0.chroma), dev[0][:4])
        return ctx

    ref_ctx = context()
    ref = _per_stream(B, ref_ctx, clips, dev)
    ref_ctx.close()
    code = {"fp16": 1, "bf16": 2, "fp8": 3}[prec]
    lw = lambda pb: pb | (1 << 12)                      # rows per wave, LDS-resident weights
    cache = tmp_path / "tune.txt"
    cache.write_text(f"prec={code} C=64 R=1 size=64x48 | {lw(2)} {lw(4)} 1\n")
    monkeypatch.setenv("NNVISR_TUNE_CACHE", str(cache))
    ctx = context()
    monkeypatch.delenv("NNVISR_TUNE_CACHE")
    probe = ctx.autotune(48, 64)                        # timed: offers only tiles that fit
    print("  tuner:", probe, flush=True)
    if "lw=" not in probe:
        ctx.close()
        pytest.skip("the device's per-workgroup LDS limit admits no LDS-weight tile for " + prec)
    monkeypatch.setenv("NNVISR_TUNE_CACHE", str(cache))
    rep = ctx.autotune(48, 64)
    print("  tiles:", rep, flush=True)
    assert "from cache" in rep
    _same(_per_stream(B, ctx, clips, dev), ref)
    _same(_batched(B, ctx, clips, dev, [[3, 3], [1, 2, 3], [6], [2, 2, 2]]), ref)
    ctx.close()


def test_fp32_two_wave_tiles_bit_identical(B, tmp_path, monkeypatch):
    """FP32 bulk convs with two waves along the output blocks (forced through the tuner's
    cache file) give the same bits as the default tiles, per stream and batched."""
    say("fp32 two-wave tiles")
    cfg = synth.NetConfig(64, 1, 8)
    blob = synth.gen_weights(cfg, seed=12)
    clips = _clips()
    dev = [[B.to_device_frame(*c.frame(t)) for t in range(N_FRAMES)] for c in clips]
    ctx0 = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision="fp32")
    ref = _per_stream(B, ctx0, clips, dev)
    ctx0.close()
    w2 = 1 << 8                                      # two waves along the output blocks
    cache = tmp_path / "tune.txt"
    cache.write_text(f"prec=0 C=64 R=1 size=64x48 | {2 | w2} {1 | w2} 2 2 2 0\n")
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision="fp32")
    monkeypatch.setenv("NNVISR_TUNE_CACHE", str(cache))
    rep = ctx.autotune(48, 64)
    monkeypatch.delenv("NNVISR_TUNE_CACHE")
    assert "from cache" in rep and "block pb2w2" in rep and "up pb1w2" in rep, rep
    _same(_per_stream(B, ctx, clips, dev), ref)
    _same(_batched(B, ctx, clips, dev, [[3, 3], [1, 2, 3], [6], [2, 2, 2]]), ref)
    ctx.close()


@pytest.mark.parametrize("prec,off_gain,C,G", [("fp16", 1.0, 64, 8), ("fp16", 12.0, 64, 8), ("bf16", 1.0, 64, 8),
                                               ("fp32", 1.0, 64, 8), ("fp32", 12.0, 64, 8), ("fp16", 1.0, 64, 16),
                                               ("fp16", 1.0, 64, 4), ("fp16", 1.0, 32, 8), ("fp32", 1.0, 64, 16)])
def test_dcn_window_tiles_bit_identical(B, prec, off_gain, C, G, tmp_path, monkeypatch):
    """The DCN forms that read a phase's sampling corners from an LDS copy of their
    window (the windowed form, tile code 2 | 16, and the staged form, 1 | 32, forced
    through the tuner's cache file) give the same bits as the plain form, per stream and
    batched.  With the offset conv's weights scaled up, most phases do not fit their
    window and read the maps directly."""
    say(f"DCN window tiles {prec} offsets x{off_gain} C={C} G={G}")
    cfg = synth.NetConfig(C, 1, G)
    blob = synth.gen_weights(cfg, seed=9)
    synth.unpack_weights(cfg, blob)["off2"][0][...] *= off_gain
    clips = _clips()
    dev = [[B.to_device_frame(*c.frame(t)) for t in range(N_FRAMES)] for c in clips]
    code = {"fp32": 0, "fp16": 1, "bf16": 2}[prec]

    def forced(dcn):
        cache = tmp_path / f"tune{dcn}.txt"
        cache.write_text(f"prec={code} C={C} R=1 size=64x48 | 2 2 {dcn} 2 2 0\n")
        ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision=prec)
        monkeypatch.setenv("NNVISR_TUNE_CACHE", str(cache))
        rep = ctx.autotune(48, 64)
        monkeypatch.delenv("NNVISR_TUNE_CACHE")
        assert "from cache" in rep, rep
        return ctx

    ref_ctx = forced(2)
    ref = _per_stream(B, ref_ctx, clips, dev)
    ref_ctx.close()
    for form in (2 | 16, 1 | 32):
        say(f"DCN tile code {form}")
        ctx = forced(form)
        _same(_per_stream(B, ctx, clips, dev), ref)
        _same(_batched(B, ctx, clips, dev, [[3, 3], [1, 2, 3], [6], [2, 2, 2]]), ref)
        ctx.close()
