"""The multi-level feature pyramid on the device against the FP64 oracle.

Section 3.1 defines the extract stage's output as a pyramid of features at several
spatial sizes; the fusion stage aligns them coarsest level first (oracle.network:
level l >= 2 = conv + LReLU of the 2x2 mean pool of level l-1; each level's offsets
add twice the x2 resize of the coarser level's, its aligned features the x2 resize of
the coarser aligned features).  Stage by stage in FP32 at the float bar (each stage fed
the device's inputs), end to end through clip streams and single groups in FP32 and
FP16 (within one code, PSNR >= 50 dB), and the allocation-free group entry against the
allocating one, bit for bit."""
import numpy as np
import pytest
import torch

import synth
from oracle import network, pipeline
from tests._helpers import max_abs, nhwc_to_chw, oracle_weights, require_gpu, say

pytestmark = pytest.mark.gpu

FLOAT_TOL = 1e-4


@pytest.fixture(scope="module")
def B():
    require_gpu()
    from paper_2308_03121_amd import binding
    return binding


def _close(got, ref, bits=8):
    d = max(int(np.abs(g.astype(np.int64) - r.astype(np.int64)).max()) for g, r in zip(got, ref))
    assert d <= 1 and pipeline.psnr_codes(ref, got, bits) >= 50.0, d


@pytest.mark.parametrize("levels,hp,wp", [(2, 40, 72), (3, 48, 64), (4, 64, 80)])
def test_pyramid_stages_match_oracle(B, levels, hp, wp):
    say(f"pyramid stages L={levels} {wp}x{hp}")
    cfg = synth.NetConfig(32, 1, 8, levels=levels)
    blob = synth.gen_weights(cfg, seed=21)
    W = oracle_weights(cfg, blob)
    G = cfg.offset_groups
    ctx = B.Context(cfg.channels, cfg.res_blocks, G, blob, levels=levels)
    rng = np.random.default_rng(hp * wp + levels)
    rgb_a = rng.uniform(0, 1, (3, hp, wp)).astype(np.float32)
    rgb_b = np.clip(rgb_a + rng.normal(0, 0.05, rgb_a.shape), 0, 1).astype(np.float32)
    ta, tb = torch.from_numpy(rgb_a).cuda(), torch.from_numpy(rgb_b).cuda()
    fa, fb = ctx.extract(ta), ctx.extract(tb)
    hr, offs, fmid = ctx.fuse(ta, tb, fa, fb, 7, want_offsets=True, want_fmid=True)
    torch.cuda.synchronize()
    ra, rb = rgb_a.astype(np.float64), rgb_b.astype(np.float64)
    pa = network.pyramid(network.extract(ra, W, cfg.res_blocks), W, levels)
    pb = network.pyramid(network.extract(rb, W, cfg.res_blocks), W, levels)
    da = [nhwc_to_chw(x) for x in ctx.pyramid_levels(fa)]
    db = [nhwc_to_chw(x) for x in ctx.pyramid_levels(fb)]
    assert [x.shape for x in da] == [x.shape for x in pa]
    for lv in range(levels):
        assert max_abs(da[lv], pa[lv]) <= FLOAT_TOL, lv
        assert max_abs(db[lv], pb[lv]) <= FLOAT_TOL, lv
    # the alignment from the device's pyramids
    o_fmid, per = network.align_pyramid(da, db, W, G)
    got = nhwc_to_chw(offs)
    assert max_abs(got[:18 * G], per[0][0]) <= FLOAT_TOL
    assert max_abs(got[18 * G:27 * G], per[0][1]) <= FLOAT_TOL
    assert max_abs(nhwc_to_chw(fmid), o_fmid) <= FLOAT_TOL
    # end to end from the same inputs
    full = network.fuse(ra, rb, pa, pb, W, G)
    for t, key in enumerate((0.0, 0.5, 1.0)):
        assert max_abs(hr[t].cpu().numpy(), full[key]) <= FLOAT_TOL, key
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
@pytest.mark.parametrize("levels", [2, 3])
def test_pyramid_stream_and_group_match_oracle(B, prec, levels):
    say(f"pyramid stream L={levels} {prec}")
    cfg = synth.NetConfig(32, 1, 8, levels=levels)
    blob = synth.gen_weights(cfg, seed=22)
    W = oracle_weights(cfg, blob)
    n, w, h = 6, 56, 40
    clip = synth.gen_clip(w, h, n, seed=23, scene_starts=[4])
    frames = [clip.frame(t) for t in range(n)]
    ref_cuts, ref = pipeline.enhance_clip(frames, 8, 420, W, cfg.res_blocks, cfg.offset_groups, levels=levels)
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision=prec, levels=levels)
    st = ctx.open_stream(B.fmt_struct(w, h, 8, 420))
    got = []
    for f in frames:
        got += st.push(B.to_device_frame(*f))
    got += st.end()
    torch.cuda.synchronize()
    assert st.cuts() == ref_cuts and len(got) == len(ref) == 2 * n
    for g, r in zip(got, ref):
        _close(B.frame_to_numpy(g, 8), r["codes"])
    st.close()
    fmt = B.fmt_struct(w, h, 8, 420)
    outs = ctx.enhance_group(fmt, B.to_device_frame(*frames[0]), B.to_device_frame(*frames[1]))
    torch.cuda.synchronize()
    ref_g = pipeline.enhance_group(frames[0], frames[1], 8, 420, W, cfg.res_blocks, cfg.offset_groups,
                                   levels=levels)
    for i, t in enumerate((0.0, 0.5, 1.0)):
        _close(B.frame_to_numpy(outs[i], 8), ref_g["codes"][t])
    # the allocation-free entry runs the same kernels on its static scratch
    outs_s = ctx.enhance_group_static(fmt, B.to_device_frame(*frames[0]), B.to_device_frame(*frames[1]))
    torch.cuda.synchronize()
    for a, b in zip(outs, outs_s):
        for pa, pb in zip(B.frame_to_numpy(a, 8), B.frame_to_numpy(b, 8)):
            assert np.array_equal(pa, pb)
    ctx.close()


def test_pyramid_validation(B):
    from paper_2308_03121_amd import _abi
    say("pyramid validation")
    cfg = synth.NetConfig(64, 1, 8, levels=2)
    blob = synth.gen_weights(cfg, seed=24)
    for kw, status in (({"precision": "fp8"}, _abi.NV_E_UNSUPPORTED), ({"levels": 5}, _abi.NV_E_INVALID)):
        args = dict(levels=2)
        args.update(kw)
        with pytest.raises(_abi.NvError) as e:
            B.Context(64, 1, 8, blob, **args)
        assert e.value.status == status, kw
    with pytest.raises(_abi.NvError) as e:
        B.Context(64, 1, 8, synth.gen_weights(synth.NetConfig(64, 1, 8, interp=False), seed=1), scale=1,
                  interp=False, levels=2)
    assert e.value.status == _abi.NV_E_INVALID
    ctx = B.Context(64, 1, 8, blob, levels=2)
    clip = synth.gen_clip(32, 16, 2, seed=1, scene_starts=[])
    st = ctx.open_stream(B.fmt_struct(32, 16, 8, 420))
    with pytest.raises(_abi.NvError) as e:
        ctx.enhance_batch([(st, [B.to_device_frame(*clip.frame(0))], None, True)])
    assert e.value.status == _abi.NV_E_UNSUPPORTED
    st.close()
    ctx.close()


def test_pyramid_general_n_clip(B):
    """A general-n clip (n = 3, b = 2, section 3.3) of a two-level network: the same pairs
    as a clip stream, bit for bit, and the oracle within the bar."""
    say("pyramid clip n=3 b=2")
    cfg = synth.NetConfig(32, 1, 8, levels=2)
    blob = synth.gen_weights(cfg, seed=25)
    T, w, h = 9, 48, 32
    clip = synth.gen_clip(w, h, T, seed=26, scene_starts=[7])
    frames = [clip.frame(t) for t in range(T)]
    _c, ref = pipeline.enhance_clip(frames, 8, 420, oracle_weights(cfg, blob), cfg.res_blocks, cfg.offset_groups,
                                    levels=2)
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, levels=2)
    fmt = B.fmt_struct(w, h, 8, 420)
    dev = [B.to_device_frame(*f) for f in frames]
    cl = B.Clip(ctx, fmt, 3, 2)
    got = []
    for f in dev:
        got += cl.push(f)
    got += cl.end()
    st = ctx.open_stream(fmt)
    alone = []
    for f in dev:
        alone += st.push(f)
    alone += st.end()
    torch.cuda.synchronize()
    assert len(got) == len(alone) == len(ref) == 2 * T
    for g, a, r in zip(got, alone, ref):
        cg = B.frame_to_numpy(g, 8)
        for pg, pa in zip(cg, B.frame_to_numpy(a, 8)):
            assert np.array_equal(pg, pa)
        _close(cg, r["codes"])
    st.close()
    cl.close()
    ctx.close()
