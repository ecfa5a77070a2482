"""The tasks of the end-user section (section 3.2) on the device against the FP64 oracle:
scale factors and the Interpolation / Extra frame / Double frame flags of section 3.1.

  denoise            scale 1, no flags: one output per frame, at the input size
  super-resolution   scale 2, no flags: one output per frame, twice the size
  deinterlace        horizontal 1, vertical 2, no flags: rows doubled
  interpolation      scale 1, Interpolation + Extra frame: the input frames pass through
                     unchanged, the network emits the frames between them
  interp + denoise   scale 1, all three flags
  space-time SR      scale 2, all three flags (the default task)

A clip of two scenes goes through a clip stream in each task; every output frame is
compared with the oracle (within 1 code and PSNR >= 50 dB; pass-through frames equal
to the inputs bit for bit), and, for the interpolating tasks, one lone group through
nv_enhance_group."""
import numpy as np
import pytest
import torch

import synth
from oracle import pipeline
from tests._helpers import oracle_weights, require_gpu, say

pytestmark = pytest.mark.gpu

TASKS = [("denoise", 1, 0, False, True), ("sr", 2, 0, False, True), ("deinterlace", 1, 2, False, True),
         ("interp-pass", 1, 0, True, False), ("interp-denoise", 1, 0, True, True), ("space-time", 2, 0, True, True)]


@pytest.fixture(scope="module")
def B():
    require_gpu()
    from paper_2308_03121_amd import binding
    return binding


def _close(got, ref, bits=8):
    d = max(int(np.abs(g.astype(np.int64) - r.astype(np.int64)).max()) for g, r in zip(got, ref))
    assert d <= 1 and pipeline.psnr_codes(ref, got, bits) >= 50.0, d


@pytest.mark.parametrize("name,scale,scale_v,interp,double", TASKS, ids=[t[0] for t in TASKS])
@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_task_stream_matches_oracle(B, name, scale, scale_v, interp, double, prec):
    say(f"task {name} {prec}")
    cfg = synth.NetConfig(32, 1, 8, scale=scale, scale_v=scale_v, interp=interp, double=double)
    blob = synth.gen_weights(cfg, seed=5)
    n, w, h = 6, 48, 32
    clip = synth.gen_clip(w, h, n, seed=17, scene_starts=[4])
    frames = [clip.frame(t) for t in range(n)]
    ref_cuts, ref = pipeline.enhance_clip(frames, 8, 420, oracle_weights(cfg, blob), cfg.res_blocks,
                                          cfg.offset_groups, scale=(cfg.sv, cfg.sh), interp=interp, double=double)
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision=prec, scale=scale,
                    scale_v=scale_v, interp=interp, double=double)
    st = ctx.open_stream(B.fmt_struct(w, h, 8, 420))
    got = []
    for f in frames:
        got += st.push(B.to_device_frame(*f))
    got += st.end()
    torch.cuda.synchronize()
    assert st.cuts() == ref_cuts
    assert len(got) == len(ref) == (2 * n if interp else n)
    for g, r in zip(got, ref):
        codes = B.frame_to_numpy(g, 8)
        assert codes[0].shape == (cfg.sv * h, cfg.sh * w)
        if r["hr"] is None:          # passed through
            assert all(np.array_equal(a, b) for a, b in zip(codes, r["codes"]))
        else:
            _close(codes, r["codes"])
    if interp:
        outs = ctx.enhance_group(B.fmt_struct(w, h, 8, 420), B.to_device_frame(*frames[0]),
                                 B.to_device_frame(*frames[1]))
        torch.cuda.synchronize()
        ref_g = pipeline.enhance_group(frames[0], frames[1], 8, 420, oracle_weights(cfg, blob), cfg.res_blocks,
                                       cfg.offset_groups, times=(0.0, 0.5, 1.0), scale=(cfg.sv, cfg.sh))
        for i, t in enumerate((0.0, 0.5, 1.0)):
            codes = B.frame_to_numpy(outs[i], 8)
            if not double and t != 0.5:
                assert all(np.array_equal(a, b) for a, b in zip(codes, frames[0 if t == 0.0 else 1]))
            else:
                _close(codes, ref_g["codes"][t])
    st.close()
    ctx.close()


def test_task_validation(B):
    """Pass-through needs scale 1; batches and FP8 run the space-time task only."""
    from paper_2308_03121_amd import _abi
    say("task validation")
    with pytest.raises(_abi.NvError) as e:
        B.Context(32, 1, 8, np.zeros(1, np.float32), scale=2, interp=True, double=False)
    assert e.value.status == _abi.NV_E_INVALID
    cfg = synth.NetConfig(32, 1, 8, scale=1, interp=False)
    ctx = B.Context(32, 1, 8, synth.gen_weights(cfg, seed=1), scale=1, interp=False)
    clip = synth.gen_clip(32, 16, 2, seed=1, scene_starts=[])
    with pytest.raises(_abi.NvError) as e:
        ctx.enhance_group(B.fmt_struct(32, 16, 8, 420), B.to_device_frame(*clip.frame(0)),
                          B.to_device_frame(*clip.frame(1)))
    assert e.value.status == _abi.NV_E_UNSUPPORTED
    st = ctx.open_stream(B.fmt_struct(32, 16, 8, 420))
    with pytest.raises(_abi.NvError) as e:
        ctx.enhance_batch([(st, [B.to_device_frame(*clip.frame(0))], None, True)])
    assert e.value.status == _abi.NV_E_UNSUPPORTED
    st.close()
    ctx.close()
