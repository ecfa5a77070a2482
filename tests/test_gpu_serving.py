"""Serving on the GPU: streams that arrive while others run are batched together, and
every stream's output is the same as when it runs alone (bit-identical: the batched
kernels compute each pixel with the per-stream arithmetic)."""
import numpy as np
import pytest
import torch

import synth
from paper_2308_03121_amd.serving import GpuExecutor, Server, StreamSpec
from tests._helpers import require_gpu, say

pytestmark = pytest.mark.gpu

FORMATS = [(64, 48, 8, 420), (48, 32, 10, 420), (80, 40, 8, 444), (40, 24, 10, 444)]


@pytest.fixture(scope="module")
def B():
    require_gpu()
    from paper_2308_03121_amd import binding
    return binding


def test_serving_mix_equals_alone(B):
    say("serving mix vs alone")
    cfg = synth.NetConfig(32, 1, 8)
    blob = synth.gen_weights(cfg, seed=8)
    rng = np.random.default_rng(1)
    specs, clips = [], {}
    for sid in range(6):
        w, h, b, c = FORMATS[sid % len(FORMATS)]
        n = int(rng.integers(4, 10))
        # bursts: three streams deliver all their frames at once, the others trickle in
        arr = [0.002 * sid] * n if sid % 2 == 0 else list(0.002 * sid + np.cumsum(rng.exponential(0.003, n)))
        clip = synth.gen_clip(w, h, n, bits=b, chroma=c, seed=50 + sid, scene_starts=[n // 2])
        clips[sid] = [B.to_device_frame(*clip.frame(t)) for t in range(n)]
        specs.append(StreamSpec(sid, w, h, b, c, arr, clip.scene_starts[1:]))
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision="fp16")
    ex = GpuExecutor(ctx, lambda spec, t: clips[spec.sid][t])
    srv = Server(ex, hbm_budget=1 << 40, keep_outputs=True)
    rep = srv.run(specs, time_scale=1.0)
    torch.cuda.synchronize()
    print("  serving:", rep, flush=True)
    assert rep["groups"] == sum(s.n_frames for s in specs)
    assert rep["batches"] < rep["groups"]          # groups of different streams shared batches
    for spec in specs:
        st = ctx.open_stream(B.fmt_struct(spec.width, spec.height, spec.bits, spec.chroma))
        alone = []
        for f in clips[spec.sid]:
            alone += st.push(f)
        alone += st.end()
        torch.cuda.synchronize()
        recs = sorted((r for r in srv.records if r.sid == spec.sid), key=lambda r: r.index)
        mixed = [o for r in recs for o in r.out]
        assert len(mixed) == len(alone) == 2 * spec.n_frames
        for a, m in zip(alone, mixed):
            for pa, pm in zip(B.frame_to_numpy(a, spec.bits), B.frame_to_numpy(m, spec.bits)):
                assert np.array_equal(pa, pm)
        st.close()
    ex.shutdown()
    ctx.close()


def test_serving_selects_network_per_colourspace(B):
    """Streams of two colourspaces are served by the network trained for each (one
    context per colourspace, one batch call per context per step); every stream's output
    is bit-identical to the same stream run alone through its own context, and a stream
    whose colourspace has no network is rejected."""
    say("serving per-colourspace networks")
    cfg = synth.NetConfig(32, 1, 8)
    ctxs = {(709, False): B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, synth.gen_weights(cfg, seed=8)),
            (601, True): B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, synth.gen_weights(cfg, seed=9),
                                   matrix=601, full=True)}
    rng = np.random.default_rng(2)
    specs, clips = [], {}
    spaces = [(709, False, False), (601, True, True), (709, False, False), (601, True, False), (2020, False, False)]
    for sid, (m, f, c) in enumerate(spaces):
        w, h, b, ch = FORMATS[sid % 2]
        n = int(rng.integers(3, 7))
        clip = synth.gen_clip(w, h, n, bits=b, chroma=ch, seed=70 + sid, scene_starts=[n // 2])
        clips[sid] = [B.to_device_frame(*clip.frame(t)) for t in range(n)]
        specs.append(StreamSpec(sid, w, h, b, ch, [0.001 * sid] * n, clip.scene_starts[1:], matrix=m, full=f,
                                centre=c))
    ex = GpuExecutor(ctxs, lambda spec, t: clips[spec.sid][t])
    srv = Server(ex, hbm_budget=1 << 40, keep_outputs=True)
    rep = srv.run(specs, time_scale=1.0)
    torch.cuda.synchronize()
    print("  serving:", rep, flush=True)
    assert rep["rejected"] == 1 and rep["admitted"] == 4
    for spec in specs[:4]:
        ctx = ctxs[(spec.matrix, spec.full)]
        st = ctx.open_stream(B.fmt_struct(spec.width, spec.height, spec.bits, spec.chroma, matrix=spec.matrix,
                                          full=spec.full, centre=spec.centre))
        alone = []
        for fr in clips[spec.sid]:
            alone += st.push(fr)
        alone += st.end()
        torch.cuda.synchronize()
        recs = sorted((r for r in srv.records if r.sid == spec.sid), key=lambda r: r.index)
        mixed = [o for r in recs for o in r.out]
        assert len(mixed) == len(alone) == 2 * spec.n_frames
        for a, m in zip(alone, mixed):
            for pa, pm in zip(B.frame_to_numpy(a, spec.bits), B.frame_to_numpy(m, spec.bits)):
                assert np.array_equal(pa, pm)
        st.close()
    ex.shutdown()
    for c in ctxs.values():
        c.close()
