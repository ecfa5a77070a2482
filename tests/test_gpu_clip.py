"""General n and batches of b groups over the Fig. 1 frame store (nv_clip_*), against the
oracle's grouping rules and frame-store layout (section 3.3, internal design; section 3.1
for n and the Extra / Double frame flags).

For each clip: the groups the device ran equal oracle.scene.groups_general scene by scene
(inputs of every group, including repeated and recycled frames); the store map of every
full block equals oracle.scene.frame_store_positions shifted to the block's first frame
(for n = 3, b = 2 the paper's Fig. 1, tests/golden/fig1_frame_store.json); the output
frames match the oracle (within 1 code, PSNR >= 50 dB) and are bit-identical to the
same clip through nv_stream_push (the same pairs, the same kernels)."""
import json
import os

import numpy as np
import pytest
import torch

import synth
from oracle import pipeline, scene
from tests._helpers import oracle_weights, require_gpu, say

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def B():
    require_gpu()
    from paper_2308_03121_amd import binding
    return binding


def _expected_batches(scene_lengths, n, b):
    """The groups of each scene, split into the full blocks of b groups the device runs
    while frames arrive and the scene's remaining groups."""
    out, start = [], 0
    for L in scene_lengths:
        gs = scene.groups_general([L], n, True)
        gs = [[f + start for f in g["inputs"]] for g in gs]
        full = (L - 1) // (n * b)            # blocks whose last frame arrived inside the scene
        for j in range(full):
            out.append((0, gs[j * b:(j + 1) * b], start + j * n * b))
        rest = gs[full * b:]
        if rest:
            out.append((1, rest, None))
        start += L
    return out


@pytest.mark.parametrize("n,b,lengths", [(3, 2, [1, 2, 3, 7]), (2, 3, [8, 5]), (1, 2, [5, 1, 4]),
                                         (3, 1, [4, 7])])
def test_clip_groups_store_and_outputs(B, n, b, lengths):
    say(f"clip n={n} b={b} scenes {lengths}")
    cfg = synth.NetConfig(32, 1, 8)
    blob = synth.gen_weights(cfg, seed=7)
    T = sum(lengths)
    starts = list(np.cumsum([0] + lengths[:-1]))[1:]
    w, h = 48, 32
    clip = synth.gen_clip(w, h, T, bits=8, chroma=420, seed=31, scene_starts=starts)
    frames = [clip.frame(t) for t in range(T)]
    ref_cuts, ref_out = pipeline.enhance_clip(frames, 8, 420, oracle_weights(cfg, blob), cfg.res_blocks,
                                              cfg.offset_groups)
    assert [t for t, c in enumerate(ref_cuts) if c] == [0] + starts
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob)
    fmt = B.fmt_struct(w, h, 8, 420)
    dev = [B.to_device_frame(*f) for f in frames]
    cl = B.Clip(ctx, fmt, n, b)
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
    assert len(got) == len(alone) == 2 * T
    for g, a, r in zip(got, alone, ref_out):
        cg = B.frame_to_numpy(g, 8)
        for pg, pa in zip(cg, B.frame_to_numpy(a, 8)):
            assert np.array_equal(pg, pa)
        d = max(int(np.abs(x.astype(np.int64) - y.astype(np.int64)).max()) for x, y in zip(cg, r["codes"]))
        assert d <= 1 and pipeline.psnr_codes(r["codes"], cg, 8) >= 50.0
    trace = cl.trace()
    expected = _expected_batches(lengths, n, b)
    assert [(k, g) for k, g, _ in trace] == [(k, g) for k, g, _ in expected]
    P = n * b + b
    for (kind, _g, store), (_k, _e, f0) in zip(trace, expected):
        if kind != 0:
            continue
        pos = scene.frame_store_positions(n, b, 0)
        want = [-1] * P
        for frame, p in pos.items():
            want[p] = frame + f0
        assert store == want
    st.close()
    cl.close()
    ctx.close()


def test_clip_store_is_fig1(B):
    """n = 3, b = 2: the first full block's store is the paper's Fig. 1 read column-first."""
    with open(os.path.join(GOLD, "fig1_frame_store.json")) as f:
        fig = json.load(f)
    n, b = fig["n"], fig["b"]
    say("clip store = Fig. 1")
    cfg = synth.NetConfig(32, 1, 8)
    blob = synth.gen_weights(cfg, seed=7)
    T = n * b + 1
    clip = synth.gen_clip(32, 16, T, seed=3, scene_starts=[])
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob)
    cl = B.Clip(ctx, B.fmt_struct(32, 16, 8, 420), n, b)
    for t in range(T):
        cl.push(B.to_device_frame(*clip.frame(t)))
    torch.cuda.synchronize()
    kind, groups, store = cl.trace()[0]
    column_first = [-1 if v is None else v for col in fig["columns"][:n + 1] for v in col]
    assert kind == 0 and store == column_first
    assert groups == [[0, 1, 2, 3], [3, 4, 5, 6]]
    cl.close()
    ctx.close()
