"""The allocation-free group entry point (nv_enhance_group_static) against
nv_enhance_group: the same frame groups give bit-identical output frames, on two calls
in a row with the second group smaller than the first (the static scratch keeps the
first call's contents), and a group whose temporaries exceed the static scratch is
rejected with NV_E_INVALID before anything is enqueued."""
import numpy as np
import pytest
import torch

import synth
from tests._helpers import require_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    require_gpu()
    from paper_2308_03121_amd import binding
    return binding


def _frame(B, rng, w, h):
    y = rng.integers(16, 236, (h, w), dtype=np.uint8)
    u = rng.integers(16, 241, (h // 2, w // 2), dtype=np.uint8)
    v = rng.integers(16, 241, (h // 2, w // 2), dtype=np.uint8)
    return B.to_device_frame(y, u, v)


@pytest.mark.parametrize("prec,C", [("fp32", 32), ("fp16", 64)])
def test_static_entry_matches_enhance_group(B, prec, C):
    cfg = synth.NetConfig(C, 2, 8)
    blob = synth.gen_weights(cfg, seed=1)
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision=prec)
    rng = np.random.default_rng(11)
    for w, h in [(64, 64), (40, 24)]:
        say(f"static entry {prec} C={C} {w}x{h}")
        fmt = B.fmt_struct(w, h, 8, 420)
        fa, fb = _frame(B, rng, w, h), _frame(B, rng, w, h)
        ref = ctx.enhance_group(fmt, fa, fb)
        got = ctx.enhance_group_static(fmt, fa, fb)
        torch.cuda.synchronize()
        for t in range(3):
            for pr, pg in zip(ref[t], got[t]):
                assert torch.equal(pr, pg), (w, h, t)
    ctx.close()


def test_static_entry_rejects_oversized_group(B):
    say("static entry oversized group")
    cfg = synth.NET_C1
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, synth.gen_weights(cfg, seed=1))
    w, h = 4096, 2048
    fmt = B.fmt_struct(w, h, 8, 420)
    z = lambda ww, hh: B.alloc_frame(ww, hh, 8, 420)   # noqa: E731
    fa, fb = z(w, h), z(w, h)
    outs = [z(2 * w, 2 * h) for _ in range(3)]
    from paper_2308_03121_amd import _abi
    with pytest.raises(_abi.NvError) as e:
        ctx.enhance_group_static(fmt, fa, fb, outs=outs)
    assert e.value.status == _abi.NV_E_INVALID and "static scratch" in str(e.value)
    ctx.close()
