"""Host-side bookkeeping of bench.py: the algorithmic work and bytes it divides by, the
counter-derived traffic figure, and the one-GPU guard.  No GPU is touched."""
import os
import re
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _layers(C, R, G):
    # (pixel factor, input channels, output channels) of every 3x3 conv of one stream
    # group: one feature extraction, the offset head and the DCN for the middle frame,
    # and the pixel-shuffle and HR convs of both output frames (HR at 4x the pixels)
    lay = [(1, 3, C)] + [(1, C, C)] * (2 * R)
    lay += [(1, 2 * C, C), (1, C, 27 * G), (1, 2 * C, C)]
    lay += [(1, C, 4 * C), (4, C, 3)] * 2
    return lay


def test_group_flops_match_layer_count():
    for C, R, G in [(64, 10, 8), (32, 2, 8), (64, 6, 8)]:
        want = sum(2 * 9 * ci * co * f for f, ci, co in _layers(C, R, G))
        assert bench.group_flops_per_px(C, R, G) == want
    # the main workload: 120 groups of 960x544 padded pixels, 165.4 TFLOP per step
    assert abs(bench.group_flops_per_px(64, 10, 8) * 960 * 544 * 120 / 1e12 - 165.4) < 0.05


def test_block_conv_work_and_bytes():
    flop, unit = bench.kernel_work("conv_block", 544, 960, 64, 8, 4)
    assert unit == "flop" and flop == 2 * 9 * 64 * 64 * 544 * 960
    # first conv: read x, write y; second: also read the skip -> 2.5 maps per launch
    m = 544 * 960 * 64 * 4
    assert bench.conv_block_bytes(544, 960, 64) == 5 * m // 2 == 334233600


def test_counter_traffic_is_near_algorithmic():
    t = bench.FP32_CONV_BLOCK_TRAFFIC
    assert re.fullmatch(r"pb[124](w2)?", t["tile"])
    traffic = bench.conv_block_traffic()
    algo = bench.conv_block_bytes(544, 960, 64)
    assert algo <= traffic <= 1.10 * algo


def test_counter_traffic_needs_the_counted_source(monkeypatch):
    """The stored counters are reported only for the device source and tile they were
    taken on."""
    t = dict(bench.FP32_CONV_BLOCK_TRAFFIC)
    line = f"block: ... -> {t['tile']}; [block {t['tile']}, up pb2w2, dcn pb2win]"
    monkeypatch.setattr(bench, "FP32_CONV_BLOCK_TRAFFIC", dict(t, source=bench.conv_source_hash()))
    assert bench.traffic_valid(line)
    assert not bench.traffic_valid(line.replace(f"[block {t['tile']},", "[block pb4,"))
    monkeypatch.setattr(bench, "FP32_CONV_BLOCK_TRAFFIC", dict(t, source="0" * 16))
    assert not bench.traffic_valid(line)
    assert re.fullmatch(r"[0-9a-f]{16}", bench.conv_source_hash())


def test_mfma_fraction_per_kind_uses_the_kind_s_mfma_type():
    """Per-kind MFMA fractions take the peak of the MFMA type each kind runs on: FP8 runs
    only the residual-block convs on e4m3 (FP8-fusion also the DCN and pixel-shuffle
    conv), the offset head stays on float16 MFMA in every reduced-precision mode."""
    hp, wp, C, G = 544, 960, 64, 8
    us = {"conv_block": 42.0, "off1": 116.0, "off2": 499.0, "dcn": 318.0, "up": 210.0, "hr": 91.0}
    pr = {k: (10, 10 * v / 1000.0) for k, v in us.items()}          # (launches, total ms)
    for prec, want in (("fp8", {"conv_block": 5000.0, "dcn": 2500.0, "up": 2500.0, "off2": 2500.0}),
                       ("fp8-fusion", {"conv_block": 5000.0, "dcn": 5000.0, "up": 5000.0, "hr": 2500.0}),
                       ("fp16", {k: 2500.0 for k in us}), ("fp32", {k: 157.3 for k in us})):
        for kind, peak in want.items():
            r = bench.mfma_share(pr, kind, hp, wp, C, G, prec)
            flop, _ = bench.kernel_work(kind, hp, wp, C, G, 0)
            assert r["peak"] == peak, (prec, kind)
            assert abs(r["frac"] - flop / (us[kind] * 1e-6) / 1e12 / peak) < 1e-4
    fr = bench.mfma_shares(pr, hp, wp, C, G, "fp16")
    assert set(fr) == set(bench.MFMA_KINDS)
    assert abs(fr["conv_block"] - 2 * 9 * 64 * 64 * hp * wp / 42e-6 / 1e12 / 2500.0) < 1e-4


def test_pixel_stage_bytes():
    # pack of one 3840x2160 10-bit 4:2:0 frame: float R'G'B' in, 1.5 codes of 2 B out
    assert bench.pixel_bytes("pack", 1920, 1080, 10, 420) == 4 * 1920 * 1080 * (12 + 3)
    # unpack of one 1920x1080 10-bit 4:2:0 frame to the padded float planes
    assert bench.pixel_bytes("unpack", 1920, 1080, 10, 420) == 1920 * 1080 * 3 + 12 * 1080 * 1920
    assert bench.pixel_bytes("scene", 1920, 1080, 8, 444) == 2 * 1920 * 1080


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_batched_pixel_rates_count_every_frame_of_the_batch():
    clips = [(640, 360, 8, 420), (1280, 720, 10, 444)]
    prof = {"unpack": (1, 0.5), "scene": (1, 0.1), "pack": (2, 2.0)}
    r = bench.batched_pixel_rates(prof, clips, 5)
    want_unpack = 5 * (bench.pixel_bytes("unpack", *clips[0]) + bench.pixel_bytes("unpack", *clips[1]))
    assert r["unpack"]["bytes_per_launch"] == want_unpack
    assert r["unpack"]["avg_us"] == 500.0 and abs(r["unpack"]["gbs"] - want_unpack / 500e3) < 0.1
    want_pack = 4 * (bench.pixel_bytes("pack", *clips[0]) + bench.pixel_bytes("pack", *clips[1]))
    assert r["pack"]["bytes_per_launch"] == want_pack and r["pack"]["avg_us"] == 1000.0


def test_mfma_share_of_a_profiled_kind():
    flop = 2 * 9 * 64 * 64 * 544 * 960
    r = bench.mfma_share({"conv_block": (10, 0.5)}, "conv_block", 544, 960, 64, 8, "fp16")
    assert r["avg_launch_us"] == 50.0 and abs(r["achieved"] - flop / 50e-6 / 1e12) < 0.01
    assert r["peak"] == 2500.0 and abs(r["frac"] - r["achieved"] / 2500.0) < 1e-4
    assert bench.mfma_share({}, "conv_block", 544, 960, 64, 8, "fp8") is None
    assert bench.mfma_share({"conv_block": (1, 1.0)}, "conv_block", 8, 8, 64, 8, "fp8-fusion")["peak"] == 5000.0
