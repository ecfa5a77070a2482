#!/usr/bin/env python3
"""Throughput of the NNVISR frame-group enhancement path on one MI355X.

One step = one 120-frame 960x540 8-bit 4:2:0 clip (scene cut every 20-40 frames)
pushed through a clip stream: unpack, scene metric, extract, and for every group
the offset head, DCNv2 alignment, x2 reconstruction of two output frames and
requantisation -- 240 output frames of 1920x1080.  Inputs are staged in HBM before
the timed region; outputs stay in HBM.

Prints one JSON line: output Mpix/s, the dominant kernel against its roofline
(per-launch HIP-event timing recorded by the library on the launch stream), and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# HBM bytes per launch of the FP32 residual-block conv (the two launch kinds of a block
# averaged, as the kernel timing is), from rocprofv3 FETCH_SIZE / WRITE_SIZE counters
# scaled by a plain device copy's readings (x2.00 and x1.00); the command lines and the
# per-kernel table are in profiles/c2_fp32_hbm_traffic.md.  Valid only for the device
# source the counters were taken on: "source" is the hash of the conv kernels' files
# (conv_source_hash), and the bench reports no traffic when it differs.
FP32_CONV_BLOCK_TRAFFIC = {
    "first conv (LReLU)": {"fetch_kib": 69840, "write_kib": 130600},
    "second conv (+ skip)": {"fetch_kib": 135500, "write_kib": 130600},
    "fetch_scale": 2.00, "write_scale": 1.00,
    "tile": "pb2w2",   # the tile the tuner chose for the counted launches
    "source": "c23dfa6b5efa41a8",
}
CONV_SOURCES = ("k_net.hip", "nv_mma.h", "nv_device.h")


def conv_source_hash():
    """First 16 hex digits of the SHA-256 of the conv kernels' device sources."""
    import hashlib
    h = hashlib.sha256()
    for f in CONV_SOURCES:
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2308_03121_amd", "csrc", f),
                  "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_valid(tuning_line):
    """The stored counters apply: same device source and the same block tile."""
    t = FP32_CONV_BLOCK_TRAFFIC
    return t["source"] == conv_source_hash() and f"[block {t['tile']}," in tuning_line


def conv_block_traffic():
    t = FP32_CONV_BLOCK_TRAFFIC
    kinds = [v for v in t.values() if isinstance(v, dict)]
    per = [1024 * (k["fetch_kib"] * t["fetch_scale"] + k["write_kib"] * t["write_scale"]) for k in kinds]
    return sum(per) / len(per)


PEAKS = {"fp32": 157.3, "fp16": 2500.0, "bf16": 2500.0, "fp8": 5000.0, "fp8-fusion": 5000.0}   # dense TFLOP/s
HBM_PEAK_GBS = 8000.0


def conv_flops(px, cin, cout):
    return 2.0 * px * cin * cout * 9


def kernel_work(kind, hp, wp, C, G, bits_out_bytes):
    """Algorithmic flops (or bytes) of one launch of each kernel kind at padded size hp x wp."""
    px = hp * wp
    if kind == "conv_block":
        return conv_flops(px, C, C), "flop"
    if kind == "conv_in":
        return conv_flops(px, 3, C), "flop"
    if kind == "off1":
        return conv_flops(px, 2 * C, C), "flop"
    if kind == "off2":
        return conv_flops(px, C, 27 * G), "flop"
    if kind == "dcn":
        return conv_flops(px, 2 * C, C), "flop"
    if kind == "up":
        return conv_flops(px, C, 4 * C), "flop"
    if kind == "hr":
        return conv_flops(4 * px, C, 3), "flop"
    return None, None


def mfma_peak(kind, prec):
    """Dense peak (TFLOP/s) of the MFMA type a conv kind runs on in a precision mode: FP32
    everything on float MFMA; 16-bit modes on their 16-bit MFMA (the offset head too, as
    float-class products of float16 parts); FP8 puts the residual-block convs on e4m3 and
    the rest on float16, FP8-fusion also the DCN and the pixel-shuffle conv."""
    if prec == "fp32":
        return PEAKS["fp32"]
    if prec == "fp8" and kind == "conv_block":
        return PEAKS["fp8"]
    if prec == "fp8-fusion" and kind in ("conv_block", "dcn", "up"):
        return PEAKS["fp8"]
    return PEAKS["fp16"]


MFMA_KINDS = ("conv_block", "off1", "off2", "dcn", "up", "hr")


def mfma_share(pr, kind, hp, wp, C, G, prec):
    """Achieved TFLOP/s of one kernel kind from a profile (launches, ms) and its share of
    the dense peak of the MFMA type it runs on."""
    n, tot = pr.get(kind, (0, 0.0))
    flop, unit = kernel_work(kind, hp, wp, C, G, 0)
    if not n or unit != "flop":
        return None
    us = 1000.0 * tot / n
    tf = flop / (us * 1e-6) / 1e12
    peak = mfma_peak(kind, prec)
    return {"kernel": kind, "avg_launch_us": round(us, 2), "achieved": round(tf, 2), "peak": peak,
            "unit": "TFLOP/s", "frac": round(tf / peak, 4)}


def mfma_shares(pr, hp, wp, C, G, prec):
    """mfma_share of every MFMA conv kind in the profile: {kind: frac}."""
    out = {}
    for kind in MFMA_KINDS:
        r = mfma_share(pr, kind, hp, wp, C, G, prec)
        if r is not None:
            out[kind] = r["frac"]
    return out


def pixel_bytes(kind, w, h, bits, chroma):
    """Algorithmic HBM bytes of one launch of a pixel-format / scene stage on a w x h
    input frame: unpack reads the codes and writes float R'G'B' at the padded size; the
    scene metric reads the luma of the frame and of its predecessor; pack reads the float
    R'G'B' of one 2w x 2h output frame and writes its codes."""
    bps = 1 if bits == 8 else 2
    per_px = 1.5 if chroma == 420 else 3.0
    hp, wp = (h + 7) // 8 * 8, (w + 7) // 8 * 8
    if kind == "unpack":
        return w * h * bps * per_px + 12 * hp * wp
    if kind == "scene":
        return 2 * w * h * bps
    if kind == "pack":
        return 4 * w * h * (12 + bps * per_px)
    return None


def pixel_rates(prof, steps, w, h, bits, chroma):
    """GB/s and fraction of the 8 TB/s HBM peak of the pixel stages from a profile."""
    out = {}
    for kind in ("unpack", "scene", "pack"):
        n, tot = prof.get(kind, (0, 0.0))
        if not n:
            continue
        us = 1000.0 * tot / n
        gbs = pixel_bytes(kind, w, h, bits, chroma) / (us * 1e3)
        out[kind] = {"avg_us": round(us, 2), "bytes_per_launch": int(pixel_bytes(kind, w, h, bits, chroma)),
                     "gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def batched_pixel_rates(prof, clips, frames_per_clip):
    """GB/s of the batched pixel stages of one batch: every clip's frames unpacked and
    scene-measured in one launch each, and one output frame per group packed per launch
    (frames_per_clip - 1 groups per clip)."""
    n_groups = frames_per_clip - 1
    per_launch = {
        "unpack": sum(frames_per_clip * pixel_bytes("unpack", *c) for c in clips),
        "scene": sum(frames_per_clip * pixel_bytes("scene", *c) for c in clips),
        "pack": sum(n_groups * pixel_bytes("pack", *c) for c in clips),
    }
    out = {}
    for kind, nbytes in per_launch.items():
        n, tot = prof.get(kind, (0, 0.0))
        if not n:
            continue
        us = 1000.0 * tot / n
        gbs = nbytes / (us * 1e3)
        out[kind] = {"avg_us": round(us, 2), "bytes_per_launch": int(nbytes), "gbs": round(gbs, 1),
                     "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def device_copy_gbs(torch, mib=1024, reps=10):
    """Measured device-to-device copy rate (read + write bytes per second), the
    achievable HBM figure quoted beside the 8 TB/s specification."""
    a = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1000.0 / reps
    del a, b
    return round(2 * mib * (1 << 20) / s / 1e9, 1)


def conv_block_bytes(hp, wp, C, elem=4):
    """Algorithmic HBM bytes of a residual-block conv launch, the two kinds averaged: the
    first reads its input and writes its output, the second also reads the skip."""
    m = hp * wp * C * elem
    return (2 * m + 3 * m) // 2


def group_flops_per_px(C, R, G):
    """Network flops per padded LR pixel of one stream group (one extract, two outputs)."""
    extract = 2 * 9 * 3 * C + R * 2 * (2 * 9 * C * C)
    fusion = 2 * 9 * 2 * C * C + 2 * 9 * C * 27 * G + 2 * 9 * 2 * C * C
    per_out = 2 * 9 * C * 4 * C + 4 * 2 * 9 * C * 3
    return extract + fusion + 2 * per_out


def cpu_baseline(clip, blob, cfg, budget_s=20.0):
    """The FP64 oracle on the first two frames of the clip, top-left crop, growing the crop
    until one run takes a few seconds (bounded by budget_s of total CPU work)."""
    from threadpoolctl import threadpool_info

    import synth
    from oracle import pipeline

    W = pipeline.weights_dict(blob, synth.weight_layout(cfg))
    crops = [(32, 64), (64, 120), (136, 240), (272, 480)]
    spent, best = 0.0, None
    for h, w in crops:
        frames = [(clip.Y[t][:h, :w], clip.U[t][:h // 2, :w // 2], clip.V[t][:h // 2, :w // 2])
                  for t in range(2)]
        t0 = time.perf_counter()
        _cuts, outs = pipeline.enhance_clip(frames, clip.bits, clip.chroma, W, cfg.res_blocks,
                                            cfg.offset_groups)
        dt = time.perf_counter() - t0
        spent += dt
        mpix = len(outs) * (2 * h) * (2 * w) / 1e6
        best = {"value": mpix / dt, "unit": "output Mpix/s", "seconds": dt,
                "sample": f"oracle enhance_clip on frames 0-1 of the clip cropped to {w}x{h} "
                          f"({len(outs)} output frames of {2 * w}x{2 * h}, {mpix:.3f} Mpix)"}
        if dt > budget_s / 4 or spent + 4 * dt > budget_s:
            break
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    best["cores"] = int(threads)
    best["kind"] = "oracle"
    best["os_cpu_count"] = os.cpu_count()
    best["cpu_model"] = cpu_model()
    # the same sample on one thread
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        pipeline.enhance_clip(frames, clip.bits, clip.chroma, W, cfg.res_blocks, cfg.offset_groups)
        dt1 = time.perf_counter() - t0
    best["single_thread"] = {"value": mpix / dt1, "unit": "output Mpix/s", "seconds": dt1, "cores": 1}
    return best


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def c1_group_bench(B, synth, torch, reps=50):
    """One frame group of two 64x64 8-bit 4:2:0 frames through nv_enhance_group (plain
    FP32, C=32, R=2, G=8): 3 output frames of 128x128; latency per group from the
    median of `reps` timed calls (inputs resident, device events on the stream)."""
    clip = synth.gen_group_c1()
    cfg = synth.NET_C1
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, synth.gen_weights(cfg, seed=1))
    tune = ctx.autotune(64, 64)     # tiles for this size: at 64x64 a launch fills few CUs
    fmt = B.fmt_struct(64, 64, 8, 420)
    fa, fb = B.to_device_frame(*clip.frame(0)), B.to_device_frame(*clip.frame(1))
    outs = [B.alloc_frame(128, 128, 8, 420) for _ in range(3)]
    for _ in range(5):
        ctx.enhance_group(fmt, fa, fb, outs=outs)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.enhance_group(fmt, fa, fb, outs=outs)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) * 1000.0)
    ctx.close()
    us = float(np.median(times))
    return {"workload": "one group of two 64x64 8-bit 4:2:0 frames, C=32 R=2 G=8, FP32",
            "latency_us": round(us, 1), "output_mpix_per_s": round(3 * 128 * 128 / us, 2), "reps": reps,
            "tuning": tune}


def c3_precision_bench(B, synth, torch, cfg, blob, precs=("fp32", "fp16", "bf16", "fp8", "fp8-fusion"), steps=2):
    """The 48-frame 1920x1080 10-bit 4:2:0 clip (cuts at 16 and 32) pushed through a
    stream in each precision: 96 output frames of 3840x2160 per step.  fp8 quantises the
    residual trunk; fp8-fusion also the DCN and pixel-shuffle conv (below the 50 dB bar
    on this network, reported for speed only)."""
    clip = synth.gen_clip_c3()
    fmt = B.fmt_struct(clip.width, clip.height, clip.bits, clip.chroma)
    frames = [B.to_device_frame(*clip.frame(t)) for t in range(clip.n_frames)]
    outs = [B.alloc_frame(2 * clip.width, 2 * clip.height, clip.bits, clip.chroma) for _ in range(2 * clip.n_frames)]
    hp, wp = (clip.height + 7) // 8 * 8, (clip.width + 7) // 8 * 8
    mpix = 2 * clip.n_frames * 4 * clip.width * clip.height / 1e6
    res = {"workload": "48-frame 1920x1080 10-bit 4:2:0 clip, cuts at 16 and 32, C=64 R=10 G=8",
           "output_mpix_per_step": round(mpix, 2)}
    for prec in precs:
        ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision=prec.split("-")[0],
                        fp8_fusion=prec == "fp8-fusion")
        ctx.autotune(hp, wp)
        if prec.startswith("fp8"):
            ctx.calibrate(fmt, frames[:4])
        st = ctx.open_stream(fmt)

        def run():
            st.reset()
            for t in range(clip.n_frames):
                o = outs[2 * (t - 1):2 * t] if t > 0 else outs[0:2]
                st.push(frames[t], outs=o)
            st.end(outs=outs[2 * clip.n_frames - 2:])

        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            run()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1000.0
        # kernel breakdown from one more pass, so the timed steps carry no launch events
        ctx.profile(True)
        run()
        torch.cuda.synchronize()
        pr = ctx.profile_read()
        ctx.profile(False)
        cuts = [t for t, c in enumerate(st.cuts()) if c]
        res[prec] = {"value": round(mpix / (ms / 1000.0), 3), "unit": "Mpix/s", "ms_per_step": round(ms, 2),
                     "cuts": cuts,
                     "kernel_ms_per_step": {k: round(v[1], 2) for k, v in pr.items() if v[0]},
                     "conv_block_mfma": mfma_share(pr, "conv_block", hp, wp, cfg.channels, cfg.offset_groups, prec),
                     "mfma_frac": mfma_shares(pr, hp, wp, cfg.channels, cfg.offset_groups, prec),
                     "meets_50db_bar": prec != "fp8-fusion"}
        if prec == "fp8-fusion":
            res[prec]["note"] = ("below the 50 dB PSNR bar against the FP64 oracle (worst 1920x1080 window "
                                 "about 46 dB, test_gpu_fp8 bar 44 dB): a speed figure only")
        if "pixel_stages" not in res:
            res["pixel_stages"] = pixel_rates(pr, 1, clip.width, clip.height, clip.bits, clip.chroma)
        print(f"# c3 {prec}: {res[prec]['value']} Mpix/s", file=sys.stderr, flush=True)
        st.close()
        ctx.close()
    if "fp32" in res:
        for prec in precs:
            if prec != "fp32" and prec in res:
                res[prec]["speedup_vs_fp32"] = round(res[prec]["value"] / res["fp32"]["value"], 3)
    return res


def _frame_bank(B, synth, w, h, bits, chroma, scenes=2, per=4, seed=0):
    """Device frames of a few scenes of one format (synthetic clip, cut between scenes)."""
    clip = synth.gen_clip(w, h, scenes * per, bits=bits, chroma=chroma, seed=seed,
                          scene_starts=[per * k for k in range(1, scenes)])
    frames = [B.to_device_frame(*clip.frame(t)) for t in range(clip.n_frames)]
    return [frames[k * per:(k + 1) * per] for k in range(scenes)]


def batching_bench(B, synth, torch, reps=3):
    """64 frame groups from 16 clips (4 consecutive groups each, the frame store of a
    5-frame chain) of mixed sizes and formats in one batched call, FP16 (and FP8) network
    C=64, R=6, tiles from the autotuner, graph replay; against the same groups one at a
    time in FP32."""
    rng = np.random.default_rng(2)
    sizes = [(640, 360), (960, 540), (1280, 720)]
    fmts = [(8, 420), (10, 420), (8, 444), (10, 444)]
    clips = []
    for i in range(16):
        w, h = sizes[rng.integers(3)]
        b, c = fmts[rng.integers(4)]
        clips.append((w, h, b, c))
    banks = {}
    for (w, h, b, c) in set(clips):
        banks[(w, h, b, c)] = _frame_bank(B, synth, w, h, b, c, scenes=1, per=5, seed=w + b + c)[0]
    cfg = synth.NET_C4
    blob = synth.gen_weights(cfg, seed=1)
    res = {}
    mpix = sum(4 * 2 * (2 * w) * (2 * h) for (w, h, _b, _c) in clips) / 1e6
    for prec in ("fp16", "fp8", "fp32"):
        ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision=prec)
        tune = ctx.autotune(544, 960)
        if prec == "fp8":
            w0, h0, b0, c0 = clips[0]
            ctx.calibrate(B.fmt_struct(w0, h0, b0, c0), banks[clips[0]])
        streams = [ctx.open_stream(B.fmt_struct(w, h, b, c)) for (w, h, b, c) in clips]

        def one_batch():
            for st in streams:
                st.reset()
                st.n_pushed = 0
            ctx.enhance_batch([(st, banks[k], None, False) for st, k in zip(streams, clips)])

        def one_at_a_time():
            for st, k in zip(streams, clips):
                st.reset()
                st.n_pushed = 0
                for f in banks[k]:
                    st.push(f)

        runs = {"batched_graph": one_batch} if prec != "fp32" else {"one_at_a_time": one_at_a_time}
        if prec == "fp16":
            runs["one_at_a_time"] = one_at_a_time
        for name, fn in runs.items():
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            res[f"{prec}_{name}"] = {"ms": round(dt * 1000, 2), "mpix_per_s": round(mpix / dt, 1)}
        if prec == "fp16":
            res["fp16_tuning"] = tune
            res["batch_workspace_gb"] = round(ctx.batch_footprint() / 2 ** 30, 2)
            # the batched pixel stages over every frame of the batch in one launch each,
            # timed with the library's events (launched directly, not replayed)
            ctx.batch_graph(False)
            ctx.profile(True)
            one_batch()
            torch.cuda.synchronize()
            prof = ctx.profile_read()
            ctx.profile(False)
            ctx.batch_graph(True)
            res["pixel_stages_batched"] = batched_pixel_rates(prof, clips, len(banks[clips[0]]))
        for st in streams:
            st.close()
        ctx.close()
    res["groups"] = 64
    res["output_mpix"] = round(mpix, 2)
    res["clips"] = [f"{w}x{h} {b}-bit {c}" for (w, h, b, c) in clips]
    res["speedup_fp16_batched_vs_fp32_single"] = round(
        res["fp32_one_at_a_time"]["ms"] / res["fp16_batched_graph"]["ms"], 2)
    res["speedup_fp8_batched_vs_fp32_single"] = round(
        res["fp32_one_at_a_time"]["ms"] / res["fp8_batched_graph"]["ms"], 2)
    return res


def next_rows_bench(B, synth, torch, n_frames=12, reps=3):
    """Throughput of the wider rows on a 12-frame 960x540 clip (cut at frame 8), FP16
    network C=64, R=10, G=8, tiles tuned per context: the feature pyramid (2 and 3
    levels) and the task modes through clip streams, a BT.2020 full-range 10-bit clip
    through the network of its colourspace, and a general-n clip (n = 3, b = 2); each
    against the same clip through the one-level space-time network."""
    clip8 = synth.gen_clip(960, 540, n_frames, seed=5, scene_starts=[8])
    clip10 = synth.gen_clip(960, 540, n_frames, bits=10, seed=5, scene_starts=[8])
    f8 = [B.to_device_frame(*clip8.frame(t)) for t in range(n_frames)]
    f10 = [B.to_device_frame(*clip10.frame(t)) for t in range(n_frames)]
    w, h = 960, 540
    res = {"workload": f"{n_frames}-frame 960x540 4:2:0 clip, cut at 8, FP16 C=64 R=10 G=8"}

    def timed(go):
        go()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            go()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def stream_run(ctx, fmt, frames):
        st = ctx.open_stream(fmt)

        def go():
            st.reset()
            n = 0
            for f in frames:
                n += len(st.push(f))
            n += len(st.end())
            return n
        dt = timed(go)
        n_out = go()
        torch.cuda.synchronize()
        st.close()
        return dt, n_out

    def record(name, dt, n_out, sv, sh, extra=None):
        mpix = n_out * sv * h * sh * w / 1e6
        res[name] = {"mpix_per_s": round(mpix / dt, 1), "ms_per_input_frame": round(1000 * dt / n_frames, 3),
                     "outputs": n_out}
        if extra:
            res[name].update(extra)

    blob_cache = {}

    def context(**kw):
        levels = kw.get("levels", 1)
        cfg = synth.NetConfig(64, 10, 8, scale=kw.get("scale", 2), scale_v=kw.get("scale_v", 0),
                              interp=kw.get("interp", True), double=kw.get("double", True), levels=levels)
        if cfg not in blob_cache:
            blob_cache[cfg] = synth.gen_weights(cfg, seed=1)
        ctx = B.Context(64, 10, 8, blob_cache[cfg], precision="fp16", **kw)
        ctx.autotune(544, 960)
        return ctx, cfg

    fmt8 = B.fmt_struct(w, h, 8, 420)
    for name, kw in (("space_time", {}), ("pyramid_2_levels", {"levels": 2}), ("pyramid_3_levels", {"levels": 3}),
                     ("denoise_x1", {"scale": 1, "interp": False}), ("sr_x2", {"scale": 2, "interp": False}),
                     ("deinterlace", {"scale": 1, "scale_v": 2, "interp": False}),
                     ("interp_pass_through", {"scale": 1, "double": False})):
        ctx, cfg = context(**kw)
        dt, n_out = stream_run(ctx, fmt8, f8)
        record(name, dt, n_out, cfg.sv, cfg.sh)
        if name == "space_time":
            # the general-n clip: n = 3 frames per run, b = 2 groups per batch
            def go_clip(cl):
                n = 0
                for f in f8:
                    n += len(cl.push(f))
                return n + len(cl.end())
            for timed_run in (False, True):      # a warm-up clip, then a timed one
                cl = B.Clip(ctx, fmt8, 3, 2)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                n_clip = go_clip(cl)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                cl.close()
            record("general_n3_b2", dt, n_clip, 2, 2)
        ctx.close()
    ctx = B.Context(64, 10, 8, blob_cache[synth.NetConfig(64, 10, 8)], precision="fp16", matrix=2020, full=True)
    ctx.autotune(544, 960)
    dt, n_out = stream_run(ctx, B.fmt_struct(w, h, 10, 420, matrix=2020, full=True), f10)
    record("bt2020_full_range_10bit", dt, n_out, 2, 2)
    ctx.close()
    return res


def serving_bench(B, synth, torch, duration=20.0, rate=40.0, budget_gb=240, tight_budget_gb=96,
                  max_batch_mpx=16.0):
    """16 streams (540p/1080p, 8/10-bit 4:2:0, 30-300 frames, cuts every 10-60 frames)
    whose frames arrive as Poisson processes totalling `rate` groups/s, truncated at
    `duration` seconds of arrivals; FP16 network C=64, R=10; admission by HBM footprint
    (stream state plus a full chain's share of the batch pools).  With budget_gb (most of
    the 288 GB card) every stream is admitted on arrival; the same arrivals under
    tight_budget_gb show the admission queue at work."""
    from paper_2308_03121_amd.serving import GpuExecutor, Server, poisson_workload

    specs = poisson_workload(n_streams=16, rate_total=rate, seed=3, max_time=duration)
    # each stream its own content: two generated scenes of six frames (its own fields,
    # textures and motion), alternating at the stream's cuts, a scene's frames cycled
    banks = {s.sid: _frame_bank(B, synth, s.width, s.height, s.bits, s.chroma, scenes=2, per=6, seed=100 + s.sid)
             for s in specs}

    def source(spec, t):
        k = sum(1 for c in spec.scene_starts if c <= t)
        start = ([0] + [c for c in spec.scene_starts if c <= t])[-1]
        scene = banks[spec.sid][k % 2]
        return scene[(t - start) % len(scene)]

    cfg = synth.NET_C2
    ctx = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, synth.gen_weights(cfg, seed=1),
                    precision="fp16")
    ctx.autotune(544, 960)
    out = {}
    saturation = [type(s)(s.sid, s.width, s.height, s.bits, s.chroma, [0.0] * s.n_frames, s.scene_starts)
                  for s in specs]
    for label, sp, gb in (("poisson", specs, budget_gb), ("saturation", saturation, budget_gb),
                          ("poisson_tight_budget", specs, tight_budget_gb)):
        ex = GpuExecutor(ctx, source, max_chain=4)   # admission counts the batch pools too
        srv = Server(ex, hbm_budget=int(gb * 2 ** 30), max_chain=4, max_batch_px=int(max_batch_mpx * 1e6))
        rep = srv.run(sp)
        torch.cuda.synchronize()
        ex.shutdown()
        out[label] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in rep.items()}
    out["streams"] = len(specs)
    out["frames"] = sum(s.n_frames for s in specs)
    out["arrival_rate_groups_per_s"] = rate
    out["hbm_budget_gb"] = budget_gb
    out["tight_hbm_budget_gb"] = tight_budget_gb
    out["max_batch_lr_mpx"] = max_batch_mpx
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=sorted(PEAKS) + ["fp8-fusion"])
    ap.add_argument("--frames", type=int, default=120)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--also", default="fp16,bf16,fp8",
                    help="other precisions timed on the same clip after the main run ('' for none)")
    ap.add_argument("--no-c3", action="store_true", help="skip the 1080p 10-bit per-precision run")
    ap.add_argument("--c3-precisions", default="fp32,fp16,bf16,fp8,fp8-fusion",
                    help="precisions of the 1080p 10-bit run (comma list)")
    ap.add_argument("--no-batching", action="store_true", help="skip the 64-group batching run")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the pyramid / task-mode / colourspace / general-n throughput leg")
    ap.add_argument("--serving-seconds", type=float, default=20.0)
    ap.add_argument("--copy-only", type=int, default=0, metavar="MIB",
                    help="only run a device copy of MIB MiB 10 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the path needs no collective and runs on a "
              f"single MI355X (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2308_03121_amd import binding as B

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_only:
        # a plain copy of known size: FETCH_SIZE / WRITE_SIZE per dispatch of this kernel
        # calibrate the counters against bytes actually moved
        n = args.copy_only * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}), flush=True)
        return
    print(f"# generating the 960x540 clip ({args.frames} frames)", file=sys.stderr, flush=True)
    clip = synth.gen_clip_c2(n_frames=args.frames)
    cfg = synth.NET_C2
    blob = synth.gen_weights(cfg, seed=1)
    W_, H_ = clip.width, clip.height
    fmt = B.fmt_struct(W_, H_, clip.bits, clip.chroma)
    frames = [B.to_device_frame(*clip.frame(t)) for t in range(clip.n_frames)]
    outs = [B.alloc_frame(2 * W_, 2 * H_, clip.bits, clip.chroma) for _ in range(2 * clip.n_frames)]
    hp, wp = (H_ + 7) // 8 * 8, (W_ + 7) // 8 * 8

    tuning = {}

    def make(prec):
        c = B.Context(cfg.channels, cfg.res_blocks, cfg.offset_groups, blob, precision=prec.split("-")[0],
                      fp8_fusion=prec == "fp8-fusion")
        tuning[prec] = c.autotune(hp, wp)
        if prec.startswith("fp8"):
            c.calibrate(fmt, frames[:4])
        return c, c.open_stream(fmt)

    def run_clip(st):
        st.reset()
        for t in range(clip.n_frames):
            o = outs[2 * (t - 1):2 * t] if t > 0 else outs[0:2]
            st.push(frames[t], outs=o)
        st.end(outs=outs[2 * clip.n_frames - 2:])

    ctx, st = make(args.precision)

    def step():
        run_clip(st)

    print(f"# warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    print(f"# timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
        torch.cuda.synchronize()
        print(f"# step {k} done", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    cuts = st.cuts()
    ms = (t1 - t0) / args.steps * 1000.0
    n_out = 2 * clip.n_frames
    mpix = n_out * (2 * W_) * (2 * H_) / 1e6
    value = mpix / (ms / 1000.0)

    kernels = {}
    for kind, (n, tot) in prof.items():
        if n == 0:
            continue
        work, unit = kernel_work(kind, hp, wp, cfg.channels, cfg.offset_groups, 1)
        ent = {"launches": n, "avg_us": round(1000.0 * tot / n, 2), "total_ms_per_step": round(tot / args.steps, 2)}
        if work is not None:
            tf = work / (tot / n / 1000.0) / 1e12
            ent.update({"tflops": round(tf, 2), "frac": round(tf / PEAKS[args.precision], 4)})
        kernels[kind] = ent
    dom = max((k for k in kernels if "tflops" in kernels[k]), key=lambda k: kernels[k]["total_ms_per_step"])
    dom_work, _ = kernel_work(dom, hp, wp, cfg.channels, cfg.offset_groups, 1)
    achieved = kernels[dom]["tflops"]
    path_flop = group_flops_per_px(cfg.channels, cfg.res_blocks, cfg.offset_groups) * hp * wp * clip.n_frames
    rec = {
        "metric": "output Mpix/s (960x540 -> 1920x1080 x2 frame rate, FP64-oracle parity)",
        "value": round(value, 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32"}.get(args.precision, args.precision),
        "data": "synthetic",
        "config": {"workload": "120-frame 960x540 8-bit 4:2:0 clip, cut every 20-40 frames, "
                               "network C=64 R=10 G=8, x2 space and time",
                   "frames_in": clip.n_frames, "frames_out": n_out, "precision": args.precision,
                   "cuts_detected": [t for t, c in enumerate(cuts) if c]},
        "roofline": {"bound": "mfma", "kernel": f"{dom} ({'3x3 conv 64->64' if dom == 'conv_block' else dom})",
                     "achieved": achieved, "peak": PEAKS[args.precision], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAKS[args.precision], 4),
                     "traffic": (round(conv_block_traffic())
                                 if args.precision == "fp32" and dom == "conv_block"
                                 and traffic_valid(tuning[args.precision])
                                 else None),
                     "traffic_algorithmic": (conv_block_bytes(hp, wp, cfg.channels) if dom == "conv_block"
                                             else None),
                     "flop_per_launch": dom_work, "avg_launch_us": kernels[dom]["avg_us"]},
        "path": {"tflop_per_step": round(path_flop / 1e12, 2),
                 "tflops": round(path_flop / (ms / 1000.0) / 1e12, 2),
                 "frac_of_peak": round(path_flop / (ms / 1000.0) / 1e12 / PEAKS[args.precision], 4)},
        "kernels": kernels,
        "pixel_stages": pixel_rates(prof, args.steps, W_, H_, clip.bits, clip.chroma),
        "hbm_copy_gbs": device_copy_gbs(torch),
    }
    others = {}
    for prec in [p for p in args.also.split(",") if p and p != args.precision]:
        print(f"# timing {prec}", file=sys.stderr, flush=True)
        c2, st2 = make(prec)
        for _ in range(max(1, args.warmup)):
            run_clip(st2)
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        for _ in range(args.steps):
            run_clip(st2)
        torch.cuda.synchronize()
        a1 = time.perf_counter()
        c2.profile(True)
        run_clip(st2)
        torch.cuda.synchronize()
        pr = c2.profile_read()
        c2.profile(False)
        ms2 = (a1 - a0) / args.steps * 1000.0
        others[prec] = {"value": round(mpix / (ms2 / 1000.0), 3), "ms_per_step": round(ms2, 3),
                        "speedup_vs_" + args.precision: round(ms / ms2, 3),
                        "kernel_ms_per_step": {k: round(v[1], 2) for k, v in pr.items() if v[0]},
                        "conv_block_mfma": mfma_share(pr, "conv_block", hp, wp, cfg.channels, cfg.offset_groups,
                                                      prec),
                        "mfma_frac": mfma_shares(pr, hp, wp, cfg.channels, cfg.offset_groups, prec)}
        st2.close()
        c2.close()
    rec["tuning"] = tuning
    if others:
        rec["other_precisions"] = others
        print("# other precisions: " + json.dumps(others), file=sys.stderr, flush=True)
    print("# C1: one 64x64 group", file=sys.stderr, flush=True)
    try:
        rec["c1_group"] = c1_group_bench(B, synth, torch)
    except Exception as e:
        rec["c1_group"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_c3:
        print("# precisions on the 48-frame 1920x1080 10-bit clip", file=sys.stderr, flush=True)
        try:
            rec["c3_precisions"] = c3_precision_bench(B, synth, torch, cfg, blob,
                                                      precs=tuple(p for p in args.c3_precisions.split(",") if p))
        except Exception as e:
            rec["c3_precisions"] = {"error": f"{type(e).__name__}: {e}"}
        print("# c3: " + json.dumps(rec["c3_precisions"]), file=sys.stderr, flush=True)
    if not args.no_batching:
        print("# batching: 64 groups of mixed clips", file=sys.stderr, flush=True)
        try:
            rec["batching"] = batching_bench(B, synth, torch)
        except Exception as e:  # report, keep the main measurement
            rec["batching"] = {"error": f"{type(e).__name__}: {e}"}
        print("# batching: " + json.dumps(rec["batching"]), file=sys.stderr, flush=True)
    if not args.no_next:
        print("# wider rows: pyramid, task modes, colourspace, general n", file=sys.stderr, flush=True)
        try:
            rec["next_rows"] = next_rows_bench(B, synth, torch)
        except Exception as e:
            rec["next_rows"] = {"error": f"{type(e).__name__}: {e}"}
        print("# next rows: " + json.dumps(rec["next_rows"]), file=sys.stderr, flush=True)
    if not args.no_serving:
        print("# serving: Poisson arrivals of 16 streams", file=sys.stderr, flush=True)
        try:
            rec["serving"] = serving_bench(B, synth, torch, duration=args.serving_seconds)
        except Exception as e:
            rec["serving"] = {"error": f"{type(e).__name__}: {e}"}
        print("# serving: " + json.dumps(rec["serving"]), file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("# timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(clip, blob, cfg)
    st.close()
    ctx.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
