"""The library's kernels and host runtime executed on the CPU (tests/cpusim/).

api.cpp, k_net.hip, k_dcn.hip, k_pyr.hip and k_pixel.hip are compiled as host C++ under AddressSanitizer
against a simulated HIP device: every work-item runs as a
fiber, __syncthreads() and the wave-wide operations (MFMA in each form the kernels use,
lane shuffles, readfirstlane) are rendezvous points, __shared__ arrays are statics, and
device memory is heap memory pre-filled with a non-zero pattern.  Any out-of-bounds
global or LDS access is an ASan report; a barrier that a live work-item never reaches,
or a wave operation not joined by every live lane, is reported as a hang (exit 3).
The MFMA forms are emulated from their documented lane layouts in float64, so results
are compared with the FP64 oracle at the GPU tests' float bar.

The 64x64, C = 64, R = 2 network case is the one kept off the GPU after a run that went
silent; here it runs through the same entry points (nv_extract, nv_fuse) with the
context's default tiles.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from oracle import network
from tests._helpers import oracle_weights

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIM = os.path.join(ROOT, "tests", "cpusim")
CSRC = os.path.join(ROOT, "paper_2308_03121_amd", "csrc")
CXX = "/opt/rocm/llvm/bin/clang++"
FLOAT_TOL = 1e-4


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = CXX if os.path.exists(CXX) else shutil.which("clang++")
    if cxx is None:
        pytest.skip("no clang++ with _Float16 and __bf16 support for the simulation build")
    out = tmp_path_factory.mktemp("cpusim")
    common = ["-std=c++17", "-g0", "-Wno-psabi", "-I" + SIM, "-I" + os.path.join(ROOT, "include")]
    asan = ["-O1", "-fsanitize=address", "-fno-omit-frame-pointer"]
    # the library's sources are instrumented; the simulator itself (scheduler, MFMA
    # emulation) is optimised and uninstrumented
    units = [(os.path.join(CSRC, "k_net.hip"), True, asan), (os.path.join(CSRC, "k_dcn.hip"), True, asan),
             (os.path.join(CSRC, "k_pyr.hip"), True, asan), (os.path.join(CSRC, "k_pixel.hip"), True, asan),
             (os.path.join(CSRC, "api.cpp"), False, asan), (os.path.join(SIM, "sim.cpp"), False, ["-O2"]),
             (os.path.join(SIM, "driver.cpp"), False, asan)]
    procs, objs = [], []
    for src, as_cxx, opt in units:
        obj = str(out / (os.path.basename(src) + ".o"))
        cmd = [cxx] + common + opt + (["-x", "c++"] if as_cxx else []) + ["-c", src, "-o", obj]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        objs.append(obj)
    for p in procs:
        log = p.communicate()[0]
        assert p.returncode == 0, log[-4000:]
    exe = str(out / "driver")
    res = subprocess.run([cxx, "-fsanitize=address", "-o", exe] + objs, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    return exe


def _run(driver, args, timeout):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:detect_stack_use_after_return=0:abort_on_error=0"
    res = subprocess.run([driver] + [str(a) for a in args], capture_output=True, text=True, env=env,
                         timeout=timeout)
    out = res.stdout + res.stderr
    assert res.returncode != 3, "simulated hang:\n" + out[-4000:]
    assert res.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out, out[-4000:]
    return out


def _chw(path, dt, h, w, c):
    return np.fromfile(path, dtype=dt).reshape(h, w, c).astype(np.float64).transpose(2, 0, 1)


@pytest.mark.parametrize("C,R,G,H,W", [(64, 2, 8, 64, 64)], ids=["C64R2-64x64"])
def test_network_case_in_simulation(driver, tmp_path, C, R, G, H, W):
    cfg = synth.NetConfig(C, R, G)
    blob = synth.gen_weights(cfg, seed=1)
    blob.astype(np.float32).tofile(tmp_path / "weights.f32")
    rng = np.random.default_rng(H * W + C)
    ra = rng.uniform(0, 1, (3, H, W)).astype(np.float32)
    rb = np.clip(ra + rng.normal(0, 0.05, ra.shape), 0, 1).astype(np.float32)
    ra.tofile(tmp_path / "rgb_a.f32")
    rb.tofile(tmp_path / "rgb_b.f32")
    _run(driver, ["net", tmp_path, C, R, G, 0, H, W], timeout=900)

    Wd = oracle_weights(cfg, blob)
    ldo = 16 * ((27 * G + 15) // 16)
    fa = _chw(tmp_path / "fa.bin", np.float32, H, W, C)
    fb = _chw(tmp_path / "fb.bin", np.float32, H, W, C)
    offs = _chw(tmp_path / "offs.bin", np.float32, H, W, ldo)
    fmid = _chw(tmp_path / "fmid.bin", np.float32, H, W, C)
    a64, b64 = ra.astype(np.float64), rb.astype(np.float64)
    ofa, ofb = network.extract(a64, Wd, R), network.extract(b64, Wd, R)
    assert np.abs(fa - ofa).max() <= FLOAT_TOL
    assert np.abs(fb - ofb).max() <= FLOAT_TOL
    o_off, o_mask = network.offset_head(fa, fb, Wd, G)
    assert np.abs(offs[:18 * G] - o_off).max() <= FLOAT_TOL
    assert np.abs(offs[18 * G:27 * G] - o_mask).max() <= FLOAT_TOL
    o_fmid = network.align(fa, fb, offs[:18 * G], offs[18 * G:27 * G], Wd, G)
    assert np.abs(fmid - o_fmid).max() <= FLOAT_TOL
    full = network.fuse(a64, b64, ofa, ofb, Wd, G)
    for t, key in enumerate((0.0, 0.5, 1.0)):
        hr = np.fromfile(tmp_path / f"hr{t}.bin", dtype=np.float32).reshape(3, 2 * H, 2 * W)
        assert np.abs(hr - full[key]).max() <= FLOAT_TOL, t


@pytest.mark.parametrize("prec,off_gain", [(1, 1.0), (1, 12.0), (0, 1.0), (2, 12.0)],
                         ids=["fp16-window", "fp16-wide-offsets", "fp32-window", "bf16-wide-offsets"])
def test_dcn_window_form_bit_identical_in_simulation(driver, tmp_path, prec, off_gain):
    """The DCN forms that read a phase's sampling corners from an LDS copy of their
    window (tile code 2 | 16, the windowed form, and 1 | 32, the staged form, forced
    through the tuner's cache file) give the same bits as the plain form: with the
    generator's offsets (every phase fits its window) and with the offset conv's weights
    scaled up (wide offsets: phases fall back to reading the map), at a padded size with
    a ragged right tile."""
    C, R, G, H, W = 64, 1, 8, 40, 56
    cfg = synth.NetConfig(C, R, G)
    blob = synth.gen_weights(cfg, seed=3)
    w_off2, _b = synth.unpack_weights(cfg, blob)["off2"]
    w_off2 *= off_gain
    rng = np.random.default_rng(5)
    ra = rng.uniform(0, 1, (3, H, W)).astype(np.float32)
    rb = np.clip(ra + rng.normal(0, 0.05, ra.shape), 0, 1).astype(np.float32)
    outs = {}
    for code in (2, 2 | 16, 1 | 32):
        d = tmp_path / f"t{code}"
        d.mkdir()
        blob.astype(np.float32).tofile(d / "weights.f32")
        ra.tofile(d / "rgb_a.f32")
        rb.tofile(d / "rgb_b.f32")
        cache = d / "tune.txt"
        cache.write_text(f"prec={prec} C={C} R={R} size={W}x{H} | 2 2 {code} 2 2 0\n")
        env_cache = os.environ.get("NNVISR_TUNE_CACHE")
        os.environ["NNVISR_TUNE_CACHE"] = str(cache)
        try:
            out = _run(driver, ["net", d, C, R, G, prec, H, W], timeout=900)
        finally:
            if env_cache is None:
                del os.environ["NNVISR_TUNE_CACHE"]
            else:
                os.environ["NNVISR_TUNE_CACHE"] = env_cache
        assert "from cache" in out, out[-2000:]
        outs[code] = {k: (d / k).read_bytes() for k in ("offs.bin", "fmid.bin", "hr0.bin", "hr1.bin", "hr2.bin")}
    ldo = 16 * ((27 * G + 15) // 16)
    offs = np.frombuffer(outs[2]["offs.bin"], np.float32).reshape(H, W, ldo)[:, :, :18 * G]
    print("max |offset|", float(np.abs(offs).max()))
    for k in outs[2]:
        assert outs[2][k] == outs[2 | 16][k], k
        assert outs[2][k] == outs[1 | 32][k], k


def test_static_group_entry_in_simulation(driver):
    """nv_enhance_group_static is bit-identical to nv_enhance_group on two groups in a
    row (the second smaller) and rejects a group too large for its static scratch."""
    out = _run(driver, ["static", 32, 2, 8, 0], timeout=600)
    assert "static ok" in out, out[-2000:]


@pytest.mark.parametrize("w,h,bits,chroma", [(40, 24, 8, 420), (38, 22, 10, 420), (30, 18, 10, 444)])
def test_pixel_stage_colourspaces_in_simulation(driver, tmp_path, w, h, bits, chroma):
    """nv_unpack and nv_pack in every matrix, range and (4:2:0) siting against the oracle:
    unpack within 1e-6, pack codes within one code (rounding ties)."""
    from oracle import pixel
    rng = np.random.default_rng(w * h + bits)
    dt = np.uint8 if bits == 8 else np.uint16
    cw, chh = (w // 2, h // 2) if chroma == 420 else (w, h)
    mats = {709: 0, 601: 1, 2020: 2}
    for matrix in (601, 709, 2020):
        for full in (False, True):
            for centre in ((False, True) if chroma == 420 else (False,)):
                planes = [rng.integers(0, 1 << bits, s).astype(dt) for s in ((h, w), (chh, cw), (chh, cw))]
                for name, a in zip("yuv", planes):
                    a.tofile(tmp_path / f"{name}.bin")
                args = [w, h, bits, chroma, mats[matrix], int(full), int(centre)]
                _run(driver, ["unpack", tmp_path] + args, timeout=120)
                hp, wp = (h + 7) // 8 * 8, (w + 7) // 8 * 8
                got = np.fromfile(tmp_path / "rgb.f32", dtype=np.float32).reshape(3, hp, wp)
                ref = pixel.pad(pixel.unpack(*planes, bits, chroma, matrix, full, centre), 8)
                assert np.abs(got - ref).max() <= 1e-6, (matrix, full, centre)
                rw = (w + 3) // 4 * 4
                x = rng.uniform(-0.1, 1.1, (3, h, rw)).astype(np.float32)
                x.tofile(tmp_path / "rgb.f32")
                _run(driver, ["pack", tmp_path] + args, timeout=120)
                want = pixel.pack(x[:, :, :w].astype(np.float64), bits, chroma, matrix, full, centre)
                for name, r in zip("yuv", want):
                    g = np.fromfile(tmp_path / f"{name}.bin", dtype=dt).reshape(r.shape)
                    assert np.abs(g.astype(np.int64) - r.astype(np.int64)).max() <= 1, (name, matrix, full, centre)


def test_general_n_clip_in_simulation(driver):
    """nv_clip_* with n = 3, b = 2 over scenes of 1, 2, 3 and 7 frames: outputs
    bit-identical to nv_stream_push, groups equal to the oracle's grouping rules and the
    full block's store equal to the Fig. 1 layout."""
    from oracle import scene
    n, b, lengths = 3, 2, [1, 2, 3, 7]
    out = _run(driver, ["clip", 32, 1, 8, n, b, 32, 16, sum(lengths), 1, 3, 6], timeout=900)
    assert "clip ok" in out
    vals = [int(v) for v in out.split("trace:")[1].split("\n")[0].split()]
    P, i, got = n * b + b, 0, []
    while i < len(vals):
        kind, g = vals[i], vals[i + 1]
        i += 2
        got.append((kind, [vals[i + j * (n + 1):i + (j + 1) * (n + 1)] for j in range(g)], vals[i + g * (n + 1):
                                                                                               i + g * (n + 1) + P]))
        i += g * (n + 1) + P
    groups = [g["inputs"] for g in scene.groups_general(lengths, n, True)]
    assert [g for _k, gs, _s in got for g in gs] == groups
    assert [k for k, _g, _s in got] == [1, 1, 1, 0, 1]
    fig = [-1] * P
    for f, p in scene.frame_store_positions(n, b, 0).items():
        fig[p] = f + 6
    assert got[3][2] == fig


@pytest.mark.parametrize("scale,scale_v,flags", [(1, 0, 0), (2, 0, 0), (1, 2, 0), (1, 0, 3), (1, 0, 7), (2, 0, 7)],
                         ids=["denoise", "sr", "deinterlace", "interp-pass", "interp-denoise", "space-time"])
def test_task_modes_in_simulation(driver, tmp_path, scale, scale_v, flags):
    """A clip stream in each task of the end-user section against the oracle: every
    output frame within one code (pass-through frames identical to the inputs)."""
    from oracle import pipeline
    interp, double = bool(flags & 1), bool(flags & 4)
    cfg = synth.NetConfig(32, 1, 8, scale=scale, scale_v=scale_v, interp=interp, double=double)
    blob = synth.gen_weights(cfg, seed=5)
    blob.astype(np.float32).tofile(tmp_path / "weights.f32")
    T, W, H = 4, 32, 16
    clip = synth.gen_clip(W, H, T, seed=9, scene_starts=[2])
    frames = [clip.frame(t) for t in range(T)]
    for t, fr in enumerate(frames):
        for name, a in zip("yuv", fr):
            np.ascontiguousarray(a).tofile(tmp_path / f"f{t}_{name}.bin")
    out = _run(driver, ["task", tmp_path, 32, 1, 8, scale, scale_v, flags, W, H, T], timeout=900)
    n = int(out.split("outputs")[1].split()[0])
    _c, ref = pipeline.enhance_clip(frames, 8, 420, oracle_weights(cfg, blob), 1, 8, scale=(cfg.sv, cfg.sh),
                                    interp=interp, double=double)
    assert n == len(ref)
    for k, r in enumerate(ref):
        got = [np.fromfile(tmp_path / f"o{k}_{name}.bin", dtype=np.uint8).reshape(p.shape)
               for name, p in zip("yuv", r["codes"])]
        d = max(int(np.abs(g.astype(np.int64) - p.astype(np.int64)).max()) for g, p in zip(got, r["codes"]))
        assert d == 0 if r["hr"] is None else d <= 1, (k, d)


@pytest.mark.parametrize("levels", [2, 3])
def test_feature_pyramid_stream_in_simulation(driver, tmp_path, levels):
    """A clip stream of a network with a feature pyramid (space-time task) against the
    oracle's cascaded alignment: every output frame within one code."""
    from oracle import pipeline
    cfg = synth.NetConfig(32, 1, 8, levels=levels)
    blob = synth.gen_weights(cfg, seed=6)
    blob.astype(np.float32).tofile(tmp_path / "weights.f32")
    T, W, H = 3, 48, 32
    clip = synth.gen_clip(W, H, T, seed=10, scene_starts=[])
    frames = [clip.frame(t) for t in range(T)]
    for t, fr in enumerate(frames):
        for name, a in zip("yuv", fr):
            np.ascontiguousarray(a).tofile(tmp_path / f"f{t}_{name}.bin")
    out = _run(driver, ["task", tmp_path, 32, 1, 8, 2, 0, 7, W, H, T, levels], timeout=1200)
    n = int(out.split("outputs")[1].split()[0])
    _c, ref = pipeline.enhance_clip(frames, 8, 420, oracle_weights(cfg, blob), 1, 8, levels=levels)
    assert n == len(ref) == 2 * T
    for k, r in enumerate(ref):
        got = [np.fromfile(tmp_path / f"o{k}_{name}.bin", dtype=np.uint8).reshape(p.shape)
               for name, p in zip("yuv", r["codes"])]
        d = max(int(np.abs(g.astype(np.int64) - p.astype(np.int64)).max()) for g, p in zip(got, r["codes"]))
        assert d <= 1, (k, d)
