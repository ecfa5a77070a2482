"""Seeded synthetic Y'CbCr clips.

Each scene is a smooth random field (Gaussian-filtered white noise) plus a
texture of analytic sinusoids that translates by a per-scene velocity, so the
sub-pixel motion is exact.  Scenes change abruptly at generator-chosen frames,
which is the ground truth the scene-change tests compare against.

Code values are produced directly in the limited-range code space of the
chosen bit depth (luma nominal span [16, 235] << (bits-8), chroma centred at
128 << (bits-8)); no colour conversion happens here.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.ndimage import gaussian_filter


@dataclass
class Clip:
    Y: np.ndarray            # [N, H, W]   uint8 (8-bit) or uint16 (10-bit, LSB aligned)
    U: np.ndarray            # [N, Hc, Wc] Cb codes
    V: np.ndarray            # [N, Hc, Wc] Cr codes
    bits: int
    chroma: int              # 420 or 444
    scene_starts: list = field(default_factory=list)  # frames that begin a scene (0 included)

    @property
    def n_frames(self) -> int:
        return int(self.Y.shape[0])

    @property
    def height(self) -> int:
        return int(self.Y.shape[1])

    @property
    def width(self) -> int:
        return int(self.Y.shape[2])

    def frame(self, t: int):
        return self.Y[t], self.U[t], self.V[t]


def clip_format(clip: Clip) -> dict:
    return {"width": clip.width, "height": clip.height, "bits": clip.bits,
            "chroma": clip.chroma}


def smooth_field(rng: np.random.Generator, h: int, w: int, sigma: float) -> np.ndarray:
    """Unit-variance Gaussian-filtered white noise (periodic boundary)."""
    f = gaussian_filter(rng.standard_normal((h, w)), sigma=sigma, mode="wrap")
    f -= f.mean()
    s = f.std()
    return f / s if s > 0 else f


class _Texture:
    """Sum of analytic sinusoids, evaluated at translated coordinates."""

    def __init__(self, rng: np.random.Generator, n: int = 6, amplitude: float = 0.1,
                 fmin: float = 0.05, fmax: float = 0.25):
        self.f = rng.uniform(fmin, fmax, n)
        self.theta = rng.uniform(0.0, 2.0 * np.pi, n)
        self.phase = rng.uniform(0.0, 2.0 * np.pi, n)
        self.amp = amplitude / n

    def __call__(self, h: int, w: int, dy: float, dx: float) -> np.ndarray:
        ys = np.arange(h, dtype=np.float64) - dy
        xs = np.arange(w, dtype=np.float64) - dx
        out = np.zeros((h, w), dtype=np.float64)
        for f, th, ph in zip(self.f, self.theta, self.phase):
            fy, fx = f * np.sin(th), f * np.cos(th)
            ay = 2.0 * np.pi * fy * ys
            ax = 2.0 * np.pi * fx * xs + ph
            # cos(ay + ax) as a difference of two rank-one products
            out += np.multiply.outer(np.cos(ay), np.cos(ax))
            out -= np.multiply.outer(np.sin(ay), np.sin(ax))
        return out * self.amp


def _to_codes(v: np.ndarray, lo: float, span: float, bits: int, dtype) -> np.ndarray:
    scale = float(1 << (bits - 8))
    c = np.rint(lo * scale + span * scale * v)
    return np.clip(c, 0, (1 << bits) - 1).astype(dtype)


def gen_clip(width: int, height: int, n_frames: int, *, bits: int = 8, chroma: int = 420,
             seed: int = 0, scene_starts=None, cut_every=(20, 40), vel_max: float = 4.0,
             garbage_high_bits: bool = False) -> Clip:
    """Generate a clip.

    scene_starts: explicit list of scene-start frames (0 is added), or None to
    draw c_{k+1} = c_k + U{cut_every[0]..cut_every[1]}.
    garbage_high_bits: for 10-bit clips, fill the unused top 6 bits of each
    16-bit container with random bits (the unpack must mask them off).
    """
    if chroma not in (420, 444):
        raise ValueError("chroma must be 420 or 444")
    if bits not in (8, 10):
        raise ValueError("bits must be 8 or 10")
    if chroma == 420 and (width % 2 or height % 2):
        raise ValueError("4:2:0 needs even sizes")
    rng = np.random.default_rng(seed)
    if scene_starts is None:
        starts = [0]
        while True:
            nxt = starts[-1] + int(rng.integers(cut_every[0], cut_every[1] + 1))
            if nxt >= n_frames:
                break
            starts.append(nxt)
    else:
        starts = sorted(set([0] + [int(s) for s in scene_starts if 0 < int(s) < n_frames]))
    hc, wc = (height // 2, width // 2) if chroma == 420 else (height, width)
    cdiv = 2.0 if chroma == 420 else 1.0
    dtype = np.uint8 if bits == 8 else np.uint16
    Y = np.empty((n_frames, height, width), dtype=dtype)
    U = np.empty((n_frames, hc, wc), dtype=dtype)
    V = np.empty((n_frames, hc, wc), dtype=dtype)
    sigma = 0.05 * min(width, height)
    prev_mean = None
    bounds = starts + [n_frames]
    for s in range(len(starts)):
        mean = rng.uniform(0.25, 0.75)
        while prev_mean is not None and abs(mean - prev_mean) < 0.2:
            mean = rng.uniform(0.25, 0.75)
        prev_mean = mean
        contrast = rng.uniform(0.08, 0.2)
        field_y = smooth_field(rng, height, width, sigma)
        field_u = smooth_field(rng, hc, wc, sigma / cdiv)
        field_v = smooth_field(rng, hc, wc, sigma / cdiv)
        mu, mv = rng.uniform(-0.07, 0.07, 2)
        tex_y = _Texture(rng)
        tex_u = _Texture(rng, amplitude=0.03)
        tex_v = _Texture(rng, amplitude=0.03)
        vy, vx = rng.uniform(-vel_max, vel_max, 2)
        for t in range(bounds[s], bounds[s + 1]):
            tau = t - bounds[s]
            y = mean + contrast * field_y + tex_y(height, width, vy * tau, vx * tau)
            u = mu + 0.03 * field_u + tex_u(hc, wc, vy * tau / cdiv, vx * tau / cdiv)
            v = mv + 0.03 * field_v + tex_v(hc, wc, vy * tau / cdiv, vx * tau / cdiv)
            Y[t] = _to_codes(np.clip(y, 0.0, 1.0), 16.0, 219.0, bits, dtype)
            U[t] = _to_codes(np.clip(u, -0.5, 0.5), 128.0, 224.0, bits, dtype)
            V[t] = _to_codes(np.clip(v, -0.5, 0.5), 128.0, 224.0, bits, dtype)
    if garbage_high_bits and bits == 10:
        for P in (Y, U, V):
            P |= (rng.integers(0, 64, P.shape, dtype=np.uint16) << 10).astype(np.uint16)
    return Clip(Y, U, V, bits, chroma, starts)


def gen_group_c1(seed: int = 0) -> Clip:
    """One frame group: two 64x64 4:2:0 8-bit frames, texture shifted by a sub-pixel vector."""
    return gen_clip(64, 64, 2, bits=8, chroma=420, seed=seed, scene_starts=[], vel_max=1.0)


def gen_clip_c2(n_frames: int = 120, seed: int = 0) -> Clip:
    """960x540 4:2:0 8-bit clip, hard cut every U{20..40} frames, motion up to 4 px/frame."""
    return gen_clip(960, 540, n_frames, bits=8, chroma=420, seed=seed)


def gen_clip_c3(n_frames: int = 48, seed: int = 0) -> Clip:
    """1920x1080 4:2:0 10-bit clip with cuts at frames 16 and 32."""
    return gen_clip(1920, 1080, n_frames, bits=10, chroma=420, seed=seed,
                    scene_starts=[16, 32])
