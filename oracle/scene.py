"""Scene changes, frame grouping and the frame-store layout (test infrastructure only).

The paper requires that frame groups never straddle a scene change (section
3.2, "End User Usage", the paragraph on scene changes, and section 3.3,
"Internal Design") and leaves the detector to the user.  The detector here is
an integer one: sum of absolute luma differences (SAD) and the L1 distance of
64-bin luma histograms, both against thresholds; a cut needs both.  An
external per-frame cut flag (the host framework's own scene-change signal) is
OR-ed in.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class SceneParams:
    mad_thresh_8bit: int = 24     # mean |dY| threshold, in 8-bit code units
    hist_frac_num: int = 1        # histogram L1 threshold as a fraction of its maximum 2N
    hist_frac_den: int = 4
    enable: bool = True           # False: only external flags decide


def luma_codes(Y: np.ndarray, bits: int) -> np.ndarray:
    return Y.astype(np.int64) & ((1 << bits) - 1)


def histogram64(y_codes: np.ndarray, bits: int) -> np.ndarray:
    """64-bin luma histogram, bin = code >> (bits - 6)."""
    return np.bincount((y_codes >> (bits - 6)).ravel(), minlength=64).astype(np.int64)


def sad(y_prev: np.ndarray, y_cur: np.ndarray) -> int:
    return int(np.abs(y_cur.astype(np.int64) - y_prev.astype(np.int64)).sum())


def hist_distance(h_prev: np.ndarray, h_cur: np.ndarray) -> int:
    return int(np.abs(h_cur.astype(np.int64) - h_prev.astype(np.int64)).sum())


def is_cut(sad_v: int, hd_v: int, n_pixels: int, bits: int, p: SceneParams) -> bool:
    """SAD > T * 2^(bits-8) * N  and  HD / (2N) > num / den, all in integers."""
    mad_ok = sad_v > p.mad_thresh_8bit * (1 << (bits - 8)) * n_pixels
    hist_ok = hd_v * p.hist_frac_den > 2 * n_pixels * p.hist_frac_num
    return bool(mad_ok and hist_ok)


def scene_metrics(Y_frames, bits: int):
    """Per-frame (SAD_t, HD_t, hist_t); frame 0 has no predecessor and reports 0, 0."""
    out = []
    prev = None
    for Y in Y_frames:
        y = luma_codes(Y, bits)
        h = histogram64(y, bits)
        if prev is None:
            out.append((0, 0, h))
        else:
            out.append((sad(prev[0], y), hist_distance(prev[1], h), h))
        prev = (y, h)
    return out


def detect_cuts(Y_frames, bits: int, params: SceneParams = SceneParams(), external=None):
    """cut[t] = 1 when frame t starts a scene.  Frame 0 always starts one."""
    mets = scene_metrics(Y_frames, bits)
    cuts = []
    for t, (s, hd, _h) in enumerate(mets):
        n_pix = int(np.asarray(Y_frames[t]).size)
        c = t == 0 or (params.enable and is_cut(s, hd, n_pix, bits, params))
        if external is not None and external[t] is not None and external[t] >= 0:
            c = c or bool(external[t])
        cuts.append(int(c))
    return cuts


def groups_n1(cuts):
    """Frame groups of an interpolating network that consumes n = 1 frame and takes
    one extra frame: group i = [i, i+1] unless frame i+1 begins a new scene or does
    not exist, in which case the last frame of the scene is duplicated: [i, i]."""
    n = len(cuts)
    return [(i, i + 1) if i + 1 < n and not cuts[i + 1] else (i, i) for i in range(n)]


def outputs_n1(cuts):
    """Emission order: each group emits its first frame (t = 0) and the interpolated
    middle frame (t = 1/2), so the output has exactly twice as many frames."""
    out = []
    for a, b in groups_n1(cuts):
        out.append((a, b, 0.0))
        out.append((a, b, 0.5))
    return out


def groups_general(scene_lengths, n: int, extra: bool):
    """Frame groups for a network consuming ``n`` frames per run, scene by scene.

    Rules (section 3.3, grouping paragraph): groups never cross a scene; with the
    extra-frame (interpolation) input the frame after the scene's last one is the
    scene's last frame duplicated; a final group short of frames recycles the
    last frames of the previous group; a scene shorter than one group
    duplicates its last frame.  Returns, per group, the list of input frame
    indices and the indices of the frames it consumes for the first time.
    """
    groups = []
    start = 0
    for L in scene_lengths:
        end = start + L
        last = end - 1
        frames = list(range(start, end))
        if L < n:
            frames = frames + [last] * (n - L)
        pos = 0
        done = set()
        while pos < len(frames):
            if pos + n > len(frames):
                pos = len(frames) - n          # recycle: slide back inside the scene
            consumed = frames[pos:pos + n]
            inp = list(consumed)
            if extra:
                nxt = pos + n
                inp.append(frames[nxt] if nxt < len(frames) else last)
            new = [f for f in dict.fromkeys(consumed) if f not in done]
            done.update(new)
            groups.append({"inputs": inp, "new": new})
            pos += n
        start = end
    return groups


def frame_store_positions(n: int, b: int, block: int):
    """Position of every frame of batch block ``block`` in the frame store (Fig. 1).

    Block j holds frames j*n*b .. j*n*b + n*b.  Its chain (every n-th frame, b+1 of
    them) occupies consecutive positions starting at P_j = (b-1) + j*n*b, so the
    batch views of input 0 and of the extra input overlap by b-1 frames; the other
    n-1 inputs follow, each as b consecutive positions.  Storing the figure's
    columns one after another gives exactly these positions.
    """
    base = (b - 1) + block * n * b
    f0 = block * n * b
    pos = {}
    for i in range(b + 1):
        pos[f0 + i * n] = base + i
    for k in range(1, n):
        for i in range(b):
            pos[f0 + i * n + k] = base + b + 1 + (k - 1) * b + i
    return pos


def frame_store_views(n: int, b: int, block: int):
    """Batch view of every network input slot: slot k -> list of b store positions."""
    base = (b - 1) + block * n * b
    views = {0: [base + i for i in range(b)], n: [base + 1 + i for i in range(b)]}
    for k in range(1, n):
        views[k] = [base + b + 1 + (k - 1) * b + i for i in range(b)]
    return views
