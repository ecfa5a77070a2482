"""Pins of the oracle's scene metric, grouping rules and frame-store layout."""
import json
import os
import random

import numpy as np
import pytest

import synth
from oracle import scene

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _flat(v, shape=(16, 24), dtype=np.uint8):
    return np.full(shape, v, dtype=dtype)


def test_hand_counted_flat_cut():
    frames = [_flat(100)] * 3 + [_flat(180)] * 3
    assert scene.detect_cuts(frames, 8) == [1, 0, 0, 1, 0, 0]


def test_metric_values_by_hand():
    a, b = _flat(100), _flat(180)
    n = a.size
    assert scene.sad(a, b) == 80 * n
    h_a, h_b = scene.histogram64(a.astype(np.int64), 8), scene.histogram64(b.astype(np.int64), 8)
    assert h_a[25] == n and h_b[45] == n and h_a.sum() == n
    assert scene.hist_distance(h_a, h_b) == 2 * n


def test_both_conditions_needed():
    rng = np.random.default_rng(0)
    tex = rng.integers(30, 220, (16, 24)).astype(np.uint8)
    # large SAD, identical histogram (spatial shuffle): no cut
    assert scene.detect_cuts([tex, np.roll(tex, 12, axis=1)], 8) == [1, 0]
    # every pixel changes bin but the mean change is only 4 codes: no cut
    assert scene.detect_cuts([_flat(100), _flat(104)], 8) == [1, 0]


@pytest.mark.parametrize("bits,lo,at,over", [(8, 100, 124, 125), (10, 400, 496, 497)])
def test_sad_threshold_is_strict(bits, lo, at, over):
    dt = np.uint8 if bits == 8 else np.uint16
    assert scene.detect_cuts([_flat(lo, dtype=dt), _flat(at, dtype=dt)], bits) == [1, 0]
    assert scene.detect_cuts([_flat(lo, dtype=dt), _flat(over, dtype=dt)], bits) == [1, 1]


def test_histogram_threshold_is_strict():
    # half of the pixels move to another bin: HD = N, i.e. HD/2N = 1/2 > 1/4 -> cut
    a = _flat(40)
    b = a.copy()
    b[:8] = 200
    assert scene.detect_cuts([a, b], 8) == [1, 1]
    # exactly a quarter of the maximum distance: HD/2N = 1/4 is not > 1/4
    c = a.copy()
    c[:4] = 250                 # 4 of 16 rows, SAD = 210 * N/4 > 24 N
    assert scene.hist_distance(scene.histogram64(a.astype(np.int64), 8),
                               scene.histogram64(c.astype(np.int64), 8)) == a.size // 2
    assert scene.detect_cuts([a, c], 8) == [1, 0]


def test_external_flags_and_disable():
    frames = [_flat(100)] * 4
    assert scene.detect_cuts(frames, 8, external=[None, -1, 1, 0]) == [1, 0, 1, 0]
    frames = [_flat(100), _flat(200), _flat(100)]
    off = scene.SceneParams(enable=False)
    assert scene.detect_cuts(frames, 8, off) == [1, 0, 0]
    assert scene.detect_cuts(frames, 8, off, external=[-1, -1, 1]) == [1, 0, 1]


def test_10bit_high_bits_ignored():
    a = _flat(400, dtype=np.uint16)
    b = a | np.uint16(0xFC00)
    assert scene.detect_cuts([a, b], 10) == [1, 0]


@pytest.mark.slow
def test_generator_cuts_recovered_c2():
    clip = synth.gen_clip_c2()
    cuts = scene.detect_cuts(list(clip.Y), clip.bits)
    assert [t for t, c in enumerate(cuts) if c] == clip.scene_starts


def test_generator_cuts_recovered_small_10bit_444():
    clip = synth.gen_clip(160, 96, 40, bits=10, chroma=444, seed=4, cut_every=(6, 12),
                          garbage_high_bits=True)
    cuts = scene.detect_cuts(list(clip.Y), 10)
    assert [t for t, c in enumerate(cuts) if c] == clip.scene_starts


def test_groups_n1_tables():
    # scenes [0,1,2] [3,4]
    assert scene.groups_n1([1, 0, 0, 1, 0]) == [(0, 1), (1, 2), (2, 2), (3, 4), (4, 4)]
    # a one-frame scene duplicates its frame
    assert scene.groups_n1([1, 1, 0]) == [(0, 0), (1, 2), (2, 2)]
    assert scene.groups_n1([1]) == [(0, 0)]
    # interpolation doubles the frame count
    assert len(scene.outputs_n1([1, 0, 0, 1, 0])) == 10


def test_groups_never_cross_a_cut():
    rng = random.Random(7)
    for _ in range(200):
        n = rng.randint(1, 30)
        cuts = [1] + [int(rng.random() < 0.2) for _ in range(n - 1)]
        sid = np.cumsum(cuts)
        for a, b in scene.groups_n1(cuts):
            assert sid[a] == sid[b] and b - a in (0, 1)


def test_general_rules_n3_extra():
    g = scene.groups_general([7], n=3, extra=True)
    assert [x["inputs"] for x in g] == [[0, 1, 2, 3], [3, 4, 5, 6], [4, 5, 6, 6]]
    assert [x["new"] for x in g] == [[0, 1, 2], [3, 4, 5], [6]]
    # a scene shorter than n duplicates its last frame
    g = scene.groups_general([2], n=3, extra=True)
    assert [x["inputs"] for x in g] == [[0, 1, 1, 1]]
    assert g[0]["new"] == [0, 1]
    # groups of the second scene start at its first frame
    g = scene.groups_general([3, 4], n=3, extra=True)
    assert [x["inputs"] for x in g] == [[0, 1, 2, 2], [3, 4, 5, 6], [4, 5, 6, 6]]


def test_general_rules_without_extra():
    g = scene.groups_general([7], n=3, extra=False)
    assert [x["inputs"] for x in g] == [[0, 1, 2], [3, 4, 5], [4, 5, 6]]
    assert sorted(sum((x["new"] for x in g), [])) == list(range(7))


def test_general_n1_matches_n1_rule():
    for cuts in ([1, 0, 0, 1, 0], [1, 1, 1], [1, 0, 0, 0, 0, 1]):
        starts = [i for i, c in enumerate(cuts) if c] + [len(cuts)]
        lengths = [b - a for a, b in zip(starts, starts[1:])]
        g = scene.groups_general(lengths, n=1, extra=True)
        assert [tuple(x["inputs"]) for x in g] == scene.groups_n1(cuts)


def test_fig1_frame_store_layout():
    with open(os.path.join(GOLD, "fig1_frame_store.json")) as f:
        fig = json.load(f)
    n, b = fig["n"], fig["b"]
    memory = [v for col in fig["columns"] for v in col]       # column-first order
    printed = {v: i for i, v in enumerate(memory) if v is not None}
    pos0 = scene.frame_store_positions(n, b, 0)
    pos1 = scene.frame_store_positions(n, b, 1)
    # block 0: frames 0..6 where the figure prints them
    assert pos0 == {f: printed[f] for f in range(0, n * b + 1)}
    # block 1: frames 7..12 where printed; frame 6 takes the place of frame 5
    for f in range(n * b + 1, 2 * n * b + 1):
        assert pos1[f] == printed[f]
    cp = fig["copy_for_next_batch"]
    assert pos1[cp["frame"]] == printed[cp["into_place_of"]]
    # batch views: each input slot is b consecutive positions, slot 0 and slot n overlap
    v = scene.frame_store_views(n, b, 0)
    inv = {p: f for f, p in pos0.items()}
    assert [inv[p] for p in v[0]] == [0, 3] and [inv[p] for p in v[3]] == [3, 6]
    assert [inv[p] for p in v[1]] == [1, 4] and [inv[p] for p in v[2]] == [2, 5]
    # no frame is stored twice within a block: b*n + 1 distinct positions
    assert len(set(pos0.values())) == n * b + 1


@pytest.mark.parametrize("n,b", [(1, 4), (2, 3), (3, 2), (4, 5)])
def test_frame_store_general(n, b):
    for blk in range(3):
        pos = scene.frame_store_positions(n, b, blk)
        views = scene.frame_store_views(n, b, blk)
        inv = {p: f for f, p in pos.items()}
        f0 = blk * n * b
        for k in range(n + 1):
            assert [inv[p] for p in views[k]] == [f0 + i * n + k for i in range(b)]
        assert len(pos) == n * b + 1 == len(set(pos.values()))
        # the next block's first frame sits where this block's last frame-slot ends
        nxt = scene.frame_store_positions(n, b, blk + 1)
        assert nxt[f0 + n * b] == max(pos.values())
