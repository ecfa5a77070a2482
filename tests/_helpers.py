"""Shared test helpers: device availability and oracle/device conversions."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import pipeline  # noqa: E402


def require_gpu():
    """On a GPU test: the device and the built library must be present (no fallback)."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2308_03121_amd import _abi
    _abi.load()


def oracle_weights(cfg, blob):
    return pipeline.weights_dict(blob, synth.weight_layout(cfg))


def nhwc_to_chw(t):
    a = t.float().cpu().numpy() if hasattr(t, "cpu") else np.asarray(t)
    return np.ascontiguousarray(a.transpose(2, 0, 1)).astype(np.float64)


def max_abs(a, b):
    return float(np.max(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64))))


def say(msg):
    """Name the case before a GPU step so a failing run shows where it stopped."""
    print(msg, flush=True)
