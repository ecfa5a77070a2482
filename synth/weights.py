"""Seeded weights for the generic frame-group enhancement network.

The network is any extract/fusion network in the sense of the paper's
network-integration section; this module fixes one concrete instance so that
the oracle and the device path can be compared.  Weights are a flat float32
blob in a fixed tensor order; every conv is 3x3 and stored OIHW followed by
its bias.

Tensor order:
  conv_in  (C, 3)            extract, first layer
  block r  a (C, C), b (C, C)  extract, residual blocks r = 0..R-1
  down l   (C, C)            extract, pyramid level l = 2..L (after a 2x2 mean pool)
  off1     (C, 2C)           offset head, first conv        (interpolating networks only)
  off2     (27G, C)          offset head, second conv (18G offsets, 9G mask logits)  (")
  dcn      (C, 2C)           modulated deformable alignment  (")
  off1.l, off2.l, dcn.l      the same three for pyramid level l = 2..L, after level 1's
  up       (sv sh C, C)      conv before the (sv, sh) pixel shuffle (4C for x2 both ways)
  hr       (3, C)            output RGB residual

The task (section 3.2, end-user usage) sets the scale (sv rows, sh columns) and the
flags: an interpolating network (Interpolation + Extra frame) fuses frame pairs and, with
Double frame, also emits its input frames enhanced; without Interpolation it enhances
each frame alone (no offset head, no alignment).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

LRELU_SLOPE = 0.1


@dataclass(frozen=True)
class NetConfig:
    channels: int = 64
    res_blocks: int = 10
    offset_groups: int = 8
    scale: int = 2            # horizontal scale factor
    align: int = 8
    scale_v: int = 0          # vertical scale factor, 0 = the same as scale
    interp: bool = True       # Interpolation + Extra frame
    double: bool = True       # Double frame
    levels: int = 1           # feature pyramid levels (1 = the trunk's output only)

    def __post_init__(self):
        if (2 * self.channels) % self.offset_groups:
            raise ValueError("2*channels must be divisible by offset_groups")

    @property
    def sv(self) -> int:
        return self.scale_v or self.scale

    @property
    def sh(self) -> int:
        return self.scale


NET_C1 = NetConfig(32, 2, 8)
NET_C2 = NetConfig(64, 10, 8)
NET_C4 = NetConfig(64, 6, 8)


def weight_layout(cfg: NetConfig):
    """List of (name, cout, cin, gain) in blob order."""
    C, G = cfg.channels, cfg.offset_groups
    layers = [("conv_in", C, 3, 1.0)]
    for r in range(cfg.res_blocks):
        layers.append((f"block{r}.a", C, C, 1.0))
        layers.append((f"block{r}.b", C, C, 0.1))
    for lv in range(2, cfg.levels + 1):
        layers.append((f"down{lv}", C, C, 1.0))
    if cfg.interp:
        for lv in range(1, cfg.levels + 1):
            sfx = "" if lv == 1 else f".l{lv}"
            layers += [("off1" + sfx, C, 2 * C, 1.0), ("off2" + sfx, 27 * G, C, 1.0), ("dcn" + sfx, C, 2 * C, 1.0)]
    layers += [("up", cfg.sv * cfg.sh * C, C, 1.0), ("hr", 3, C, 0.1)]
    return layers


def gen_weights(cfg: NetConfig, seed: int = 1) -> np.ndarray:
    """He-initialised weights (gain for LeakyReLU 0.1) and N(0, 0.01^2) biases."""
    rng = np.random.default_rng(seed)
    he = np.sqrt(2.0 / (1.0 + LRELU_SLOPE ** 2))
    parts = []
    for _name, cout, cin, gain in weight_layout(cfg):
        std = gain * he / np.sqrt(cin * 9)
        parts.append((rng.standard_normal((cout, cin, 3, 3)) * std).astype(np.float32).ravel())
        parts.append((rng.standard_normal(cout) * 0.01).astype(np.float32))
    return np.concatenate(parts)


def unpack_weights(cfg: NetConfig, blob: np.ndarray) -> dict:
    """Views {name: (w OIHW, b)} into a blob."""
    out, off = {}, 0
    for name, cout, cin, _gain in weight_layout(cfg):
        n = cout * cin * 9
        w = blob[off:off + n].reshape(cout, cin, 3, 3)
        off += n
        b = blob[off:off + cout]
        off += cout
        out[name] = (w, b)
    if off != blob.size:
        raise ValueError(f"blob has {blob.size} floats, layout needs {off}")
    return out
