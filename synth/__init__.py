"""Seeded synthetic inputs shared, as data only, by the oracle and the HIP path.

Nothing here performs any step of the enhancement method: the clip generator
writes Y'CbCr code values directly (it never converts colours), and the weight
generator only draws random numbers.  Both the oracle (``oracle/``) and the
device path (``paper_2308_03121_amd``) receive these arrays as inputs.
"""
from .clips import (Clip, gen_clip, gen_group_c1, gen_clip_c2, gen_clip_c3,
                    smooth_field, clip_format)
from .weights import (NetConfig, NET_C1, NET_C2, NET_C4, LRELU_SLOPE, gen_weights,
                      weight_layout, unpack_weights)

__all__ = ["Clip", "gen_clip", "gen_group_c1", "gen_clip_c2", "gen_clip_c3",
           "smooth_field", "clip_format", "NetConfig", "NET_C1", "NET_C2", "NET_C4",
           "LRELU_SLOPE", "gen_weights", "weight_layout", "unpack_weights"]
