"""MI355X-native frame-group enhancement path of NNVISR (ACM MM 2023).

The work happens in libnnvisr.so (hand-written HIP kernels for gfx950 behind the C-ABI
declared in include/nnvisr.h).  ``paper_2308_03121_amd.binding`` only marshals
arguments; loading fails loudly when the library has not been built.
"""
from ._abi import NvError, header_functions, load  # noqa: F401

__all__ = ["NvError", "header_functions", "load"]
