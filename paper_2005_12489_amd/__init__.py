"""MI355X-native per-pixel tile masks (display-driven computing, HiVision).

The hot path is hand-written HIP for gfx950 behind the C ABI in
include/hv.h; ``hv`` is its thin Python binding.
"""
from . import hv  # noqa: F401  (fails loudly if libhv.so is not built)
