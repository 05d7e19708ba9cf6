"""MI355X-native exact k-NN over an iSAX index (MESSI's data-parallel hot path).

The compute lives in ``libmessi.so`` (hand-written HIP for gfx950, C ABI in
``include/messi.h``); this package is its ctypes binding.
"""
from .messi import (  # noqa: F401
    MODE_BF16, MODE_FP32, Index, MessiError, Server, breakpoints, last_error, load, znorm_,
)
