"""MI355X-native w-stacking imaging (gridding, per-plane FFT, w-screen).

The compute path is libwstack.so (hand-written HIP kernels for gfx950 behind
a C ABI, include/wstack.h); this package is its thin Python binding.
"""
from ._abi import WStackError, lib  # noqa: F401
from .api import WStackPlan, make_params, validate, workspace_bytes  # noqa: F401

__all__ = ["WStackPlan", "WStackError", "make_params", "validate",
           "workspace_bytes", "lib"]
