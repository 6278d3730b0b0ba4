"""MI355X-native IEWPF ensemble forecast + analysis (arXiv:1910.01031).

The compute path is libiewpf.so (HIP kernels for gfx950, C ABI in include/iewpf.h);
this package is its ctypes binding (`abi`) and the in-tree build step (`build`).
"""
from . import abi
from .abi import (Batch, Context, IewpfError, Net, forecast_drifters_surrogate, load,
                  surrogate_window, surrogate_window_async)

__all__ = ["abi", "Batch", "Context", "IewpfError", "Net", "forecast_drifters_surrogate", "load",
           "surrogate_window", "surrogate_window_async"]
