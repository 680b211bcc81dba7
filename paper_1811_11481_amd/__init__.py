"""MI355X TPC sector tracker (arXiv:1811.11481 hot path): HIP kernels for gfx950
behind the C ABI of include/tpcca.h, with a thin ctypes binding."""
from .tpcca import (DeviceClusters, Params, Tracker, Tracks, TpccaError, Tuning, default_params,  # noqa: F401
                    default_tuning, fp32_selfcheck, load)
