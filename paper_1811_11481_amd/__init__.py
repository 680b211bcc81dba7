"""MI355X TPC sector tracker (arXiv:1811.11481 hot path): HIP kernels for gfx950
behind the C ABI of include/tpcca.h, with a thin ctypes binding."""
from .tpcca import (FLAG_ADJOINT_F64, FLAG_MERGE, FLAG_STATS, FLAG_TIMING, MAP_SHAPE, MAP_SIZE,  # noqa: F401
                    DeviceClusters, DeviceNativeClusters, Params, RefitSet, Tracker, Tracks, TpccaError, Tuning,
                    default_params,
                    default_tuning, fp32_selfcheck, load, refit_chi2, sqrt_step_check)
