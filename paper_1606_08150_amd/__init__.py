"""Workload consolidation of nested parallel work on AMD MI355X (gfx950).

The compute lives in libwc.so (HIP kernels behind the C ABI of include/wc.h);
``paper_1606_08150_amd.wc`` is the thin ctypes binding.
"""
from .wc import (BLOCK, FLAT, GRID, MODES, WAVE, Context, DeviceCSR, DeviceTree, Stats, Tune, WcError,  # noqa: F401
                 default_tune, kc_config, load_library, make_tune, per_buffer_size)
