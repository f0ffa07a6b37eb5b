"""GPU compaction of LSM-tree tables on MI355X (gfx950).

The compute path lives in HIP kernels behind the C-ABI of include/luda.h;
this package holds those sources (csrc/), the build script and the ctypes
binding.
"""
from .binding import (  # noqa: F401
    Context, Server, Result, Error, STATUS, EXPORTS, LIB_PATH, lib, selftest_crc, pin_reserve, pool_trim,
)
