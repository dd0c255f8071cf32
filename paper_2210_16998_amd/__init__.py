"""MI355X-native prime-path and test-path generation (HIP, gfx950).

The compute path lives in libtpg.so (C ABI declared in include/tpg.h); the
binding in :mod:`paper_2210_16998_amd.tpg` only marshals arguments.  Import
is light: the library is loaded on first use and a missing build raises.
"""

__all__ = ["tpg", "cfggen"]
