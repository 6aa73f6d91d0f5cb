"""mrx: MI355X-native SENSE / CG / MoDL / VarNet hot path (arXiv 2202.14005).

The compute lives in libmrx.so (HIP, gfx950), reached through the C-ABI in
include/mrx.h; this package is its thin Python binding.  Build the library
with ``python -m paper_2202_14005_amd.build``.
"""
from ._lib import MrxError, lib  # noqa: F401

__all__ = ["MrxError", "lib", "ops"]
