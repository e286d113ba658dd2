"""MI355X (gfx950) moist anelastic LES time step: HIP kernels behind a C ABI.

`paper_2301_04698_amd.les` is the ctypes binding of include/les.h; the
library itself is built by `paper_2301_04698_amd.build`.
"""
from . import les  # noqa: F401

__all__ = ["les"]
