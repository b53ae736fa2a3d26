"""MI355X-native explicit HOPU convection hot path (C-ABI library + binding).

The compute lives in libhopu.so (hand-written HIP for gfx950); this package
only marshals arguments.  Importing it does not load the library or touch the
GPU; `Hopu(...)` does, and fails loudly if the library is missing.
"""
from ._lib import (FP64, FP32_MFMA, BF16X2, BF16X3, TERM_VOLUME, TERM_CENTRAL, TERM_UPWIND, TERM_ALL,  # noqa: F401
                   HopuError, LIB_PATH, lib)


def __getattr__(name):
    if name in ("Hopu", "SubstepChain", "MassEnergy"):
        from . import hopu
        return getattr(hopu, name)
    raise AttributeError(name)
