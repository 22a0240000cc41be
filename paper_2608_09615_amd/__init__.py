"""MI355X-native Spectral Difference right-hand side with the compact
(three-element) and standard BR1 treatments of second-order fluxes.

The compute path is the HIP library ``libsd.so`` (C ABI declared in
``include/sd.h``); :mod:`paper_2608_09615_amd.sd` is a thin ctypes binding
that marshals torch device tensors into it.  There is no CPU fallback.
"""
from .sd import SD, SDError, load_library  # noqa: F401

__all__ = ["SD", "SDError", "load_library"]
