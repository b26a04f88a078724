"""MI355X (gfx950) inverse spherical harmonic transform (alm2map) and its adjoint.

The transform runs in hand-written HIP kernels behind the C ABI of
``include/sht.h`` (library ``libsht.so`` in this package); this package is the
Python binding.  Importing it without the built library raises ImportError.
"""
from . import _lib
from ._lib import ShtError, load

load()

from .sht import AlmToMap, Batch, Plan, alm2map  # noqa: E402

__all__ = ["Plan", "Batch", "AlmToMap", "alm2map", "ShtError", "load", "_lib"]
__version__ = "0.1.0"
