"""MI355X-native implicit flux-limited-diffusion (FLD) radiation update.

The product is the HIP library ``lib/libfld.so`` (C ABI in include/fld.h);
``fld`` is its ctypes binding and ``solver`` a thin convenience layer that
drives a whole split step (opacity, diffusion, exchange) on torch tensors.
"""
from . import fld  # noqa: F401
