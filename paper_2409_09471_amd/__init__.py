"""MI355X (gfx950) hot path of randomized sketched TT-GMRES.

The numerical work lives in the HIP library libttsg.so (C ABI in
include/ttsg.h); `ttsg` is its ctypes binding.
"""
from . import ttsg  # noqa: F401
