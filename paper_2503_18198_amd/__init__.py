"""MI355X-native sparse MTTKRP and CP-ALS (HIP kernels behind a C ABI).

``capi`` is the thin binding of ``include/mttkrp.h``; ``build`` compiles the
HIP library.  Importing ``capi`` raises if the library has not been built.
"""

__all__ = ["capi", "build"]
