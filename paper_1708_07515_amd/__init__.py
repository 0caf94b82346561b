"""MI355X-native FDK-OD cone-beam backprojection.

A thin ctypes binding over libfdkod.so (C ABI in include/fdkod.h).  Every step
of the reconstruction runs in the library's HIP kernels; this package only
marshals arguments.  Torch tensors supply device memory and streams.
"""

from ._lib import (FdkodError, Plan, STORE_TYPES, library_path, load_library,  # noqa: F401
                   validate)

__all__ = ["Plan", "FdkodError", "validate", "load_library", "library_path", "STORE_TYPES"]
