"""MI355X-native FDK-OD cone-beam backprojection.

A thin ctypes binding over libfdkod.so (C ABI in include/fdkod.h).  Every step
of the reconstruction runs in the library's HIP kernels; this package only
marshals arguments.  Torch tensors supply device memory and streams.
"""

from ._lib import (Batch, FdkodError, Plan, STORE_TYPES, library_path,  # noqa: F401
                   load_library, validate)

__all__ = ["Plan", "Batch", "FdkodError", "validate", "load_library", "library_path", "STORE_TYPES"]
