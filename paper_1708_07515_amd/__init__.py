"""MI355X-native FDK-OD cone-beam backprojection.

A thin ctypes binding over libfdkod.so (C ABI in include/fdkod.h).  Every step
of the reconstruction runs in the library's HIP kernels; this package only
marshals arguments.  Torch tensors supply device memory and streams.
"""

from ._lib import (DECIM_TYPES, INTERP_TYPES, LEARNED_PARAMS, NOALLOC_SCRATCH_BYTES, ROWS_TYPES,  # noqa: F401
                   Batch, FdkodError, Plan, STORE_TYPES,
                   MI355X_COSTS, adamw_step, check_counts, choose_s, cost_counts, library_path, load_library,
                   sq_residual, sq_residual_weighted, validate)
from .learned import LearnedDecimation  # noqa: F401

__all__ = ["Plan", "Batch", "FdkodError", "validate", "load_library", "library_path", "STORE_TYPES",
           "DECIM_TYPES", "ROWS_TYPES", "INTERP_TYPES", "LEARNED_PARAMS", "NOALLOC_SCRATCH_BYTES", "sq_residual", "sq_residual_weighted", "adamw_step", "check_counts",
           "cost_counts", "choose_s", "MI355X_COSTS",
           "LearnedDecimation"]
