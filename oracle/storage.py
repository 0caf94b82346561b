"""Rounding emulation of the half-precision storage forms (FP16 / BF16).

The GPU path can store the filtered sinogram and the decimated sub-sinograms
in 16-bit types while computing in FP32.  These helpers round FP64 data to the
values such storage can hold, and return FP64 again, so that the oracle can
predict the error floor that storage alone causes.

Pinned by: exactly representable values pass unchanged; round-to-nearest-even
ties; agreement with NumPy's float16 cast and with torch's bfloat16 cast on
random data (tests/test_oracle_storage.py).
"""

import numpy as np


def round_f16(x):
    """Round to IEEE binary16 (round to nearest even) and back to FP64."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float16).astype(np.float64)


def round_bf16(x):
    """Round to bfloat16 (round to nearest even on the FP32 bit pattern)."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    bits = (bits + 0x7FFF + lsb) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def round_f32(x):
    """Round to IEEE binary32 and back to FP64."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


ROUNDERS = {"f32": round_f32, "f16": round_f16, "bf16": round_bf16}
