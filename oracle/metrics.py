"""Error metrics used to state parity against the FP64 oracle."""

import numpy as np


def rel_rmse(f, ref):
    """||f - ref||_2 / ||ref||_2 over the evaluated voxels."""
    f = np.asarray(f, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(f - ref) / den) if den > 0 else float(np.linalg.norm(f))


def max_abs(f, ref):
    """max |f - ref| and the same divided by max |ref|."""
    f = np.asarray(f, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    m = float(np.max(np.abs(f - ref))) if f.size else 0.0
    scale = float(np.max(np.abs(ref))) if ref.size else 0.0
    return m, (m / scale if scale > 0 else m)


def sampled_slices(nz, count=16):
    """l = round(linspace(0, N_z - 1, count)): includes the top and bottom
    slices, where the cone angle is largest."""
    return np.unique(np.round(np.linspace(0, nz - 1, count)).astype(np.int64))
