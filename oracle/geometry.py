"""Cone-beam geometry of the paper (Sec. 2.1 eq. (1), Sec. 2.2 eq. (9)), FP64.

Conventions (the paper fixes only the two formulas; the rest is our reading):

* Units are voxels.  The voxel pitch equals the pitch of a virtual detector
  through the rotation axis, so eq. (1) as printed (magnification 1 at the
  axis) gives a detector column coordinate directly.  R is the constant of
  eq. (1); the source sits at distance R from the axis.
* Voxel centre coordinates: x_i = i - c, y_j = j - c with c = (N-1)/2, and
  z_l = l - c_z with c_z = (N_z-1)/2.  Volumes are stored ``vol[l, j, i]``.
* Detector index coordinates: column u = a + c_u, row v = b + c_v with
  c_u = c_v = (N-1)/2.  Projections are stored ``proj[p, v, u]``.
* Angles: beta_p = 2 pi p / P over a full circle.  The source is at
  -R (cos beta, sin beta, 0); the detector column axis is (-sin beta, cos beta, 0)
  and the row axis is z, so eq. (1) is R * lateral / depth and eq. (9) is
  z * R / depth with depth = R + x cos beta + y sin beta.
"""

import numpy as np


def centre(n):
    """Index of the geometric centre of an axis with ``n`` samples."""
    return (n - 1) / 2.0


def angles(p):
    """beta_p = 2 pi p / P, p = 0..P-1 (full 360 degree orbit)."""
    return 2.0 * np.pi * np.arange(p, dtype=np.float64) / p


def depth(x, y, beta, r):
    """Distance along the central ray from the source: R + x cos b + y sin b."""
    return r + x * np.cos(beta) + y * np.sin(beta)


def pix_pos(x, y, beta, r):
    """Detector column coordinate a(x, y, beta) of point (x, y), Sec. 2.1 eq. (1).

    Pinned by: an explicit ray/plane intersection in the tests (the point, the
    source and the detector point are collinear), and the vertex-extremum
    brute force of the bounds.
    """
    cb, sb = np.cos(beta), np.sin(beta)
    return r * (y * cb - x * sb) / (r + x * cb + y * sb)


def row_pos(x, y, z, beta, r):
    """Detector row coordinate b(x, y, z, beta) of voxel (x, y, z), Sec. 2.2 eq. (9)."""
    return z * r / depth(x, y, beta, r)


def blocks(n, parts):
    """Split range(n) into ``parts`` contiguous blocks, sizes as equal as possible,
    larger blocks first (the 2^s x 2^s squares of Sec. 2.1 when 2^s does not
    divide N).  Returns a list of (start, stop) pairs."""
    if parts < 1 or parts > n:
        raise ValueError("need 1 <= parts <= n")
    base, extra = divmod(n, parts)
    out, start = [], 0
    for k in range(parts):
        size = base + (1 if k < extra else 0)
        out.append((start, start + size))
        start += size
    return out


def squares(n, s):
    """The 4^s squares of Sec. 2.1: list of (x0, x1, y0, y1) index ranges
    (half-open), ordered with the y block major: q = by * 2^s + bx."""
    b = blocks(n, 2 ** s)
    return [(x0, x1, y0, y1) for (y0, y1) in b for (x0, x1) in b]


def valid_radius(n, r):
    """True when every voxel of the N x N slice has a positive depth at every
    angle (the denominator of eq. (1) never reaches zero): R > (N-1)/sqrt(2)."""
    return r > (n - 1) / np.sqrt(2.0)
