"""Textbook FDK in FP64 (the paper cites FDK in Sec. 1 and uses it in Sec. 2.1).

The paper gives no FDK formulas, so this is the standard Feldkamp-Davis-Kress
reconstruction for a circular orbit and a flat (virtual) detector:

1. cosine pre-weight  p~ = p * R / sqrt(R^2 + a^2 + b^2);
2. row-wise ramp filter, a linear convolution with the spatial Ram-Lak kernel
   h[0] = 1/4, h[n odd] = -1/(pi^2 n^2), h[n even != 0] = 0 (unit spacing),
   zero outside the detector;
3. backprojection  f(x, y, z) = (pi / P) * sum_p U^-2 * Bil(q_p, u*, v*), with
   U = depth / R, a from eq. (1), b from eq. (9), u* = a + c_u, v* = b + c_v,
   bilinear interpolation with zero extension outside the detector.

The factor pi/P is (1/2) * (2 pi / P): the 1/2 removes the double coverage of
a full orbit.

Pinned by (tests/test_oracle_fdk.py): FFT filtering equals the direct
convolution; the kernel sums to zero over the integers (closed form); the
interior means and centroids of reconstructed off-centre spheres match the
analytic phantom; linearity.
"""

import numpy as np

from . import geometry as g


def cosine_weight(n, r, rows=None):
    """R / sqrt(R^2 + a^2 + b^2) for detector rows ``rows`` (all by default),
    shape [len(rows), n]."""
    c = g.centre(n)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    a = np.arange(n, dtype=np.float64) - c
    b = rows.astype(np.float64) - c
    return r / np.sqrt(r * r + a[None, :] ** 2 + b[:, None] ** 2)


def ramlak(offsets):
    """Spatial Ram-Lak kernel h[n] at integer offsets n (unit detector spacing)."""
    n = np.asarray(offsets, dtype=np.int64)
    h = np.zeros(n.shape, dtype=np.float64)
    h[n == 0] = 0.25
    odd = (n % 2) != 0
    h[odd] = -1.0 / (np.pi ** 2 * n[odd].astype(np.float64) ** 2)
    return h


def ramp_matrix(n):
    """Toeplitz matrix T with T[u', u] = h[u - u'], so that rows @ T is the
    linear convolution restricted to the detector (zero outside)."""
    idx = np.arange(n)
    return ramlak(idx[None, :] - idx[:, None])


def ramp_filter(rows):
    """Linear convolution of every detector row with Ram-Lak: q[u] = sum_u' h[u-u'] p[u'].

    Written as a matrix product with the Toeplitz matrix of the definition."""
    rows = np.asarray(rows, dtype=np.float64)
    return rows @ ramp_matrix(rows.shape[-1])


def ramp_filter_fft(rows):
    """The same linear convolution computed with an FFT of length M >= 2N-1 and
    the DFT of the spatial kernel (not a sampled |omega|).  Used as a pin."""
    rows = np.asarray(rows, dtype=np.float64)
    n = rows.shape[-1]
    m = 1 << int(np.ceil(np.log2(2 * n - 1)))
    k = np.arange(m)
    k = np.where(k < m // 2 + 1, k, k - m)       # circular offsets
    hk = np.fft.rfft(ramlak(k))
    out = np.fft.irfft(np.fft.rfft(rows, n=m, axis=-1) * hk, n=m, axis=-1)
    return out[..., :n]


class FilteredRows:
    """Filtered detector rows kept for a subset of rows.

    ``data[p, k, u]`` holds row ``rows[k]`` of projection p.  ``slot[v]`` maps a
    detector row to k, or -1.  Reading a row inside the detector that was not
    filtered raises, so a wrong row selection cannot pass silently."""

    def __init__(self, rows, data, nv):
        self.rows = np.asarray(rows, dtype=np.int64)
        self.data = data
        self.nv = nv
        self.slot = np.full(nv, -1, dtype=np.int64)
        self.slot[self.rows] = np.arange(len(self.rows))

    def sample(self, p, v, u):
        """Bilinear sample of filtered projection p at index coordinates (v, u),
        zero outside the detector."""
        return bilinear(self.data[p], self.slot, self.nv, v, u)


def bilinear(img, slot, nv, v, u):
    """Bilinear interpolation of ``img[k, u]`` (rows mapped through ``slot``) at
    index coordinates (v, u), with zero extension outside [0, nv) x [0, nu)."""
    nu = img.shape[-1]
    if img.shape[0] == 0:
        img = np.zeros((1, nu))
    v = np.asarray(v, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    iv = np.floor(v).astype(np.int64)
    iu = np.floor(u).astype(np.int64)
    fv = v - iv
    fu = u - iu
    out = np.zeros(np.broadcast(v, u).shape, dtype=np.float64)
    for dv, wv in ((0, 1.0 - fv), (1, fv)):
        vi = iv + dv
        vin = (vi >= 0) & (vi < nv)
        k = slot[np.clip(vi, 0, nv - 1)]
        if np.any(vin & (k < 0)):
            raise KeyError("detector row needed but not filtered")
        for du, wu in ((0, 1.0 - fu), (1, fu)):
            ui = iu + du
            ok = vin & (ui >= 0) & (ui < nu)
            val = img[np.clip(k, 0, None), np.clip(ui, 0, nu - 1)]
            out += np.where(ok, wv * wu * val, 0.0)
    return out


def filter_rows(proj, r, rows):
    """Steps 1-2 of FDK for detector rows ``rows`` of every projection.

    ``proj`` is indexable as proj[p, v, :] (numpy array or any object with that
    slicing); returns a FilteredRows."""
    rows = np.unique(np.asarray(rows, dtype=np.int64))
    n = proj.shape[2]
    nv = proj.shape[1]
    pw = np.asarray(proj[:, rows, :], dtype=np.float64) * cosine_weight(n, r, rows)[None]
    # the Toeplitz product is the definition; above 512 columns the same linear
    # convolution is taken by FFT (equal to 1e-10, see the filter pins)
    filt = ramp_filter(pw) if n <= 512 else ramp_filter_fft(pw)
    return FilteredRows(rows, filt, nv)


def rows_for_points(n, r, betas, x, y, z):
    """Detector rows that bilinear sampling of the points (x, y, z) can touch
    at the given angles (eq. (9) plus the +1 interpolation neighbour)."""
    cv = g.centre(n)
    need = np.zeros(n, dtype=bool)
    for beta in betas:
        iv = np.floor(g.row_pos(x, y, z, beta, r) + cv)
        lo = int(max(iv.min(), 0)) if iv.size else 0
        hi = int(min(iv.max() + 1, n - 1)) if iv.size else -1
        if hi >= lo:
            need[lo:hi + 1] = True      # a contiguous superset is harmless
    return np.nonzero(need)[0]


def backproject_points(frows, r, betas, x, y, z):
    """Step 3 of FDK at arbitrary voxel coordinates (x, y, z) (arrays, voxels)."""
    n = frows.data.shape[-1]
    cu = cv = g.centre(n)
    p_count = len(betas)
    f = np.zeros(np.broadcast(x, y, z).shape, dtype=np.float64)
    for p, beta in enumerate(betas):
        dep = g.depth(x, y, beta, r)
        u_mag = dep / r
        a = g.pix_pos(x, y, beta, r)
        b = g.row_pos(x, y, z, beta, r)
        f += frows.sample(p, b + cv, a + cu) / (u_mag * u_mag)
    return (np.pi / p_count) * f


def voxel_grid(n, nz, slices):
    """Coordinates of all voxels of the listed slices, each shaped [S, N, N]."""
    c, cz = g.centre(n), g.centre(nz)
    zs = np.asarray(slices, dtype=np.float64) - cz
    ys = np.arange(n, dtype=np.float64) - c
    xs = np.arange(n, dtype=np.float64) - c
    z, y, x = np.meshgrid(zs, ys, xs, indexing="ij")
    return x, y, z


def fdk(proj, r, slices=None, nz=None):
    """Direct FDK of the listed slices (all by default).  Returns [S, N, N]."""
    p_count, nv, n = proj.shape
    nz = n if nz is None else nz
    slices = np.arange(nz) if slices is None else np.asarray(slices)
    betas = g.angles(p_count)
    x, y, z = voxel_grid(n, nz, slices)
    rows = rows_for_points(n, r, betas, x, y, z)
    frows = filter_rows(proj, r, rows)
    return backproject_points(frows, r, betas, x, y, z)


def fdk_points(proj, r, idx, nz=None):
    """Direct FDK at voxel indices ``idx`` ([K, 3] array of (l, j, i))."""
    p_count, nv, n = proj.shape
    nz = n if nz is None else nz
    idx = np.asarray(idx)
    x = idx[:, 2] - g.centre(n)
    y = idx[:, 1] - g.centre(n)
    z = idx[:, 0] - g.centre(nz)
    betas = g.angles(p_count)
    rows = rows_for_points(n, r, betas, x, y, z)
    frows = filter_rows(proj, r, rows)
    return backproject_points(frows, r, betas, x, y, z)
