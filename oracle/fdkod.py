"""FDK-OD in FP64 (Sec. 2.1 and Sec. 2.2 of the paper), test infrastructure only.

Steps, in the paper's order:

1. Split every slice into 4^s squares of side N/2^s (Sec. 2.1).
2. For every square and angle, evaluate eq. (1) at the four vertices; the
   minimum and maximum bound the part of each detector row the square uses
   (Sec. 2.1).  The square's centre trajectory a_c(beta) = a(x_c, y_c, beta) is
   the column that the shift makes constant (Sec. 2.1, "centers ... on one
   column").
3. Crop and shift every row, with linear interpolation (Sec. 2.1).
4. Angular decimation: low-pass filter plus downsampling, P -> P' (Sec. 2.1).
5. Backproject the square from the P' decimated angles; the second shift back
   to detector positions is folded into the sample coordinate (Sec. 2.1 and
   Sec. 2.2, "only one interpolation").

Readings where the paper is silent:

* squares: near-equal contiguous blocks, larger first, when 2^s does not
  divide N; vertices are the four corner voxel centres and (x_c, y_c) their
  mean;
* local grid: local column j of square q at angle beta sits at detector index
  u_j(beta) = a_c(beta) + u0_q + j, an integer offset from the centre
  trajectory, with u0_q = floor(e_min + c_u) and
  W_q = floor(e_max + c_u) - u0_q + 2, where e_min / e_max are the extremes of
  a_min - a_c and a_max - a_c over the decimated angles;
* decimation filter: a triangle (Bartlett) window of half-width
  Delta' = 2 pi / P' centred on each decimated angle beta'_m = 2 pi m / P',
  circular in beta and normalised to unit sum, with D = 2^(s-k) and
  P' = ceil(P / D) (k = skipped decimation stages, Sec. 2.2).  When D divides
  P it equals s-k cascaded [1, 2, 1]/4 half-band stages with keep-even;
* each detector row is decimated on its own (Sec. 2.1, the bounds do not
  depend on the row).

Pinned by (tests/test_oracle_fdkod.py): s = 0 reproduces direct FDK; D = 1 is
the identity; triangle weights equal the [1,2,1]/4 cascade; brute-force vertex
containment of every voxel of every square and every bilinear footprint;
linearity; interior means and centroids of analytic spheres; the update and
crop counters of eq. (6) and eq. (7).  The quality knobs (windowed-sinc
decimation, cubic shift) are pinned in tests/test_oracle_knobs.py against
scipy's windowed-sinc design, the identity at D = 1, exact reproduction of
quadratics and the Catmull-Rom Hermite form.
"""

from dataclasses import dataclass

import numpy as np

from . import fdk as fdk_mod
from . import geometry as g


@dataclass
class Square:
    """One of the 4^s squares: voxel index ranges, centre, local column grid."""
    x0: int
    x1: int
    y0: int
    y1: int
    xc: float
    yc: float
    u0: int = 0
    width: int = 0


def decimation_factor(s, k):
    """D = 2^(s-k): s decomposition stages with k decimation stages skipped."""
    if not 0 <= k <= s:
        raise ValueError("need 0 <= k <= s")
    return 1 << (s - k)


def decimated_count(p, d):
    """P' = ceil(P / D)."""
    return -(-p // d)


def make_squares(n, s):
    """The squares of step 1 with their vertex-mean centres (coordinates)."""
    c = g.centre(n)
    out = []
    for (x0, x1, y0, y1) in g.squares(n, s):
        xc = 0.5 * ((x0 - c) + (x1 - 1 - c))
        yc = 0.5 * ((y0 - c) + (y1 - 1 - c))
        out.append(Square(x0, x1, y0, y1, xc, yc))
    return out


def vertices(sq, n):
    """The four corner voxel centres of a square, as coordinate arrays."""
    c = g.centre(n)
    xs = np.array([sq.x0 - c, sq.x1 - 1 - c, sq.x0 - c, sq.x1 - 1 - c])
    ys = np.array([sq.y0 - c, sq.y0 - c, sq.y1 - 1 - c, sq.y1 - 1 - c])
    return xs, ys


def centre_track(sq, betas, r):
    """a_c(beta) = eq. (1) at the square's centre."""
    return g.pix_pos(sq.xc, sq.yc, np.asarray(betas), r)


def vertex_bounds(sq, n, betas, r):
    """a_min(beta), a_max(beta): extremes of eq. (1) over the four vertices."""
    xs, ys = vertices(sq, n)
    a = g.pix_pos(xs[:, None], ys[:, None], np.asarray(betas)[None, :], r)
    return a.min(axis=0), a.max(axis=0)


def local_grid(sq, n, betas_dec, r):
    """Fill sq.u0 and sq.width from the bounds at the decimated angles."""
    cu = g.centre(n)
    ac = centre_track(sq, betas_dec, r)
    amin, amax = vertex_bounds(sq, n, betas_dec, r)
    e_min = float(np.min(amin - ac))
    e_max = float(np.max(amax - ac))
    sq.u0 = int(np.floor(e_min + cu))
    sq.width = int(np.floor(e_max + cu)) - sq.u0 + 2
    return sq


def plan(n, p, r, s, k):
    """Squares with their local grids, the original and decimated angles."""
    d = decimation_factor(s, k)
    pd = decimated_count(p, d)
    betas = g.angles(p)
    betas_dec = g.angles(pd)
    sqs = [local_grid(sq, n, betas_dec, r) for sq in make_squares(n, s)]
    return sqs, betas, betas_dec


def triangle_weights(p, pd):
    """w[m, p]: triangle of half-width 2 pi / P' around beta'_m, circular in
    beta, normalised so every row sums to one (decimation, step 4).

    The distance between beta_p = 2 pi p / P and beta'_m = 2 pi m / P',
    measured in decimated steps, is |p P' - m P| / P (circularly modulo P'),
    so the unnormalised weight max(0, 1 - distance) is computed exactly from
    integers: max(0, P - e) / P with e = circular |p P' - m P|."""
    pp = np.arange(p, dtype=np.int64)[None, :]
    mm = np.arange(pd, dtype=np.int64)[:, None]
    period = p * pd
    e = np.abs(pp * pd - mm * p) % period
    e = np.minimum(e, period - e)
    w = np.maximum(0, p - e).astype(np.float64)
    return w / w.sum(axis=1, keepdims=True)


# ------------------------------------------------------------ quality knobs
#
# Two extensions beyond the paper, cheaper than a learned decimation filter:
# Sec. 2.1 leaves the low-pass kernel open ("filters with small kernel"), and
# the discussion of interpolation counts in Sec. 2.2 notes that a more precise
# interpolation reduces smoothing.
#
# * windowed-sinc decimation: the ideal low-pass for the decimated rate (cut
#   off at half a decimated step's frequency) truncated to K decimated steps
#   by a Hann window, normalised per window like the triangle;
# * cubic shift: Keys' cubic convolution kernel (a = -1/2, Catmull-Rom) in u
#   for the crop and shift of step 3.

def sinc_weights(p, pd, taps):
    """w[m, p] proportional to sinc(t) (1 + cos(2 pi t / K)) / 2 for |t| < K / 2,
    zero beyond, with t the circular distance between beta_p and beta'_m in
    decimated steps (|p P' - m P| / P, as in triangle_weights) and K = taps
    (even); normalised so every row sums to one.  K = 2 has the triangle's
    support."""
    if taps < 2 or taps % 2:
        raise ValueError("taps must be an even number >= 2")
    pp = np.arange(p, dtype=np.int64)[None, :]
    mm = np.arange(pd, dtype=np.int64)[:, None]
    period = p * pd
    e = np.abs(pp * pd - mm * p) % period
    e = np.minimum(e, period - e)
    t = e / p
    inside = e * 2 < taps * p                      # |t| < K / 2, decided in integers
    w = np.where(inside, np.sinc(t) * 0.5 * (1.0 + np.cos(2.0 * np.pi * t / taps)), 0.0)
    return w / w.sum(axis=1, keepdims=True)


def decimation_weights(p, pd, window="triangle", taps=2):
    if window == "triangle":
        return triangle_weights(p, pd)
    if window == "sinc":
        return sinc_weights(p, pd, taps)
    raise ValueError(f"unknown decimation window {window!r}")


def keys_cubic(d):
    """Keys' cubic convolution kernel with a = -1/2 at distance d (samples):
    (a+2)|d|^3 - (a+3)|d|^2 + 1 on [0, 1], a|d|^3 - 5a|d|^2 + 8a|d| - 4a on
    (1, 2), zero beyond."""
    d = np.abs(np.asarray(d, dtype=np.float64))
    a = -0.5
    near = (a + 2.0) * d ** 3 - (a + 3.0) * d ** 2 + 1.0
    far = a * d ** 3 - 5.0 * a * d ** 2 + 8.0 * a * d - 4.0 * a
    return np.where(d <= 1.0, near, np.where(d < 2.0, far, 0.0))


def cascade121_weights(p, stages):
    """Decimation by 2^stages built as ``stages`` rounds of circular [1, 2, 1]/4
    smoothing followed by keeping the even samples (a half-band decimator).
    Returns the equivalent [P / 2^stages, P] matrix.  Requires 2^stages | P.
    Used only to pin ``triangle_weights``."""
    if p % (1 << stages):
        raise ValueError("cascade needs 2^stages to divide P")
    mat = np.eye(p)
    cur = p
    for _ in range(stages):
        smooth = np.zeros((cur, cur))
        for i in range(cur):
            smooth[i, (i - 1) % cur] += 0.25
            smooth[i, i] += 0.5
            smooth[i, (i + 1) % cur] += 0.25
        keep = smooth[0::2]
        mat = keep @ mat
        cur //= 2
    return mat


def u_taps(fu, interp):
    """Offsets from floor(u) and weights of the shift's interpolation in u:
    linear (Sec. 2.1), or Keys' cubic convolution (see keys_cubic)."""
    if interp == "linear":
        return ((0, 1.0 - fu), (1, fu))
    if interp == "cubic":
        return tuple((d, keys_cubic(fu - d)) for d in (-1, 0, 1, 2))
    raise ValueError(f"unknown interpolation {interp!r}")


def crop_shift(frows, sq, betas, r, n, interp="linear"):
    """Step 3: S[p, k, j] = Lin_u(q[p, rows[k], :], a_c(beta_p) + u0 + j), zero
    outside the detector, for every filtered row k (``interp="cubic"``: Keys'
    cubic kernel instead of the linear one)."""
    ac = centre_track(sq, betas, r)
    j = np.arange(sq.width, dtype=np.float64)
    nrow = len(frows.rows)
    out = np.zeros((len(betas), nrow, sq.width))
    for p in range(len(betas)):
        u = ac[p] + sq.u0 + j                          # index coordinates
        iu = np.floor(u).astype(np.int64)
        fu = u - iu
        row = frows.data[p]                            # [nrow, N]
        for d, w in u_taps(fu, interp):
            ui = iu + d
            ok = (ui >= 0) & (ui < n)
            out[p] += np.where(ok[None, :], w[None, :] * row[:, np.clip(ui, 0, n - 1)], 0.0)
    return out


def decimate(s_sub, weights):
    """Step 4: Y[m, k, j] = sum_p w[m, p] S[p, k, j]."""
    return np.tensordot(weights, s_sub, axes=(1, 0))


def backproject_square(y_sub, slot, nv, sq, betas_dec, r, n, x, y, z):
    """Step 5: f = (pi / P') sum_m U^-2 Bil(Y[m], v*, tau), with
    tau = a - a_c(beta'_m) + c_u - u0 (the folded second shift) and
    v* = b + c_v.  Rows outside the detector read zero; tau must lie in
    [0, W-1) by construction of the local grid, which is asserted."""
    cu = cv = g.centre(n)
    pd = len(betas_dec)
    ac = centre_track(sq, betas_dec, r)
    f = np.zeros(np.broadcast(x, y, z).shape)
    for m, beta in enumerate(betas_dec):
        u_mag = g.depth(x, y, beta, r) / r
        a = g.pix_pos(x, y, beta, r)
        b = g.row_pos(x, y, z, beta, r)
        tau = a - ac[m] + cu - sq.u0
        if tau.size and (tau.min() < 0.0 or tau.max() >= sq.width - 1):
            raise AssertionError("local column outside the square's grid")
        f += fdk_mod.bilinear(y_sub[m], slot, nv, b + cv, tau) / (u_mag * u_mag)
    return (np.pi / pd) * f


def _square_points(sq, n, nz, slices):
    c, cz = g.centre(n), g.centre(nz)
    zs = np.asarray(slices, dtype=np.float64) - cz
    ys = np.arange(sq.y0, sq.y1, dtype=np.float64) - c
    xs = np.arange(sq.x0, sq.x1, dtype=np.float64) - c
    return np.meshgrid(zs, ys, xs, indexing="ij")


def square_pipeline(frows, r, sq, betas, betas_dec, weights, x, y, z, store=None, interp="linear"):
    """Steps 3-5 for one square at the voxel coordinates (x, y, z) that lie
    inside it, from the filtered rows ``frows`` (which must hold every row the
    points touch).  ``store`` optionally rounds the decimated data to a storage
    type (see oracle.storage); the filtered rows are rounded by the caller."""
    n = frows.data.shape[-1]
    s_sub = crop_shift(frows, sq, betas, r, n, interp)
    y_sub = decimate(s_sub, weights)
    if store is not None:
        y_sub = store(y_sub)
    return backproject_square(y_sub, frows.slot, frows.nv, sq, betas_dec, r, n, x, y, z)


def _filtered(proj, r, betas_dec, pts, store):
    """Filter (once) every detector row that any of the point sets touches."""
    n = proj.shape[2]
    rows = np.unique(np.concatenate(
        [fdk_mod.rows_for_points(n, r, betas_dec, x, y, z) for (x, y, z) in pts] + [np.zeros(0, np.int64)]))
    frows = fdk_mod.filter_rows(proj, r, rows)
    if store is not None:
        frows.data = store(frows.data)
    return frows


def _rows_subset(frows, x, y, z, betas_dec, r):
    """Restrict filtered rows to those a square's points touch (keeps the
    crop of step 3 to the rows that square needs)."""
    n = frows.data.shape[-1]
    rows = fdk_mod.rows_for_points(n, r, betas_dec, x, y, z)
    sub = fdk_mod.FilteredRows(rows, frows.data[:, frows.slot[rows], :], frows.nv)
    return sub


def fdkod(proj, r, s, k=0, slices=None, nz=None, store=None, window="triangle", taps=2, interp="linear"):
    """FDK-OD of the listed slices (all by default).  Returns [S, N, N].
    ``window``, ``taps`` and ``interp`` select the decimation window and the
    shift's interpolation (the defaults are the paper's method)."""
    p_count, nv, n = proj.shape
    nz = n if nz is None else nz
    slices = np.arange(nz) if slices is None else np.asarray(slices)
    sqs, betas, betas_dec = plan(n, p_count, r, s, k)
    weights = decimation_weights(p_count, len(betas_dec), window, taps)
    pts = [tuple(reversed(_square_points(sq, n, nz, slices))) for sq in sqs]
    frows = _filtered(proj, r, betas_dec, pts, store)
    out = np.zeros((len(slices), n, n))
    for sq, (x, y, z) in zip(sqs, pts):
        sub = _rows_subset(frows, x, y, z, betas_dec, r)
        out[:, sq.y0:sq.y1, sq.x0:sq.x1] = square_pipeline(
            sub, r, sq, betas, betas_dec, weights, x, y, z, store, interp)
    return out


# ------------------------------------------------ cone-corrected decimation
#
# An extension beyond the paper (its Sec. 2.1 crops and shifts every detector
# row on its own and notes that the bounds stay roughly the same for all
# slices).  Off the mid-plane a voxel's detector row b = z R / D(beta)
# (eq. (9)) moves with the angle, so averaging a row over the decimation
# window blurs it.  The cone-corrected crop also resamples the rows, by the
# square centre's depth D_c(beta) = R + x_c cos beta + y_c sin beta:
#
#   S[p][v'][j] = Bil(q[p], (v' - c_v) R / D_c(beta_p) + c_v, a_c(beta_p) + u0 + j)
#
# so that a point above the square's centre keeps one warped row v' = z + c_v
# at every angle.  The reconstruction samples the warped data at
# v' = z D_c(beta') / D(beta') + c_v (the same eq. (9) in warped rows).

def cone_row_scale(sq, beta, r):
    """R / D_c(beta): detector row offset per warped row offset."""
    return r / g.depth(sq.xc, sq.yc, beta, r)


def crop_shift_cone(frows, sq, betas, r, n, interp="linear"):
    """Cone-corrected step 3 for every warped row v' = 0..N-1: S[p, v', j]
    (frows must hold every detector row); linear in v, ``interp`` in u."""
    if len(frows.rows) != frows.nv:
        raise ValueError("the cone-corrected crop needs every filtered row")
    cv = g.centre(n)
    ac = centre_track(sq, betas, r)
    j = np.arange(sq.width, dtype=np.float64)
    vw = np.arange(frows.nv, dtype=np.float64)
    out = np.zeros((len(betas), frows.nv, sq.width))
    for p, beta in enumerate(betas):
        rows = (vw - cv) * cone_row_scale(sq, beta, r) + cv
        out[p] = sample_vu(frows.data[p], frows.slot, frows.nv, rows[:, None],
                           (ac[p] + sq.u0 + j)[None, :], interp)
    return out


def sample_vu(img, slot, nv, v, u, interp="linear"):
    """img sampled at index coordinates (v, u): linear in v, ``interp`` in u,
    zero outside [0, nv) x [0, nu) (bilinear for interp="linear")."""
    if interp == "linear":
        return fdk_mod.bilinear(img, slot, nv, v, u)
    nu = img.shape[-1]
    v = np.asarray(v, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    iv = np.floor(v).astype(np.int64)
    iu = np.floor(u).astype(np.int64)
    fv = v - iv
    out = np.zeros(np.broadcast(v, u).shape)
    for dv, wv in ((0, 1.0 - fv), (1, fv)):
        vi = iv + dv
        vin = (vi >= 0) & (vi < nv)
        kk = slot[np.clip(vi, 0, nv - 1)]
        if np.any(vin & (kk < 0)):
            raise KeyError("detector row needed but not filtered")
        for du, wu in u_taps(u - iu, interp):
            ui = iu + du
            ok = vin & (ui >= 0) & (ui < nu)
            out += np.where(ok, wv * wu * img[np.clip(kk, 0, None), np.clip(ui, 0, nu - 1)], 0.0)
    return out


def cone_row(sq, x, y, z, beta, r):
    """Warped row offset v' - c_v = z D_c(beta) / D(beta) of voxel (x, y, z)."""
    return z * g.depth(sq.xc, sq.yc, beta, r) / g.depth(x, y, beta, r)


def backproject_square_cone(y_sub, nv, sq, betas_dec, r, n, x, y, z, slot=None):
    """Step 5 on cone-corrected data Y[m, v', j]: as backproject_square, with
    the row coordinate cone_row + c_v.  ``slot`` maps warped rows to the rows
    of y_sub (all rows by default; -1 = not computed)."""
    cu = cv = g.centre(n)
    pd = len(betas_dec)
    ac = centre_track(sq, betas_dec, r)
    slot = np.arange(nv) if slot is None else slot
    f = np.zeros(np.broadcast(x, y, z).shape)
    for m, beta in enumerate(betas_dec):
        u_mag = g.depth(x, y, beta, r) / r
        a = g.pix_pos(x, y, beta, r)
        tau = a - ac[m] + cu - sq.u0
        if tau.size and (tau.min() < 0.0 or tau.max() >= sq.width - 1):
            raise AssertionError("local column outside the square's grid")
        f += fdk_mod.bilinear(y_sub[m], slot, nv, cone_row(sq, x, y, z, beta, r) + cv, tau) / (u_mag * u_mag)
    return (np.pi / pd) * f


def fdkod_cone(proj, r, s, k=0, slices=None, nz=None, store=None, window="triangle", taps=2,
               interp="linear"):
    """FDK-OD with the cone-corrected decimation, listed slices (all by
    default).  Filters every detector row.  Returns [S, N, N]."""
    p_count, nv, n = proj.shape
    nz = n if nz is None else nz
    slices = np.arange(nz) if slices is None else np.asarray(slices)
    sqs, betas, betas_dec = plan(n, p_count, r, s, k)
    weights = decimation_weights(p_count, len(betas_dec), window, taps)
    frows = fdk_mod.filter_rows(proj, r, np.arange(nv))
    if store is not None:
        frows.data = store(frows.data)
    out = np.zeros((len(slices), n, n))
    for sq in sqs:
        z, y, x = _square_points(sq, n, nz, slices)
        y_sub = decimate(crop_shift_cone(frows, sq, betas, r, n, interp), weights)
        if store is not None:
            y_sub = store(y_sub)
        out[:, sq.y0:sq.y1, sq.x0:sq.x1] = backproject_square_cone(y_sub, nv, sq, betas_dec, r, n, x, y, z)
    return out


def cone_rows_for_points(n, nv, r, sq, betas, betas_dec, x, y, z):
    """Warped rows that the cone-corrected backprojection of the points reads
    (both bilinear neighbours, at every decimated angle) and the detector rows
    that those warped rows are resampled from at every original angle."""
    cv = g.centre(n)
    iv = np.floor(np.array([cone_row(sq, x, y, z, b, r) for b in betas_dec]) + cv).astype(np.int64)
    warped = np.unique(np.concatenate([iv.ravel(), iv.ravel() + 1]))
    warped = warped[(warped >= 0) & (warped < nv)]
    det = set()
    for beta in betas:
        f = np.floor((warped - cv) * cone_row_scale(sq, beta, r) + cv).astype(np.int64)
        det.update(f.tolist())
        det.update((f + 1).tolist())
    det = np.array(sorted(d for d in det if 0 <= d < nv), dtype=np.int64)
    return warped, det


def fdkod_cone_points(proj, r, s, k, idx, nz=None, store=None, window="triangle", taps=2, interp="linear"):
    """Cone-corrected FDK-OD at voxel indices ``idx`` ([K, 3] array of
    (l, j, i)): the same steps as fdkod_cone, restricted to the warped rows
    the voxels read and the detector rows those are resampled from."""
    p_count, nv, n = proj.shape
    nz = n if nz is None else nz
    idx = np.asarray(idx)
    sqs, betas, betas_dec = plan(n, p_count, r, s, k)
    weights = decimation_weights(p_count, len(betas_dec), window, taps)
    qid = np.array([square_of(n, s, i, j) for (_, j, i) in idx])
    c, cz = g.centre(n), g.centre(nz)
    groups, det_all = [], []
    for q in np.unique(qid):
        sel = qid == q
        x, y, z = idx[sel, 2] - c, idx[sel, 1] - c, idx[sel, 0] - cz
        warped, det = cone_rows_for_points(n, nv, r, sqs[q], betas, betas_dec, x, y, z)
        groups.append((q, sel, (x, y, z), warped))
        det_all.append(det)
    rows = np.unique(np.concatenate(det_all + [np.zeros(0, np.int64)]))
    frows = fdk_mod.filter_rows(proj, r, rows)
    if store is not None:
        frows.data = store(frows.data)
    cv = g.centre(n)
    out = np.zeros(len(idx))
    for q, sel, (x, y, z), warped in groups:
        sq = sqs[q]
        ac = centre_track(sq, betas, r)
        j = np.arange(sq.width, dtype=np.float64)
        s_sub = np.zeros((len(betas), len(warped), sq.width))
        for p, beta in enumerate(betas):
            rp = (warped - cv) * cone_row_scale(sq, beta, r) + cv
            s_sub[p] = sample_vu(frows.data[p], frows.slot, frows.nv, rp[:, None],
                                 (ac[p] + sq.u0 + j)[None, :], interp)
        y_sub = decimate(s_sub, weights)
        if store is not None:
            y_sub = store(y_sub)
        slot = np.full(nv, -1, dtype=np.int64)
        slot[warped] = np.arange(len(warped))
        out[sel] = backproject_square_cone(y_sub, nv, sq, betas_dec, r, n, x, y, z, slot)
    return out


def square_of(n, s, i, j):
    """Index q of the square that holds voxel column i, row j."""
    b = g.blocks(n, 2 ** s)
    bx = next(t for t, (a0, a1) in enumerate(b) if a0 <= i < a1)
    by = next(t for t, (a0, a1) in enumerate(b) if a0 <= j < a1)
    return by * (2 ** s) + bx


def fdkod_points(proj, r, s, k, idx, nz=None, store=None, window="triangle", taps=2, interp="linear"):
    """FDK-OD at voxel indices ``idx`` ([K, 3] array of (l, j, i))."""
    p_count, nv, n = proj.shape
    nz = n if nz is None else nz
    idx = np.asarray(idx)
    sqs, betas, betas_dec = plan(n, p_count, r, s, k)
    weights = decimation_weights(p_count, len(betas_dec), window, taps)
    qid = np.array([square_of(n, s, i, j) for (_, j, i) in idx])
    c, cz = g.centre(n), g.centre(nz)
    groups = []
    for q in np.unique(qid):
        sel = qid == q
        groups.append((q, sel, (idx[sel, 2] - c, idx[sel, 1] - c, idx[sel, 0] - cz)))
    frows = _filtered(proj, r, betas_dec, [pt for (_, _, pt) in groups], store)
    out = np.zeros(len(idx))
    for q, sel, (x, y, z) in groups:
        sub = _rows_subset(frows, x, y, z, betas_dec, r)
        out[sel] = square_pipeline(sub, r, sqs[q], betas, betas_dec, weights, x, y, z, store, interp)
    return out


def cost_counts(n, nz, p, r, s, k):
    """Counters of the two costs of Sec. 2.2: cropped samples of the
    decomposition (eq. (7): 4^s squares x N rows x W_q columns x P angles) and
    voxel-angle updates of the reconstruction (eq. (6): N^2 N_z P')."""
    sqs, betas, betas_dec = plan(n, p, r, s, k)
    cropped = sum(sq.width for sq in sqs) * p * n
    updates = n * n * nz * len(betas_dec)
    return cropped, updates
