"""Pins of the cone-corrected decimation in the oracle (an extension beyond
the paper: rows resampled by the square centre's depth before the angular
decimation)."""

import numpy as np
import pytest

from oracle import fdk, fdkod, geometry as g
from synth import phantom


def _thin_discs():
    """Thin discs far off the mid-plane plus a faint body (normalised units)."""
    return phantom.Ellipsoids(
        np.array([[0.0, 0.0, 0.55], [0.2, -0.3, -0.5], [-0.3, 0.2, 0.45], [0.0, 0.0, 0.0]]),
        np.array([[0.6, 0.6, 0.04], [0.4, 0.4, 0.05], [0.3, 0.3, 0.04], [0.7, 0.7, 0.7]]),
        np.array([1.0, 1.0, 1.0, 0.2]))


def _rel(a, b):
    return np.sqrt(np.mean((a - b) ** 2)) / np.sqrt(np.mean(b ** 2))


def test_one_square_is_direct_fdk():
    """s = 0: the square's centre is the axis, D_c = R, the warp is the identity."""
    n, p, r = 33, 40, 64.0
    proj = phantom.project(phantom.random_ellipsoids(6, 1), n, p, r).double().numpy()
    a = fdkod.fdkod_cone(proj, r, 0)
    b = fdk.fdk(proj, r)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_mid_plane_equals_plain_decimation():
    """z = 0 maps to warped row c_v, which the crop reads from detector row c_v
    (N odd, so c_v is a row): the mid-plane slice is the plain FDK-OD's."""
    n, p, r = 33, 48, 64.0
    proj = phantom.project(phantom.random_ellipsoids(6, 2), n, p, r).double().numpy()
    mid = [n // 2]
    a = fdkod.fdkod_cone(proj, r, 2, slices=mid)
    b = fdkod.fdkod(proj, r, 2, slices=mid)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_crop_scales_rows_by_r_over_centre_depth():
    """Rows linear in v, q[p, v, u] = (v - c_v) h[p, u]: bilinear sampling is
    exact on them, so the crop must give (v' - c_v) R / D_c(beta_p) times the
    plain crop of h, on every warped row that stays inside the detector."""
    n, p, r = 41, 12, 60.0
    rng = np.random.default_rng(3)
    h = rng.standard_normal((p, n))
    cv = g.centre(n)
    data = (np.arange(n) - cv)[None, :, None] * h[:, None, :]
    frows = fdk.FilteredRows(np.arange(n), data, n)
    sqs, betas, _ = fdkod.plan(n, p, r, 2, 0)
    sq = sqs[5]
    got = fdkod.crop_shift_cone(frows, sq, betas, r, n)                # [P, v', W]
    flat = fdk.FilteredRows(np.arange(1), h[:, None, :], 1)
    base = fdkod.crop_shift(flat, sq, betas, r, n)[:, 0, :]             # [P, W]
    for pp, beta in enumerate(betas):
        sc = r / g.depth(sq.xc, sq.yc, beta, r)
        vw = np.arange(n) - cv
        inside = np.abs(vw * sc) <= cv - 1.0
        want = (vw * sc)[:, None] * base[pp][None, :]
        assert np.allclose(got[pp][inside], want[inside], atol=1e-12 * np.max(np.abs(want)))


def test_backprojection_row_is_z_times_centre_over_voxel_depth():
    """Warped data linear in v' and constant along columns, Y = v' - c_v: the
    reconstruction is (pi / P') sum_m (R / D_m)^2 z D_c,m / D_m."""
    n, p, r = 41, 24, 60.0
    sqs, betas, betas_dec = fdkod.plan(n, p, r, 2, 0)
    sq = sqs[9]
    pd = len(betas_dec)
    cv = g.centre(n)
    y_sub = np.broadcast_to((np.arange(n) - cv)[None, :, None], (pd, n, sq.width)).copy()
    c = g.centre(n)
    x = np.array([sq.x0 - c, sq.x1 - 1 - c, 0.5 * (sq.x0 + sq.x1 - 1) - c])
    y = np.array([sq.y0 - c, sq.y1 - 1 - c, 0.5 * (sq.y0 + sq.y1 - 1) - c])
    z = np.array([7.0, -9.0, 11.0])
    got = fdkod.backproject_square_cone(y_sub, n, sq, betas_dec, r, n, x, y, z)
    want = np.zeros(3)
    for beta in betas_dec:
        d = r + x * np.cos(beta) + y * np.sin(beta)
        dc = r + sq.xc * np.cos(beta) + sq.yc * np.sin(beta)
        want += (r / d) ** 2 * z * dc / d
    want *= np.pi / pd
    assert np.allclose(got, want, rtol=1e-12)


def test_cone_correction_reduces_off_midplane_error():
    """Thin discs at z = +-0.5 N/2, D = 16: the plain decimation averages rows
    that a voxel's trajectory crosses; the corrected one follows the square's
    centre.  Error against direct FDK on two off-midplane slices."""
    n, p, r, s = 96, 96, 192.0, 4
    proj = phantom.project(_thin_discs(), n, p, r).double().numpy()
    cz = (n - 1) / 2.0
    sl = [int(cz + 0.55 * n / 2), int(cz - 0.5 * n / 2)]
    ref = fdk.fdk(proj, r, slices=sl)
    plain = _rel(fdkod.fdkod(proj, r, s, 0, slices=sl), ref)
    cone = _rel(fdkod.fdkod_cone(proj, r, s, 0, slices=sl), ref)
    assert cone <= 0.7 * plain, (plain, cone)


@pytest.mark.parametrize("knobs", [{}, dict(window="sinc", taps=4, interp="cubic")])
def test_points_form_equals_volume_form(knobs):
    """The sampled-voxel form (only the rows the voxels need) gives the volume
    form's values, top and bottom slices and a ragged square included."""
    n, nz, p, r, s = 40, 36, 48, 96.0, 2
    proj = phantom.project(phantom.random_ellipsoids(6, 8), n, p, r).double().numpy()
    vol = fdkod.fdkod_cone(proj, r, s, 0, nz=nz, **knobs)
    rng = np.random.default_rng(4)
    idx = np.stack([rng.integers(0, nz, 25), rng.integers(0, n, 25), rng.integers(0, n, 25)], axis=1)
    idx = np.concatenate([idx, [[0, 3, 37], [nz - 1, 39, 0], [nz // 2, 20, 20]]])
    got = fdkod.fdkod_cone_points(proj, r, s, 0, idx, nz=nz, **knobs)
    want = vol[idx[:, 0], idx[:, 1], idx[:, 2]]
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * np.max(np.abs(vol)))
