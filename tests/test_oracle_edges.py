"""Pins of the oracle's zero extension at the detector's edges.

The library reads interpolation outside the detector as zero, with no field-of-
view mask and no clamping: every neighbour with an index outside [0, N) adds
nothing.  These are fixed values worked out by hand for samples straddling
the first and last column and row, so that clamping to the edge, wrapping
around, or an off-by-one at the upper bound fails here."""

import numpy as np
import pytest

from oracle import fdk, fdkod, geometry as g


NV, NU = 6, 7


def _ramp_image():
    # every entry non-zero and distinct: img[v, u] = 10 v + u + 1
    v, u = np.meshgrid(np.arange(NV), np.arange(NU), indexing="ij")
    return (10.0 * v + u + 1.0)


@pytest.mark.parametrize("v,u,want", [
    (2.0, NU - 0.5, 1.5),          # half a pixel beyond the last column: half the constant
    (2.0, -0.5, 1.5),              # half a pixel before the first column
    (NV - 0.5, 3.0, 1.5),          # half a pixel beyond the last row
    (-0.5, 3.0, 1.5),              # half a pixel before the first row
    (-0.5, -0.5, 0.75),            # a corner: one of four neighbours inside
    (NV - 0.5, NU - 0.5, 0.75),
    (2.0, -0.25, 2.25),            # u in (-1, 0): weight 0.75 on column 0
    (2.0, NU - 0.75, 3.0 * 0.75),  # u in (N-1, N): weight 0.75 on column N-1
    (2.0, float(NU), 0.0),         # at column N: both neighbours outside
    (2.0, -1.0, 0.0),              # at column -1: all weight on column -1
    (float(NV), 3.0, 0.0),
    (-1.0, 3.0, 0.0),
    (2.0, NU + 3.7, 0.0),          # far outside
    (-5.2, 3.0, 0.0),
])
def test_bilinear_zero_extension_constant(v, u, want):
    img = np.full((NV, NU), 3.0)
    got = fdk.bilinear(img, np.arange(NV), NV, np.array([v]), np.array([u]))[0]
    assert got == pytest.approx(want, abs=1e-14)


def test_bilinear_edges_read_zero_not_the_edge_value():
    img = _ramp_image()
    slot = np.arange(NV)
    # (v, u) -> the hand-computed value: only the inside neighbour, with its weight
    cases = [((2.0, -0.3), 0.7 * 21.0),                 # not 21 (clamp), not 0.3*27 + 0.7*21 (wrap)
             ((2.0, NU - 1 + 0.4), 0.6 * 27.0),         # not 27 (clamp)
             ((-0.3, 3.0), 0.7 * 4.0),
             ((NV - 1 + 0.4, 3.0), 0.6 * 54.0),
             ((-0.5, -0.5), 0.25 * 1.0),
             ((NV - 1 + 0.25, NU - 1 + 0.5), 0.75 * 0.5 * 57.0)]
    for (v, u), want in cases:
        got = fdk.bilinear(img, slot, NV, np.array([v]), np.array([u]))[0]
        assert got == pytest.approx(want, abs=1e-12), (v, u)


def test_backprojection_of_points_beyond_the_last_row():
    # on the rotation axis (x = y = 0) every angle has depth R, U = 1, a = 0
    # and b = z (eq. (1), eq. (9)), so the sample sits at column c_u and row
    # z + c_v for every projection: f = (pi / P) P Bil = pi Bil.
    n, r, p = 7, 50.0, 4
    cv = g.centre(n)
    betas = g.angles(p)
    frows = fdk.FilteredRows(np.arange(n), np.full((p, n, n), 2.0), n)
    zs = np.array([n - 0.5 - cv, -0.5 - cv, n - cv, -1.0 - cv, 0.0, n - 0.75 - cv])
    want = np.pi * np.array([1.0, 1.0, 0.0, 0.0, 2.0, 0.75 * 2.0])   # row n - 0.75: 0.75 on row n - 1
    got = fdk.backproject_points(frows, r, betas, np.zeros(6), np.zeros(6), zs)
    assert np.allclose(got, want, atol=1e-13)
    # the folded FDK-OD backprojection reads its decimated rows the same way
    sq = fdkod.Square(0, n, 0, n, 0.0, 0.0, u0=0, width=n)
    y_sub = np.full((p, n, n), 2.0)                       # [P', rows, W]
    got = fdkod.backproject_square(y_sub, np.arange(n), n, sq, betas, r, n, np.zeros(6), np.zeros(6), zs)
    assert np.allclose(got, want, atol=1e-13)


def test_backprojection_of_a_point_projecting_off_the_detector():
    # one angle (beta = 0): a = y, b = z; a point whose column lies beyond the
    # last one reads zero, half a column beyond reads half
    n, r = 7, 50.0
    cu = g.centre(n)
    frows = fdk.FilteredRows(np.arange(n), np.full((1, n, n), 2.0), n)
    ys = np.array([n - 0.5 - cu, n + 0.2 - cu, -0.5 - cu, -1.5 - cu])
    got = fdk.backproject_points(frows, r, np.array([0.0]), np.zeros(4), ys, np.zeros(4))
    assert np.allclose(got, np.pi * np.array([1.0, 0.0, 1.0, 0.0]), atol=1e-13)


def test_crop_shift_zero_extension():
    # A square centred at (0, 1/4): at beta = 0, eq. (1) gives a_c = R (1/4) / R
    # = 1/4, so local column j sits at detector column 1/4 + u0 + j.  With
    # u0 = -2 and W = N + 4 the crop runs from column -1.75 to N + 0.25.
    n, r = 9, 40.0
    row = np.arange(n, dtype=np.float64) + 1.0            # q[u] = u + 1, non-zero
    frows = fdk.FilteredRows(np.array([0]), row[None, None, :], n)
    sq = fdkod.Square(0, 1, 0, 1, 0.0, 0.25, u0=-2, width=n + 4)
    got = fdkod.crop_shift(frows, sq, np.array([0.0]), r, n)[0, 0]
    want = np.zeros(n + 4)
    want[0] = 0.0                                         # column -1.75: both neighbours outside
    want[1] = 0.25 * row[0]                               # column -0.75: fu = 0.25 on column 0
    for j in range(2, n + 1):                             # columns 0.25 .. n - 1.75: inside
        want[j] = 0.75 * row[j - 2] + 0.25 * row[j - 1]
    want[n + 1] = 0.75 * row[n - 1]                       # column n - 0.75: column n is outside
    want[n + 2] = 0.0                                     # column n + 0.25
    want[n + 3] = 0.0
    assert np.allclose(got, want, atol=1e-13)
    # an integer trajectory (a square centred on the axis) is an exact copy,
    # with zeros where the grid leaves the detector
    sq0 = fdkod.Square(0, 1, 0, 1, 0.0, 0.0, u0=-3, width=n + 5)
    frows3 = fdk.FilteredRows(np.array([0]), np.tile(row, (3, 1, 1)), n)
    got0 = fdkod.crop_shift(frows3, sq0, np.array([0.0, 1.3, 4.0]), r, n)[:, 0]
    want0 = np.concatenate([np.zeros(3), row, np.zeros(2)])
    assert np.allclose(got0, want0[None, :], atol=1e-12)
