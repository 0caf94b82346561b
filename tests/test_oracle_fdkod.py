"""Pins of the oracle's FDK-OD (Sec. 2.1 and 2.2 of the paper)."""

import os

import numpy as np
import pytest
import torch

from oracle import fdk, fdkod, geometry as g, metrics
from synth import phantom

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def small_scan():
    ell = phantom.random_ellipsoids(10, 1)
    n, p, r = 32, 48, 256.0
    proj = phantom.project(ell, n, p, r, out_dtype=torch.float64).numpy()
    return proj, r


def test_s0_equals_direct_fdk(small_scan):
    # with one square the centre trajectory is the detector centre, the local
    # grid is the detector grid and D = 1: FDK-OD is FDK (Sec. 2.2 with s = 0)
    proj, r = small_scan
    slices = [0, 9, 16, 31]
    ref = fdk.fdk(proj, r, slices=slices)
    got = fdkod.fdkod(proj, r, 0, 0, slices=slices)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_decimation_d1_is_identity():
    assert np.array_equal(fdkod.triangle_weights(37, 37), np.eye(37))


@pytest.mark.parametrize("p,pd", [(90, 23), (179, 45), (717, 90), (720, 45), (7, 4)])
def test_decimation_rows_sum_to_one_and_are_symmetric(p, pd):
    w = fdkod.triangle_weights(p, pd)
    assert np.allclose(w.sum(axis=1), 1.0, atol=1e-14)
    assert np.all(w >= 0)
    # support: only angles closer than one decimated step contribute
    betas, bd = g.angles(p), g.angles(pd)
    diff = np.abs(betas[None, :] - bd[:, None])
    dc = np.minimum(diff, 2 * np.pi - diff)
    assert np.all(w[dc >= 2 * np.pi / pd - 1e-12] == 0)
    # symmetric in angle about every decimated angle when D divides P
    if p % pd == 0:
        d = p // pd
        for m in range(pd):
            for t in range(1, d):
                assert w[m, (m * d + t) % p] == pytest.approx(w[m, (m * d - t) % p], abs=1e-15)


@pytest.mark.parametrize("stages", [1, 2, 3, 4])
def test_triangle_equals_cascade_of_halfband_stages(stages):
    # Sec. 2.1: filtering + downsampling by 2 per stage; cascading the
    # [1, 2, 1]/4 half-band filter with keep-even gives the triangle of
    # half-width D = 2^stages (built independently here by repeated stages)
    p = 96
    d = 1 << stages
    cas = fdkod.cascade121_weights(p, stages)
    tri = fdkod.triangle_weights(p, p // d)
    assert np.allclose(cas, tri, atol=1e-14)


def test_triangle_d4_matches_golden():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "triangle_D4.txt"))
            if not l.startswith("#")]
    golden = {int(o): int(nm) / 16.0 for o, nm in rows}
    w = fdkod.triangle_weights(64, 16)
    for m in (0, 5, 15):
        for off, val in golden.items():
            assert w[m, (4 * m + off) % 64] == pytest.approx(val, abs=1e-15)
        assert np.count_nonzero(w[m]) == 7


CASES = [(8, 1, 20.0, 7), (12, 2, 9.0, 16), (16, 2, 64.0, 90), (16, 3, 12.0, 16),
         (32, 3, 100.0, 90), (32, 2, 25.0, 7), (10, 2, 40.0, 16)]


@pytest.mark.parametrize("n,s,r,p", CASES)
def test_vertex_bounds_contain_every_voxel_bruteforce(n, s, r, p):
    # Sec. 2.1: the extremes of eq. (1) over a square are at its vertices.
    # Brute force over every voxel centre and a dense grid of points of each
    # square, at every angle.
    c = g.centre(n)
    betas = g.angles(p)
    for sq in fdkod.make_squares(n, s):
        amin, amax = fdkod.vertex_bounds(sq, n, betas, r)
        xs = np.linspace(sq.x0 - c, sq.x1 - 1 - c, 23)
        ys = np.linspace(sq.y0 - c, sq.y1 - 1 - c, 23)
        x, y = np.meshgrid(xs, ys)
        for t, beta in enumerate(betas):
            a = g.pix_pos(x, y, beta, r)
            assert a.min() >= amin[t] - 1e-9 and a.max() <= amax[t] + 1e-9


@pytest.mark.parametrize("n,s,r,p", CASES)
@pytest.mark.parametrize("k", [0, 1])
def test_local_grid_covers_every_bilinear_footprint(n, s, r, p, k):
    # every voxel of the square, at every decimated angle, lands on local
    # columns tau in [0, W-1), so both bilinear neighbours exist
    if k > s:
        pytest.skip("k > s")
    sqs, betas, bd = fdkod.plan(n, p, r, s, k)
    c = g.centre(n)
    for sq in sqs:
        ac = fdkod.centre_track(sq, bd, r)
        i, j = np.meshgrid(np.arange(sq.x0, sq.x1), np.arange(sq.y0, sq.y1))
        for m, beta in enumerate(bd):
            tau = g.pix_pos(i - c, j - c, beta, r) - ac[m] + c - sq.u0
            assert tau.min() >= 0.0 and tau.max() < sq.width - 1


def test_fdkod_is_linear(small_scan):
    proj, r = small_scan
    rng = np.random.default_rng(7)
    q2 = rng.standard_normal(proj.shape)
    sl = [3, 16]
    f1 = fdkod.fdkod(proj, r, 2, 0, slices=sl)
    f2 = fdkod.fdkod(q2, r, 2, 0, slices=sl)
    f12 = fdkod.fdkod(1.5 * proj + q2, r, 2, 0, slices=sl)
    assert np.allclose(f12, 1.5 * f1 + f2, rtol=0, atol=1e-11 * np.abs(f12).max())


@pytest.mark.parametrize("s,k", [(1, 0), (2, 0), (2, 1)])
def test_fdkod_keeps_uniform_regions_and_positions(s, k):
    # Sec. 4: decomposition leaves uniform regions almost unchanged and moves
    # nothing; the interior of an off-centre sphere stays at its density
    n, p, r = 64, 360, 128.0
    centre = (0.3, -0.35, 0.0)
    ell = phantom.sphere(centre, 0.25, 1.0)
    proj = phantom.project(ell, n, p, r, out_dtype=torch.float64).numpy()
    vol = fdkod.fdkod(proj, r, s, k, slices=[31, 32])
    x, y, z = fdk.voxel_grid(n, n, [31, 32])
    dist = np.sqrt((x - centre[0] * 32) ** 2 + (y - centre[1] * 32) ** 2 + z ** 2)
    assert vol[dist < 8 - 3].mean() == pytest.approx(1.0, abs=0.015)
    wgt = np.clip(vol, 0, None) * (dist < 8 + 3)
    assert np.sum(wgt * x) / np.sum(wgt) == pytest.approx(centre[0] * 32, abs=0.25)
    assert np.sum(wgt * y) / np.sum(wgt) == pytest.approx(centre[1] * 32, abs=0.25)


def test_skipping_a_stage_moves_closer_to_fdk():
    # Sec. 2.2: skipping a decimation stage improves sharpness; with k = s no
    # decimation is left and only the interpolation difference remains
    ell = phantom.random_ellipsoids(10, 1)
    n, p, r = 64, 90, 512.0
    proj = phantom.project(ell, n, p, r, out_dtype=torch.float64).numpy()
    sl = [20, 32, 44]
    ref = fdk.fdk(proj, r, slices=sl)
    errs = [metrics.rel_rmse(fdkod.fdkod(proj, r, 2, k, slices=sl), ref) for k in (0, 1, 2)]
    assert errs[0] > errs[1] > errs[2]


def test_points_driver_matches_slices(small_scan):
    proj, r = small_scan
    n = proj.shape[2]
    sl = [0, 13, 31]
    vol = fdkod.fdkod(proj, r, 2, 1, slices=sl)
    rng = np.random.default_rng(2)
    idx = np.stack([rng.choice(sl, 50), rng.integers(0, n, 50), rng.integers(0, n, 50)], axis=1)
    got = fdkod.fdkod_points(proj, r, 2, 1, idx)
    lut = {l: t for t, l in enumerate(sl)}
    ref = np.array([vol[lut[l], j, i] for l, j, i in idx])
    assert np.allclose(got, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n,p,s,k", [(64, 90, 2, 0), (64, 96, 2, 0), (48, 96, 3, 1), (2000, 720, 4, 0)])
def test_cost_counters(n, p, s, k):
    # eq. (6): reconstruction visits every voxel once per decimated angle;
    # when 2^(s-k) divides P that is N^3 P / 2^(s-k).  eq. (7): cropping reads
    # W_q columns of every row at every angle for each of the 4^s squares,
    # W_q ~ N / 2^s plus the spread of the square's footprint.
    cropped, updates = fdkod.cost_counts(n, n, p, 4.0 * n, s, k)
    d = 1 << (s - k)
    assert updates == n ** 3 * (-(-p // d))
    if p % d == 0:
        assert updates * d == n ** 3 * p
    # W_q lies between the square's side and its diagonal magnified by the
    # largest R / depth, plus the two interpolation columns
    per_square = cropped / (4 ** s * n * p)
    side = n / 2 ** s
    r = 4.0 * n
    assert side <= per_square <= np.sqrt(2) * side * r / (r - (n - 1) / np.sqrt(2)) + 2
