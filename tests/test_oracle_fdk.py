"""Pins of the oracle's FDK (textbook FDK, which the paper builds on)."""

import numpy as np
import pytest
import torch

from oracle import fdk, geometry as g, metrics
from synth import phantom


def test_ramlak_sums_to_zero():
    # sum_n h[n] = 1/4 - (2/pi^2) sum_{odd n>0} 1/n^2 = 1/4 - (2/pi^2)(pi^2/8) = 0;
    # the tail beyond K is below 1/(pi^2 K)
    k = 20001
    total = fdk.ramlak(np.arange(-k, k + 1)).sum()
    assert abs(total) < 1.0 / (np.pi ** 2 * k)


def test_ramlak_frequency_response_is_ramp():
    # the kernel is the band-limited ramp: its DTFT is |w| for |w| <= 1/2
    # (w in cycles per detector pixel); truncation error is O(1/K)
    k = 4000
    n = np.arange(-k, k + 1)
    h = fdk.ramlak(n)
    for w in (0.02, 0.1, 0.25, 0.4, 0.49):
        resp = np.sum(h * np.cos(2 * np.pi * w * n))
        assert resp == pytest.approx(abs(w), abs=2e-4)


@pytest.mark.parametrize("n", [8, 64, 101])
def test_fft_filter_equals_direct_convolution(n):
    rng = np.random.default_rng(n)
    rows = rng.standard_normal((5, n)) * 100 + 50
    direct = np.array([[np.sum(fdk.ramlak(u - np.arange(n)) * row) for u in range(n)]
                       for row in rows])
    assert np.allclose(fdk.ramp_filter(rows), direct, rtol=0, atol=1e-11)
    assert np.allclose(fdk.ramp_filter_fft(rows), direct, rtol=0, atol=1e-10)


def test_cosine_weight_is_ray_obliquity():
    # R / |Q - S| with the source at distance R and Q on the virtual detector
    n, r = 16, 40.0
    w = fdk.cosine_weight(n, r)
    c = g.centre(n)
    for v in (0, 7, 15):
        for u in (0, 3, 15):
            src = np.array([-r, 0.0, 0.0])
            q = np.array([0.0, u - c, v - c])
            assert w[v, u] == pytest.approx(r / np.linalg.norm(q - src), rel=1e-14)


def _sphere_recon(centre, radius, slices, n=64, p=180, r=60.0):
    ell = phantom.sphere(centre, radius, 1.0)
    proj = phantom.project(ell, n, p, r, out_dtype=torch.float64).numpy()
    vol = fdk.fdk(proj, r, slices=list(slices))
    x, y, z = fdk.voxel_grid(n, n, list(slices))
    scale = n / 2
    dist = np.sqrt((x - centre[0] * scale) ** 2 + (y - centre[1] * scale) ** 2
                   + (z - centre[2] * scale) ** 2)
    return vol, (x, y, z), dist, radius * scale


@pytest.mark.parametrize("centre", [(0.0, 0.0, 0.0), (0.45, -0.3, 0.0), (-0.4, 0.35, 0.0)])
def test_fdk_recovers_density_and_position(centre):
    # central slices: FDK reduces to fan-beam FBP, so the interior of a
    # uniform sphere reconstructs to its density.  R = 60 for N = 64 is close
    # to the validity limit (44.5), so the distance weight U^-2 and the cosine
    # weight change the off-centre interior by 4-8 % when wrong.
    vol, (x, y, z), dist, rad = _sphere_recon(centre, 0.25, (31, 32))
    interior = dist < rad - 3.0
    assert vol[interior].mean() == pytest.approx(1.0, abs=0.01)
    wgt = np.clip(vol, 0, None) * (dist < rad + 3)
    assert np.sum(wgt * x) / np.sum(wgt) == pytest.approx(centre[0] * 32, abs=0.25)
    assert np.sum(wgt * y) / np.sum(wgt) == pytest.approx(centre[1] * 32, abs=0.25)


def test_fdk_off_midplane_sphere():
    # a sphere above the mid-plane: FDK is approximate there, but for a
    # 9-degree cone the interior stays within 2 % and the z position holds
    centre = (0.1, -0.15, 0.4)
    slices = list(range(10, 64))
    vol, (x, y, z), dist, rad = _sphere_recon(centre, 0.22, slices, r=96.0)
    interior = dist < rad - 3.0
    assert vol[interior].mean() == pytest.approx(1.0, abs=0.02)
    wgt = np.clip(vol, 0, None) * (dist < rad + 3)
    assert np.sum(wgt * z) / np.sum(wgt) == pytest.approx(centre[2] * 32, abs=0.3)


def _ray_plane(x, y, z, beta, r):
    """Source-through-point line meets the plane through the axis normal to
    the central ray: returns (lateral, vertical, depth along central ray)."""
    d = np.array([np.cos(beta), np.sin(beta), 0.0])
    src = -r * d
    pt = np.array([x, y, z])
    t = -np.dot(src, d) / np.dot(pt - src, d)
    q = src + t * (pt - src)
    lat = np.dot(q, np.array([-np.sin(beta), np.cos(beta), 0.0]))
    return lat, q[2], np.dot(pt - src, d)


def test_backprojection_of_affine_data_is_exact():
    # bilinear interpolation reproduces affine data exactly, so backprojecting
    # q_p(u, v) = al_p u + ga_p v + de_p must give the weighted sum of the
    # affine values at the projected positions (positions from an explicit
    # ray / plane intersection; distance weight (R / depth)^2)
    n, p, r = 20, 9, 50.0
    rng = np.random.default_rng(5)
    al, ga, de = rng.standard_normal((3, p))
    uu = np.arange(n)[None, None, :]
    vv = np.arange(n)[None, :, None]
    data = al[:, None, None] * uu + ga[:, None, None] * vv + de[:, None, None]
    frows = fdk.FilteredRows(np.arange(n), data, n)
    betas = g.angles(p)
    c = g.centre(n)
    pts = rng.uniform(-4, 4, (30, 3))
    got = fdk.backproject_points(frows, r, betas, pts[:, 0], pts[:, 1], pts[:, 2])
    for k, (x, y, z) in enumerate(pts):
        tot = 0.0
        for t, beta in enumerate(betas):
            lat, vert, dep = _ray_plane(x, y, z, beta, r)
            tot += (r / dep) ** 2 * (al[t] * (lat + c) + ga[t] * (vert + c) + de[t])
        assert got[k] == pytest.approx(np.pi / p * tot, rel=1e-12, abs=1e-12)


def test_fdk_is_linear():
    rng = np.random.default_rng(3)
    q1 = rng.standard_normal((12, 16, 16))
    q2 = rng.standard_normal((12, 16, 16))
    a = 2.5
    f1 = fdk.fdk(q1, 40.0, slices=[0, 7, 15])
    f2 = fdk.fdk(q2, 40.0, slices=[0, 7, 15])
    f12 = fdk.fdk(a * q1 + q2, 40.0, slices=[0, 7, 15])
    assert np.allclose(f12, a * f1 + f2, rtol=0, atol=1e-12 * np.abs(f12).max())


def test_fdk_points_matches_slices():
    ell = phantom.random_ellipsoids(5, 11)
    n, p, r = 24, 30, 80.0
    proj = phantom.project(ell, n, p, r, out_dtype=torch.float64).numpy()
    vol = fdk.fdk(proj, r, slices=[0, 11, 23])
    rng = np.random.default_rng(1)
    idx = np.stack([rng.choice([0, 11, 23], 40), rng.integers(0, n, 40),
                    rng.integers(0, n, 40)], axis=1)
    pts = fdk.fdk_points(proj, r, idx)
    lut = {0: 0, 11: 1, 23: 2}
    ref = np.array([vol[lut[l], j, i] for l, j, i in idx])
    assert np.allclose(pts, ref, rtol=0, atol=1e-12)


def test_metrics():
    assert metrics.rel_rmse([1.0, 2.0], [1.0, 2.0]) == 0.0
    assert metrics.rel_rmse([1.0, 0.0], [0.0, 1.0]) == pytest.approx(np.sqrt(2))
    assert list(metrics.sampled_slices(64, 16))[:2] == [0, 4]
    assert metrics.sampled_slices(64, 16)[-1] == 63
