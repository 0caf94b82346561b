"""Checks of the seeded input generator (analytic ellipsoid line integrals)."""

import math

import numpy as np
import pytest
import torch

from synth import phantom


def test_sphere_line_integral_closed_form():
    # a ray at distance d from a sphere's centre crosses it over 2 sqrt(r^2 - d^2)
    n, p, r = 32, 8, 100.0
    c_norm, rad_norm = (0.2, -0.1, 0.15), 0.4
    proj = phantom.project(phantom.sphere(c_norm, rad_norm), n, p, r,
                           out_dtype=torch.float64).numpy()
    scale = n / 2
    cen = np.array(c_norm) * scale
    rad = rad_norm * scale
    c = (n - 1) / 2
    for t in range(p):
        beta = 2 * math.pi * t / p
        src = -r * np.array([math.cos(beta), math.sin(beta), 0.0])
        for v in (0, 9, 16, 31):
            for u in (2, 15, 16, 29):
                q = (u - c) * np.array([-math.sin(beta), math.cos(beta), 0.0]) + np.array([0, 0, v - c])
                d = (q - src) / np.linalg.norm(q - src)
                w = cen - src
                dist2 = np.dot(w, w) - np.dot(w, d) ** 2
                want = 2 * math.sqrt(rad * rad - dist2) if dist2 < rad * rad else 0.0
                assert proj[t, v, u] == pytest.approx(want, rel=1e-10, abs=1e-10)


def test_ellipsoid_line_integral_quadrature():
    # brute-force midpoint quadrature of the indicator along a few rays
    ell = phantom.random_ellipsoids(4, 9)
    n, p, r = 24, 3, 60.0
    proj = phantom.project(ell, n, p, r, out_dtype=torch.float64).numpy()
    c = (n - 1) / 2
    scale = n / 2
    rng = np.random.default_rng(0)
    for _ in range(12):
        t, v, u = rng.integers(0, p), rng.integers(0, n), rng.integers(0, n)
        beta = 2 * math.pi * t / p
        src = -r * np.array([math.cos(beta), math.sin(beta), 0.0])
        q = (u - c) * np.array([-math.sin(beta), math.cos(beta), 0.0]) + np.array([0, 0, v - c])
        d = (q - src) / np.linalg.norm(q - src)
        h = 2e-3
        ts = np.arange(r - 2 * n, r + 2 * n, h) + h / 2
        pts = src[None, :] + ts[:, None] * d[None, :]
        dens = phantom.density(ell, n, n, pts[:, 0], pts[:, 1], pts[:, 2])
        assert proj[t, v, u] == pytest.approx(dens.sum() * h, abs=2e-2)


def test_random_ellipsoids_seeded_and_in_range():
    a = phantom.random_ellipsoids(20, 2)
    b = phantom.random_ellipsoids(20, 2)
    assert np.array_equal(a.centres, b.centres) and np.array_equal(a.density, b.density)
    assert np.all(np.abs(a.centres) <= 0.6)
    assert np.all((a.axes >= 0.05) & (a.axes <= 0.4))
    assert np.all((a.density >= -0.5) & (a.density <= 1.0))


def test_poisson_noise_statistics():
    n = 64
    p = torch.full((4, 64, 64), 10.0, dtype=torch.float32)
    noisy = phantom.poisson_noise(p, n, 1e5, seed=3)
    lam = 1e5 * math.exp(-10.0 / 32)
    # delta method: std of -(N/2) ln(n/I0) is (N/2)/sqrt(lambda)
    assert float(noisy.mean()) == pytest.approx(10.0, abs=0.02)
    assert float(noisy.std()) == pytest.approx(32 / math.sqrt(lam), rel=0.05)


def test_box_line_integral_quadrature():
    # a rotated box: brute-force midpoint quadrature of its indicator, also on
    # the mid-plane row whose rays are parallel to the z faces
    bx = phantom.Boxes(np.array([[0.1, -0.05, 0.1], [-0.2, 0.3, -0.1]]),
                       np.array([[0.5, 0.3, 0.4], [0.2, 0.25, 0.3]]),
                       np.array([0.3, -1.1]), np.array([1.0, 0.5]))
    n, p, r = 25, 5, 60.0
    proj = phantom.project(bx, n, p, r, out_dtype=torch.float64).numpy()
    c = (n - 1) / 2
    rng = np.random.default_rng(1)
    picks = [(rng.integers(0, p), rng.integers(0, n), rng.integers(0, n)) for _ in range(12)]
    picks += [(0, 12, u) for u in (5, 12, 18)]          # v = c: rays in the plane z = 0
    hit = 0
    for t, v, u in picks:
        beta = 2 * math.pi * t / p
        src = -r * np.array([math.cos(beta), math.sin(beta), 0.0])
        q = (u - c) * np.array([-math.sin(beta), math.cos(beta), 0.0]) + np.array([0, 0, v - c])
        d = (q - src) / np.linalg.norm(q - src)
        h = 1e-3
        ts = np.arange(r - 2 * n, r + 2 * n, h) + h / 2
        pts = src[None, :] + ts[:, None] * d[None, :]
        dens = phantom.density(bx, n, n, pts[:, 0], pts[:, 1], pts[:, 2])
        assert proj[t, v, u] == pytest.approx(dens.sum() * h, abs=1e-2)
        hit += proj[t, v, u] > 0
    assert hit >= 5


def test_box_density_axis_aligned():
    bx = phantom.box((0.0, 0.0, 0.0), (0.5, 0.25, 0.5), 0.0, 2.0)
    n = 16                                  # half sizes 4 and 2 voxels
    x = np.array([3.9, 4.1, 0.0, 0.0])
    y = np.array([0.0, 0.0, 1.9, 2.1])
    assert np.array_equal(phantom.density(bx, n, n, x, y, np.zeros(4)), [2.0, 0.0, 2.0, 0.0])
