"""Pins of the quality study's estimators (CPU): the slanted-edge MTF and the
edge width of a Gaussian-blurred edge against their closed forms, the cost
fit on exact data, and the interior mask of a sphere."""

import math

import numpy as np
import pytest
from scipy.special import erfc

import study
from synth import phantom


def blurred_box_slice(n, half, angle, sigma):
    dist, _ = study.face_coordinates(n, (0.0, 0.0), angle, (half, half))
    return 0.5 * erfc(dist / (sigma * math.sqrt(2.0)))


@pytest.mark.parametrize("sigma", [0.7, 1.0, 1.6, 3.0])
def test_gaussian_edge_mtf_and_width(sigma):
    """ESF = Phi(-d / sigma): MTF(f) = exp(-2 pi^2 sigma^2 f^2), 10-90 % width
    2 z_0.9 sigma with z_0.9 = 1.2816."""
    n, half, angle = 160, 50.0, math.radians(5.0)
    img = blurred_box_slice(n, half, angle, sigma)
    got = study.slanted_edge(img, (0.0, 0.0), angle, (half, half))
    want10 = math.sqrt(math.log(10.0) / (2 * math.pi ** 2 * sigma ** 2))
    want50 = math.sqrt(math.log(2.0) / (2 * math.pi ** 2 * sigma ** 2))
    assert got["mtf10"] == pytest.approx(want10, rel=0.04)
    assert got["mtf50"] == pytest.approx(want50, rel=0.04)
    assert got["width_10_90"] == pytest.approx(2 * 1.2815516 * sigma, rel=0.04)


def test_edge_spread_rejects_an_unslanted_face():
    n, half = 64, 20.0
    img = blurred_box_slice(n, half, 0.0, 1.0)
    with pytest.raises(ValueError):
        study.slanted_edge(img, (0.0, 0.0), 0.0, (half, half))


def test_first_crossing_interpolates():
    f = np.array([0.0, 0.1, 0.2, 0.3])
    m = np.array([1.0, 0.8, 0.4, 0.0])
    assert study.first_crossing(f, m, 0.5) == pytest.approx(0.175)
    assert study.first_crossing(f, m, -1.0) is None


def test_cost_fit_recovers_constants():
    c1, c2 = 3e-9, 7e-8
    rows = [{"n": n, "p": p, "s": s, "reconstruct_ms": c1 * n ** 3 * p / 2 ** s,
             "decompose_ms": c2 * n ** 2 * p * 2 ** s}
            for n, p in ((256, 360), (512, 720)) for s in range(1, 6)]
    got1, got2 = study.fit_costs(rows)
    assert got1 == pytest.approx(c1, rel=1e-12) and got2 == pytest.approx(c2, rel=1e-12)


def test_interior_mask_of_a_sphere():
    n = 32
    ball = phantom.sphere((0.0, 0.0, 0.0), 0.5, 1.0)          # radius 8 voxels
    sl, mask = study.interior_mask(ball, n, margin=3.0, step=1)
    c = (n - 1) / 2.0
    g = np.arange(n) - c
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    rad = np.sqrt(x ** 2 + y ** 2 + z ** 2)
    assert np.all(rad[mask] <= 8.0)
    # the axis-aligned +-3 probes stay inside for every point within 8 - 3 of the centre
    assert np.all(mask[rad <= 5.0])
    assert not np.any(mask[rad > 8.0])


def test_ratio_map_blocks_and_profiles():
    """E4 ratio map: a volume that is 1.02 times the reference reads 1.02 in
    every block where the reference is large, None where it is small; the
    profiles are the band-averaged central rows, subsampled."""
    n = 64
    ref = np.zeros((n, n, n))
    ref[:, 16:48, 16:48] = 2.0
    v = 1.02 * ref
    m = study.ratio_map(v, ref, n, grid=8, band=4)
    blocks = np.array([[np.nan if x is None else x for x in row] for row in m["ratio_blocks"]])
    assert np.allclose(blocks[2:6, 2:6], 1.02) and np.isnan(blocks[0, 0]) and np.isnan(blocks[7, 7])
    assert m["profile_step"] == 1 and len(m["profile_fdk"]) == n
    assert m["profile_fdk"][32] == 2.0 and m["profile_fdkod"][32] == 2.04 and m["profile_fdk"][0] == 0.0
