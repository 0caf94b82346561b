"""Pins of the oracle's geometry (Sec. 2.1 eq. (1), Sec. 2.2 eq. (9))."""

import numpy as np
import pytest

from oracle import geometry as g


def _ray_plane(x, y, z, beta, r):
    """Intersect the line from the source through (x, y, z) with the plane
    through the rotation axis perpendicular to the central ray, and return the
    in-plane coordinates (lateral, vertical).  Plain vector algebra, written
    independently of eq. (1) / eq. (9)."""
    d = np.array([np.cos(beta), np.sin(beta), 0.0])
    src = -r * d
    pt = np.array([x, y, z])
    # (src + t (pt - src)) . d = 0
    t = -np.dot(src, d) / np.dot(pt - src, d)
    q = src + t * (pt - src)
    lateral_axis = np.array([-np.sin(beta), np.cos(beta), 0.0])
    return float(np.dot(q, lateral_axis)), float(q[2])


def test_pix_pos_and_row_pos_match_ray_intersection():
    rng = np.random.default_rng(0)
    for _ in range(200):
        r = rng.uniform(50, 500)
        x, y, z = rng.uniform(-30, 30, 3)
        beta = rng.uniform(0, 2 * np.pi)
        lat, vert = _ray_plane(x, y, z, beta, r)
        assert g.pix_pos(x, y, beta, r) == pytest.approx(lat, rel=1e-12, abs=1e-12)
        assert g.row_pos(x, y, z, beta, r) == pytest.approx(vert, rel=1e-12, abs=1e-12)


def test_pix_pos_on_axis_is_zero_and_magnification_one():
    # the axis projects to the detector centre; near the axis a = lateral offset
    for beta in np.linspace(0, 2 * np.pi, 13):
        assert g.pix_pos(0.0, 0.0, beta, 100.0) == pytest.approx(0.0, abs=1e-14)
        eps = 1e-6
        lat = g.pix_pos(-eps * np.sin(beta), eps * np.cos(beta), beta, 100.0)
        assert lat / eps == pytest.approx(1.0, rel=1e-6)


@pytest.mark.parametrize("n,parts", [(64, 4), (2000, 16), (2000, 32), (7, 7), (10, 4)])
def test_blocks_cover_and_balance(n, parts):
    b = g.blocks(n, parts)
    sizes = [e - s for s, e in b]
    assert b[0][0] == 0 and b[-1][1] == n
    assert all(b[i][1] == b[i + 1][0] for i in range(len(b) - 1))
    assert max(sizes) - min(sizes) <= 1
    assert sizes == sorted(sizes, reverse=True)


def test_squares_count_and_order():
    sq = g.squares(64, 2)
    assert len(sq) == 16
    assert sq[1] == (16, 32, 0, 16)      # x block advances first
    assert sq[4] == (0, 16, 16, 32)


def test_valid_radius():
    assert g.valid_radius(64, 45.0)
    assert not g.valid_radius(64, 44.0)
