"""Pins of the oracle's quality knobs (extensions beyond the paper): the
windowed-sinc decimation window and the cubic (Keys, a = -1/2) shift."""

import numpy as np
import pytest
from scipy import signal

from oracle import fdk, fdkod
from synth import phantom


@pytest.mark.parametrize("p,d,taps", [(64, 4, 2), (64, 4, 4), (96, 8, 6), (48, 2, 4), (120, 4, 6)])
def test_sinc_weights_are_scipys_windowed_sinc_when_d_divides_p(p, d, taps):
    """With D | P, window m is centred on projection m D; scipy's firwin with
    K D + 1 taps, cutoff 1/D of Nyquist and a Hann window is the same filter
    (firwin scales it to unit DC gain, as the weights sum to one)."""
    w = fdkod.sinc_weights(p, p // d, taps)
    h = signal.firwin(taps * d + 1, 1.0 / d, window="hann")
    half = taps * d // 2
    for m in range(p // d):
        want = np.zeros(p)
        for i, hv in enumerate(h):
            want[(m * d + i - half) % p] += hv
        assert np.allclose(w[m], want, atol=1e-14)


def test_sinc_weights_at_d1_are_the_identity_and_rows_sum_to_one():
    assert np.allclose(fdkod.sinc_weights(37, 37, 4), np.eye(37), atol=1e-15)
    for p, pd, taps in ((100, 13, 4), (90, 23, 2), (97, 25, 6)):
        w = fdkod.sinc_weights(p, pd, taps)
        assert np.allclose(w.sum(axis=1), 1.0)


def test_sinc_support_k2_is_the_triangles():
    for p, pd in ((90, 23), (64, 16), (97, 13)):
        tri = fdkod.triangle_weights(p, pd)
        sinc = fdkod.sinc_weights(p, pd, 2)
        assert np.array_equal(tri > 0, np.abs(sinc) > 0)


def test_sinc_passband_cutoff_and_stopband():
    """Frequency response of window 0 (D = 8 | P) in cycles per projection: the
    windowed sinc is cut off at the decimated rate's Nyquist frequency 1/(2D)
    (response 1/2 there, the window being symmetric about the cut-off), its
    pass band is flatter than the triangle's and its stop band deeper,
    more so for more taps."""
    p, d = 256, 8
    f = np.fft.rfftfreq(p)
    at = lambda h, x: float(h[np.argmin(np.abs(f - x / d))])
    resp = lambda w: np.abs(np.fft.rfft(w[0]))
    ht = resp(fdkod.triangle_weights(p, p // d))
    h4 = resp(fdkod.sinc_weights(p, p // d, 4))
    h6 = resp(fdkod.sinc_weights(p, p // d, 6))
    # the discrete triangle of half-width D: (sin(pi f D) / (D sin(pi f)))^2
    f0 = 0.25 / d
    assert at(ht, 0.25) == pytest.approx((np.sin(np.pi * f0 * d) / (d * np.sin(np.pi * f0))) ** 2, abs=1e-9)
    assert at(h4, 0.25) >= at(ht, 0.25) + 0.05 and at(h6, 0.25) >= 0.98
    assert at(h4, 0.5) == pytest.approx(0.5, abs=0.01) and at(h6, 0.5) == pytest.approx(0.5, abs=0.01)
    assert at(h4, 0.75) <= 0.1 and at(h6, 0.75) <= 0.02
    assert max(at(h4, 1.25), at(h6, 1.25)) <= 0.005 < at(ht, 1.25)


def test_keys_kernel_interpolates_and_sums_to_one():
    k = fdkod.keys_cubic
    assert k(0.0) == 1.0 and k(1.0) == 0.0 and k(2.0) == 0.0 and k(-1.0) == 0.0
    f = np.linspace(0, 1, 17)
    total = sum(k(f - d) for d in (-1, 0, 1, 2))
    assert np.allclose(total, 1.0, atol=1e-15)


def _square_and_rows(n, p, r, s, q_idx, data):
    sqs, betas, _ = fdkod.plan(n, p, r, s, 0)
    frows = fdk.FilteredRows(np.arange(data.shape[1]), data, data.shape[1])
    return sqs[q_idx], betas, frows


def test_cubic_crop_reproduces_quadratics():
    """Rows quadratic in u are reproduced exactly by the cubic shift where all
    four taps lie on the detector (the linear shift is not exact there)."""
    n, p, r = 40, 10, 80.0
    u = np.arange(n, dtype=np.float64)
    coef = np.array([0.3, -0.02, 0.0015])
    row = coef[0] + coef[1] * u + coef[2] * u ** 2
    data = np.broadcast_to(row, (p, 1, n)).copy()
    sq, betas, frows = _square_and_rows(n, p, r, 2, 6, data)
    cub = fdkod.crop_shift(frows, sq, betas, r, n, "cubic")[:, 0, :]
    lin = fdkod.crop_shift(frows, sq, betas, r, n, "linear")[:, 0, :]
    ac = fdkod.centre_track(sq, betas, r)
    pos = ac[:, None] + sq.u0 + np.arange(sq.width)[None, :]
    inside = (np.floor(pos) >= 1) & (np.floor(pos) + 2 <= n - 1)
    want = coef[0] + coef[1] * pos + coef[2] * pos ** 2
    assert inside.sum() > 20
    assert np.allclose(cub[inside], want[inside], atol=1e-12)
    assert not np.allclose(lin[inside], want[inside], atol=1e-6)


def test_cubic_crop_is_catmull_rom_hermite():
    """Catmull-Rom written as a cubic Hermite segment with tangents
    (q[i+1] - q[i-1]) / 2 (an independent form of the same kernel)."""
    n, p, r = 36, 7, 70.0
    rng = np.random.default_rng(5)
    data = rng.standard_normal((p, 2, n))
    sq, betas, frows = _square_and_rows(n, p, r, 1, 3, data)
    got = fdkod.crop_shift(frows, sq, betas, r, n, "cubic")
    ac = fdkod.centre_track(sq, betas, r)
    for pp in range(p):
        for j in range(sq.width):
            x = ac[pp] + sq.u0 + j
            i = int(np.floor(x))
            t = x - i
            if i - 1 < 0 or i + 2 > n - 1:
                continue
            for v in range(2):
                q = data[pp, v]
                m0, m1 = 0.5 * (q[i + 1] - q[i - 1]), 0.5 * (q[i + 2] - q[i])
                h = ((2 * t ** 3 - 3 * t ** 2 + 1) * q[i] + (t ** 3 - 2 * t ** 2 + t) * m0
                     + (-2 * t ** 3 + 3 * t ** 2) * q[i + 1] + (t ** 3 - t ** 2) * m1)
                assert got[pp, v, j] == pytest.approx(h, abs=1e-12)


def test_knobs_at_s0_are_direct_fdk():
    """s = 0: one square centred on the axis, an integer shift and D = 1, so
    neither knob changes anything."""
    n, p, r = 33, 40, 64.0
    proj = phantom.project(phantom.random_ellipsoids(6, 4), n, p, r).double().numpy()
    want = fdk.fdk(proj, r)
    got = fdkod.fdkod(proj, r, 0, window="sinc", taps=4, interp="cubic")
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_knobs_change_the_result_and_keep_uniform_interiors():
    """A sphere: the interior mean stays the density for every knob setting,
    and the settings give different volumes."""
    n, p, r, s = 48, 96, 192.0, 2
    ball = phantom.sphere((0.05, -0.05, 0.0), 0.5, 1.0)
    proj = phantom.project(ball, n, p, r).double().numpy()
    mid = [n // 2]
    vols = {}
    for window, taps, interp in (("triangle", 2, "linear"), ("sinc", 2, "linear"), ("sinc", 4, "linear"),
                                 ("triangle", 2, "cubic"), ("sinc", 4, "cubic")):
        v = fdkod.fdkod(proj, r, s, slices=mid, window=window, taps=taps, interp=interp)[0]
        c = (n - 1) / 2
        jj, ii = np.mgrid[0:n, 0:n]
        rad = np.hypot(ii - c - 0.05 * n / 2, jj - c + 0.05 * n / 2)
        assert abs(v[rad < 0.5 * n / 2 - 4].mean() - 1.0) < 0.02
        vols[(window, taps, interp)] = v
    keys = list(vols)
    for a in range(len(keys)):
        for b in range(a + 1, len(keys)):
            assert np.max(np.abs(vols[keys[a]] - vols[keys[b]])) > 1e-4
