"""Pins of the learned-decimation oracle (conv net over (angle, column))."""

import numpy as np
import pytest
import torch

from oracle import fdk, fdkod, geometry as g, learned
from synth import phantom


def _direct_correction(s_sub, net, d_factor, pd):
    """R by plain loops over the definition (one row)."""
    p, w = s_sub.shape
    d = learned.dilation(d_factor)
    sv = lambda pp, jj: s_sub[pp % p, jj] if 0 <= jj < w else 0.0  # noqa: E731
    out = np.zeros((pd, w))
    for m in range(pd):
        c = int(((2 * m * p + pd) // (2 * pd)) % p)
        for j in range(w):
            acc = net["b2"][0]
            for a2 in range(5):
                pa = (c + (a2 - 2) * d) % p
                for b2 in range(5):
                    jj = j + b2 - 2
                    if not 0 <= jj < w:
                        continue
                    for k in range(16):
                        hk = net["b1"][k]
                        for a1 in range(5):
                            for b1 in range(5):
                                hk += net["w1"][k, a1, b1] * sv(pa + (a1 - 2) * d, jj + b1 - 2)
                        acc += net["w2"][k, a2, b2] * max(hk, 0.0)
            out[m, j] = acc
    return out


def _random_net(seed):
    rng = np.random.default_rng(seed)
    net = learned.init_weights(seed, scale=0.5)
    net["w2"] = rng.standard_normal((16, 5, 5)) * 0.05
    net["b1"] = rng.standard_normal(16) * 0.1
    net["b2"] = rng.standard_normal(1) * 0.1
    return net


@pytest.mark.parametrize("d_factor,p,pd", [(4, 24, 6), (8, 40, 5), (2, 11, 6)])
def test_correction_matches_direct_loops(d_factor, p, pd):
    rng = np.random.default_rng(d_factor)
    s_sub = rng.standard_normal((p, 7))
    net = _random_net(3)
    r, _ = learned.forward(s_sub, net, d_factor, pd)
    assert np.allclose(r, _direct_correction(s_sub, net, d_factor, pd), atol=1e-12)


def test_zero_conv2_is_plain_decimation():
    rng = np.random.default_rng(0)
    s_sub = rng.standard_normal((3, 48, 9))
    tri = fdkod.triangle_weights(48, 12)
    net = learned.init_weights(1)
    y = learned.decimate_learned(s_sub, tri, net, 4, 12)
    plain = np.moveaxis(np.tensordot(s_sub, tri.T, axes=(1, 0)), -1, 1)
    assert np.array_equal(y, plain)


def test_dilation_reaches_the_triangle_support():
    # the two 5-tap layers reach +-4 d original angles; the triangle of
    # decimation factor D spans +-D, so d = D / 4 once D >= 4
    for d_factor in (4, 8, 16, 32, 64):
        assert 4 * learned.dilation(d_factor) == d_factor
    assert learned.dilation(1) == learned.dilation(2) == 1
    assert list(learned.centre_angle(np.arange(5), 40, 5)) == [0, 8, 16, 24, 32]
    assert list(learned.centre_angle(np.arange(4), 10, 4)) == [0, 3, 5, 8]   # round half up


def _case():
    # s = 3, k = 0: D = 8, dilation 2
    ell = phantom.random_ellipsoids(5, 3)
    n, p, r, s, k = 16, 32, 64.0, 3, 0
    proj = phantom.project(ell, n, p, r, out_dtype=torch.float64).numpy()
    idx = np.array([(l, j, i) for l in (6, 7, 9) for j in range(0, 2) for i in range(0, 2)])
    target = fdk.fdk_points(proj, r, idx)
    return proj, r, s, k, idx, target


def test_gradients_match_central_differences():
    proj, r, s, k, idx, target = _case()
    net = _random_net(5)
    loss, grads, _ = learned.loss_and_grads(proj, r, s, k, net, target, idx)
    rng = np.random.default_rng(9)
    for name in ("w1", "b1", "w2", "b2"):
        for _ in range(4):
            pos = tuple(rng.integers(0, dim) for dim in net[name].shape)
            eps = 1e-6
            hi = {kk: v.copy() for kk, v in net.items()}
            lo = {kk: v.copy() for kk, v in net.items()}
            hi[name][pos] += eps
            lo[name][pos] -= eps
            fd = (learned.loss_and_grads(proj, r, s, k, hi, target, idx)[0]
                  - learned.loss_and_grads(proj, r, s, k, lo, target, idx)[0]) / (2 * eps)
            an = grads[name][pos]
            assert fd == pytest.approx(an, rel=1e-5, abs=1e-9 * max(1.0, abs(loss)))


def test_backprojection_adjoint_identity():
    proj, r, s, k, idx, target = _case()
    n = proj.shape[2]
    sqs, betas, bd = fdkod.plan(n, proj.shape[0], r, s, k)
    sq = sqs[0]
    c = g.centre(n)
    x, y, z = idx[:, 2] - c, idx[:, 1] - c, idx[:, 0] - c
    frows, s_sub = learned.square_rows(proj, r, sq, betas, bd, x, y, z)
    rng = np.random.default_rng(1)
    yv = rng.standard_normal((s_sub.shape[0], len(bd), s_sub.shape[2]))
    res = rng.standard_normal(len(idx))
    lhs = np.dot(learned.bp_square(yv, frows.slot, proj.shape[1], sq, bd, r, n, x, y, z), res)
    yt = learned.bp_square_adjoint(res, frows.slot, proj.shape[1], sq, bd, r, n, x, y, z,
                                   s_sub.shape[0], s_sub.shape[2])
    assert lhs == pytest.approx(np.sum(yv * yt), rel=1e-12)


def test_bf16_form_rounds_inputs_and_weights():
    rng = np.random.default_rng(2)
    s_sub = rng.standard_normal((2, 32, 6))
    net = _random_net(4)
    r32, _ = learned.forward(s_sub, learned.rounded(net), 4, 8, bf16=True)
    r64, _ = learned.forward(s_sub, net, 4, 8)
    assert not np.array_equal(r32, r64)
    assert np.max(np.abs(r32 - r64)) < 0.05 * np.max(np.abs(r64))


def _bf(x):
    """BF16 rounding (nearest even) of an FP32 value, by torch's cast."""
    return float(torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64))


def _direct_bf16_grads(s_sub, net, d_factor, pd, d_r):
    """Gradients of sum R dR in the BF16 form, by plain loops over the
    definition: conv1 takes BF16 S, conv2 the BF16 activation, the gradients
    hold those roundings fixed (dW2 from the rounded activation, dA passed
    through the rounding, db1 from dH, dW1 from BF16 dH times BF16 S)."""
    p, w = s_sub.shape
    d = learned.dilation(d_factor)
    sb = [[_bf(s_sub[pp, jj]) for jj in range(w)] for pp in range(p)]
    sv = lambda pp, jj: sb[pp % p][jj] if 0 <= jj < w else 0.0  # noqa: E731
    g = {k: np.zeros_like(v) for k, v in net.items()}
    for m in range(pd):
        c = int(((2 * m * p + pd) // (2 * pd)) % p)
        for j in range(w):
            g["b2"][0] += d_r[m, j]
        for a2 in range(5):
            pa = (c + (a2 - 2) * d) % p
            for jj in range(w):                    # activation column
                for k in range(16):
                    hk = net["b1"][k]
                    for a1 in range(5):
                        for b1 in range(5):
                            hk += net["w1"][k, a1, b1] * sv(pa + (a1 - 2) * d, jj + b1 - 2)
                    act = _bf(max(hk, 0.0))
                    da = 0.0
                    for b2 in range(5):             # A[jj] feeds R[jj - b2 + 2]
                        j = jj - b2 + 2
                        if 0 <= j < w:
                            g["w2"][k, a2, b2] += d_r[m, j] * act
                            da += net["w2"][k, a2, b2] * d_r[m, j]
                    dh = da if hk > 0.0 else 0.0
                    g["b1"][k] += dh
                    dhb = _bf(dh)
                    for a1 in range(5):
                        for b1 in range(5):
                            g["w1"][k, a1, b1] += dhb * sv(pa + (a1 - 2) * d, jj + b1 - 2)
    return g


@pytest.mark.parametrize("d_factor,p,pd", [(4, 24, 6), (2, 11, 6)])
def test_bf16_backward_matches_direct_loops(d_factor, p, pd):
    rng = np.random.default_rng(10 + d_factor)
    s_sub = rng.standard_normal((p, 6))
    net = learned.rounded(_random_net(7))
    d_r = rng.standard_normal((pd, 6))
    _, cache = learned.forward(s_sub, net, d_factor, pd, bf16=True)
    got = learned.backward(s_sub, net, d_factor, pd, d_r, cache, bf16=True)
    want = _direct_bf16_grads(s_sub, net, d_factor, pd, d_r)
    for key in ("w1", "b1", "w2", "b2"):
        assert np.allclose(got[key], want[key], rtol=1e-10, atol=1e-12), key
    # the BF16 form differs from the FP64 form (the roundings are placed)
    g64 = learned.backward(s_sub, net, d_factor, pd, d_r, learned.forward(s_sub, net, d_factor, pd)[1])
    assert not np.allclose(g64["w1"], want["w1"], rtol=1e-6)
