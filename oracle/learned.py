"""Learned angular decimation, FP64 oracle (test infrastructure only).

Sec. 2.1 of the paper leaves the low-pass filter of the angular decimation
open ("Quality can be adjusted by changing size of filter kernel and the
low-pass filter implementation").  This module defines the learned filter the
GPU library implements and checks it:

    Y_q[m][j] = T[m][j] + R[m][j]
    T = plain triangle decimation of the cropped, shifted sub-sinogram S
    R = conv2(ReLU(conv1(S))), evaluated at the original angle c(m) nearest
        to the decimated angle beta'_m = 2 pi m / P'

for every square q and detector row v separately, with

    conv1: H_k(p, j) = b1_k + sum_{a,b=0..4} W1[k,a,b] S((p + (a-2) d) mod P, j + b - 2)
    A_k(p, j) = max(H_k(p, j), 0) on the columns [0, W), zero outside
    R(m, j)  = b2 + sum_k sum_{a,b=0..4} W2[k,a,b] A_k((c(m) + (a-2) d) mod P, j + b - 2)

S is zero outside the columns [0, W); the angle index is circular.
c(m) = floor(m P / P' + 1/2) mod P; the angle dilation d = max(1, D / 4), so
that the two layers together reach +-D original angles, the support of the
triangle.  16 channels, 5 x 5 taps: 817 parameters.  conv2 starts at zero,
so the untrained network is exactly the plain decimation.

Precision form of the GPU kernels (emulated here when bf16=True): weights are
BF16 (rounded from an FP32 master copy); both convolutions multiply BF16
operands with FP32 accumulation on matrix cores: conv1 takes BF16 S, conv2
takes the BF16-rounded activations.  The gradients are those of this rounded
forward with the roundings held fixed: dW2 uses the BF16 activations, dA
passes through the rounding unchanged, and the conv1 weight gradient
multiplies BF16 dH by BF16 S.

Pinned by (tests/test_oracle_learned.py): zero conv2 gives the plain
decimation exactly; central finite differences of the loss match the analytic
gradients (FP64 form); the backprojection adjoint satisfies
<BP y, r> = <y, BP^T r>; forward and backward equal an independent direct
loop implementation on tiny inputs.
"""

import numpy as np

from . import fdk as fdk_mod
from . import fdkod
from . import geometry as g
from . import storage

CH = 16
TAPS = 5


def dilation(d_factor):
    """Angle dilation of both convolutions for decimation factor D."""
    return max(1, d_factor // 4)


def centre_angle(m, p, pd):
    """Original angle index nearest to beta'_m: floor(m P / P' + 1/2) mod P."""
    return ((2 * np.asarray(m) * p + pd) // (2 * pd)) % p


def init_weights(seed, scale=0.1):
    """W1 ~ N(0, scale^2 / 25), b1 = 0, W2 = 0, b2 = 0 (untrained = plain)."""
    rng = np.random.default_rng(seed)
    return dict(w1=rng.standard_normal((CH, TAPS, TAPS)) * scale / TAPS,
                b1=np.zeros(CH), w2=np.zeros((CH, TAPS, TAPS)), b2=np.zeros(1))


def rounded(net):
    """The BF16 values the GPU uses for a set of FP32/FP64 master weights."""
    return {k: storage.round_bf16(v) for k, v in net.items()}


def _shift_cols(x, off):
    """x[..., j + off] with zeros outside [0, W)."""
    out = np.zeros_like(x)
    w = x.shape[-1]
    if off >= 0:
        out[..., :w - off] = x[..., off:]
    else:
        out[..., -off:] = x[..., :w + off]
    return out


def _used_angles(p, pd, d):
    """[P', 5] original angles at which conv1 feeds conv2 (c(m) + (a-2) d)."""
    c = centre_angle(np.arange(pd), p, pd)
    return (c[:, None] + (np.arange(TAPS)[None, :] - 2) * d) % p


def conv1(s_sub, net, angles, d, bf16=False):
    """H[..., n, k, j] at the original angles ``angles`` (array [n]) from
    S[..., p, j]; returns H with shape S.shape[:-2] + (n, 16, W)."""
    p = s_sub.shape[-2]
    w1 = net["w1"]
    src = storage.round_bf16(s_sub) if bf16 else s_sub
    shp = s_sub.shape[:-2] + (len(angles), CH, s_sub.shape[-1])
    h = np.zeros(shp) + net["b1"][:, None]
    for a in range(TAPS):
        rows = src[..., (angles + (a - 2) * d) % p, :]            # [..., n, W]
        for b in range(TAPS):
            x = _shift_cols(rows, b - 2)
            h += w1[:, a, b][:, None] * x[..., :, None, :]
    return h


def forward(s_sub, net, d_factor, pd, bf16=False):
    """Correction R[..., m, j] and the cache for the backward pass.
    s_sub: S[..., p, j] for one square (any leading axes, e.g. rows)."""
    p = s_sub.shape[-2]
    d = dilation(d_factor)
    used = _used_angles(p, pd, d)                                   # [P', 5]
    h = conv1(s_sub, net, used.reshape(-1), d, bf16)                 # [..., P'*5, 16, W]
    h = h.reshape(s_sub.shape[:-2] + (pd, TAPS, CH, s_sub.shape[-1]))
    a_act = np.maximum(h, 0.0)
    if bf16:
        a_act = storage.round_bf16(a_act)
    w2 = net["w2"]
    r = np.zeros(s_sub.shape[:-2] + (pd, s_sub.shape[-1])) + net["b2"][0]
    for a in range(TAPS):
        for b in range(TAPS):
            r += np.einsum("k,...mkj->...mj", w2[:, a, b], _shift_cols(a_act[..., a, :, :], b - 2))
    return r, dict(h=h, used=used, d=d)


def decimate_learned(s_sub, tri, net, d_factor, pd, bf16=False):
    """Y = T + R for S[..., p, j]; tri: the [P', P] triangle weights."""
    t = np.tensordot(s_sub, tri.T, axes=(-2, 0))                     # [..., W, P']
    t = np.moveaxis(t, -1, -2)
    r, _ = forward(s_sub, net, d_factor, pd, bf16)
    return t + r


def backward(s_sub, net, d_factor, pd, d_r, cache, bf16=False):
    """Gradients of sum(R * d_r) with respect to w1, b1, w2, b2."""
    p = s_sub.shape[-2]
    d = cache["d"]
    h = cache["h"]                                                   # [..., P', 5, 16, W]
    a_act = np.maximum(h, 0.0)
    if bf16:
        a_act = storage.round_bf16(a_act)
    w2 = net["w2"]
    lead = tuple(range(d_r.ndim - 2))
    grads = dict(b2=np.array([d_r.sum()]))
    gw2 = np.zeros_like(w2)
    d_a = np.zeros_like(h)
    for a in range(TAPS):
        for b in range(TAPS):
            sh = _shift_cols(a_act[..., a, :, :], b - 2)             # [..., P', 16, W]
            gw2[:, a, b] = np.einsum("...mj,...mkj->...k", d_r, sh).reshape(-1, CH).sum(axis=0)
            # A[j + b - 2] feeds R[j]: scatter back by the opposite shift
            d_a[..., a, :, :] += w2[:, a, b][:, None] * _shift_cols(d_r, -(b - 2))[..., :, None, :]
    grads["w2"] = gw2
    d_h = d_a * (h > 0)
    grads["b1"] = d_h.sum(axis=lead + (-4, -3, -1))
    if bf16:
        d_h = storage.round_bf16(d_h)
    src = storage.round_bf16(s_sub) if bf16 else s_sub
    used = cache["used"]
    gw1 = np.zeros_like(net["w1"])
    for a1 in range(TAPS):
        rows = src[..., (used + (a1 - 2) * d) % p, :]                # [..., P', 5, W]
        for b1 in range(TAPS):
            x = _shift_cols(rows, b1 - 2)
            gw1[:, a1, b1] = np.einsum("...makj,...maj->...k", d_h, x).reshape(-1, CH).sum(axis=0)
    grads["w1"] = gw1
    return grads


# ------------------------------------------------------------ square pipeline

def square_rows(proj, r, sq, betas, betas_dec, x, y, z):
    """Filtered rows and the cropped, shifted full-rate S[rows, P, W] for the
    voxels (x, y, z) of one square (steps 2-3 of FDK-OD)."""
    n = proj.shape[2]
    rows = fdk_mod.rows_for_points(n, r, betas_dec, x, y, z)
    frows = fdk_mod.filter_rows(proj, r, rows)
    s_sub = fdkod.crop_shift(frows, sq, betas, r, n)                 # [P, rows, W]
    return frows, np.moveaxis(s_sub, 0, 1)                           # [rows, P, W]


def bp_square(y_sub, slot, nv, sq, betas_dec, r, n, x, y, z):
    """Backprojection of Y[rows, P', W] (step 5 of FDK-OD) at points."""
    return fdkod.backproject_square(np.moveaxis(y_sub, 1, 0), slot, nv, sq, betas_dec, r, n, x, y, z)


def bp_square_adjoint(res, slot, nv, sq, betas_dec, r, n, x, y, z, nrows, width):
    """Exact transpose of bp_square: scatter the residual at the points into
    dY[rows, P', W] with the same bilinear weights and (pi / P') U^-2."""
    cu = cv = g.centre(n)
    pd = len(betas_dec)
    ac = fdkod.centre_track(sq, betas_dec, r)
    out = np.zeros((nrows, pd, width))
    res = np.asarray(res, dtype=np.float64).ravel()
    x, y, z = (np.asarray(t, dtype=np.float64).ravel() for t in (x, y, z))
    for m, beta in enumerate(betas_dec):
        u_mag = g.depth(x, y, beta, r) / r
        a = g.pix_pos(x, y, beta, r)
        b = g.row_pos(x, y, z, beta, r)
        tau = a - ac[m] + cu - sq.u0
        v = b + cv
        iv = np.floor(v).astype(np.int64)
        iu = np.floor(tau).astype(np.int64)
        fv = v - iv
        fu = tau - iu
        wgt = (np.pi / pd) * res / (u_mag * u_mag)
        for dv, wv in ((0, 1.0 - fv), (1, fv)):
            vi = iv + dv
            ok = (vi >= 0) & (vi < nv)
            k = slot[np.clip(vi, 0, nv - 1)]
            for du, wu in ((0, 1.0 - fu), (1, fu)):
                ui = iu + du
                np.add.at(out, (k[ok], m, ui[ok]), (wgt * wv * wu)[ok])
    return out


def loss_and_grads(proj, r, s, k, net, target, idx, nz=None, bf16=False):
    """Loss sum over the voxels idx ([K, 3] of (l, j, i), one square) of
    (FDK-OD-learned - target)^2 and its gradients with respect to the net."""
    p_count, nv, n = proj.shape
    nz = n if nz is None else nz
    sqs, betas, betas_dec = fdkod.plan(n, p_count, r, s, k)
    tri = fdkod.triangle_weights(p_count, len(betas_dec))
    d_factor = fdkod.decimation_factor(s, k)
    idx = np.asarray(idx)
    q = fdkod.square_of(n, s, idx[0, 2], idx[0, 1])
    sq = sqs[q]
    c, cz = g.centre(n), g.centre(nz)
    x, y, z = idx[:, 2] - c, idx[:, 1] - c, idx[:, 0] - cz
    frows, s_sub = square_rows(proj, r, sq, betas, betas_dec, x, y, z)
    wnet = rounded(net) if bf16 else net
    t = np.moveaxis(np.tensordot(s_sub, tri.T, axes=(1, 0)), -1, 1)   # [rows, P', W]
    r_corr, cache = forward(s_sub, wnet, d_factor, len(betas_dec), bf16)
    y_sub = t + r_corr
    f = bp_square(y_sub, frows.slot, nv, sq, betas_dec, r, n, x, y, z)
    diff = f - target
    loss = float(np.sum(diff * diff))
    d_y = bp_square_adjoint(2.0 * diff, frows.slot, nv, sq, betas_dec, r, n, x, y, z,
                            s_sub.shape[0], s_sub.shape[2])
    grads = backward(s_sub, wnet, d_factor, len(betas_dec), d_y, cache, bf16)
    return loss, grads, dict(f=f, y=y_sub, dy=d_y, s=s_sub, rows=frows.rows)
