"""Seeded synthetic inputs: random-ellipsoid and box phantoms and their exact
cone-beam line integrals.

This module only makes inputs.  It holds none of the reconstruction method's
arithmetic and is imported by the tests and the benchmark, never by the
oracle or the GPU library.  The paper measured on a Shepp-Logan-3D phantom
and on scanner data (Sec. 3); seeded random ellipsoids with closed-form
projections stand in for both.

Geometry (the same conventions as the reconstruction): voxel units; source at
-R (cos beta, sin beta, 0); detector point Q(a, b) = a (-sin beta, cos beta, 0)
+ b (0, 0, 1) on a virtual detector through the axis; pixel (u, v) of
projection p sits at a = u - (N-1)/2, b = v - (N-1)/2, beta_p = 2 pi p / P.
Ellipsoids are given in normalised units, 1.0 = N/2 voxels, axis aligned, and
densities add where they overlap.  Boxes (the slanted-edge phantom of the
resolution study, Sec. 4) are given in the same units and may be rotated about
the z axis.
"""

import math
from dataclasses import dataclass

import numpy as np
import torch


@dataclass
class Ellipsoids:
    centres: np.ndarray     # [M, 3] normalised (x, y, z)
    axes: np.ndarray        # [M, 3] normalised semi-axes
    density: np.ndarray     # [M]


def random_ellipsoids(count, seed, centre_range=0.6, axis_range=(0.05, 0.4),
                      density_range=(-0.5, 1.0)):
    """``count`` ellipsoids drawn with numpy.random.default_rng(seed); per
    ellipsoid the draw order is centre (3), semi-axes (3), density (1)."""
    rng = np.random.default_rng(seed)
    c = np.zeros((count, 3))
    a = np.zeros((count, 3))
    d = np.zeros(count)
    for e in range(count):
        c[e] = rng.uniform(-centre_range, centre_range, 3)
        a[e] = rng.uniform(axis_range[0], axis_range[1], 3)
        d[e] = rng.uniform(density_range[0], density_range[1])
    return Ellipsoids(c, a, d)


@dataclass
class Boxes:
    centres: np.ndarray     # [M, 3] normalised (x, y, z)
    half: np.ndarray        # [M, 3] normalised half sizes along the box's own axes
    angle: np.ndarray       # [M] rotation about z (radians): box axis x is (cos, sin, 0)
    density: np.ndarray     # [M]


def box(centre, half, angle=0.0, density=1.0):
    """A single box (normalised units) rotated by ``angle`` about z."""
    return Boxes(np.array([centre], dtype=np.float64), np.array([half], dtype=np.float64),
                 np.array([angle], dtype=np.float64), np.array([density], dtype=np.float64))


def sphere(centre, radius, density=1.0):
    """A single sphere (normalised units), for closed-form checks."""
    return Ellipsoids(np.array([centre], dtype=np.float64),
                      np.array([[radius] * 3], dtype=np.float64),
                      np.array([density], dtype=np.float64))


def _chords(src, dirn, ell, scale, device):
    """Sum over ellipsoids of density x chord length (voxel units) of the
    lines src + t dirn (dirn unit vectors), shapes [..., 3]."""
    out = torch.zeros(dirn.shape[:-1], dtype=torch.float64, device=device)
    for e in range(len(ell.density)):
        c = torch.tensor(ell.centres[e] * scale, dtype=torch.float64, device=device)
        ax = torch.tensor(ell.axes[e] * scale, dtype=torch.float64, device=device)
        o = (src - c) / ax
        dd = dirn / ax
        a2 = (dd * dd).sum(-1)
        b = (o * dd).sum(-1)
        cc = (o * o).sum(-1) - 1.0
        disc = b * b - a2 * cc
        chord = 2.0 * torch.sqrt(torch.clamp(disc, min=0.0)) / a2
        out += float(ell.density[e]) * chord
    return out


def _box_chords(src, dirn, boxes, scale, device):
    """Sum over boxes of density x chord length (slab intersection: the ray
    is inside the box between the largest entry and the smallest exit of the
    three pairs of parallel faces)."""
    out = torch.zeros(dirn.shape[:-1], dtype=torch.float64, device=device)
    for e in range(len(boxes.density)):
        c = torch.tensor(boxes.centres[e] * scale, dtype=torch.float64, device=device)
        h = boxes.half[e] * scale
        ca, sa = math.cos(boxes.angle[e]), math.sin(boxes.angle[e])
        axes = ((ca, sa, 0.0), (-sa, ca, 0.0), (0.0, 0.0, 1.0))
        o = src - c
        t_in = torch.full(out.shape, -math.inf, dtype=torch.float64, device=device)
        t_out = torch.full(out.shape, math.inf, dtype=torch.float64, device=device)
        for k in range(3):
            ax = torch.tensor(axes[k], dtype=torch.float64, device=device)
            ok = (o * ax).sum(-1)                 # source coordinate along the axis
            dk = (dirn * ax).sum(-1)
            par = dk.abs() < 1e-15                # parallel to the faces: inside or never
            safe = torch.where(par, torch.ones_like(dk), dk)
            t1 = (-h[k] - ok) / safe
            t2 = (h[k] - ok) / safe
            inside = ok.abs() <= h[k]
            lo = torch.where(par, torch.where(inside, -math.inf, math.inf), torch.minimum(t1, t2))
            hi = torch.where(par, torch.where(inside, math.inf, -math.inf), torch.maximum(t1, t2))
            t_in = torch.maximum(t_in, lo)
            t_out = torch.minimum(t_out, hi)
        out += float(boxes.density[e]) * torch.clamp(t_out - t_in, min=0.0)
    return out


def project(ell, n, p, r, device="cpu", out_dtype=torch.float32, angles=None,
            rows=None, chunk_rays=1 << 24):
    """Exact line integrals [P, N_v, N] of the phantom (voxel-length units).

    ``angles`` / ``rows`` restrict the output to some projections / detector
    rows (default: all).  Computed in float64 for chunks of angles (about
    ``chunk_rays`` rays at a time), returned in ``out_dtype``."""
    scale = n / 2.0
    c = (n - 1) / 2.0
    angles = np.arange(p) if angles is None else np.asarray(angles)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    a = torch.arange(n, dtype=torch.float64, device=device) - c
    b = torch.tensor(rows, dtype=torch.float64, device=device) - c
    bb, aa = torch.meshgrid(b, a, indexing="ij")
    out = torch.empty((len(angles), len(rows), n), dtype=out_dtype, device=device)
    per = max(1, int(chunk_rays // (len(rows) * n)))
    for t0 in range(0, len(angles), per):
        idx = angles[t0:t0 + per]
        beta = torch.tensor(2.0 * np.pi * idx.astype(np.float64) / p, dtype=torch.float64, device=device)
        cb = torch.cos(beta)[:, None, None]
        sb = torch.sin(beta)[:, None, None]
        src = torch.stack([-r * cb, -r * sb, torch.zeros_like(cb)], dim=-1)      # [A, 1, 1, 3]
        q = torch.stack([-aa[None] * sb, aa[None] * cb, bb[None].expand(len(idx), -1, -1)], dim=-1)
        d = q - src
        d = d / torch.linalg.norm(d, dim=-1, keepdim=True)
        chords = _box_chords if isinstance(ell, Boxes) else _chords
        out[t0:t0 + len(idx)] = chords(src, d, ell, scale, device).to(out_dtype)
    return out


def poisson_noise(proj, n, i0, seed):
    """Photon-counting noise: lambda = I0 exp(-p / (N/2)), counts ~ Poisson,
    p_hat = -(N/2) ln(max(counts, 1) / I0).  Seeded torch generator on the
    tensor's device; returns a tensor of the input's dtype."""
    gen = torch.Generator(device=proj.device)
    gen.manual_seed(seed)
    scale = n / 2.0
    lam = i0 * torch.exp(-proj.double() / scale)
    counts = torch.poisson(lam, generator=gen)
    return (-scale * torch.log(torch.clamp(counts, min=1.0) / i0)).to(proj.dtype)


def density(ell, n, nz, x, y, z):
    """True phantom density at voxel coordinates (x, y, z) (numpy arrays)."""
    scale = n / 2.0
    out = np.zeros(np.broadcast(x, y, z).shape)
    if isinstance(ell, Boxes):
        for e in range(len(ell.density)):
            c = ell.centres[e] * scale
            h = ell.half[e] * scale
            ca, sa = np.cos(ell.angle[e]), np.sin(ell.angle[e])
            lx = (x - c[0]) * ca + (y - c[1]) * sa
            ly = -(x - c[0]) * sa + (y - c[1]) * ca
            inside = (np.abs(lx) <= h[0]) & (np.abs(ly) <= h[1]) & (np.abs(z - c[2]) <= h[2])
            out += ell.density[e] * inside
        return out
    for e in range(len(ell.density)):
        c = ell.centres[e] * scale
        ax = ell.axes[e] * scale
        inside = (((x - c[0]) / ax[0]) ** 2 + ((y - c[1]) / ax[1]) ** 2
                  + ((z - c[2]) / ax[2]) ** 2) <= 1.0
        out += ell.density[e] * inside
    return out
