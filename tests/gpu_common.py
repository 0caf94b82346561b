"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and the FP64 oracle on the same seeded inputs."""

import functools
import sys
import time

import numpy as np
import pytest
import torch

import paper_1708_07515_amd as pkg
from oracle import fdk as ofdk, fdkod as ofdkod, metrics, storage
from synth import phantom

DEV = "cuda:0"


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pkg.load_library()     # a GPU without the built library is a failure, not a skip


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=8)
def scan(n, p, r, ellipsoids, seed, photons=0.0, on_gpu=False):
    """Seeded phantom projections, float32, as a CPU tensor (cached)."""
    ell = phantom.random_ellipsoids(ellipsoids, seed)
    dev = DEV if on_gpu else "cpu"
    proj = phantom.project(ell, n, p, r, device=dev)
    if photons:
        proj = phantom.poisson_noise(proj, n, photons, seed + 1000)
    return proj.cpu().contiguous()


def gpu_reconstruct(proj, n, p, r, s, skip=0, nz=0, store="f32", stream=None):
    """Filter + backproject on the GPU; returns (volume numpy f64, filtered numpy f64)."""
    with pkg.Plan(n, p, r, s=s, skip=skip, nz=nz, store=store) as plan:
        d_proj = proj.to(DEV)
        filt = plan.empty_filtered()
        vol = plan.empty_volume()
        ws = plan.empty_workspace()
        plan.filter(d_proj, filt, stream=stream)
        plan.backproject(filt, vol, ws, stream=stream)
        torch.cuda.synchronize()
        return vol.cpu().double().numpy(), filt.cpu().double().numpy()


def oracle_reconstruct(proj, r, s, skip=0, slices=None, nz=None, store=None):
    arr = proj.numpy() if isinstance(proj, torch.Tensor) else proj
    rounder = storage.ROUNDERS[store] if store else None
    if s == 0 and rounder is None:
        return ofdk.fdk(arr, r, slices=slices, nz=nz)
    return ofdkod.fdkod(arr, r, s, skip, slices=slices, nz=nz, store=rounder)


def report(tag, got, ref):
    err = metrics.rel_rmse(got, ref)
    mx, mxr = metrics.max_abs(got, ref)
    log(f"{tag}: rel-RMSE {err:.3e}  max-abs {mx:.3e} ({mxr:.3e} of max|ref|)")
    return err, mxr


class Timer:
    def __enter__(self):
        self.t = time.time()
        return self

    def __exit__(self, *a):
        self.dt = time.time() - self.t
