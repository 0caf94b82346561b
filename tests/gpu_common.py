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


# what the oracle's worker processes read: set before the pool forks, so the
# projections are shared with the children (copy on write), never pickled
_POOL = {}


def _oracle_job(task):
    from threadpoolctl import threadpool_limits
    vi, l = task
    c = _POOL["scans"][vi]
    with threadpool_limits(limits=1):
        if c["s"] == 0:
            return ofdk.fdk(c["proj"], c["r"], slices=[l], nz=c["nz"])[0]
        return ofdkod.fdkod(c["proj"], c["r"], c["s"], c["k"], slices=[l], nz=c["nz"])[0]


def oracle_slices_many(scans, tasks, workers=16):
    """FP64 oracle slices of several scans, one slice per task on forked
    worker processes (numpy pools limited to one thread each).  scans: list
    of dict(proj, r, s, k, nz), proj a CPU tensor or array [P][N][N]; tasks:
    list of (scan index, slice).  Returns the slices in task order."""
    import multiprocessing as mp
    import os
    _POOL["scans"] = [dict(c, proj=c["proj"].numpy() if isinstance(c["proj"], torch.Tensor)
                           else np.asarray(c["proj"])) for c in scans]
    nw = max(1, min(len(tasks), workers, len(os.sched_getaffinity(0))))
    try:
        with mp.get_context("fork").Pool(processes=nw) as pool:
            return pool.map(_oracle_job, [(int(a), int(b)) for a, b in tasks], chunksize=1)
    finally:
        _POOL.clear()


def oracle_slices_parallel(proj, r, s, k, slices, nz, workers=16):
    """The FP64 oracle's slices (a list of indices) of one scan, one slice per
    worker process: [len(slices)][N][N]."""
    scans = [dict(proj=proj, r=r, s=s, k=k, nz=nz)]
    return np.stack(oracle_slices_many(scans, [(0, l) for l in slices], workers))


def report(tag, got, ref, bar=None, factor=20.0):
    """rel-RMSE and max-abs of got against ref, logged; with a rel-RMSE bar,
    also asserts that the largest single error is at most factor x bar of
    max |ref| (a bad square edge or tail column that the RMSE over a whole
    volume would average away fails this)."""
    err = metrics.rel_rmse(got, ref)
    mx, mxr = metrics.max_abs(got, ref)
    log(f"{tag}: rel-RMSE {err:.3e}  max-abs {mx:.3e} ({mxr:.3e} of max|ref|)")
    if bar is not None:
        assert mxr <= factor * bar, f"{tag}: max-abs {mxr:.3e} of max|ref| above {factor:g} x {bar:g}"
    return err, mxr


class Timer:
    def __enter__(self):
        self.t = time.time()
        return self

    def __exit__(self, *a):
        self.dt = time.time() - self.t
