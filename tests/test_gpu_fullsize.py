"""GPU parity at the full workload sizes, on outputs the FP64 oracle can
compute one by one: sampled slices (1024^3) and sampled voxel clusters
(2000^3), in the same launch configuration that bench.py times."""

import numpy as np
import pytest
import torch

import paper_1708_07515_amd as pkg
from oracle import fdkod as ofdkod, metrics
import time

from gpu_common import DEV, log, oracle_slices_parallel, report, require_gpu
from synth import configs, phantom

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


class DeviceRows:
    """Array-like view of projections resident on the GPU: the oracle's
    proj[:, rows, :] copies only those detector rows to the host."""

    def __init__(self, t):
        self.t = t
        self.shape = tuple(t.shape)

    def __getitem__(self, key):
        _, rows, _ = key
        idx = torch.as_tensor(np.asarray(rows), device=self.t.device)
        return self.t.index_select(1, idx).cpu().numpy()


def reconstruct(proj, wl, s, store, **knobs):
    with pkg.Plan(wl.n, wl.p, wl.r, s=s, skip=wl.k, nz=wl.nzv, store=store, **knobs) as plan:
        filt = plan.empty_filtered()
        vol = plan.empty_volume()
        ws = plan.empty_workspace()
        plan.filter(proj, filt)
        plan.backproject(filt, vol, ws)
        torch.cuda.synchronize()
        del filt, ws
        return vol


def scan_on_gpu(wl):
    ell = phantom.random_ellipsoids(wl.ellipsoids, wl.seed)
    proj = phantom.project(ell, wl.n, wl.p, wl.r, device=DEV).contiguous()
    torch.cuda.synchronize()
    return proj


# 16 slices of the 1024^3 volume: both ends (largest cone angle), the centre
# and 13 spread between them
C3_SLICES = sorted(set([0, 1023, 512] + [int(x) for x in np.linspace(37, 990, 13)]))


def test_precision_forms_1024():
    # cone1024_p720, s=3: filtered and decimated data stored as FP32, FP16 and
    # BF16 with FP32 arithmetic; rel-RMSE and max-abs against the plain FP64
    # oracle on 16 slices per storage type (one oracle slice per host worker)
    wl = configs.C3
    s = 3
    proj = scan_on_gpu(wl)
    slices = C3_SLICES
    assert len(slices) == 16
    t0 = time.time()
    ref = oracle_slices_parallel(proj.cpu(), wl.r, s, wl.k, slices, wl.nzv)
    log(f"oracle: {len(slices)} slices of cone1024_p720 in {time.time() - t0:.1f} s")
    tol = {"f32": 1e-4, "f16": 2e-3, "bf16": 2e-3}
    for store in ("f32", "f16", "bf16"):
        vol = reconstruct(proj, wl, s, store)
        got = vol[slices].double().cpu().numpy()
        del vol
        torch.cuda.empty_cache()
        tag = f"cone1024_p720 s=3 {store} 16 slices"
        err, _ = report(tag, got, ref, bar=tol[store])
        per = [metrics.rel_rmse(got[i], ref[i]) for i in range(len(slices))]
        log(f"{tag}: per-slice rel-RMSE " + " ".join(f"{l}:{e:.1e}" for l, e in zip(slices, per)))
        assert err <= tol[store]


def _clusters(n, nz):
    # 4x4 (x, y) patches on two slices at the centre, an edge and a corner,
    # the top and bottom slices included
    out = []
    for (l, j, i) in [(0, n // 2 - 2, n // 2 - 2), (nz - 1, 3, n - 7), (nz // 2, n - 5, 2),
                      (nz // 3, n // 4, 3 * n // 4)]:
        for dl in (0, 1):
            for dj in range(4):
                for di in range(4):
                    out.append((min(l + dl, nz - 1), j + dj, i + di))
    return np.array(out)


@pytest.mark.parametrize("store,tol", [("bf16", 2e-3), ("f32", 1e-4)])
def test_n2000_sampled_voxels(store, tol):
    wl = configs.C5
    s = max(wl.s)
    proj = scan_on_gpu(wl)
    idx = _clusters(wl.n, wl.nzv)
    vol = reconstruct(proj, wl, s, store)
    got = vol[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
    del vol
    torch.cuda.empty_cache()
    log(f"oracle on {len(idx)} voxels of cone2000_p720")
    ref = ofdkod.fdkod_points(DeviceRows(proj), wl.r, s, wl.k, idx, nz=wl.nzv)
    err, _ = report(f"cone2000_p720 s={s} {store} {len(idx)} voxels", got, ref, bar=tol)
    assert err <= tol


@pytest.mark.parametrize("knobs", [dict(rows="cone"), dict(decim="sinc", taps=4, interp="cubic")])
def test_n2000_sampled_voxels_extensions(knobs):
    """cone2000_p720, s = 4, BF16 storage (the bench's configuration) with
    cone-corrected rows, or with the windowed sinc and the cubic shift."""
    wl = configs.C5
    s = max(wl.s)
    proj = scan_on_gpu(wl)
    idx = _clusters(wl.n, wl.nzv)
    vol = reconstruct(proj, wl, s, "bf16", **knobs)
    got = vol[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
    del vol
    torch.cuda.empty_cache()
    log(f"oracle on {len(idx)} voxels of cone2000_p720 with {knobs}")
    ok = {"window": knobs.get("decim", "triangle"), "taps": knobs.get("taps", 2),
          "interp": knobs.get("interp", "linear")}
    if knobs.get("rows") == "cone":
        ref = ofdkod.fdkod_cone_points(DeviceRows(proj), wl.r, s, wl.k, idx, nz=wl.nzv, **ok)
    else:
        ref = ofdkod.fdkod_points(DeviceRows(proj), wl.r, s, wl.k, idx, nz=wl.nzv, **ok)
    err, _ = report(f"cone2000_p720 s={s} bf16 {knobs} {len(idx)} voxels", got, ref, bar=2e-3)
    assert err <= 2e-3
