"""GPU tests of the low-memory slab mode (band calls and the streaming driver):
band results equal the whole-volume results bit for bit, the streamed
reconstruction equals the in-memory one and the oracle, and the device memory
it needs is a fraction of the whole-volume path's."""

import numpy as np
import pytest
import torch

import paper_1708_07515_amd as pkg
from gpu_common import DEV, log, oracle_reconstruct, report, require_gpu, scan

pytestmark = pytest.mark.gpu

# N, N_z, P, R, s, k, store
CASES = [(64, 64, 90, 256.0, 2, 0, "f32"), (48, 40, 67, 150.0, 2, 1, "f32"),
         (64, 64, 90, 256.0, 0, 0, "f32"), (64, 64, 90, 256.0, 3, 0, "bf16")]
# N above 1024 (the four-step 4096-point filter) on bands: equality only
BAND_CASES = CASES + [(1100, 64, 24, 4400.0, 3, 0, "f32")]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def full_run(plan, proj):
    filt, ws, vol = plan.empty_filtered(), plan.empty_workspace(), plan.empty_volume()
    plan.filter(proj, filt)
    plan.backproject(filt, vol, ws)
    return filt, ws, vol


def ws_rows(plan, ws_flat, v0, nrows):
    """The rows [v0, v0 + nrows) of every square's block of a whole-volume
    workspace, laid out as a band workspace."""
    widths = plan.get_bounds()["width"]
    pd, n = plan.p_dec, plan.n
    out, off = [], 0
    for w in widths:
        blk = ws_flat[off:off + pd * n * int(w)].reshape(pd, n, int(w))
        out.append(blk[:, v0:v0 + nrows, :].reshape(-1))
        off += pd * n * int(w)
    return torch.cat(out)


@pytest.mark.parametrize("case", BAND_CASES)
def test_band_calls_equal_whole_volume(case):
    n, nz, p, r, s, k, store = case
    proj = scan(n, p, r, 6, 70 + n).to(DEV)
    with pkg.Plan(n, p, r, s=s, skip=k, nz=nz, store=store) as plan:
        filt, ws, vol = full_run(plan, proj)
        zr = plan.get_tuning()["z_run"]
        for z0 in range(0, nz, zr):
            nzs = min(zr, nz - z0)
            v0, nr = plan.band_rows(z0, nzs)
            assert 0 <= v0 and v0 + nr <= n and nr >= 2
            pb, fb, wb = plan.empty_band(nr)
            pb.copy_(proj[:, v0:v0 + nr, :])
            plan.filter_band(pb, v0, fb)
            slab = torch.empty((nzs, n, n), dtype=torch.float32, device=DEV)
            plan.decompose_band(fb, v0, wb)
            plan.reconstruct_slab(fb, wb, v0, nr, z0, slab)
            torch.cuda.synchronize()
            assert torch.equal(fb, filt[:, v0:v0 + nr, :]), f"filtered band z0={z0}"
            if s > 0:
                e = plan.band_workspace_elems(nr)
                assert torch.equal(wb[:e], ws_rows(plan, ws.view(plan.store_torch_dtype())[:plan.workspace_elems],
                                                   v0, nr)), f"workspace band z0={z0}"
            assert torch.equal(slab, vol[z0:z0 + nzs]), f"slab z0={z0}"
        log(f"band calls {case}: {nz // zr} slabs bitwise equal")


def test_band_rows_follow_eq9_and_reject_short_bands():
    n, nz, p, r = 64, 64, 90, 256.0
    with pkg.Plan(n, p, r, s=2, nz=nz) as plan:
        # the mid-plane slab maps to the central rows; the top slab to the top
        v0, nr = plan.band_rows(nz // 2 - 1, 2)
        assert v0 <= n // 2 - 1 and v0 + nr >= n // 2 + 1 and nr <= 8
        v0t, nrt = plan.band_rows(nz - 8, 8)
        assert v0t + nrt == n and v0t > n // 2
        # every sample of every voxel of the slab lies in the band (eq. (9), FP64)
        c = (n - 1) / 2.0
        z = np.arange(nz - 8, nz) - (nz - 1) / 2.0
        d = r + np.array([-c * np.sqrt(2.0), c * np.sqrt(2.0)])
        b = (z[:, None] * r / d[None, :]).ravel() + c
        assert v0t <= np.floor(b.min()) and min(np.floor(b.max()) + 1, n - 1) <= v0t + nrt - 1
        pb, fb, wb = plan.empty_band(nrt)
        slab = torch.empty((8, n, n), dtype=torch.float32, device=DEV)
        with pytest.raises(pkg.FdkodError) as ei:
            plan.reconstruct_slab(fb, wb, v0t + 1, nrt - 1, nz - 8, slab)
        assert ei.value.code == "E_ARG"


@pytest.mark.parametrize("case", [CASES[0], CASES[2], CASES[3]])
def test_streamed_equals_in_memory_and_oracle(case):
    n, nz, p, r, s, k, store = case
    proj_cpu = scan(n, p, r, 6, 80 + n)
    with pkg.Plan(n, p, r, s=s, skip=k, nz=nz, store=store) as plan:
        _, _, vol = full_run(plan, proj_cpu.to(DEV))
        host_proj = proj_cpu.pin_memory()
        host_vol = torch.zeros((nz, n, n), dtype=torch.float32).pin_memory()
        nbytes = plan.streamed_bytes(16)
        work = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
        copy = torch.cuda.Stream()
        plan.reconstruct_streamed(host_proj, host_vol, 16, work, copy_stream=copy)
        torch.cuda.synchronize()
        assert torch.equal(host_vol, vol.cpu()), "streamed != in-memory"
        ref = oracle_reconstruct(proj_cpu, r, s, k, nz=nz, store=store if store != "f32" else None)
        err, _ = report(f"streamed {case}", host_vol.double().numpy(), ref, bar=(1e-4 if store == "f32" else 2e-3))
        assert err <= (1e-4 if store == "f32" else 2e-3)
        # the same on one stream, and with too small a work buffer
        host_vol.zero_()
        plan.reconstruct_streamed(host_proj, host_vol, 16, work)
        assert torch.equal(host_vol, vol.cpu())
        with pytest.raises(pkg.FdkodError) as ei:
            plan.reconstruct_streamed(host_proj, host_vol, 16, work[: nbytes // 2])
        assert ei.value.code == "E_ARG"


def test_streamed_memory_is_a_fraction_of_the_whole_volume_path():
    """2000^3, P = 720, s = 4, BF16 (plans only: no data)."""
    n, p, r = 2000, 720, 8000.0
    with pkg.Plan(n, p, r, s=4, store="bf16") as plan:
        whole = 4 * p * n * n + plan.filtered_bytes + plan.workspace_bytes + 4 * n * n * n
        slab = plan.streamed_bytes(64)
        log(f"device bytes: whole-volume FDK-OD {whole / 1e9:.1f} GB, streamed (64-slice slabs) "
            f"{slab / 1e9:.1f} GB ({whole / slab:.1f}x less)")
        assert slab * 4 < whole
