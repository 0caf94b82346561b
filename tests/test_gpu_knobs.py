"""GPU tests of the quality knobs (extensions beyond the paper): the
windowed-sinc decimation window (2, 4 or 6 taps) and the cubic (Keys) shift,
alone, together and with cone-corrected rows.  Parity with the FP64 oracle's
pipeline with the same knobs (rel-RMSE <= 1e-4 FP32, <= 2e-3 BF16 storage),
the chunk count not changing a bit of the result, the slab mode equal to the
in-memory path, and the calls that reject the knobs."""

import numpy as np
import pytest
import torch

import paper_1708_07515_amd as pkg
from oracle import fdkod as ofdkod, metrics, storage
from gpu_common import DEV, log, report, require_gpu, scan

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-4
TOL_HALF = 2e-3

# N, N_z, P, R, s, k, store, window, taps, interp, rows
CASES = [
    (64, 64, 90, 512.0, 2, 0, "f32", "sinc", 2, "linear", "detector"),
    (64, 64, 90, 512.0, 2, 0, "f32", "sinc", 4, "linear", "detector"),
    (72, 72, 97, 300.0, 3, 1, "f32", "sinc", 6, "linear", "detector"),
    (48, 40, 67, 150.0, 2, 1, "f32", "triangle", 2, "cubic", "detector"),
    (80, 80, 120, 320.0, 3, 0, "f32", "sinc", 4, "cubic", "detector"),
    (64, 64, 90, 256.0, 3, 0, "bf16", "sinc", 4, "cubic", "detector"),
    (96, 96, 96, 192.0, 4, 0, "f32", "sinc", 4, "cubic", "cone"),
    (64, 64, 90, 256.0, 2, 0, "bf16", "sinc", 6, "cubic", "cone"),
]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def run(proj, n, p, r, s, k=0, nz=0, store="f32", chunks=None, **knobs):
    with pkg.Plan(n, p, r, s=s, skip=k, nz=nz, store=store, **knobs) as plan:
        if chunks is not None:
            plan.set_tuning(decim_chunks=chunks)
        filt, ws, vol = plan.empty_filtered(), plan.empty_workspace(), plan.empty_volume()
        plan.filter(proj.to(DEV), filt)
        plan.backproject(filt, vol, ws)
        torch.cuda.synchronize()
        return vol.cpu().double().numpy()


def oracle(proj, r, s, k, nz, store, window, taps, interp, rows):
    rounder = storage.ROUNDERS[store] if store != "f32" else None
    fn = ofdkod.fdkod_cone if rows == "cone" else ofdkod.fdkod
    return fn(proj.double().numpy(), r, s, k, nz=nz, store=rounder, window=window, taps=taps, interp=interp)


@pytest.mark.parametrize("case", CASES)
def test_knobs_match_oracle(case):
    n, nz, p, r, s, k, store, window, taps, interp, rows = case
    log(f"knobs parity {case}")
    proj = scan(n, p, r, 8, 120 + n)
    got = run(proj, n, p, r, s, k, nz, store, decim=window, taps=taps, interp=interp, rows=rows)
    ref = oracle(proj, r, s, k, nz, store, window, taps, interp, rows)
    err, _ = report(f"knobs {case}", got, ref, bar=(TOL_F32 if store == "f32" else TOL_HALF))
    assert err <= (TOL_F32 if store == "f32" else TOL_HALF)
    plain = run(proj, n, p, r, s, k, nz, store, rows=rows)
    assert metrics.rel_rmse(plain, ref) > 10 * err, "the knobs left the result unchanged"


@pytest.mark.parametrize("knobs,chunks", [(dict(decim="sinc", taps=6, interp="cubic"), (1, 2, 4)),
                                          ({}, (1, 2, 4, 8))])
def test_chunk_count_does_not_change_the_result(knobs, chunks):
    """Several column groups per square, several open windows, and (the plain
    linear shift at one chunk) two detector rows per task: every chunk count
    the kernels exist for gives the same bits; 8 chunks do not exist with more
    than two windows."""
    for n, p, r, s in ((200, 120, 800.0, 1), (97, 90, 300.0, 3)):
        proj = scan(n, p, r, 8, 5)
        vols = [run(proj, n, p, r, s, chunks=c, **knobs) for c in chunks]
        assert all(np.array_equal(vols[0], v) for v in vols[1:]), (n, s)
    with pkg.Plan(200, 120, 800.0, s=1, **knobs) as plan:
        assert plan.info.max_width > 64           # several column groups at 1 chunk
        if knobs:
            with pytest.raises(pkg.FdkodError) as ei:
                plan.set_tuning(decim_chunks=8)
            assert ei.value.code == "E_UNSUPPORTED"


def test_streamed_knobs_equal_in_memory():
    n, nz, p, r, s = 64, 64, 90, 256.0, 2
    knobs = dict(decim="sinc", taps=4, interp="cubic")
    proj_cpu = scan(n, p, r, 6, 31)
    want = run(proj_cpu, n, p, r, s, nz=nz, **knobs)
    with pkg.Plan(n, p, r, s=s, nz=nz, **knobs) as plan:
        host_proj = proj_cpu.pin_memory()
        host_vol = torch.zeros((nz, n, n), dtype=torch.float32).pin_memory()
        work = torch.empty(plan.streamed_bytes(16), dtype=torch.uint8, device=DEV)
        plan.reconstruct_streamed(host_proj, host_vol, 16, work)
        torch.cuda.synchronize()
    assert np.array_equal(host_vol.double().numpy(), want)


def test_c2_sampled_slices_with_knobs():
    """The 512^3, P = 360, s = 3 workload (noisy phantom) with the windowed
    sinc (4 taps) and the cubic shift, on two slices."""
    n, p, r, s = 512, 360, 2048.0, 3
    proj = scan(n, p, r, 20, 2, 1e5, on_gpu=True)
    slices = [0, 300]
    got = run(proj, n, p, r, s, decim="sinc", taps=4, interp="cubic")
    ref = ofdkod.fdkod(proj.double().numpy(), r, s, slices=slices, window="sinc", taps=4, interp="cubic")
    err, _ = report(f"c2 s=3 sinc4 cubic slices {slices}", got[slices], ref, bar=TOL_F32)
    assert err <= TOL_F32


def test_learned_and_batch_reject_knobs():
    """Batches keep to the paper's knobs.  The learned filter takes the
    windowed sinc and the cubic shift: with zero weights it returns the
    plan's plain decomposition exactly."""
    n, p, r = 64, 90, 256.0
    w = torch.zeros(pkg.LEARNED_PARAMS, dtype=torch.bfloat16, device=DEV)
    for knobs in (dict(decim="sinc", taps=4), dict(interp="cubic")):
        with pkg.Plan(n, p, r, s=2, **knobs) as plan:
            filt = plan.empty_filtered().normal_(generator=torch.Generator(device=DEV).manual_seed(3))
            ws_l, ws_t = plan.empty_workspace(), plan.empty_workspace()
            plan.learned_decompose(filt, ws_l, w)
            plan.decompose(filt, ws_t)
            torch.cuda.synchronize()
            e = plan.workspace_elems
            assert torch.equal(ws_l.view(torch.float32)[:e], ws_t.view(torch.float32)[:e])
        with pytest.raises(pkg.FdkodError) as ei:
            pkg.Batch([dict(n=n, p=p, r=r, s=2), dict(n=n, p=p, r=r, s=2, **knobs)])
        assert ei.value.code == "E_UNSUPPORTED"
