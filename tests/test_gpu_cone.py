"""GPU tests of the cone-corrected decimation (FDKOD_ROWS_CONE): parity with
the FP64 oracle's fdkod_cone (rel-RMSE <= 1e-4 FP32, <= 2e-3 BF16 storage),
s = 0 unchanged, the quality property it exists for (less off-midplane error
than the plain decimation at a large D), and the calls that reject it."""

import numpy as np
import pytest
import torch

import paper_1708_07515_amd as pkg
from oracle import fdkod as ofdkod, metrics, storage
from synth import phantom
from gpu_common import DEV, log, report, require_gpu, scan

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-4
TOL_HALF = 2e-3

# N, N_z, P, R, s, k, store: several tiles, ragged squares and slabs, skipped
# stages, both storage widths
CASES = [(64, 64, 90, 512.0, 2, 0, "f32"), (48, 40, 67, 150.0, 2, 1, "f32"),
         (72, 72, 97, 300.0, 3, 1, "f32"), (64, 64, 90, 256.0, 3, 0, "bf16"),
         (96, 96, 96, 192.0, 4, 0, "f32")]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def run(proj, n, p, r, s, k=0, nz=0, store="f32", rows="cone"):
    with pkg.Plan(n, p, r, s=s, skip=k, nz=nz, store=store, rows=rows) as plan:
        filt, ws, vol = plan.empty_filtered(), plan.empty_workspace(), plan.empty_volume()
        plan.filter(proj.to(DEV), filt)
        plan.backproject(filt, vol, ws)
        torch.cuda.synchronize()
        return vol.cpu().double().numpy()


def thin_discs():
    """Thin discs far off the mid-plane plus a faint body (normalised units)."""
    return phantom.Ellipsoids(
        np.array([[0.0, 0.0, 0.55], [0.2, -0.3, -0.5], [-0.3, 0.2, 0.45], [0.0, 0.0, 0.0]]),
        np.array([[0.6, 0.6, 0.04], [0.4, 0.4, 0.05], [0.3, 0.3, 0.04], [0.7, 0.7, 0.7]]),
        np.array([1.0, 1.0, 1.0, 0.2]))


@pytest.mark.parametrize("case", CASES)
def test_cone_matches_oracle(case):
    n, nz, p, r, s, k, store = case
    log(f"cone parity {case}")
    proj = scan(n, p, r, 8, 90 + n)
    got = run(proj, n, p, r, s, k, nz, store)
    rounder = storage.ROUNDERS[store] if store != "f32" else None
    ref = ofdkod.fdkod_cone(proj.double().numpy(), r, s, k, nz=nz, store=rounder)
    err, _ = report(f"cone {case}", got, ref, bar=(TOL_F32 if store == "f32" else TOL_HALF))
    assert err <= (TOL_F32 if store == "f32" else TOL_HALF)
    # the plain decimation differs from the cone-corrected one off the mid-plane
    plain = run(proj, n, p, r, s, k, nz, store, rows="detector")
    assert metrics.rel_rmse(plain, ref) > 10 * err


def test_cone_is_plain_fdkod_at_s0():
    n, p, r = 48, 60, 200.0
    proj = scan(n, p, r, 6, 7)
    a = run(proj, n, p, r, 0, rows="cone")
    b = run(proj, n, p, r, 0, rows="detector")
    assert np.array_equal(a, b)


def test_cone_reduces_off_midplane_error_against_direct_fdk():
    """Thin discs at |z| ~ N/4, D = 16: against the HIP direct FDK, the
    cone-corrected decimation's error on the off-midplane slices is well below
    the plain decimation's."""
    n, p, r, s = 96, 96, 192.0, 4
    proj = phantom.project(thin_discs(), n, p, r).contiguous()
    direct = run(proj, n, p, r, 0, rows="detector")
    plain = run(proj, n, p, r, s, rows="detector")
    cone = run(proj, n, p, r, s)
    cz = (n - 1) / 2.0
    sl = [int(cz + 0.55 * n / 2), int(cz - 0.5 * n / 2)]
    e_plain = metrics.rel_rmse(plain[sl], direct[sl])
    e_cone = metrics.rel_rmse(cone[sl], direct[sl])
    log(f"off-midplane rel-RMSE vs direct FDK: plain {e_plain:.4f}, cone {e_cone:.4f}")
    assert e_cone <= 0.7 * e_plain


def test_calls_that_need_detector_rows_reject_cone():
    n, p, r = 64, 90, 256.0
    with pkg.Plan(n, p, r, s=2, rows="cone") as plan:
        for call in (lambda: plan.band_rows(0, 8),
                     lambda: plan.learned_decompose(plan.empty_filtered(), plan.empty_workspace(),
                                                    torch.zeros(pkg.LEARNED_PARAMS, dtype=torch.bfloat16,
                                                                device=DEV))):
            with pytest.raises(pkg.FdkodError) as ei:
                call()
            assert ei.value.code == "E_UNSUPPORTED"
    with pytest.raises(pkg.FdkodError) as ei:
        pkg.Batch([dict(n=n, p=p, r=r, s=2), dict(n=n, p=p, r=r, s=2, rows="cone")])
    assert ei.value.code == "E_UNSUPPORTED"
