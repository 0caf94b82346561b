"""The row-staged decimation kernel (the default for the paper's plain
decimation) against the per-square kernel, through the C ABI: both add the
same interpolated samples with the same weights in the same order, so the
decimated sub-sinograms must be bitwise equal.  Covers one, two and four
64-column chunks per lane, ragged squares, skipped stages, the three storage
types, a band of detector rows, and the N = 2000, P = 720 workload at s = 4
and s = 5."""

import pytest
import torch

import paper_1708_07515_amd as pkg
from gpu_common import DEV, log, require_gpu, scan

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


# n, p, r, s, k, store
CASES = [(64, 90, 512.0, 1, 0, "f32"), (64, 90, 512.0, 2, 0, "f32"), (64, 90, 512.0, 2, 1, "bf16"),
         (37, 50, 150.0, 3, 1, "f32"), (96, 128, 384.0, 3, 0, "f16"), (160, 120, 640.0, 2, 0, "f32"),
         (300, 96, 1200.0, 2, 1, "bf16"), (512, 360, 2048.0, 3, 0, "f32")]


def _decimate_both(plan, filt, v0=None, nrows=None, filt_band=None):
    shape = plan.get_tuning()
    assert shape["decim_chunks"] == 0, "the row-staged kernel is the default"
    chunks = 1
    while 64 * chunks < plan.info.max_width:
        chunks *= 2
    outs = []
    for c in (0, chunks):
        plan.set_tuning(decim_chunks=c)
        if v0 is None:
            ws = plan.empty_workspace()
            ws.fill_(7)
            plan.decompose(filt, ws)
        else:
            ws = plan.empty_band(nrows)[2]
            ws.fill_(7)
            plan.decompose_band(filt_band, v0, ws)
        torch.cuda.synchronize()
        outs.append(ws)
    plan.set_tuning(decim_chunks=0)
    return outs


@pytest.mark.parametrize("case", CASES)
def test_staged_equals_per_square_kernel(case):
    n, p, r, s, k, store = case
    proj = scan(n, p, r, 8, 40 + n)
    with pkg.Plan(n, p, r, s=s, skip=k, store=store) as plan:
        filt = plan.empty_filtered()
        plan.filter(proj.to(DEV), filt)
        staged, chunked = _decimate_both(plan, filt)
        e = plan.workspace_bytes
        log(f"staged decimation {case}: max width {plan.info.max_width}, "
            f"equal {torch.equal(staged[:e], chunked[:e])}")
        assert torch.equal(staged[:e], chunked[:e])


def test_staged_band_equals_per_square_kernel():
    n, p, r, s, k = 96, 120, 384.0, 3, 0
    proj = scan(n, p, r, 8, 77)
    with pkg.Plan(n, p, r, s=s, skip=k) as plan:
        v0, nrows = plan.band_rows(40, 16)
        pb = proj[:, v0:v0 + nrows, :].contiguous().to(DEV)
        fb = plan.empty_band(nrows)[1]
        plan.filter_band(pb, v0, fb)
        staged, chunked = _decimate_both(plan, None, v0, nrows, fb)
        assert torch.equal(staged, chunked)


@pytest.mark.parametrize("s", [4, 5])
def test_staged_full_size(s):
    from synth import configs, phantom
    wl = configs.C5
    proj = phantom.project(phantom.random_ellipsoids(wl.ellipsoids, wl.seed), wl.n, wl.p, wl.r,
                           device=DEV).contiguous()
    with pkg.Plan(wl.n, wl.p, wl.r, s=s, store="f32") as plan:
        filt = plan.empty_filtered()
        plan.filter(proj, filt)
        del proj
        staged, chunked = _decimate_both(plan, filt)
        same = torch.equal(staged, chunked)
        log(f"staged decimation cone2000_p720 s={s}: max width {plan.info.max_width}, equal {same}")
        assert same
