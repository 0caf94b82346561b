"""fdkod_backproject_noalloc (the entry point for callers that cannot
allocate device memory) against fdkod_backproject with a caller workspace,
through the C ABI: the same kernels, so the volumes must be bitwise equal.
Two calls in a row, the second with a smaller plan, share the library's
fixed device array; a plan whose workspace exceeds it is refused."""

import ctypes

import pytest
import torch

import paper_1708_07515_amd as pkg
from gpu_common import DEV, log, require_gpu, scan

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _inputs(n, p, r, s, store, nz=0, seed=31):
    plan = pkg.Plan(n, p, r, s=s, nz=nz, store=store)
    proj = scan(n, p, r, 8, seed).to(DEV)
    filt = plan.empty_filtered()
    plan.filter(proj, filt)
    return plan, filt


def _check(case):
    n, p, r, s, store, nz = case
    plan, filt = _inputs(n, p, r, s, store, nz)
    assert plan.workspace_bytes <= pkg.NOALLOC_SCRATCH_BYTES
    ref = plan.empty_volume()
    ws = plan.empty_workspace()
    plan.backproject(filt, ref, ws)
    got = torch.full_like(ref, float("nan"))
    torch.cuda.synchronize()
    lib = pkg.load_library()
    st = lib.fdkod_backproject_noalloc(plan._h, ctypes.c_void_p(filt.data_ptr()),
                                       ctypes.c_void_p(got.data_ptr()),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, lib.fdkod_last_error()
    torch.cuda.synchronize()
    log(f"noalloc {case}: workspace {plan.workspace_bytes} bytes, "
        f"max |diff| {float((got - ref).abs().max()):.3e}")
    assert torch.equal(got, ref)
    plan.close()


def test_noalloc_matches_workspace_call_twice():
    # first a larger plan, then a smaller one: the second call reuses the
    # array that still holds the first call's sub-sinograms
    _check((96, 120, 384.0, 3, "f32", 0))
    _check((40, 50, 160.0, 2, "bf16", 24))


def test_noalloc_direct_and_refusal():
    _check((48, 60, 192.0, 0, "f32", 0))
    # N = 512, P = 360, s = 3, FP32: 589 MB of sub-sinograms, beyond the array
    with pkg.Plan(512, 360, 2048.0, s=3) as plan:
        assert plan.workspace_bytes > pkg.NOALLOC_SCRATCH_BYTES
        filt = torch.empty(1, dtype=torch.float32, device=DEV)
        vol = torch.empty(1, dtype=torch.float32, device=DEV)
        lib = pkg.load_library()
        st = lib.fdkod_backproject_noalloc(plan._h, ctypes.c_void_p(filt.data_ptr()),
                                           ctypes.c_void_p(vol.data_ptr()), None)
        assert pkg._lib.STATUS_NAMES[st] == "E_UNSUPPORTED"
