"""Canary guard bands: every output buffer handed to the library is a view
into a larger allocation whose bytes before and after it hold a canary
pattern; after the whole path runs (filter, decomposition, reconstruction;
the learned filter's forward, transpose and gradient; bands and slabs), the
canaries are unchanged, so no kernel writes outside the buffers the header
gives it."""

import numpy as np
import pytest
import torch

import paper_1708_07515_amd as pkg
from gpu_common import DEV, require_gpu, scan

pytestmark = pytest.mark.gpu

GUARD = 4096            # elements of canary before and after each buffer
CANARY = 0x7FC0DEAD     # a NaN pattern no kernel writes


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


class Guarded:
    """A buffer of ``shape`` and ``dtype`` inside a canary-filled allocation."""

    def __init__(self, shape, dtype):
        n = int(np.prod(shape))
        es = torch.empty(0, dtype=dtype).element_size()
        words = (GUARD * es + 3) // 4
        self.pre = words
        total = 2 * words + (n * es + 3) // 4
        self.raw = torch.full((total,), CANARY, dtype=torch.int32, device=DEV)
        self.t = self.raw[words:].view(torch.uint8)[:n * es].view(dtype).view(shape)
        self.tail0 = words + (n * es + 3) // 4

    def intact(self):
        torch.cuda.synchronize()
        head = self.raw[:self.pre]
        tail = self.raw[self.tail0:]
        return bool((head == CANARY).all()) and bool((tail == CANARY).all())


CASES = [dict(n=64, p=90, r=256.0, s=0), dict(n=64, p=90, r=256.0, s=2),
         dict(n=37, p=50, r=150.0, s=3, skip=1), dict(n=64, p=96, r=256.0, s=3, store="bf16"),
         dict(n=48, p=64, r=192.0, s=2, store="f16"), dict(n=64, p=90, r=256.0, s=2, rows="cone"),
         dict(n=64, p=90, r=256.0, s=2, decim="sinc", taps=6, interp="cubic"),
         dict(n=48, p=72, r=192.0, s=1, nz=20)]


@pytest.mark.parametrize("case", CASES, ids=[str(i) for i in range(len(CASES))])
def test_outputs_stay_within_their_buffers(case):
    n, p, r = case["n"], case["p"], case["r"]
    kw = {k: v for k, v in case.items() if k not in ("n", "p", "r")}
    proj = scan(n, p, r, 6, 77).to(DEV)
    with pkg.Plan(n, p, r, **kw) as plan:
        filt = Guarded(tuple(plan.empty_filtered().shape), plan.store_torch_dtype())
        vol = Guarded((plan.nz, n, n), torch.float32)
        ws = Guarded((max(plan.workspace_elems, 1),), plan.store_torch_dtype()) if plan.s > 0 else None
        plan.filter(proj, filt.t)
        plan.backproject(filt.t, vol.t, None if ws is None else ws.t)
        assert filt.intact() and vol.intact() and (ws is None or ws.intact())
        assert bool(torch.isfinite(vol.t).all())


def test_learned_and_band_outputs_stay_within_their_buffers():
    n, p, r, s = 64, 96, 256.0, 3
    proj = scan(n, p, r, 6, 78).to(DEV)
    with pkg.Plan(n, p, r, s=s) as plan:
        filt = plan.empty_filtered()
        plan.filter(proj, filt)
        net = pkg.LearnedDecimation(DEV, seed=1)
        net.load(torch.randn(pkg.LEARNED_PARAMS, generator=torch.Generator().manual_seed(2)) * 0.05)
        ws = Guarded((plan.workspace_elems,), torch.float32)
        vol = Guarded((plan.nz, n, n), torch.float32)
        dws = Guarded((plan.workspace_elems,), torch.float32)
        grad = Guarded((pkg.LEARNED_PARAMS,), torch.float32)
        plan.learned_decompose(filt, ws.t, net.weights)
        plan.reconstruct(filt, ws.t, vol.t)
        plan.reconstruct_adjoint(torch.randn_like(vol.t), dws.t)
        plan.learned_backward(filt, dws.t, net.weights, grad.t)
        for g in (ws, vol, dws, grad):
            assert g.intact()
        # a band of rows and its slab
        z0, nzs = 16, 16
        v0, nr = plan.band_rows(z0, nzs)
        fb = Guarded((p, nr, n), torch.float32)
        wb = Guarded((plan.band_workspace_elems(nr),), torch.float32)
        dwb = Guarded((plan.band_workspace_elems(nr),), torch.float32)
        slab = Guarded((nzs, n, n), torch.float32)
        plan.filter_band(proj[:, v0:v0 + nr, :].contiguous(), v0, fb.t)
        plan.decompose_band(fb.t, v0, wb.t)
        plan.reconstruct_slab(fb.t, wb.t, v0, nr, z0, slab.t)
        plan.learned_decompose_band(fb.t, v0, wb.t, net.weights)
        plan.reconstruct_adjoint_slab(torch.randn_like(slab.t), v0, nr, z0, dwb.t)
        plan.learned_backward_band(fb.t, v0, dwb.t, net.weights, grad.t)
        for g in (fb, wb, dwb, slab, grad):
            assert g.intact()
