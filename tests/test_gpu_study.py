"""GPU check of the quality study's claims on a small case (N = 96, P = 120):
uniform interiors keep their value (Sec. 4: the decomposition hardly affects
uniform regions), each skipped decimation stage moves the result closer to
direct FDK (Sec. 2.2), and edges are blurred by the decimation, less with a
stage skipped (Sec. 4)."""

import numpy as np
import pytest
import torch

import paper_1708_07515_amd as pkg
import study
from gpu_common import log, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def test_quality_sweep_properties():
    res = study.quality_sweep(torch, pkg, 96, 120, 384.0, 3)
    rows = res["rows"]
    fdk_w = res["fdk_edge"]["width_10_90"]
    log(f"direct FDK 10-90 edge width {fdk_w:.2f} voxels, {res['interior_voxels']} interior voxels")
    assert res["interior_voxels"] > 1000
    for r in rows:
        assert abs(r["interior_ratio_mean"] - 1.0) <= 5e-3, r
        assert r["width_10_90"] > fdk_w, r
    by = {(r["s"], r["k"], r["rows"]): r for r in rows}
    for (s, k, rw), r in by.items():
        if (s, k + 1, rw) in by:
            assert by[(s, k + 1, rw)]["rel_rmse_vs_fdk"] < r["rel_rmse_vs_fdk"], (s, k, rw)
    w0 = np.mean([r["width_10_90"] for r in rows if r["k"] == 0])
    w1 = np.mean([r["width_10_90"] for r in rows if r["k"] == 1])
    log(f"mean 10-90 edge width: k=0 {w0:.2f}, k=1 {w1:.2f}")
    assert w1 < w0 - 0.2
