"""Reconstructions run under the checked build of the library (loaded through
FDKOD_LIB by tests/test_gpu_checked.py, in a process of their own): the small
parity cases of the GPU suite, each compared with the FP64 oracle, and the
kernels' event counters read after each.  Prints one JSON line per case."""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import numpy as np  # noqa: E402
import torch  # noqa: E402

import paper_1708_07515_amd as pkg  # noqa: E402
from oracle import fdkod as ofdkod, metrics  # noqa: E402
from synth import phantom  # noqa: E402

# n, p, r, s, k, store, rows: direct FDK, FDK-OD at s = 1..4, ragged sizes,
# skipped stages, half storage, cone-corrected rows and a close source whose
# block footprints are large
CASES = [(48, 60, 192.0, 0, 0, "f32", "detector"), (64, 90, 512.0, 1, 0, "f32", "detector"),
         (64, 90, 512.0, 2, 1, "bf16", "detector"), (37, 50, 150.0, 3, 1, "f32", "detector"),
         (96, 120, 384.0, 3, 0, "f16", "detector"), (128, 64, 512.0, 4, 0, "f32", "detector"),
         (64, 48, 100.0, 2, 0, "f32", "detector"), (48, 60, 192.0, 2, 0, "f32", "cone")]


def main():
    dev = "cuda:0"
    pkg.check_counts(reset=True)
    for (n, p, r, s, k, store, rows) in CASES:
        proj = phantom.project(phantom.random_ellipsoids(8, 50 + n), n, p, r).contiguous()
        with pkg.Plan(n, p, r, s=s, skip=k, store=store, rows=rows) as plan:
            filt, ws, vol = plan.empty_filtered(), plan.empty_workspace(), plan.empty_volume()
            plan.filter(proj.to(dev), filt)
            plan.backproject(filt, vol, ws)
            torch.cuda.synchronize()
            got = vol.cpu().double().numpy()
        counts = pkg.check_counts(reset=True)
        arr = proj.numpy().astype(np.float64)
        fn = ofdkod.fdkod_cone if rows == "cone" else ofdkod.fdkod
        ref = fn(arr, r, s, k)
        print(json.dumps({"case": [n, p, r, s, k, store, rows], "counts": counts,
                          "rel_rmse": metrics.rel_rmse(got, ref)}), flush=True)


if __name__ == "__main__":
    main()
