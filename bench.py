"""Benchmark: FDK-OD against direct FDK on one MI355X, in GVUPS.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cone512_p360] [--s 3]

A step is one pass of the whole hot path over one scan already resident in
HBM: bounds kernel (eq. (1) at the square vertices), ramp filter, crop + shift
+ angular decimation, backprojection of every square.  GVUPS (voxel-angle
updates per second) counts the direct-equivalent work N*N*N_z*P per step, so
FDK-OD and direct FDK are on the same scale.  Prints one JSON line.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GVUPS FDK-OD vs direct FDK on 1 MI355X at stated rel-RMSE vs FP64 oracle"
HBM_PEAK_GBS = 8000.0
# FP32 VALU peak without packed FP32: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2
VALU_PEAK_TFLOPS = 78.6
FLOPS_PER_UPDATE = 14     # row coordinate FMA, fraction, 3 lerps (sub + FMA), weighted FMA


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cone512_p360")
    ap.add_argument("--s", type=int, default=None)
    ap.add_argument("--skip", type=int, default=None)
    ap.add_argument("--store", default=None)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-direct", action="store_true", help="skip timing direct FDK")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed_steps(torch, stages, steps, warmup):
    """Run ``stages`` (list of (name, fn)) warmup + steps times; per-stage HIP
    event times on the current stream, and the wall time of the timed steps."""
    for _ in range(warmup):
        for _, fn in stages:
            fn()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        for i, (_, fn) in enumerate(stages):
            fn()
            ev[k][i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = {name: sum(ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(steps)) / steps
           for i, (name, _) in enumerate(stages)}
    total = sum(ev[k][0].elapsed_time(ev[k][-1]) for k in range(steps)) / steps
    return per, total, wall


def cpu_baseline(proj_cpu, wl, s, k, gpu_vol):
    """Time the FP64 oracle (single thread) on one slice of the same workload,
    and compare that slice with the GPU result."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import fdk as ofdk, fdkod as ofdkod, metrics

    sl = [wl.nzv // 2 + 7]
    arr = proj_cpu.numpy()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        if s == 0:
            ref = ofdk.fdk(arr, wl.r, slices=sl)
        else:
            ref = ofdkod.fdkod(arr, wl.r, s, k, slices=sl)
        dt = time.perf_counter() - t0
    got = gpu_vol[sl].cpu().double().numpy()
    err = metrics.rel_rmse(got, ref)
    mx, mxr = metrics.max_abs(got, ref)
    gv = wl.n * wl.n * len(sl) * wl.p / dt / 1e9
    return dict(value=gv, unit="GVUPS", cores=1, kind="oracle",
                sample=f"1 slice (l={sl[0]}) of {wl.name}, s={s}, k={k}: {dt:.1f} s",
                seconds=dt), dict(rel_rmse=err, max_abs=mx, max_abs_rel=mxr, slices=sl)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path "
              "shards by z-slab across GPUs but that is not built here", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1708_07515_amd as pkg
    from synth import configs, phantom

    wl = configs.ALL[args.workload]
    s = args.s if args.s is not None else max(wl.s)
    k = args.skip if args.skip is not None else wl.k
    store = args.store or wl.store[0]
    n, p, r, nz = wl.n, wl.p, wl.r, wl.nzv
    dev = "cuda:0"

    log(f"[bench] generating {wl.name} on the GPU")
    ell = phantom.random_ellipsoids(wl.ellipsoids, wl.seed)
    proj = phantom.project(ell, n, p, r, device=dev)
    if wl.photons:
        proj = phantom.poisson_noise(proj, n, wl.photons, wl.seed + 1000)
    proj = proj.contiguous()
    torch.cuda.synchronize()

    plan = pkg.Plan(n, p, r, s=s, skip=k, nz=nz, store=store)
    filt = plan.empty_filtered()
    ws = plan.empty_workspace()
    vol = plan.empty_volume()
    stages = [("bounds", lambda: plan.bounds()),
              ("filter", lambda: plan.filter(proj, filt)),
              ("decompose", lambda: plan.decompose(filt, ws)),
              ("reconstruct", lambda: plan.reconstruct(filt, ws, vol))]
    log(f"[bench] FDK-OD s={s} k={k} store={store}: P'={plan.p_dec}, squares={plan.squares}, "
        f"workspace {plan.workspace_bytes / 1e9:.2f} GB")
    per, step_ms, wall = timed_steps(torch, stages, args.steps, args.warmup)
    log(f"[bench] FDK-OD per stage (ms): " + ", ".join(f"{a}={b:.3f}" for a, b in per.items()))

    direct = None
    if not args.no_direct:
        dplan = pkg.Plan(n, p, r, s=0, nz=nz, store=store)
        dvol = dplan.empty_volume()
        dstages = [("filter", lambda: dplan.filter(proj, filt)),
                   ("reconstruct", lambda: dplan.reconstruct(filt, None, dvol))]
        dsteps = max(1, min(args.steps, 3))
        dper, dstep_ms, _ = timed_steps(torch, dstages, dsteps, 1)
        direct = dict(ms_per_step=dstep_ms, stage_ms=dper,
                      gvups=n * n * nz * p / (dstep_ms * 1e-3) / 1e9,
                      gvups_reconstruct=n * n * nz * p / (dper["reconstruct"] * 1e-3) / 1e9)
        log(f"[bench] direct FDK per stage (ms): " + ", ".join(f"{a}={b:.3f}" for a, b in dper.items()))
        # the filter buffer was overwritten with the same values; rerun once to
        # leave the FDK-OD output in place for the parity sample
        for _, fn in stages:
            fn()
        torch.cuda.synchronize()

    updates_eq = n * n * nz * p
    value = updates_eq / (step_ms * 1e-3) / 1e9
    paper_ms = per["bounds"] + per["decompose"] + per["reconstruct"]
    rec_ms = per["reconstruct"]
    flops = FLOPS_PER_UPDATE * plan.updates
    achieved = flops / (rec_ms * 1e-3) / 1e12
    roofline = dict(bound="alu", kernel="k_backproject", achieved=round(achieved, 3),
                    peak=VALU_PEAK_TFLOPS, unit="TFLOP/s", frac=round(achieved / VALU_PEAK_TFLOPS, 4),
                    traffic=None, flops_per_update=FLOPS_PER_UPDATE, updates=plan.updates)

    cpu = parity = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on a bounded sample")
        cpu, parity = cpu_baseline(proj.cpu(), wl, s, k, vol)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GVUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if store == "f32" else f"{store}-storage/f32",
        "data": f"synthetic: seeded {wl.ellipsoids}-ellipsoid phantom"
                + (f", Poisson noise {wl.photons:g} photons" if wl.photons else ""),
        "config": {"workload": wl.name, "n": n, "nz": nz, "p": p, "r": r, "s": s, "k": k,
                   "p_dec": plan.p_dec, "store": store},
        "stage_ms": {a: round(b, 4) for a, b in per.items()},
        "gvups_paper_scope": round(updates_eq / (paper_ms * 1e-3) / 1e9, 3),
        "gvups_exec_reconstruct": round(plan.updates / (rec_ms * 1e-3) / 1e9, 3),
        "direct_fdk": None if direct is None else {
            "ms_per_step": round(direct["ms_per_step"], 4),
            "gvups": round(direct["gvups"], 3),
            "stage_ms": {a: round(b, 4) for a, b in direct["stage_ms"].items()}},
        "speedup_vs_direct": None if direct is None else round(direct["ms_per_step"] / step_ms, 3),
        "speedup_vs_direct_paper_scope": None if direct is None else
            round(direct["stage_ms"]["reconstruct"] / paper_ms, 3),
        "parity": parity,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "wall_s_timed": round(wall, 4),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
