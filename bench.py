"""Benchmark: FDK-OD against direct FDK on one MI355X, in GVUPS.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cone2000_p720] [--s 4]

A step is one pass of the whole hot path over one scan already resident in
HBM: bounds kernel (eq. (1) at the square vertices), ramp filter, crop + shift
+ angular decimation, backprojection of every square.  GVUPS (voxel-angle
updates per second) counts the direct-equivalent work N*N*N_z*P per step, so
FDK-OD and direct FDK are on the same scale.  The main line is the paper's
headline size, N = 2000, P = 720 (volume 2000^3), s = 4, no skipped stage,
FP32 storage; BF16 storage, s = 5 and one skipped decimation stage are
reported beside it (``variants``), and the 512^3 workload as
``small_workload``.  Prints one JSON line.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GVUPS FDK-OD vs direct FDK on 1 MI355X at stated rel-RMSE vs FP64 oracle"
# FP32 VALU peak without packed FP32 (the library is built without packed
# FP32 instructions): 256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2 flops per FMA
VALU_PEAK_TFLOPS = 78.6
# the published FP32 vector figure, which counts packed FP32 (reported beside)
VALU_PACKED_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
# LDS: 128 bytes per clock per compute unit, 256 CUs at 2.4 GHz
LDS_PEAK_GBS = 128 * 256 * 2.4
# VALU issue limit: one 64-lane instruction per compute unit per cycle (four
# SIMDs, each taking four cycles for a wave's instruction), 256 CUs at 2.4 GHz
VALU_ISSUE_PEAK = 256 * 2.4e9
# algorithmic FP32 work of one voxel-angle update of the backprojection: three
# linear interpolations (a subtraction and an FMA each, counted as one flop
# and two) and the weighted accumulation (one FMA): 3 x 2 + 2 = 8
FLOPS_PER_UPDATE = 8
# on-chip bytes of one update: the bilinear sample's quad (value, column,
# row and mixed differences), FP32 (one 16-byte LDS read)
LDS_BYTES_PER_UPDATE = 16
# the workers of the CPU oracle baseline: the machine's CPU share for one GPU
CPU_WORKERS_MAX = 16


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cone2000_p720")
    ap.add_argument("--s", type=int, default=None)
    ap.add_argument("--skip", type=int, default=None)
    ap.add_argument("--store", default=None)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-direct", action="store_true", help="skip timing direct FDK")
    ap.add_argument("--no-small", action="store_true", help="skip the 512^3 workload")
    ap.add_argument("--no-variants", action="store_true", help="skip the BF16 / s / k variants")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-filter step")
    ap.add_argument("--no-streamed", action="store_true", help="skip the low-memory slab mode run")
    ap.add_argument("--no-cone", action="store_true", help="skip the cone-corrected decimation run")
    ap.add_argument("--slab", type=int, default=64, help="slices per slab in the slab mode")
    ap.add_argument("--cpu-workers", type=int, default=0, help="oracle worker processes (0: all, at most 16)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy (for HBM counter calibration)")
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
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)]
          for _ in range(steps)]
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


def measure_copy_peak(torch, reps=5):
    """Device-to-device copy of a 1 GiB FP32 buffer (1 GiB read + 1 GiB
    written), timed with HIP events: the HBM bandwidth a plain streaming
    kernel reaches, the practical ceiling of the HBM-bound stages."""
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 2 * a.numel() * a.element_size()
    del a, b
    torch.cuda.empty_cache()
    gbs = nbytes / (ms * 1e-3) / 1e9
    log(f"[bench] device copy: {ms:.3f} ms per 2 GiB moved, {gbs:.0f} GB/s")
    return {"value": round(gbs, 1), "unit": "GB/s", "ms": round(ms, 4), "bytes": nbytes,
            "what": "device copy of a 1 GiB FP32 buffer (read + write)"}


def make_scan(torch, wl, dev):
    from synth import phantom
    ell = phantom.random_ellipsoids(wl.ellipsoids, wl.seed)
    proj = phantom.project(ell, wl.n, wl.p, wl.r, device=dev)
    if wl.photons:
        proj = phantom.poisson_noise(proj, wl.n, wl.photons, wl.seed + 1000)
    proj = proj.contiguous()
    torch.cuda.synchronize()
    return proj


def run_workload(torch, pkg, wl, s, k, store, steps, warmup, direct=True, proj=None):
    """Time FDK-OD steps (and direct FDK) on one workload; returns a dict."""
    n, p, r, nz = wl.n, wl.p, wl.r, wl.nzv
    if proj is None:
        log(f"[bench] generating {wl.name} on the GPU")
        proj = make_scan(torch, wl, "cuda:0")
    plan = pkg.Plan(n, p, r, s=s, skip=k, nz=nz, store=store)
    filt = plan.empty_filtered()
    ws = plan.empty_workspace()
    vol = plan.empty_volume()
    stages = [("bounds", lambda: plan.bounds()),
              ("filter", lambda: plan.filter(proj, filt)),
              ("decompose", lambda: plan.decompose(filt, ws)),
              ("reconstruct", lambda: plan.reconstruct(filt, ws, vol))]
    log(f"[bench] {wl.name} FDK-OD s={s} k={k} store={store}: P'={plan.p_dec}, "
        f"squares={plan.squares}, workspace {plan.workspace_bytes / 1e9:.2f} GB")
    per, step_ms, wall = timed_steps(torch, stages, steps, warmup)
    log(f"[bench] FDK-OD per stage (ms): " + ", ".join(f"{a}={b:.3f}" for a, b in per.items()))
    out = dict(plan=plan, proj=proj, vol=vol, filt=filt, ws=ws, per=per, step_ms=step_ms, wall=wall,
               direct=None)
    if direct:
        dplan = pkg.Plan(n, p, r, s=0, nz=nz, store=store)
        dvol = dplan.empty_volume()
        dstages = [("filter", lambda: dplan.filter(proj, filt)),
                   ("reconstruct", lambda: dplan.reconstruct(filt, None, dvol))]
        dsteps = max(1, min(steps, 3))
        dper, dstep_ms, _ = timed_steps(torch, dstages, dsteps, 1)
        log(f"[bench] direct FDK per stage (ms): " + ", ".join(f"{a}={b:.3f}" for a, b in dper.items()))
        out["direct"] = dict(ms_per_step=dstep_ms, stage_ms=dper)
        del dvol
        # the filter buffer was rewritten with the same values; rerun one
        # FDK-OD step so vol holds its result for the parity sample
        for _, fn in stages:
            fn()
        torch.cuda.synchronize()
    return out


def summarise(wl, s, k, store, res):
    n, p, nz = wl.n, wl.p, wl.nzv
    per, step_ms = res["per"], res["step_ms"]
    updates_eq = n * n * nz * p
    paper_ms = per["bounds"] + per["decompose"] + per["reconstruct"]
    d = res["direct"]
    return {
        "workload": wl.name, "n": n, "nz": nz, "p": p, "r": wl.r, "s": s, "k": k,
        "p_dec": res["plan"].p_dec, "store": store,
        "ms_per_step": round(step_ms, 4),
        "gvups": round(updates_eq / (step_ms * 1e-3) / 1e9, 3),
        "stage_ms": {a: round(b, 4) for a, b in per.items()},
        "gvups_paper_scope": round(updates_eq / (paper_ms * 1e-3) / 1e9, 3),
        "gvups_exec_reconstruct": round(res["plan"].updates / (per["reconstruct"] * 1e-3) / 1e9, 3),
        "direct_fdk": None if d is None else {
            "ms_per_step": round(d["ms_per_step"], 4),
            "gvups": round(updates_eq / (d["ms_per_step"] * 1e-3) / 1e9, 3),
            "stage_ms": {a: round(b, 4) for a, b in d["stage_ms"].items()}},
        "speedup_vs_direct": None if d is None else round(d["ms_per_step"] / step_ms, 3),
        "speedup_vs_direct_paper_scope": None if d is None else
            round(d["stage_ms"]["reconstruct"] / paper_ms, 3),
    }


def run_learned(torch, pkg, wl, res, steps):
    """The FDK-OD step with the learned decimation filter on the main workload
    (seeded random weights: the cost does not depend on their values), timed
    like the triangle step; None where the learned kernels do not apply."""
    plan = res["plan"]
    if plan.s == 0 or plan.info.max_width > 252 or plan.p > 2048:
        return None
    proj, filt, ws, vol = res["proj"], res["filt"], res["ws"], res["vol"]
    # the triangle step's volume, the target of the timed training steps (the
    # random weights make the residual non-zero); volumes up to 1024^3 only
    train_target = vol.clone() if wl.n <= 1024 else None
    net = pkg.LearnedDecimation("cuda:0", seed=0)
    net.load(torch.randn(pkg.LEARNED_PARAMS, generator=torch.Generator().manual_seed(1)) * 0.05)
    stages = [("bounds", lambda: plan.bounds()),
              ("filter", lambda: plan.filter(proj, filt)),
              ("decompose_learned", lambda: plan.learned_decompose(filt, ws, net.weights)),
              ("reconstruct", lambda: plan.reconstruct(filt, ws, vol))]
    per, step_ms, _ = timed_steps(torch, stages, steps, 1)
    log("[bench] FDK-OD with the learned filter, per stage (ms): "
        + ", ".join(f"{a}={b:.3f}" for a, b in per.items()))
    updates_eq = wl.n * wl.n * wl.nzv * wl.p
    train = None
    if train_target is not None:
        resid = torch.empty_like(vol)
        dws = torch.empty(plan.workspace_elems, dtype=torch.float32, device=vol.device)
        tstages = [("train_step", lambda: net.train_step(plan, filt, ws, vol, train_target, resid, dws))]
        _, train_ms, _ = timed_steps(torch, tstages, 3, 1)
        log(f"[bench] learned filter, one AdamW step on the volume: {train_ms:.3f} ms")
        train = {"ms_per_step": round(train_ms, 3), "steps": 3,
                 "step": "learned decomposition, backprojection, squared residual against the "
                         "triangle step's volume, transpose of the backprojection, weight gradient, AdamW"}
        del resid, dws, train_target
    out = {"ms_per_step": round(step_ms, 4),
           "gvups": round(updates_eq / (step_ms * 1e-3) / 1e9, 3),
           "stage_ms": {a: round(b, 4) for a, b in per.items()},
           "decompose_triangle_ms": round(res["per"]["decompose"], 4),
           "weights": "817 BF16 parameters, seeded random",
           "training_step": train}
    if wl.name == "cone2000_p720" and plan.s == 4:
        out["trained"] = run_learned_slabs(torch, pkg, wl)
    return out


def run_learned_slabs(torch, pkg, wl, nzs=32):
    """The filter trained at this geometry (weights written by the quality
    study's --learned-c5 run) on held-out slabs: rel-RMSE against direct FDK
    of the triangle, the learned filter and the windowed sinc + cubic shift;
    and the time of one AdamW step on a slab (learned decomposition of the
    slab's band, slab reconstruction, residual, slab transpose, weight
    gradient, update)."""
    import study
    net = study.load_learned_c5(pkg)
    if net is None:
        return None
    scans = study.SlabScans(torch, pkg, wl, 4, nzs, wl.ellipsoids)
    seeds, positions = [9200, 9201, 9202, 9203], [384, 768, 1152, 1536]
    held = study.held_out_slabs(torch, pkg, scans, net, seeds, positions)
    log("[bench] trained learned filter, held-out slabs, rel-RMSE vs direct FDK: "
        + ", ".join(f"{a} {b:.4f}" for a, b in held["mean"].items()))
    # one training step on the last held-out slab (a copy of the net: the
    # trained weights stay as they are)
    trainer = study.load_learned_c5(pkg)
    z0 = positions[-1]
    v0, nr, fb = scans.slab(seeds[-1], z0)
    w = 1.0 / scans.energy(scans.tgt)
    tstages = [("train_step_slab", lambda: trainer.train_step_slab(
        scans.plan, fb, v0, scans.ws(nr), z0, scans.vol, scans.tgt, scans.resid, scans.dws(nr), weight=w))]
    _, train_ms, _ = timed_steps(torch, tstages, 3, 1)
    scans.close()
    return {"held_out": {k: [round(x, 5) for x in v] if k != "slabs" else v for k, v in held.items() if k != "mean"},
            "held_out_mean": {k: round(v, 5) for k, v in held["mean"].items()},
            "reference": "direct FDK (s = 0) of the same slab from the same filtered band",
            "slab_slices": nzs, "weights": "paper_1708_07515_amd/learned_c5_weights.txt",
            "train_step_slab_ms": round(train_ms, 3), "train_step_slab_rows": nr}


def _rel_rmse_regions(torch, vol, ref, regions, chunk=32):
    """rel-RMSE of vol against ref (device volumes) over slice ranges, in FP64
    chunks of slices so that no full-volume temporary is made."""
    out = {}
    for name, (z0, z1) in regions.items():
        num = den = 0.0
        for a in range(z0, z1, chunk):
            b = min(a + chunk, z1)
            r = ref[a:b].double()
            num += float(((vol[a:b].double() - r) ** 2).sum())
            den += float((r ** 2).sum())
        out[name] = (num / den) ** 0.5 if den > 0 else None
    return out


def run_cone(torch, pkg, wl, s, k, store, res, steps):
    """The FDK-OD step with the cone-corrected decimation on the same scan,
    timed like the triangle step, and the error of both decimations against
    the HIP direct FDK on the whole volume, on its top and bottom eighths
    (where the cone angle is largest) and on the central eighth."""
    if s == 0:
        return None
    n, p, r, nz = wl.n, wl.p, wl.r, wl.nzv
    proj, filt, vol = res["proj"], res["filt"], res["vol"]
    cplan = pkg.Plan(n, p, r, s=s, skip=k, nz=nz, store=store, rows="cone")
    cws = cplan.empty_workspace()
    cvol = cplan.empty_volume()
    stages = [("bounds", lambda: cplan.bounds()),
              ("filter", lambda: cplan.filter(proj, filt)),
              ("decompose", lambda: cplan.decompose(filt, cws)),
              ("reconstruct", lambda: cplan.reconstruct(filt, cws, cvol))]
    per, step_ms, _ = timed_steps(torch, stages, steps, 1)
    log("[bench] FDK-OD with the cone-corrected decimation, per stage (ms): "
        + ", ".join(f"{a}={b:.3f}" for a, b in per.items()))
    del cws
    # the triangle result (vol may hold another decimation's since)
    plan, ws = res["plan"], res["ws"]
    plan.decompose(filt, ws)
    plan.reconstruct(filt, ws, vol)
    dplan = pkg.Plan(n, p, r, s=0, nz=nz, store=store)
    dvol = dplan.empty_volume()
    dplan.filter(proj, filt)
    dplan.reconstruct(filt, None, dvol)
    torch.cuda.synchronize()
    e = max(1, nz // 8)
    regions = {"whole": (0, nz), "top_eighth": (nz - e, nz), "bottom_eighth": (0, e),
               "central_eighth": ((nz - e) // 2, (nz - e) // 2 + e)}
    tri = _rel_rmse_regions(torch, vol, dvol, regions)
    cone = _rel_rmse_regions(torch, cvol, dvol, regions)
    log("[bench] rel-RMSE vs direct FDK, triangle / cone: "
        + ", ".join(f"{a} {tri[a]:.4f} / {cone[a]:.4f}" for a in regions))
    del dvol, cvol
    updates_eq = n * n * nz * p
    paper_ms = per["bounds"] + per["decompose"] + per["reconstruct"]
    return {"ms_per_step": round(step_ms, 4),
            "gvups": round(updates_eq / (step_ms * 1e-3) / 1e9, 3),
            "gvups_paper_scope": round(updates_eq / (paper_ms * 1e-3) / 1e9, 3),
            "stage_ms": {a: round(b, 4) for a, b in per.items()},
            "rel_rmse_vs_direct_fdk": {"triangle": {a: round(b, 6) for a, b in tri.items()},
                                       "cone": {a: round(b, 6) for a, b in cone.items()}},
            "regions": {a: list(b) for a, b in regions.items()}}


def run_streamed(torch, res, slab):
    """The same reconstruction in the low-memory slab mode: projections and
    volume in page-locked host memory, bands of detector rows streamed through
    a device work buffer (PCIe included in the time).  Compared bit for bit
    with the in-memory result."""
    plan, vol = res["plan"], res["vol"]
    work_bytes = plan.streamed_bytes(slab)
    whole = 4 * plan.p * plan.n * plan.n + plan.filtered_bytes + plan.workspace_bytes + 4 * plan.nz * plan.n * plan.n
    direct = 4 * plan.p * plan.n * plan.n + plan.filtered_bytes + 4 * plan.nz * plan.n * plan.n
    log(f"[bench] streamed slab mode: work buffer {work_bytes / 1e9:.2f} GB "
        f"(in-memory FDK-OD {whole / 1e9:.1f} GB, direct FDK {direct / 1e9:.1f} GB)")
    host_proj = torch.empty(res["proj"].shape, dtype=torch.float32, pin_memory=True)
    host_proj.copy_(res["proj"])
    host_vol = torch.empty(vol.shape, dtype=torch.float32, pin_memory=True)
    work = torch.empty(work_bytes, dtype=torch.uint8, device="cuda:0")
    copy = torch.cuda.Stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.reconstruct_streamed(host_proj, host_vol, slab, work, copy_stream=copy)
    dt = time.perf_counter() - t0
    same = bool(torch.equal(host_vol[::97], vol[::97].cpu()))
    updates_eq = plan.n * plan.n * plan.nz * plan.p
    log(f"[bench] streamed slab mode: {dt:.3f} s including PCIe, sampled slices equal in-memory: {same}")
    del work, host_proj, host_vol
    return {"slab_slices": slab, "device_work_bytes": work_bytes, "in_memory_fdkod_bytes": whole,
            "direct_fdk_bytes": direct, "memory_reduction_vs_in_memory": round(whole / work_bytes, 2),
            "seconds_including_pcie": round(dt, 4),
            "gvups_including_pcie": round(updates_eq / dt / 1e9, 3),
            "bitwise_equal_sampled_slices": same}


def batch_volumes(bw, pkg):
    """The batched workload's volumes: sizes drawn with the workload's seed,
    s per volume from the cost model (eq. (8) over the exact counts, with the
    MI355X cost constants)."""
    import numpy as np
    rng = np.random.default_rng(bw.seed)
    sizes = rng.choice(np.array(bw.sizes), bw.count)
    out = []
    for n in sizes:
        n, p, r = int(n), int(round(bw.p_per_n * n)), float(bw.r_per_n * n)
        s, _ = pkg.choose_s(n, p, r, s_max=bw.s_max, store="bf16")
        out.append(dict(n=n, p=p, r=r, s=s))
    return out


def run_batch(torch, pkg, bw, steps):
    """Time the batched workload: one captured hipGraph replay per step, after
    the autotuner; and, for comparison, the same volumes one plan at a time."""
    from synth import phantom
    vols = batch_volumes(bw, pkg)
    log(f"[bench] batch {bw.name}: {len(vols)} volumes, sizes {sorted(v['n'] for v in vols)}")
    b = pkg.Batch(vols, store="bf16")
    projs = []
    for i, v in enumerate(vols):
        ell = phantom.random_ellipsoids(bw.ellipsoids, 400 + i)
        projs.append(phantom.project(ell, v["n"], v["p"], v["r"], device="cuda:0").contiguous())
    filts = [pl.empty_filtered() for pl in b.plans]
    wss = [pl.empty_workspace() if pl.s > 0 else None for pl in b.plans]
    outs = [pl.empty_volume() for pl in b.plans]
    b.bind(projs, filts, wss, outs)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        tuning = b.tune(st)
        b.capture(st)
        b.replay(st)
        st.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(steps):
            b.replay(st)
        e1.record(st)
        st.synchronize()
        graph_ms = e0.elapsed_time(e1) / steps
        # one plan after another, eager launches, same kernels per volume
        def sequential():
            for pl, pr, f, w, o in zip(b.plans, projs, filts, wss, outs):
                pl.bounds(st)
                pl.filter(pr, f, st)
                pl.decompose(f, w, st)
                pl.reconstruct(f, w, o, st)
        sequential()
        e0.record(st)
        sequential()
        e1.record(st)
        st.synchronize()
        seq_ms = e0.elapsed_time(e1)
    info = b.info()
    b.close()
    return {
        "workload": bw.name, "volumes": len(vols), "store": "bf16",
        "sizes": {str(n): sum(1 for v in vols if v["n"] == n) for n in bw.sizes},
        "s_by_size": {str(v["n"]): v["s"] for v in vols},
        "s_rule": "cost model (eq. (8) over the exact counts), MI355X cost constants",
        "updates_eq": info["updates_eq"], "work_items": info["items"],
        "persistent_blocks": info["blocks"], "tuning": {k: (round(x, 4) if isinstance(x, float) else x)
                                                         for k, x in tuning.items()},
        "ms_per_run_graph": round(graph_ms, 4),
        "gvups": round(info["updates_eq"] / (graph_ms * 1e-3) / 1e9, 3),
        "ms_one_plan_at_a_time": round(seq_ms, 4),
        "speedup_vs_one_plan_at_a_time": round(seq_ms / graph_ms, 3),
    }


def profiled(kernel, wl, s, k, store):
    """The committed rocprofv3 summary record of ``kernel``
    (profiles/hbm_traffic.json), or None when the kernel's source or the
    workload differs from the one that was profiled."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "hbm_traffic.json")) as f:
            rec = json.load(f)[kernel]
        with open(os.path.join(ROOT, "paper_1708_07515_amd", "csrc", rec["source"]), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, KeyError, ValueError):
        return None
    if sha != rec["source_sha256"] or (rec["workload"], rec["s"], rec["k"], rec["store"]) != (wl.name, s, k, store):
        return None
    return rec


def measured_traffic(kernel, wl, s, k, store):
    """HBM bytes per launch of ``kernel`` (FETCH_SIZE + WRITE_SIZE, scaled by
    the copy-kernel calibration) from the committed counter summary."""
    rec = profiled(kernel, wl, s, k, store)
    return None if rec is None else rec["read_bytes"] + rec["write_bytes"]


def measured_counter(kernel, wl, s, k, store, key):
    """A derived counter figure (e.g. VALU instructions per work unit) from
    the committed counter summary."""
    rec = profiled(kernel, wl, s, k, store)
    return None if rec is None else rec.get(key)


def kernel_rooflines(wl, s, k, store, res):
    """Per-kernel rooflines of one FDK-OD step from the stage times (HIP events
    on the launch stream, averaged over the timed steps) and the algorithmic
    work of each stage: the ramp filter and the decimation against HBM (each
    input read once, each output written once), the backprojection against
    the FP32 VALU (8 flops per update) with its LDS and HBM rates beside."""
    plan, per = res["plan"], res["per"]
    n, p, nz = wl.n, wl.p, wl.nzv
    bs = {"f32": 4, "f16": 2, "bf16": 2}[store]
    ws_bytes = plan.workspace_bytes
    vol_bytes = 4 * n * n * nz

    def hbm(kernel, name, nbytes, what):
        ms = per[name]
        gbs = nbytes / (ms * 1e-3) / 1e9
        return {"kernel": kernel, "bound": "hbm", "avg_ms": round(ms, 4), "algorithmic_bytes": nbytes,
                "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes": what,
                "traffic": measured_traffic(kernel, wl, s, k, store)}

    out = {
        "filter": hbm("k_filter4096" if plan.info.fft_len == 4096 else "k_filter", "filter", n * n * p * (4 + bs),
                      "projections read once (FP32) + filtered rows written once (store type)"),
        "decompose": hbm("k_decimate_staged" if plan.get_tuning()["decim_chunks"] == 0 else "k_decimate",
                         "decompose", n * n * p * bs + ws_bytes,
                         "filtered rows read once + decimated sub-sinograms written once"),
    }
    ms = per["reconstruct"]
    ups = plan.updates / (ms * 1e-3)
    tflops = FLOPS_PER_UPDATE * ups / 1e12
    out["reconstruct"] = {
        "kernel": "k_backproject", "bound": "alu", "avg_ms": round(ms, 4), "updates": plan.updates,
        "updates_per_s": round(ups, 1), "flops_per_update": FLOPS_PER_UPDATE,
        "achieved": round(tflops, 3), "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": round(tflops / VALU_PEAK_TFLOPS, 4),
        "frac_of_packed_peak": round(tflops / VALU_PACKED_PEAK_TFLOPS, 4),
        "lds": {"bytes_per_update": LDS_BYTES_PER_UPDATE,
                "achieved": round(LDS_BYTES_PER_UPDATE * ups / 1e9, 1), "peak": round(LDS_PEAK_GBS, 1),
                "unit": "GB/s", "frac": round(LDS_BYTES_PER_UPDATE * ups / 1e9 / LDS_PEAK_GBS, 4)},
        "hbm": {"algorithmic_bytes": ws_bytes + vol_bytes,
                "achieved": round((ws_bytes + vol_bytes) / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "bytes": "decimated sub-sinograms read once + volume written once"},
        "traffic": measured_traffic("k_backproject", wl, s, k, store),
    }
    # the backprojection's VALU instructions per update (all of them: the
    # inner loop, the per-angle set-up and the staging) from the committed
    # counter summary, when it was taken on this kernel and workload
    vipu = measured_counter("k_backproject", wl, s, k, store, "valu_instr_per_update")
    out["reconstruct"]["valu_instr_per_update"] = vipu
    # the rate at which those instructions issue (64-lane instructions per
    # second) against the issue limit of one per compute unit per cycle:
    # the kernel's bound once the instructions per update are fixed
    if vipu is not None:
        rate = vipu * ups / 64.0
        out["reconstruct"]["valu_issue"] = {
            "achieved": round(rate / 1e9, 1), "peak": round(VALU_ISSUE_PEAK / 1e9, 1),
            "unit": "G wave-instructions/s", "frac": round(rate / VALU_ISSUE_PEAK, 4),
            "instructions": "counter-measured VALU instructions per update (profiles/) x the live update rate"}
    return out


def host_description():
    """CPU model, the cores this process may run on, and the BLAS pools."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        blas = [{"api": i.get("internal_api"), "threads": i.get("num_threads")} for i in threadpool_info()]
    except Exception:           # threadpoolctl missing: report nothing
        blas = []
    return {"cpu_model": model, "affinity_cores": len(os.sched_getaffinity(0)), "blas_pools": blas}


# State the oracle's worker processes read: set before the pool forks, so the
# projections are shared with the children (copy on write), never pickled.
_ORACLE = {}


def _oracle_task(task):
    from threadpoolctl import threadpool_limits
    from oracle import fdk as ofdk, fdkod as ofdkod
    c = _ORACLE
    kind, what = task
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        if kind == "slice":
            if c["s"] == 0:
                ref = ofdk.fdk(c["proj"], c["r"], slices=[what], nz=c["nz"])[0]
            else:
                ref = ofdkod.fdkod(c["proj"], c["r"], c["s"], c["k"], slices=[what], nz=c["nz"])[0]
        else:
            ref = ofdkod.fdkod_points(c["proj"], c["r"], c["s"], c["k"], what, nz=c["nz"])
        return ref, time.perf_counter() - t0


def voxel_clusters(n, nz):
    """4 x 4 (x, y) patches on two slices at the top slice (centre), the bottom
    slice (an edge), the centre slice (a corner) and a third of the way up:
    where the cone angle is largest and where the squares meet the border."""
    import numpy as np
    groups = []
    for (l, j, i) in [(0, n // 2 - 2, n // 2 - 2), (nz - 1, 3, n - 7), (nz // 2, n - 5, 2),
                      (nz // 3, n // 4, 3 * n // 4)]:
        g = [(min(l + dl, nz - 1), j + dj, i + di) for dl in (0, 1) for dj in range(4) for di in range(4)]
        groups.append(np.array(g))
    return groups


def cpu_baseline(proj_cpu, wl, s, k, store, gpu_vol, workers):
    """The FP64 oracle timed on the host's cores (one worker process per core,
    one thread each): each worker reconstructs one slice near the centre of
    the volume (the rows eq. (9) maps them to are few, so the time is the
    oracle's decomposition and backprojection), while four more workers
    compute voxel clusters at the top and bottom slices for the parity
    record.  The GPU result is compared with both."""
    import multiprocessing as mp
    import numpy as np
    from oracle import metrics

    host = host_description()
    cores = max(1, min(workers or host["affinity_cores"], CPU_WORKERS_MAX, host["affinity_cores"]))
    groups = voxel_clusters(wl.n, wl.nzv)
    nsl = max(1, cores - len(groups)) if cores > len(groups) else cores
    sl = sorted(set(int(x) for x in np.round(np.linspace(0.45 * (wl.nzv - 1), 0.55 * (wl.nzv - 1), nsl))))
    _ORACLE.update(proj=proj_cpu.numpy(), r=wl.r, s=s, k=k, nz=wl.nzv)
    tasks = [("slice", l) for l in sl] + [("points", g) for g in groups]
    log(f"[bench] CPU oracle: {len(sl)} slices and {len(groups)} voxel clusters on {cores} worker processes")
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(processes=cores) as pool:
        out = pool.map(_oracle_task, tasks, chunksize=1)
    wall = time.perf_counter() - t0
    _ORACLE.clear()
    refs = [o[0] for o in out]
    times = [o[1] for o in out]
    slice_t = max(times[:len(sl)])
    gpu_sl = gpu_vol[sl].cpu().double().numpy()
    ref_sl = np.stack(refs[:len(sl)])
    idx = np.concatenate(groups)
    gpu_pts = gpu_vol[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().double().numpy()
    ref_pts = np.concatenate(refs[len(sl):])
    err_sl = metrics.rel_rmse(gpu_sl, ref_sl)
    mx_sl, mxr_sl = metrics.max_abs(gpu_sl, ref_sl)
    err_pt = metrics.rel_rmse(gpu_pts, ref_pts)
    mx_pt, mxr_pt = metrics.max_abs(gpu_pts, ref_pts)
    updates = wl.n * wl.n * len(sl) * wl.p
    gv = updates / slice_t / 1e9
    conc = min(len(sl), cores)
    log(f"[bench] CPU oracle: {len(sl)} slices in {slice_t:.1f} s ({gv:.3f} GVUPS on {conc} cores), "
        f"all tasks {wall:.1f} s; parity slices {err_sl:.2e}, clusters {err_pt:.2e}")
    cpu = dict(value=round(gv, 5), unit="GVUPS", cores=conc, kind="oracle",
               sample=f"{len(sl)} slices of {wl.name} near the centre (l = {sl[0]}..{sl[-1]}), s={s}, k={k}, "
                      f"FP64 NumPy, one slice per worker process, one thread each; "
                      f"the longest took {slice_t:.1f} s",
               seconds=round(slice_t, 2), threads_per_worker=1, host=host)
    parity = dict(bar=1e-4 if store == "f32" else 2e-3, store=store, rel_rmse=err_sl, max_abs=mx_sl, max_abs_rel=mxr_sl, slices=sl,
                  clusters=dict(rel_rmse=err_pt, max_abs=mx_pt, max_abs_rel=mxr_pt, voxels=int(len(idx)),
                                where="4x4x2 voxel patches at the top slice (centre), the bottom slice (edge), "
                                      "the centre slice (corner) and a third of the way up"),
                  oracle="FP64 FDK-OD of the same (s, k), plain storage")
    return cpu, parity


def run_variant(torch, pkg, wl, s, k, store, base, steps, direct_ms):
    """Time FDK-OD steps of another (s, k, store) on the main scan; the direct
    FDK time of the main run serves as the reference (the same kernel at s = 0)."""
    proj = base["proj"]
    plan = pkg.Plan(wl.n, wl.p, wl.r, s=s, skip=k, nz=wl.nzv, store=store)
    same = {"f32": 0, "f16": 1, "bf16": 2}[store] == base["plan"].store
    filt = base["filt"] if same else plan.empty_filtered()
    ws = plan.empty_workspace()
    vol = base["vol"]
    stages = [("bounds", lambda: plan.bounds()),
              ("filter", lambda: plan.filter(proj, filt)),
              ("decompose", lambda: plan.decompose(filt, ws)),
              ("reconstruct", lambda: plan.reconstruct(filt, ws, vol))]
    per, step_ms, _ = timed_steps(torch, stages, steps, 1)
    log(f"[bench] variant s={s} k={k} store={store}, per stage (ms): "
        + ", ".join(f"{a}={b:.3f}" for a, b in per.items()))
    updates_eq = wl.n * wl.n * wl.nzv * wl.p
    paper_ms = per["bounds"] + per["decompose"] + per["reconstruct"]
    out = {"s": s, "k": k, "store": store, "p_dec": plan.p_dec, "ms_per_step": round(step_ms, 4),
           "gvups": round(updates_eq / (step_ms * 1e-3) / 1e9, 3),
           "gvups_paper_scope": round(updates_eq / (paper_ms * 1e-3) / 1e9, 3),
           "stage_ms": {a: round(b, 4) for a, b in per.items()},
           "speedup_vs_direct": None if direct_ms is None else round(direct_ms["step"] / step_ms, 3),
           "speedup_vs_direct_paper_scope": None if direct_ms is None else
               round(direct_ms["reconstruct"] / paper_ms, 3),
           "steps": steps}
    del ws, filt
    plan.close()
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library has "
              "no multi-GPU path (it would shard the volume by z-slab across GPUs)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1708_07515_amd as pkg
    from synth import configs

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 1 GiB read + 1 GiB written")
        del a, b
    copy_peak = measure_copy_peak(torch)

    wl = configs.ALL[args.workload]
    s = args.s if args.s is not None else max(wl.s)
    k = args.skip if args.skip is not None else wl.k
    store = args.store or wl.store[0]
    res = run_workload(torch, pkg, wl, s, k, store, args.steps, args.warmup,
                       direct=not args.no_direct)
    main_sum = summarise(wl, s, k, store, res)
    kernels = kernel_rooflines(wl, s, k, store, res)
    bp = kernels["reconstruct"]
    roofline = dict(bound="alu", kernel="k_backproject", achieved=bp["achieved"], peak=VALU_PEAK_TFLOPS,
                    unit="TFLOP/s", frac=bp["frac"], traffic=bp["traffic"],
                    flops_per_update=FLOPS_PER_UPDATE, updates=bp["updates"], avg_ms=bp["avg_ms"])
    direct_ms = None
    if res["direct"] is not None:
        direct_ms = {"step": res["direct"]["ms_per_step"], "reconstruct": res["direct"]["stage_ms"]["reconstruct"]}

    cpu = parity = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on a bounded sample")
        cpu, parity = cpu_baseline(res["proj"].cpu(), wl, s, k, store, res["vol"], args.cpu_workers)

    variants = None
    if not args.no_variants and s > 0:
        variants = []
        alt_store = "bf16" if store == "f32" else "f32"
        for (vs, vk, vst) in [(s, k, alt_store), (s + 1, k, store), (s, k + 1, store), (s + 1, k + 1, store)]:
            if (1 << vs) > wl.n:
                continue
            variants.append(run_variant(torch, pkg, wl, vs, vk, vst, res, max(1, min(args.steps, 3)), direct_ms))
        # the main volume again (parity and the extensions below compare with it)
        res["plan"].decompose(res["filt"], res["ws"])
        res["plan"].reconstruct(res["filt"], res["ws"], res["vol"])
        torch.cuda.synchronize()

    learned = None if args.no_learned else run_learned(torch, pkg, wl, res, max(1, min(args.steps, 5)))
    cone = None if args.no_cone else run_cone(torch, pkg, wl, s, k, store, res, max(1, min(args.steps, 3)))
    streamed = None if args.no_streamed else run_streamed(torch, res, args.slab)
    del res
    torch.cuda.empty_cache()

    small = None
    if not args.no_small and wl.name != "cone512_p360":
        sw = configs.C2
        sres = run_workload(torch, pkg, sw, max(sw.s), sw.k, sw.store[0], max(1, min(args.steps, 10)), 2,
                            direct=not args.no_direct)
        small = summarise(sw, max(sw.s), sw.k, sw.store[0], sres)
        small["kernels"] = kernel_rooflines(sw, max(sw.s), sw.k, sw.store[0], sres)
        del sres
        torch.cuda.empty_cache()

    batch = batch_small = None
    if not args.no_batch:
        batch = run_batch(torch, pkg, configs.C4, 3)
        log(f"[bench] batch: {batch['ms_per_run_graph']} ms per graph replay, "
            f"{batch['ms_one_plan_at_a_time']} ms one plan at a time")
        torch.cuda.empty_cache()
        batch_small = run_batch(torch, pkg, configs.C4S, 10)
        log(f"[bench] small batch: {batch_small['ms_per_run_graph']} ms per graph replay, "
            f"{batch_small['ms_one_plan_at_a_time']} ms one plan at a time")
        torch.cuda.empty_cache()

    out = {
        "metric": METRIC,
        "value": main_sum["gvups"],
        "unit": "GVUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_sum["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if store == "f32" else f"{store}-storage/f32",
        "data": f"synthetic: seeded {wl.ellipsoids}-ellipsoid phantom"
                + (f", Poisson noise {wl.photons:g} photons" if wl.photons else ""),
        "config": {"workload": wl.name, "n": wl.n, "nz": wl.nzv, "p": wl.p, "r": wl.r,
                   "s": s, "k": k, "p_dec": main_sum["p_dec"], "store": store},
        "stage_ms": main_sum["stage_ms"],
        "gvups_paper_scope": main_sum["gvups_paper_scope"],
        "gvups_exec_reconstruct": main_sum["gvups_exec_reconstruct"],
        "direct_fdk": main_sum["direct_fdk"],
        "speedup_vs_direct": main_sum["speedup_vs_direct"],
        "speedup_vs_direct_paper_scope": main_sum["speedup_vs_direct_paper_scope"],
        "parity": parity,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "variants": variants,
        "learned_decimation": learned,
        "cone_decimation": cone,
        "streamed": streamed,
        "small_workload": small,
        "batch_workload": batch,
        "batch_small_workload": batch_small,
        "copy_peak": copy_peak,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
