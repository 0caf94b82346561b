"""GPU tests of the batched form (grouped decimation + persistent
backprojection over uneven volumes, hipGraph capture) and of the autotuner."""

import os

import numpy as np
import pytest
import torch

import paper_1708_07515_amd as pkg
from gpu_common import DEV, gpu_reconstruct, log, oracle_reconstruct, report, require_gpu, scan

pytestmark = pytest.mark.gpu

# uneven volumes: sizes, P = round(1.4 N), R = 4 N, s per size, a short volume,
# a skipped stage and a direct (s = 0) volume
VOLS = [dict(n=32, p=45, r=128.0, s=1), dict(n=48, p=67, r=192.0, s=2, nz=20),
        dict(n=40, p=56, r=160.0, s=2, skip=1), dict(n=64, p=90, r=256.0, s=3),
        dict(n=24, p=34, r=96.0, s=0)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def scans():
    return [scan(v["n"], v["p"], v["r"], 6, 40 + i) for i, v in enumerate(VOLS)]


def make_batch(store="f32"):
    b = pkg.Batch(VOLS, store=store)
    projs = [p.to(DEV) for p in scans()]
    filts = [pl.empty_filtered() for pl in b.plans]
    wss = [pl.empty_workspace() if pl.s > 0 else None for pl in b.plans]
    vols = [pl.empty_volume() for pl in b.plans]
    b.bind(projs, filts, wss, vols)
    return b, vols


def test_batch_matches_oracle_and_single_plans():
    b, vols = make_batch()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        b.run(st)
    st.synchronize()
    log(f"batch info {b.info()}")
    for i, (v, proj) in enumerate(zip(VOLS, scans())):
        got = vols[i].double().cpu().numpy()
        ref = oracle_reconstruct(proj, v["r"], v.get("s", 0), v.get("skip", 0), nz=v.get("nz", v["n"]))
        err, _ = report(f"batch volume {i} {v}", got, ref, bar=1e-4)
        assert err <= 1e-4
        single, _ = gpu_reconstruct(proj, v["n"], v["p"], v["r"], s=v.get("s", 0),
                                    skip=v.get("skip", 0), nz=v.get("nz", 0))
        assert np.max(np.abs(got - single)) <= 1e-5 * np.max(np.abs(single))
    b.close()


def test_batch_graph_replays_match_eager():
    b, vols = make_batch()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        b.run(st)
    st.synchronize()
    eager = [v.clone() for v in vols]
    with torch.cuda.stream(st):
        b.capture(st)
    st.synchronize()
    for rep in range(3):
        for v in vols:
            v.zero_()                       # eager work between replays
        junk = torch.randn(1 << 20, device=DEV).sum()
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            b.replay(st)
        st.synchronize()
        for i, v in enumerate(vols):
            assert torch.equal(v, eager[i]), f"replay {rep} volume {i} differs"
        assert torch.isfinite(junk)
    b.close()


def test_batch_bf16_storage():
    b, vols = make_batch("bf16")
    b.run()
    torch.cuda.synchronize()
    for i, (v, proj) in enumerate(zip(VOLS, scans())):
        ref = oracle_reconstruct(proj, v["r"], v.get("s", 0), v.get("skip", 0), nz=v.get("nz", v["n"]))
        err, _ = report(f"batch bf16 volume {i}", vols[i].double().cpu().numpy(), ref, bar=2e-3)
        assert err <= 2e-3
    b.close()


def test_batch_tune_keeps_results():
    b, vols = make_batch()
    choice = b.tune()
    log(f"batch tuning {choice}")
    assert choice["z_run"] in (16, 32) and choice["decim_chunks"] in (1, 2, 4, 8)
    b.run()
    torch.cuda.synchronize()
    for i, (v, proj) in enumerate(zip(VOLS, scans())):
        ref = oracle_reconstruct(proj, v["r"], v.get("s", 0), v.get("skip", 0), nz=v.get("nz", v["n"]))
        err, _ = report(f"tuned batch volume {i}", vols[i].double().cpu().numpy(), ref, bar=1e-4)
        assert err <= 1e-4
    b.close()


def test_plan_tune_variants_and_cache(tmp_path, monkeypatch):
    n, p, r, s = 64, 90, 512.0, 2
    proj = scan(n, p, r, 10, 1)
    ref = oracle_reconstruct(proj, r, s)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("FDKOD_TUNE_CACHE", str(cache))
    with pkg.Plan(n, p, r, s=s) as plan:
        filt, ws, vol = plan.empty_filtered(), plan.empty_workspace(), plan.empty_volume()
        plan.filter(proj.to(DEV), filt)
        # every variant that holds the geometry gives the oracle's result
        outs = []
        for zr in (16, 32):
            for tw in (32, 64):
                for th in (48, 64):
                    for g in (1, 2, 4):
                        try:
                            plan.set_tuning(z_run=zr, tile_w=tw, tile_h=th, angles_per_stage=g)
                        except pkg.FdkodError as e:
                            assert e.code == "E_UNSUPPORTED"
                            continue
                        plan.backproject(filt, vol, ws)
                        torch.cuda.synchronize()
                        outs.append(((zr, tw, th, g), vol.double().cpu().numpy()))
        assert len(outs) >= 6
        for key, out in outs:
            err, _ = report(f"variant {key}", out, ref, bar=1e-4)
            assert err <= 1e-4
        with pytest.raises(pkg.FdkodError) as ei:
            plan.set_tuning(z_run=8)
        assert ei.value.code == "E_UNSUPPORTED"
        choice = plan.tune(filt, ws, vol)
        log(f"plan tuning {choice}")
        plan.backproject(filt, vol, ws)
        torch.cuda.synchronize()
        err, _ = report("tuned plan", vol.double().cpu().numpy(), ref, bar=1e-4)
        assert err <= 1e-4
    assert cache.exists() and cache.read_text().strip()
    with pkg.Plan(n, p, r, s=s) as again:
        t = again.get_tuning()
        for k in ("z_run", "tile_w", "tile_h", "angles_per_stage", "decim_chunks"):
            assert t[k] == choice[k]


@pytest.mark.parametrize("name", ["batch32_mixed", "batch256_small"])
def test_batched_workload_matches_oracle_on_sampled_slices(name):
    """The benchmark's batched workloads themselves (32 volumes, N in {128,
    ..., 512}; 256 volumes, N in {32, 48, 64}; P = 1.4 N, R = 4 N, s from
    the cost model, BF16 storage), tuned, captured and replayed as the
    benchmark times them: slices of every volume (top, bottom, centre, a
    third of the way up; for the small volumes the centre and the slice
    through the largest ellipsoid) against the FP64 oracle, one oracle
    slice per host worker."""
    import time

    import bench
    from gpu_common import oracle_slices_many
    from synth import configs, phantom
    bw = {"batch32_mixed": configs.C4, "batch256_small": configs.C4S}[name]
    vols = bench.batch_volumes(bw, pkg)
    assert len(vols) == bw.count
    b = pkg.Batch(vols, store="bf16")
    ells = [phantom.random_ellipsoids(bw.ellipsoids, 400 + i) for i in range(len(vols))]
    projs = [phantom.project(e, v["n"], v["p"], v["r"], device=DEV).contiguous() for e, v in zip(ells, vols)]
    filts = [pl.empty_filtered() for pl in b.plans]
    wss = [pl.empty_workspace() if pl.s > 0 else None for pl in b.plans]
    outs = [pl.empty_volume() for pl in b.plans]
    b.bind(projs, filts, wss, outs)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        b.tune(st)
        b.capture(st)
        b.replay(st)
    st.synchronize()
    if bw.count > 64:
        # a small phantom of few ellipsoids can leave fixed slices nearly
        # empty, where the relative error is that of the rounding of the
        # other slices' projections: take the centre slice and the slice
        # through the centre of the phantom's largest ellipsoid
        def through_largest(e, n):
            big = int(np.argmax(np.abs(e.density) * np.prod(e.axes, axis=1)))
            return int(np.clip(round((n - 1) / 2 + e.centres[big, 2] * n / 2), 0, n - 1))
        slices = {i: sorted({v["n"] // 2, through_largest(ells[i], v["n"])}) for i, v in enumerate(vols)}
    else:
        slices = {i: sorted({0, v["n"] - 1, v["n"] // 2, v["n"] // 3}) for i, v in enumerate(vols)}
    scans = [dict(proj=pr.cpu(), r=v["r"], s=v["s"], k=0, nz=v["n"]) for pr, v in zip(projs, vols)]
    tasks = [(i, l) for i in range(len(vols)) for l in slices[i]]
    t0 = time.time()
    refs = oracle_slices_many(scans, tasks)
    log(f"oracle: {len(tasks)} slices of {len(vols)} volumes in {time.time() - t0:.1f} s")
    pos = 0
    worst = 0.0
    for i, v in enumerate(vols):
        ref = np.stack(refs[pos:pos + len(slices[i])])
        pos += len(slices[i])
        got = outs[i][slices[i]].double().cpu().numpy()
        err, _ = report(f"{name} volume {i} n={v['n']} s={v['s']} slices {slices[i]}", got, ref, bar=2e-3)
        assert err <= 2e-3
        worst = max(worst, err)
    log(f"{name}: worst rel-RMSE {worst:.2e} over {len(vols)} volumes")
    b.close()
