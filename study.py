"""Quality and cost study of FDK-OD on one GPU, after the paper's own
evaluations (Sec. 2.2 cost model, Sec. 4 quality), on synthetic phantoms:

1. s x k sweep on a noise-free random-ellipsoid phantom (standing in for the
   Shepp-Logan-3D phantom, whose parameter table the paper does not give):
   rel-RMSE against direct FDK, and the voxel-wise ratio FDK-OD / FDK on the
   uniform interiors of the objects (the paper's ratio maps, reduced to their
   mean and spread where the ratio is meaningful: away from borders and from
   near-zero densities).
2. Slanted-edge resolution (Sec. 4) on an analytic box phantom rotated by 5
   degrees: the edge spread function of one face in the central slice,
   binned at a quarter voxel by distance to the known face, its derivative
   (tapered beyond half the reach) and Fourier magnitude; MTF50, MTF10 and the 10-90 % edge
   width for direct FDK and every (s, k, decimation).
3. Time split vs s (Sec. 2.2): decomposition and reconstruction kernel times
   for s = 1..5 at several N, and the constants of the cost model
   Total = C1 N^3 P / 2^s + C2 N^2 P 2^s fitted by least squares (one
   constant per term), with the optimum 2^s = sqrt(C1 N / C2) against the
   measured best s.
4. The non-learned quality knobs (windowed-sinc decimation, cubic shift)
   against the learned decimation filter on the same held-out phantoms (the
   learned filter trained as in its GPU test), and the decomposition cost of
   each at 512^3, P = 360, s = 3.

Usage: python study.py [--quick] > study.json (progress on stderr).  Every
reconstruction runs in the HIP library; the analysis is plain NumPy.
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ analysis

def face_coordinates(n, centre, angle, half):
    """Signed distance to the face x' = +half[0] of a box rotated by ``angle``
    about z (positive outside) and the coordinate along that face, for every
    pixel of an N x N slice indexed [j (y), i (x)]; centre and half in voxels."""
    c = (n - 1) / 2.0
    j, i = np.mgrid[0:n, 0:n].astype(np.float64)
    x, y = i - c - centre[0], j - c - centre[1]
    ca, sa = math.cos(angle), math.sin(angle)
    lx = x * ca + y * sa
    ly = -x * sa + y * ca
    return lx - half[0], ly


def edge_spread(img, dist, along, half_len, reach=20.0, bin_w=0.25):
    """Edge spread function: pixel values averaged in bins of ``bin_w`` voxels
    of distance to the face, over pixels within ``reach`` of it and within
    ``half_len`` of the face's middle.  Returns (bin centres, ESF)."""
    sel = (np.abs(dist) < reach) & (np.abs(along) <= half_len)
    nb = int(round(2 * reach / bin_w))
    b = np.clip(np.floor((dist[sel] + reach) / bin_w).astype(np.int64), 0, nb - 1)
    sums = np.bincount(b, weights=img[sel], minlength=nb)
    cnt = np.bincount(b, minlength=nb)
    if np.any(cnt == 0):
        raise ValueError("empty distance bin: the face is not slanted enough or too short")
    centres = -reach + (np.arange(nb) + 0.5) * bin_w
    return centres, sums / cnt


def mtf_from_esf(esf, bin_w=0.25):
    """MTF (frequencies in cycles per voxel, magnitude normalised at 0) of an
    edge spread function sampled every ``bin_w`` voxels, centred on the edge.
    The line spread function is kept whole within half the reach and tapered
    by a raised cosine beyond it (a full Hann window would narrow it)."""
    lsf = np.gradient(esf, bin_w)
    u = np.abs(np.arange(len(lsf)) + 0.5 - len(lsf) / 2.0) / (len(lsf) / 2.0)
    lsf = lsf * np.where(u <= 0.5, 1.0, 0.5 * (1.0 + np.cos(2.0 * np.pi * (u - 0.5))))
    spec = np.abs(np.fft.rfft(lsf))
    return np.fft.rfftfreq(len(lsf), d=bin_w), spec / spec[0]


def first_crossing(f, m, level):
    """Frequency where m first falls below ``level`` (linear interpolation)."""
    k = np.nonzero(m < level)[0]
    if len(k) == 0:
        return None
    k = int(k[0])
    if k == 0:
        return float(f[0])
    t = (m[k - 1] - level) / (m[k - 1] - m[k])
    return float(f[k - 1] + t * (f[k] - f[k - 1]))


def edge_width(centres, esf, reach_frac=0.5):
    """10-90 % rise distance of a falling edge (inside level at negative
    distance, outside level at positive distance)."""
    far = np.abs(centres) >= reach_frac * np.abs(centres).max()
    hi = esf[far & (centres < 0)].mean()
    lo = esf[far & (centres > 0)].mean()
    t = (esf - lo) / (hi - lo)
    def cross(level):
        k = np.nonzero(t < level)[0]
        k = int(k[0])
        return centres[k - 1] + (t[k - 1] - level) / (t[k - 1] - t[k]) * (centres[k] - centres[k - 1])
    return float(cross(0.1) - cross(0.9))


def slanted_edge(img, centre, angle, half, reach=20.0, bin_w=0.25, along_frac=0.6):
    dist, along = face_coordinates(img.shape[0], centre, angle, half)
    d, esf = edge_spread(img, dist, along, along_frac * half[1], reach, bin_w)
    f, m = mtf_from_esf(esf, bin_w)
    return {"mtf50": first_crossing(f, m, 0.5), "mtf10": first_crossing(f, m, 0.1),
            "width_10_90": edge_width(d, esf)}


def interior_mask(ell, n, margin=3.0, min_density=0.2, step=2):
    """Voxels (every ``step``-th in each direction) whose true density is the
    same at +-margin voxels along x, y and z and at least ``min_density`` in
    magnitude.  Returns (slice tuple, boolean mask on that grid)."""
    from synth import phantom
    c = (n - 1) / 2.0
    g = np.arange(0, n, step, dtype=np.float64) - c
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    d0 = phantom.density(ell, n, n, x, y, z)
    same = np.abs(d0) >= min_density
    for dx, dy, dz in ((margin, 0, 0), (-margin, 0, 0), (0, margin, 0), (0, -margin, 0),
                       (0, 0, margin), (0, 0, -margin)):
        same &= phantom.density(ell, n, n, x + dx, y + dy, z + dz) == d0
    sl = (slice(0, n, step),) * 3
    return sl, same


def ratio_map(v, ref, n, grid=16, band=8):
    """The E4 picture in numbers: FDK-OD / direct FDK on the central slice,
    averaged over grid x grid blocks of voxels where direct FDK is at least a
    fifth of its largest magnitude (None elsewhere), and the two
    reconstructions along the central row, every n // 64 voxels, averaged
    over `band` rows."""
    mid = n // 2
    a, b = v[mid], ref[mid]
    keep = np.abs(b) >= 0.2 * np.abs(b).max()
    bs = n // grid
    out = []
    for i in range(grid):
        row = []
        for j in range(grid):
            blk = (slice(i * bs, (i + 1) * bs), slice(j * bs, (j + 1) * bs))
            kk = keep[blk]
            row.append(round(float((a[blk][kk] / b[blk][kk]).mean()), 4) if kk.sum() >= bs else None)
        out.append(row)
    step = max(n // 64, 1)
    rows = slice(mid - band // 2, mid + band // 2)
    prof_od = a[rows].mean(axis=0)[::step]
    prof_fdk = b[rows].mean(axis=0)[::step]
    return {"ratio_blocks": out, "block_voxels": bs,
            "profile_step": step, "profile_fdkod": [round(float(x), 5) for x in prof_od],
            "profile_fdk": [round(float(x), 5) for x in prof_fdk]}


def rel_rmse(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2) / np.mean(b ** 2)))


def fit_costs(rows):
    """Least-squares constants of Dec = C2 N^2 P 2^s and Rec = C1 N^3 P / 2^s
    (each a one-parameter fit through the origin)."""
    a1 = np.array([r["n"] ** 3 * r["p"] / 2 ** r["s"] for r in rows], dtype=np.float64)
    a2 = np.array([r["n"] ** 2 * r["p"] * 2 ** r["s"] for r in rows], dtype=np.float64)
    rec = np.array([r["reconstruct_ms"] for r in rows])
    dec = np.array([r["decompose_ms"] for r in rows])
    c1 = float(a1 @ rec / (a1 @ a1))
    c2 = float(a2 @ dec / (a2 @ a2))
    return c1, c2


# ----------------------------------------------------------------- GPU runs

def reconstruct(torch, pkg, proj, n, p, r, s, k=0, rows="detector", reps=0, **knobs):
    """Volume (device tensor) and, with reps > 0, the median decomposition and
    reconstruction kernel times (ms) over ``reps`` runs.  ``knobs``: decim,
    taps, interp of the plan."""
    with pkg.Plan(n, p, r, s=s, skip=k, rows=rows, **knobs) as plan:
        filt, ws, vol = plan.empty_filtered(), plan.empty_workspace(), plan.empty_volume()
        plan.filter(proj, filt)
        plan.decompose(filt, ws)
        plan.reconstruct(filt, ws, vol)
        times = None
        if reps:
            dec, rec = [], []
            for _ in range(reps):
                e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                e[0].record()
                plan.decompose(filt, ws)
                e[1].record()
                plan.reconstruct(filt, ws, vol)
                e[2].record()
                torch.cuda.synchronize()
                dec.append(e[0].elapsed_time(e[1]))
                rec.append(e[1].elapsed_time(e[2]))
            times = (float(np.median(dec)), float(np.median(rec)))
        torch.cuda.synchronize()
        del filt, ws
        return vol, times


def combos(smax):
    out = []
    for s in range(1, smax + 1):
        for k in range(0, min(2, s) + 1):
            for rows in ("detector", "cone"):
                out.append((s, k, rows))
    return out


def quality_sweep(torch, pkg, n, p, r, smax):
    from synth import phantom
    ell = phantom.random_ellipsoids(20, 11)
    proj = phantom.project(ell, n, p, r, device="cuda:0").contiguous()
    box_half_norm, box_angle = 0.6, math.radians(5.0)
    bx = phantom.box((0.0, 0.0, 0.0), (box_half_norm,) * 3, box_angle, 1.0)
    bproj = phantom.project(bx, n, p, r, device="cuda:0").contiguous()
    half_vox = (box_half_norm * n / 2.0,) * 2
    mid = n // 2
    log(f"[study] quality sweep N={n} P={p} R={r}: interior mask")
    sl, mask = interior_mask(ell, n)
    ref, _ = reconstruct(torch, pkg, proj, n, p, r, 0)
    ref_np = ref.cpu().double().numpy()
    ref_in = ref_np[sl][mask]
    bref, _ = reconstruct(torch, pkg, bproj, n, p, r, 0)
    edge_ref = slanted_edge(bref[mid].cpu().double().numpy(), (0.0, 0.0), box_angle, half_vox)
    log(f"[study] direct FDK edge: {edge_ref}")
    rows = []
    for s, k, rw in combos(smax):
        vol, _ = reconstruct(torch, pkg, proj, n, p, r, s, k, rw)
        v = vol.cpu().double().numpy()
        ratio = v[sl][mask] / ref_in
        bvol, _ = reconstruct(torch, pkg, bproj, n, p, r, s, k, rw)
        edge = slanted_edge(bvol[mid].cpu().double().numpy(), (0.0, 0.0), box_angle, half_vox)
        row = {"s": s, "k": k, "d": 2 ** (s - k), "rows": rw,
               "rel_rmse_vs_fdk": rel_rmse(v, ref_np),
               "interior_ratio_mean": float(ratio.mean()), "interior_ratio_std": float(ratio.std()),
               "interior_ratio_p01": float(np.percentile(ratio, 1)),
               "interior_ratio_p99": float(np.percentile(ratio, 99)), **edge,
               "e4_central_slice": ratio_map(v, ref_np, n)}
        log(f"[study] s={s} k={k} {rw} rows: rel-RMSE {row['rel_rmse_vs_fdk']:.4f}, interior ratio "
            f"{row['interior_ratio_mean']:.4f} +- {row['interior_ratio_std']:.4f}, MTF50 {edge['mtf50']:.3f} "
            f"MTF10 {edge['mtf10']:.3f}, 10-90 {edge['width_10_90']:.2f}")
        rows.append(row)
        del vol, bvol
    return {"n": n, "p": p, "r": r, "phantom": "20 random ellipsoids, seed 11, noise-free",
            "edge_phantom": f"box, half size {box_half_norm} (normalised), rotated 5 degrees, face x' = +half",
            "interior_voxels": int(mask.sum()), "fdk_edge": edge_ref, "rows": rows}


def time_split(torch, pkg, sizes, smax, reps):
    from synth import phantom
    out = []
    for n, p in sizes:
        r = 4.0 * n
        ell = phantom.random_ellipsoids(20, 3)
        proj = phantom.project(ell, n, p, r, device="cuda:0").contiguous()
        rows = []
        for s in range(1, smax + 1):
            _, (dec, rec) = reconstruct(torch, pkg, proj, n, p, r, s, 0, "detector", reps)
            rows.append({"n": n, "p": p, "s": s, "decompose_ms": dec, "reconstruct_ms": rec,
                         "total_ms": dec + rec})
            log(f"[study] N={n} P={p} s={s}: decompose {dec:.3f} ms, reconstruct {rec:.3f} ms")
        c1, c2 = fit_costs(rows)
        best = min(rows, key=lambda x: x["total_ms"])["s"]
        s_model = 0.5 * math.log2(c1 * n / c2)
        out.append({"n": n, "p": p, "r": r, "rows": rows, "c1_ms": c1, "c2_ms": c2,
                    "s_opt_model": s_model, "s_opt_measured": best})
        log(f"[study] N={n}: C1 {c1:.3e} ms, C2 {c2:.3e} ms, optimum s model {s_model:.2f}, measured {best}")
        del proj
        torch.cuda.empty_cache()
    return out


KNOBS = [("triangle", {}), ("sinc2", dict(decim="sinc", taps=2)), ("sinc4", dict(decim="sinc", taps=4)),
         ("sinc6", dict(decim="sinc", taps=6)), ("cubic", dict(interp="cubic")),
         ("sinc4+cubic", dict(decim="sinc", taps=4, interp="cubic")),
         ("sinc6+cubic", dict(decim="sinc", taps=6, interp="cubic"))]


def _filtered_scans(torch, pkg, direct, n, p, r, seeds):
    """Filtered projections and direct-FDK volumes of seeded phantoms."""
    from synth import phantom
    out = []
    for sd in seeds:
        proj = phantom.project(phantom.random_ellipsoids(8, sd), n, p, r, device="cuda:0").contiguous()
        filt = direct.empty_filtered()
        direct.filter(proj, filt)
        tgt = direct.empty_volume()
        direct.reconstruct(filt, None, tgt)
        out.append((filt, tgt))
    return out


def knobs_vs_learned(torch, pkg, steps=600, cost_reps=5):
    """Held-out error against direct FDK of every knob setting and of the
    trained learned filter (N = 96, N_z = 24, P = 128, R = 384, s = 2; 8
    training and 4 held-out phantoms of 8 ellipsoids), and the decomposition
    time of each at 512^3, P = 360, R = 2048, s = 3, FP32."""
    n, nz, p, r, s = 96, 24, 128, 384.0, 2
    direct = pkg.Plan(n, p, r, s=0, nz=nz)
    train = _filtered_scans(torch, pkg, direct, n, p, r, range(100, 108))
    held = _filtered_scans(torch, pkg, direct, n, p, r, range(200, 204))

    def rel(a, b):
        return float(torch.linalg.norm((a - b).double()) / torch.linalg.norm(b.double()))

    err = {}
    for name, knobs in KNOBS:
        with pkg.Plan(n, p, r, s=s, nz=nz, **knobs) as plan:
            ws, vol = plan.empty_workspace(), plan.empty_volume()
            e = []
            for filt, tgt in held:
                plan.decompose(filt, ws)
                plan.reconstruct(filt, ws, vol)
                e.append(rel(vol, tgt))
            err[name] = float(np.mean(e))
    with pkg.Plan(n, p, r, s=s, nz=nz) as plan:
        ws, vol = plan.empty_workspace(), plan.empty_volume()
        resid = torch.empty_like(vol)
        dws = torch.empty(plan.workspace_elems, dtype=torch.float32, device="cuda:0")
        net = pkg.LearnedDecimation("cuda:0", seed=0, lr=3e-3)
        for it in range(steps):
            filt, tgt = train[it % len(train)]
            net.train_step(plan, filt, ws, vol, tgt, resid, dws)
        e = []
        for filt, tgt in held:
            net.forward(plan, filt, ws, vol)
            e.append(rel(vol, tgt))
        err["learned"] = float(np.mean(e))
    direct.close()
    log("[study] held-out rel-RMSE vs direct FDK: " + ", ".join(f"{a} {b:.4f}" for a, b in err.items()))

    from synth import phantom
    n2, p2, r2, s2 = 512, 360, 2048.0, 3
    proj = phantom.project(phantom.random_ellipsoids(20, 2), n2, p2, r2, device="cuda:0").contiguous()
    cost = {}

    def median_ms(fn):
        fn()
        t = []
        for _ in range(cost_reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            t.append(e0.elapsed_time(e1))
        return float(np.median(t))

    for name, knobs in KNOBS + [("learned", None)]:
        with pkg.Plan(n2, p2, r2, s=s2, **(knobs or {})) as plan:
            filt, ws = plan.empty_filtered(), plan.empty_workspace()
            plan.filter(proj, filt)
            if knobs is None:
                w = pkg.LearnedDecimation("cuda:0", seed=0).weights
                cost[name] = median_ms(lambda: plan.learned_decompose(filt, ws, w))
            else:
                cost[name] = median_ms(lambda: plan.decompose(filt, ws))
            del filt, ws
    log("[study] decomposition ms at 512^3, s=3: " + ", ".join(f"{a} {b:.3f}" for a, b in cost.items()))
    return {"held_out": {"n": n, "nz": nz, "p": p, "r": r, "s": s, "train_phantoms": 8, "held_out_phantoms": 4,
                         "learned_steps": steps, "rel_rmse_vs_fdk": err},
            "decompose_ms_512_p360_s3": cost}


LEARNED_C5_WEIGHTS = os.path.join(ROOT, "paper_1708_07515_amd", "learned_c5_weights.txt")


class SlabScans:
    """Slabs of seeded phantoms at the N = 2000, P = 720 geometry: only the
    detector rows a slab samples (eq. (9), the slab mode's band) are
    projected and filtered; the target is the direct FDK reconstruction of
    the slab from the same band."""

    def __init__(self, torch, pkg, wl, s, nzs, ellipsoids):
        self.torch, self.pkg, self.wl, self.nzs, self.ellipsoids = torch, pkg, wl, nzs, ellipsoids
        n, p, r = wl.n, wl.p, wl.r
        self.plan = pkg.Plan(n, p, r, s=s, store="f32")
        self.direct = pkg.Plan(n, p, r, s=0, store="f32")
        self.vol = torch.empty((nzs, n, n), device="cuda:0")
        self.tgt = torch.empty_like(self.vol)
        self.resid = torch.empty_like(self.vol)
        self.zs = list(range(0, (wl.nz or wl.n) - nzs + 1, 32))
        maxrows = max(self.plan.band_rows(z0, nzs)[1] for z0 in self.zs)
        self.ws_all = self.plan.empty_band(maxrows)[2]
        self.dws_all = torch.empty(self.plan.band_workspace_elems(maxrows), dtype=torch.float32, device="cuda:0")

    def slab(self, seed, z0):
        """(v0, rows, filtered band) of phantom ``seed`` for slices
        [z0, z0 + nzs); self.tgt receives its direct FDK slab."""
        from synth import phantom
        n, p, r = self.wl.n, self.wl.p, self.wl.r
        v0, nr = self.plan.band_rows(z0, self.nzs)
        ell = phantom.random_ellipsoids(self.ellipsoids, seed)
        pb = phantom.project(ell, n, p, r, device="cuda:0", rows=np.arange(v0, v0 + nr)).contiguous()
        fb = self.torch.empty((p, nr, n), dtype=self.torch.float32, device="cuda:0")
        self.plan.filter_band(pb, v0, fb)
        self.direct.reconstruct_slab(fb, None, v0, nr, z0, self.tgt)
        return v0, nr, fb

    def ws(self, nr):
        return self.ws_all[:self.plan.band_workspace_elems(nr)]

    def dws(self, nr):
        return self.dws_all[:self.plan.band_workspace_elems(nr)]

    def energy(self, t):
        """sum t^2 on the device (the library's squared residual against zero)."""
        loss = self.torch.zeros(1, dtype=self.torch.float64, device="cuda:0")
        self.pkg.sq_residual(t, self.torch.zeros_like(t), self.resid, loss)
        return float(loss)

    def close(self):
        self.plan.close()
        self.direct.close()


def train_learned_slabs(torch, pkg, scans, steps, lr, seed0, rng_seed=7, log_every=64, positions=None,
                        lr_end=None):
    """AdamW on one slab per step (phantom seed0 + step, slab position drawn
    with rng_seed from ``positions``, default every position), each slab's
    squared error weighted by the inverse of its target's energy; with
    lr_end, the step size falls from lr to lr_end along a half cosine.
    Returns the trained LearnedDecimation and the training time split (ms of
    library kernels per step, seconds of data generation)."""
    net = pkg.LearnedDecimation("cuda:0", seed=0, lr=lr)
    rng = np.random.default_rng(rng_seed)
    t_gen = t_train = 0.0
    skipped = 0
    positions = scans.zs if positions is None else positions
    for it in range(steps):
        z0 = int(rng.choice(positions))
        t0 = time.time()
        v0, nr, fb = scans.slab(seed0 + it, z0)
        e = scans.energy(scans.tgt)
        if e <= 0.0:                 # the slab misses the phantom
            skipped += 1
            continue
        w = 1.0 / e
        torch.cuda.synchronize()
        t1 = time.time()
        if lr_end is not None:
            net.lr = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * it / max(steps - 1, 1)))
        net.train_step_slab(scans.plan, fb, v0, scans.ws(nr), z0, scans.vol, scans.tgt, scans.resid,
                            scans.dws(nr), weight=w)
        torch.cuda.synchronize()
        t2 = time.time()
        t_gen += t1 - t0
        t_train += t2 - t1
        if it % log_every == 0 or it == steps - 1:
            log(f"[study] learned c5 step {it}: slab z0={z0} ({nr} rows), weighted loss {float(net.loss):.4e}")
    return net, {"train_ms_per_step": 1e3 * t_train / max(steps - skipped, 1), "data_seconds": t_gen,
                 "empty_slabs_skipped": skipped}


def held_out_slabs(torch, pkg, scans, net, seeds, positions):
    """Relative error against direct FDK, per held-out slab, of the triangle,
    the trained learned filter and the windowed sinc (6 taps) with the cubic
    shift, all FDK-OD at the scans' s."""
    wl = scans.wl
    knob = pkg.Plan(wl.n, wl.p, wl.r, s=scans.plan.s, store="f32", decim="sinc", taps=6, interp="cubic")

    def rel(a, b):
        return float(torch.linalg.norm((a - b).double()) / torch.linalg.norm(b.double()))

    out = {"triangle": [], "learned": [], "sinc6_cubic": [], "slabs": []}
    for sd, z0 in zip(seeds, positions):
        v0, nr, fb = scans.slab(sd, z0)
        if scans.energy(scans.tgt) <= 0.0:
            continue
        ws = scans.ws(nr)
        scans.plan.decompose_band(fb, v0, ws)
        scans.plan.reconstruct_slab(fb, ws, v0, nr, z0, scans.vol)
        out["triangle"].append(rel(scans.vol, scans.tgt))
        if net is not None:
            net.forward_slab(scans.plan, fb, v0, ws, z0, scans.vol)
            out["learned"].append(rel(scans.vol, scans.tgt))
        knob.decompose_band(fb, v0, ws)
        knob.reconstruct_slab(fb, ws, v0, nr, z0, scans.vol)
        out["sinc6_cubic"].append(rel(scans.vol, scans.tgt))
        out["slabs"].append([int(sd), int(z0)])
    knob.close()
    out["mean"] = {k: float(np.mean(v)) for k, v in out.items() if k != "slabs" and v}
    return out


def load_learned_c5(pkg, path=LEARNED_C5_WEIGHTS, device="cuda:0"):
    """A LearnedDecimation holding the weights learned_c5 wrote (None when the
    file is absent)."""
    if not os.path.exists(path):
        return None
    vals = [float(x) for x in open(path).read().split("\n") if x.strip() and not x.startswith("#")]
    net = pkg.LearnedDecimation(device, seed=0)
    net.load(np.asarray(vals, dtype=np.float32))
    return net


def learned_c5(torch, pkg, steps=512, lr=1e-3, nzs=32, held=16, out_path=LEARNED_C5_WEIGHTS, lr_end=None):
    """The learned decimation at the N = 2000, P = 720, s = 4 workload (D = 16,
    dilation 4): trained on ``steps`` seeded 30-ellipsoid phantoms (seeds
    5000 + i), one slab of nzs slices each, and compared on ``held`` other
    phantoms (seeds 9000 + i, slabs spread over the volume) with the
    triangle, the windowed sinc + cubic shift and direct FDK.  Writes the
    trained weights to paper_1708_07515_amd/learned_c5_weights.txt."""
    from synth import configs
    wl = configs.C5
    scans = SlabScans(torch, pkg, wl, 4, nzs, wl.ellipsoids)
    # training slabs from the central half of the volume: towards its ends a
    # slab can hold little of the phantom, and its inverse-energy weight then
    # lets a few nearly empty slabs drive the updates (training on every
    # position diverged at lr 2e-3)
    nzv = wl.nz or wl.n
    central = [z for z in scans.zs if abs(z + nzs / 2 - nzv / 2) < nzv / 4]
    net, timing = train_learned_slabs(torch, pkg, scans, steps, lr, 5000, positions=central, log_every=32,
                                      lr_end=lr_end)
    # held-out slabs spread over the central three quarters of the volume
    lo, hi = (wl.nz or wl.n) // 8, (wl.nz or wl.n) - (wl.nz or wl.n) // 8 - nzs
    positions = [z for z in (int(x) // 32 * 32 for x in np.linspace(lo, hi, held))]
    res = held_out_slabs(torch, pkg, scans, net, [9000 + i for i in range(held)], positions)
    log("[study] learned c5 held-out mean rel-RMSE vs direct FDK: "
        + ", ".join(f"{a} {b:.4f}" for a, b in res["mean"].items()))
    w = net.master.detach().cpu().double().numpy()
    with open(out_path, "w") as f:
        f.write("# learned decimation filter for N = 2000, P = 720, R = 8000, s = 4 (D = 16): 817 FP32 master\n"
                f"# weights (W1 [16][5][5], b1 [16], W2 [16][5][5], b2), AdamW lr {lr}"
                + (f" falling to {lr_end} (half cosine)" if lr_end is not None else "") + f", {steps} slabs of "
                f"{nzs} slices; written by study.py --learned-c5\n")
        for x in w:
            f.write(f"{x:.9e}\n")
    scans.close()
    return {"n": wl.n, "p": wl.p, "r": wl.r, "s": 4, "d": 16, "slab_slices": nzs, "train_phantoms": steps,
            "held_out_phantoms": held, "lr": lr, "lr_end": lr_end, "train_slices": [central[0], central[-1] + nzs],
            "timing": timing, "held_out": res,
            "weights_file": os.path.relpath(os.path.abspath(out_path), ROOT)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="smaller sizes (a few seconds)")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--learned-c5", action="store_true",
                    help="only train and evaluate the learned filter at N = 2000, P = 720, s = 4")
    ap.add_argument("--c5-steps", type=int, default=512)
    ap.add_argument("--c5-lr", type=float, default=1e-3)
    ap.add_argument("--c5-out", default=LEARNED_C5_WEIGHTS, help="where the trained weights are written")
    ap.add_argument("--c5-lr-end", type=float, default=None, help="final step size (half-cosine decay)")
    args = ap.parse_args()
    import torch

    import paper_1708_07515_amd as pkg

    t0 = time.time()
    if args.learned_c5:
        res = learned_c5(torch, pkg, steps=args.c5_steps, lr=args.c5_lr, out_path=args.c5_out,
                         lr_end=args.c5_lr_end)
        print(json.dumps({"study": "learned decimation at N = 2000, P = 720, s = 4 on one MI355X",
                          "data": "synthetic", "learned_c5": res, "seconds": round(time.time() - t0, 1)}),
              flush=True)
        return
    if args.quick:
        sweep = quality_sweep(torch, pkg, 96, 120, 384.0, 3)
        split = time_split(torch, pkg, [(128, 180)], 3, 2)
        knobs = knobs_vs_learned(torch, pkg, steps=50, cost_reps=2)
    else:
        sweep = quality_sweep(torch, pkg, 256, 360, 1024.0, 5)
        split = time_split(torch, pkg, [(256, 360), (512, 360), (1024, 720)], 5, args.reps)
        knobs = knobs_vs_learned(torch, pkg)
    print(json.dumps({"study": "FDK-OD quality and cost on one MI355X", "data": "synthetic",
                      "quality": sweep, "time_split": split, "knobs": knobs,
                      "seconds": round(time.time() - t0, 1)}), flush=True)


if __name__ == "__main__":
    main()
