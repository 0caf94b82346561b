"""The benchmark and test workloads, with their seeds.

Each workload is a circular-orbit cone-beam scan of a seeded random-ellipsoid
phantom: detector N x N pixels, P angles over 360 degrees, eq. (1) constant R
(source-to-axis distance in voxel units, virtual detector through the axis),
volume N x N x N_z.  ``s`` lists the decomposition levels exercised and ``k``
the skipped decimation stages.  Where a workload description leaves R or the
ellipsoid count open, the value chosen here keeps R / N = 4.
"""

from dataclasses import dataclass


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    p: int
    r: float
    s: tuple
    ellipsoids: int
    seed: int
    nz: int = 0                 # 0 -> n
    k: int = 0
    photons: float = 0.0        # Poisson incident photons per ray, 0 = noise free
    store: tuple = ("f32",)
    note: str = ""

    @property
    def nzv(self):
        return self.nz or self.n


# small case: the oracle reconstructs the whole volume in seconds
C1 = Workload("cone64_p90", n=64, p=90, r=512.0, s=(0, 1, 2), ellipsoids=10, seed=1,
              note="detector 64x64, P=90, R=512, volume 64^3, 10 ellipsoids")

# the metric's workload: FDK-OD s in {1,2,3} against direct FDK
C2 = Workload("cone512_p360", n=512, p=360, r=2048.0, s=(1, 2, 3), ellipsoids=20, seed=2,
              photons=1e5,
              note="detector 512x512, P=360, R=2048, volume 512^3, 20 ellipsoids, "
                   "Poisson noise at 1e5 photons per ray")

# precision form: FP16 / BF16 storage of the filtered and decimated sinograms
C3 = Workload("cone1024_p720", n=1024, p=720, r=4096.0, s=(3,), ellipsoids=30, seed=3,
              store=("f32", "f16", "bf16"),
              note="detector 1024x1024, P=720, volume 1024^3, s=3, 30 ellipsoids")

# large case: N = 2000, P = 720, s = 4 (the paper's headline size)
C5 = Workload("cone2000_p720", n=2000, p=720, r=8000.0, s=(4,), ellipsoids=30, seed=5000,
              store=("f32", "bf16"),
              note="detector 2000x2000, P=720, volume 2000^3, s=4, 30 ellipsoids")


@dataclass(frozen=True)
class BatchWorkload:
    """Many volumes of uneven size reconstructed in one persistent launch."""
    name: str = "batch32_mixed"
    count: int = 32
    sizes: tuple = (128, 192, 256, 384, 512)
    p_per_n: float = 1.4
    r_per_n: float = 4.0
    ellipsoids: int = 10
    seed: int = 4
    s_max: int = 5              # s per volume: the cost model's choice up to s_max


C4 = BatchWorkload()
# many small volumes, where one volume alone is far from filling the GPU
C4S = BatchWorkload(name="batch256_small", count=256, sizes=(32, 48, 64), ellipsoids=6, seed=6)

ALL = {w.name: w for w in (C1, C2, C3, C5)}
