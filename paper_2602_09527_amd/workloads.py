"""Synthetic workloads shaped like the paper's experiments (sizes and solver settings only).

The paper reconstructs one real 2D slice (400 angles x 347 bins, Sec. 2.1) and a simulated
foam phantom (Sec. 2.2); neither dataset is available, so seeded random-ellipse phantoms with
analytic projections stand in for them at the sizes below.  Seeds: phantom = seed, noise =
seed + 1, subset/coin streams = seed + 2.
"""
from __future__ import annotations

import dataclasses


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    n_angles: int
    n_bins: int
    n_subsets: int
    nz: int = 1
    p: float = 0.1
    alpha: float = 0.01
    fgp_inner: int = 100
    n_epochs: int = 30
    seed: int = 101
    noise: str = "gaussian"
    nonneg: bool = True

    @property
    def key(self) -> str:
        return f"{self.nx}x{self.ny}x{self.nz}_a{self.n_angles}_b{self.n_bins}"


# 128^2 FP64-oracle problem: 180 angles x 128 bins, 10 subsets, p = 0.1, 100 FGP iterations,
# alpha = 0.01, 30 epochs.
SMALL_2D = Workload("2d-128-a180", 128, 128, 180, 128, 10, p=0.1, alpha=0.01, fgp_inner=100,
                    n_epochs=30, seed=101)

# Single 512^2 solve: 720 angles x 768 bins, 20 subsets, alpha = 0.005, 50 FGP iterations;
# p swept over {1, 0.1, 0.02} against non-skipped ProxSVRG.
SINGLE_2D = Workload("2d-512-a720", 512, 512, 720, 768, 20, p=0.1, alpha=0.005, fgp_inner=50,
                     n_epochs=30, seed=202)

# Differentiation check: batch of 64 images 256^2, 360 angles x 384 bins (full operator).
AUTOGRAD_BATCH = Workload("autograd-64x256-a360", 256, 256, 360, 384, 1, nz=64, seed=303)

# Batched volume: 256 slices of 1024^2, 1800 angles x 1448 bins, 30 subsets, p = 0.05,
# 3D TV, Poisson-log noise; and its reduced parity shape.
VOLUME_3D = Workload("3d-256x1024-a1800", 1024, 1024, 1800, 1448, 30, nz=256, p=0.05,
                     alpha=0.005, fgp_inner=50, n_epochs=10, seed=404, noise="poisson-log")
VOLUME_3D_REDUCED = Workload("3d-8x128-a180", 128, 128, 180, 192, 10, nz=8, p=0.05, alpha=0.005,
                             fgp_inner=50, n_epochs=10, seed=404, noise="poisson-log")

# Serving mix: sizes N in {128, 256, 512, 1024}, angles in {90, 360, 720, 1800}, bins = 1.5 N.
SERVE_SIDES = (128, 256, 512, 1024)
SERVE_ANGLES = (90, 360, 720, 1800)
SERVE_SUBSETS = {90: 10, 360: 20, 720: 20, 1800: 30}

ALL = {w.name: w for w in (SMALL_2D, SINGLE_2D, AUTOGRAD_BATCH, VOLUME_3D, VOLUME_3D_REDUCED)}
