"""Workload table: the five synthetic workloads the path is tested and timed on.

Scanner constants follow Sec. "Acquisition parameters" (G_max 40 mT/m,
S_max 180 T/m/s, raster 10 us, 20.48 ms readout) and Sec. "From trajectories
to actual k-space data" (ADC dwell 2 us).  The k-space domain is [-L, L]^3
with L = 1/2; K_max is matrix/(2 FOV) as in Sec. "3D K-space sampling".
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import inputs

GAMMA_BAR = 42.576e6      # Hz/T, the proton gyromagnetic ratio divided by 2 pi
GMAX = 40e-3              # T/m
SMAX = 180.0              # T/m/s
RASTER_DT = 10e-6         # s, gradient raster time
DWELL_DT = 2e-6           # s, ADC dwell time


@dataclass(frozen=True)
class Workload:
    name: str
    n_shots: int
    n_samples: int
    grid: int
    half_width: float
    density_C: float
    density_D: float
    jitter: float
    seed: int
    fov: float            # m
    matrix: int           # matrix side that fixes K_max = matrix / (2 FOV)
    n_pit: int
    n_iters: int
    oracle_targets: int   # 0 = every target
    precision: str

    @property
    def p(self) -> int:
        return self.n_shots * self.n_samples

    @property
    def n_voxels(self) -> int:
        return self.grid ** 3

    @property
    def kmax(self) -> float:
        return self.matrix / (2.0 * self.fov)

    @property
    def eta_fixed(self) -> float:
        # a quarter of the mean sample spacing per unit of |p * grad_i F|
        return 0.25 * (2.0 * self.half_width) * float(self.p) ** (2.0 / 3.0)

    def trajectory(self) -> np.ndarray:
        return inputs.radial_spokes(self.n_shots, self.n_samples, self.half_width,
                                    self.seed, self.jitter)

    def density(self) -> np.ndarray:
        return inputs.radial_density(self.grid, self.half_width,
                                     self.density_C, self.density_D)


# c1: plain FP64 gradient + 5 iterations, 64 x 64 spokes, 32^3 density min(1, (0.05/|k|)^2)
C1 = Workload("c1_plain_fp64_loop", 64, 64, 32, 0.5, 0.05, 2.0, 0.0, 1,
              0.24, 32, 200, 5, 0, "plain_fp64")
# c2: FP32 gradient, 1024 x 512 jittered spokes, 128^3 density with a 1/8-radius flat centre
C2 = Workload("c2_fp32_grad", 1024, 512, 128, 0.5, 0.0625, 2.0, 0.05, 2,
              0.24, 128, 200, 0, 4096, "fp32_comp")
# c3: FP32-compensated, 4096 x 2048 (384x384x208 at 0.6 mm), 192^3 density, flat radius 0.1
C3 = Workload("c3_fp32_comp_8p4M", 4096, 2048, 192, 0.5, 0.1, 2.0, 0.05, 3,
              384 * 0.6e-3, 384, 200, 0, 1024, "fp32_comp")
# c4: autograd, 128 x 512, 32^3 density (c1 law)
C4 = Workload("c4_autograd", 128, 512, 32, 0.5, 0.05, 2.0, 0.05, 4,
              0.24, 32, 200, 0, 0, "fp32_comp")
# c5: 100 projected-gradient iterations, 2048 x 1024, 128^3 density (c2 law)
C5 = Workload("c5_loop", 2048, 1024, 128, 0.5, 0.0625, 2.0, 0.05, 5,
              0.24, 128, 200, 100, 0, "fp32_comp")

WORKLOADS = {w.name: w for w in (C1, C2, C3, C4, C5)}
