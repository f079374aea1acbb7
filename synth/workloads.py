"""Named synthetic workloads (sizes only; no method arithmetic).

Each workload fixes the image grid, coil count, ACS block, kernel radius,
low-resolution grid and output grid of one scan family.  The shapes follow the
paper's setting (Q = 15-32 channels, 24^2 to 32^2 calibration regions, kernel
radius 2-3 in the paper's experiments, Sec. III-E and Sec. IV) extended to the
larger sizes this implementation is measured on.
"""
from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np

from .generator import Scan, make_acs_scan, make_scan


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    grid: Tuple[int, ...]       # output (full) grid
    Q: int
    acs: Tuple[int, ...]
    radius: float
    grid_lr: Tuple[int, ...]    # low-resolution estimation grid
    n_shapes: int
    snr_db: float
    seeds: Tuple[int, ...]
    acs_only: bool = False      # scan too large for full k-space: ACS block only

    @property
    def D(self) -> int:
        return len(self.grid)

    def scan(self, seed: int | None = None, keep_kspace: bool = True) -> Scan:
        s = self.seeds[0] if seed is None else seed
        if self.acs_only:
            return make_acs_scan(s, self.grid, self.Q, self.acs, self.n_shapes,
                                 self.snr_db)
        return make_scan(s, self.grid, self.Q, self.acs, self.n_shapes,
                         self.snr_db, keep_kspace=keep_kspace)


# 2D 64x64, 8 coils, 24x24 ACS, radius 3, maps on 32x32 (small case)
SMALL_2D = Workload("2d_64x64_q8_acs24_r3", (64, 64), 8, (24, 24), 3.0,
                    (32, 32), 6, 40.0, (1000, 1001, 1002, 1003, 1004))

# 2D 256x256, 32 coils, 32x32 ACS, radius 5; low-res grid = ACS + 24 per dim
BRAIN_2D = Workload("2d_256x256_q32_acs32_r5", (256, 256), 32, (32, 32), 5.0,
                    (56, 56), 20, 30.0, (2000, 2001, 2002, 2003, 2004))

# 3D 160x160x96 (z=96 slowest is stored first), 16 coils, 24^3 ACS, radius 4
VOLUME_3D = Workload("3d_96x160x160_q16_acs24_r4", (96, 160, 160), 16,
                     (24, 24, 24), 4.0, (24, 40, 40), 20, 30.0,
                     (3000, 3001, 3002))

# 3D 256x256x128 (z = 128 slowest), 32 coils, 32^3 ACS, radius 5 (n = 16480);
# low-res grid ACS + 24 = 56 per dim; the application size of the learned
# warm start.  Shapes and SNR as the other 3D volume; drawn ACS-only.
APP_3D = Workload("3d_128x256x256_q32_acs32_r5", (128, 256, 256), 32,
                  (32, 32, 32), 5.0, (56, 56, 56), 20, 30.0, (20000,),
                  acs_only=True)

ALL = {w.name: w for w in (SMALL_2D, BRAIN_2D, VOLUME_3D, APP_3D)}


def tiny(seed: int = 7, Q: int = 4, grid=(32, 32), acs=(16, 16), radius=2.0,
         grid_lr=(16, 16), n_shapes=4, snr_db=40.0) -> Workload:
    """A tiny workload for exhaustive (brute force) oracle checks."""
    return Workload(f"tiny_{len(grid)}d", tuple(grid), Q, tuple(acs), radius,
                    tuple(grid_lr), n_shapes, snr_db, (seed,))


def batch_slices(seed: int = 4000, count: int = 64) -> List[Workload]:
    """Uneven 2D slices: grids from {128^2, 192^2, 256^2, 256x320}, Q from
    {8, 16, 32}, ACS even in [24, 40], radius in {3, 4, 5, 6}, 30 dB; the
    low-res grid is ACS + 24 capped at the output grid."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grids = [(128, 128), (192, 192), (256, 256), (256, 320)]
    out = []
    for i in range(count):
        g = grids[int(rng.integers(0, 4))]
        Q = int((8, 16, 32)[int(rng.integers(0, 3))])
        A = int(rng.integers(12, 21)) * 2
        r = float(rng.integers(3, 7))
        lr = tuple(min(A + 24, n) for n in g)
        out.append(Workload(f"slice{i}", g, Q, (A, A), r, lr, 20, 30.0,
                            (seed + i,)))
    return out
