"""Seeded synthetic workloads: grid fields with no-fly cells.

This module only draws inputs (grid shapes, no-fly masks, batch mixes).  It
holds none of the method's arithmetic, and it is the one module that both the
oracle-side tests and the HIP path consume.

The paper's fields are plain M x N grids with the start cell c_{0,0}
(Sec. II).  The workloads below add seeded no-fly cells (removed from the
visit list) and batches of uneven sizes.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Grid:
    rows: int
    cols: int
    nofly: np.ndarray                     # uint8 [rows*cols], 1 = excluded
    depot: int = 0                        # row-major index of the start cell
    inst_id: int = 0                      # instance id (addresses the random streams)
    density: float = 0.0

    @property
    def n_free(self) -> int:
        return int(self.rows * self.cols - 1 - int(self.nofly.sum()))


def _rng(seed: int, stream: int, inst: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, stream, inst])))


def grid(rows: int, cols: int, density: float = 0.0, seed: int = 1, inst: int = 0) -> Grid:
    """rows x cols field; each non-depot cell is no-fly with probability ``density``."""
    nofly = np.zeros(rows * cols, np.uint8)
    if density > 0:
        u = _rng(seed, 2, inst).random(rows * cols)
        nofly[:] = (u < density).astype(np.uint8)
        nofly[0] = 0
    return Grid(rows, cols, nofly, 0, inst, float(density))


def batch(n: int, seed: int = 1, side_lo: int = 4, side_hi: int = 10, density_hi: float = 0.2,
          first_id: int = 0, side: Optional[int] = None) -> List[Grid]:
    """``n`` instances with ids first_id.. ; side uniform in side_lo..side_hi (or fixed
    ``side``) and no-fly density uniform in [0, density_hi]."""
    out = []
    for i in range(n):
        iid = first_id + i
        r = _rng(seed, 3, iid)
        s = int(side) if side is not None else int(r.integers(side_lo, side_hi + 1))
        d = float(r.uniform(0.0, density_hi))
        out.append(grid(s, s, d, seed, iid))
    return out


@dataclass
class Workload:
    name: str
    grids: List[Grid]
    replicas: int
    sweeps: int
    T0: float
    T1: float
    seed: int = 1
    notes: str = ""


def workload(name: str) -> Workload:
    """The named workloads (shapes and schedules of the evaluation configs)."""
    if name == "grid3x3":
        return Workload(name, [grid(3, 3)], 64, 1000, 100.0, 0.5, 1,
                        "3x3, no obstacles, 8 free cells, 64 vars")
    if name == "grid8x8_nofly0.1":
        return Workload(name, [grid(8, 8, 0.1, 1, 0)], 1024, 2000, 200.0, 0.5, 1,
                        "8x8, Bernoulli(0.1) no-fly cells, ~57 free cells, ~3249 vars")
    if name == "grid12x12":
        return Workload(name, [grid(12, 12)], 4096, 4000, 200.0, 0.5, 1,
                        "12x12, no obstacles, 143 free cells, 20449 vars")
    if name == "grid16x16":
        return Workload(name, [grid(16, 16)], 4096, 1000, 200.0, 0.5, 1,
                        "16x16, no obstacles, 255 free cells, 65025 vars (the largest factored class)")
    if name == "grid19x19":
        return Workload(name, [grid(19, 19)], 4096, 1000, 200.0, 0.5, 1,
                        "19x19, no obstacles, 360 free cells, 129600 vars (the largest field with 8-bit costs)")
    if name == "grid20x20":
        return Workload(name, [grid(20, 20)], 4096, 1000, 200.0, 0.5, 1,
                        "20x20, no obstacles, 399 free cells, 159201 vars, costs up to 269 (16-bit)")
    if name == "grid24x24":
        return Workload(name, [grid(24, 24)], 4096, 1000, 200.0, 0.5, 1,
                        "24x24, no obstacles, 575 free cells, 330625 vars, costs up to 325 (16-bit)")
    if name == "batch256":
        return Workload(name, batch(256, 1), 256, 2000, 200.0, 0.5, 1,
                        "256 instances, side U{4..10}, density U[0,0.2]")
    raise KeyError(name)
