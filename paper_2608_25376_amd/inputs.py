"""Seeded synthetic workloads: grid fields with no-fly cells.

This module only draws inputs (grid shapes, no-fly masks, batch mixes).  It
holds none of the method's arithmetic, and it is the one module that both the
oracle-side tests and the HIP path consume.

The paper's fields are plain M x N grids with the start cell c_{0,0}
(Sec. II).  The workloads below add seeded no-fly cells (removed from the
visit list) and batches of uneven sizes.
"""
import json
import os
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


CONFIG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")


def fields_from_spec(spec: dict) -> List[Grid]:
    """The grids a config's field spec names: {"kind": "grid", rows, cols, density, seed, inst}
    or {"kind": "batch", n, seed, first_id, side | side_lo and side_hi, density_hi}."""
    kind = spec["kind"]
    if kind == "grid":
        return [grid(int(spec["rows"]), int(spec["cols"]), float(spec.get("density", 0.0)),
                     int(spec.get("seed", 1)), int(spec.get("inst", 0)))]
    if kind == "batch":
        return batch(int(spec["n"]), int(spec.get("seed", 1)), int(spec.get("side_lo", 4)),
                     int(spec.get("side_hi", 10)), float(spec.get("density_hi", 0.2)),
                     int(spec.get("first_id", 0)), spec.get("side"))
    raise ValueError(f"unknown field kind {kind!r}")


def load_config(path: str) -> Workload:
    """A workload from a JSON config: name, fields (see fields_from_spec),
    replicas, sweeps, T0, T1, seed, notes."""
    with open(path) as f:
        c = json.load(f)
    return Workload(c["name"], fields_from_spec(c["fields"]), int(c["replicas"]), int(c["sweeps"]),
                    float(c["T0"]), float(c["T1"]), int(c.get("seed", 1)), c.get("notes", ""))


def workload_names() -> List[str]:
    return sorted(os.path.splitext(f)[0] for f in os.listdir(CONFIG_DIR)
                  if f.endswith(".json") and "fields" in json.load(open(os.path.join(CONFIG_DIR, f))))


def workload(name: str) -> Workload:
    """The named workloads (shapes and schedules of the evaluation configs),
    one JSON file each under configs/."""
    path = os.path.join(CONFIG_DIR, name + ".json")
    if not os.path.exists(path):
        raise KeyError(name)
    return load_config(path)
