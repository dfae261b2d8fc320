"""Seeded scenario sets and request streams on the district mesh (inputs only).

Batches: many independent scenarios traced together.  Serving: requests arriving as a
Poisson process.  Sources stand on the street centre lines (where the district has no
buildings) 0.5 m above the ground; microphones are subsets of the district's 4 m grid.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# the district's microphone grid: x, y = -998 + 4 i, i < 500, at 1.5 m
GRID = (np.float32(-998.0), np.float32(-998.0), np.float32(1.5), np.float32(4.0), np.float32(4.0), 500, 500)
LEVEL_OF_BEAMS = {1280: 3, 5120: 4, 20480: 5, 81920: 6}


@dataclasses.dataclass
class ScenarioSpec:
    """One scenario or request: sources, power, icosphere level, depth and microphones
    (a grid (x0, y0, z, dx, dy, nx, ny) and optionally a subset of its indices)."""
    sources: np.ndarray
    power: np.ndarray
    level: int
    depth: int
    grid: tuple
    subset: np.ndarray | None = None
    arrival: float = 0.0     # seconds from the start of a request stream

    @property
    def n_beams0(self) -> int:
        return int(self.sources.shape[0]) * 20 * 4 ** self.level

    @property
    def n_mic(self) -> int:
        return len(self.subset) if self.subset is not None else int(self.grid[5]) * int(self.grid[6])


def street_points(rng, n: int) -> np.ndarray:
    """n points on the interior street centre lines x or y = -1000 + 200 k (k = 1..9),
    uniform along the line, 0.5 m above the ground."""
    k = rng.integers(1, 10, size=n)
    along = rng.uniform(-990.0, 990.0, size=n)
    line = -1000.0 + 200.0 * k
    vertical = rng.random(n) < 0.5
    x = np.where(vertical, line, along)
    y = np.where(vertical, along, line)
    return np.stack([x, y, np.full(n, 0.5)], 1).astype(np.float32)


def batch_scenarios(seed: int = 0, n: int = 256, mics: int = 10_000) -> list[ScenarioSpec]:
    """Uneven scenarios: floor(exp(U(0, ln 65))) sources at street points, one beam count
    per scenario from {1280, 5120, 20480, 81920} per source, depth U{2..10}, and a
    random `mics`-point subset of the 4 m grid."""
    rng = np.random.default_rng(seed)
    out = []
    n_grid = GRID[5] * GRID[6]
    for _ in range(n):
        ns = int(math.floor(math.exp(rng.uniform(0.0, math.log(65.0)))))
        ns = min(max(ns, 1), 64)
        beams = int(rng.choice([1280, 5120, 20480, 81920]))
        depth = int(rng.integers(2, 11))
        subset = np.sort(rng.choice(n_grid, size=mics, replace=False)).astype(np.int32)
        out.append(ScenarioSpec(street_points(rng, ns), np.ones(ns, np.float32), LEVEL_OF_BEAMS[beams], depth, GRID,
                                subset))
    return out


def serving_requests(seed: int = 0, n: int = 2200, rate: float = 200.0) -> list[ScenarioSpec]:
    """Poisson arrivals at `rate` requests/s: floor(exp(U(0, ln 33))) sources at street
    points, depth U{3..8}, 5120 or 20480 beams per source, and an axis-aligned rectangle
    of the 4 m grid with N ~ log-U[1k, 50k] microphones and aspect ratio U(0.5, 2)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for k in range(n):
        ns = int(math.floor(math.exp(rng.uniform(0.0, math.log(33.0)))))
        ns = min(max(ns, 1), 32)
        depth = int(rng.integers(3, 9))
        beams = int(rng.choice([5120, 20480]))
        nm = math.exp(rng.uniform(math.log(1000.0), math.log(50000.0)))
        aspect = rng.uniform(0.5, 2.0)
        nx = int(min(max(round(math.sqrt(nm * aspect)), 1), 500))
        ny = int(min(max(round(nm / nx), 1), 500))
        i0 = int(rng.integers(0, 500 - nx + 1))
        j0 = int(rng.integers(0, 500 - ny + 1))
        grid = (np.float32(-998.0 + 4.0 * i0), np.float32(-998.0 + 4.0 * j0), np.float32(1.5), np.float32(4.0),
                np.float32(4.0), nx, ny)
        out.append(ScenarioSpec(street_points(rng, ns), np.ones(ns, np.float32), LEVEL_OF_BEAMS[beams], depth, grid,
                                None, float(t[k])))
    return out
