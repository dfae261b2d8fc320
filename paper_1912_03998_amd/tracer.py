"""Convenience session over the C ABI: one context and one resident mesh, many runs.

Every step runs in libbt.so's kernels; this module only allocates torch device
buffers for optional per-beam outputs and sequences the C calls.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import bt


@dataclasses.dataclass
class RunResult:
    e_strict: np.ndarray            # float64 [n_mic]
    e_flag: np.ndarray              # float64 [n_mic]
    level_db: np.ndarray            # float64 [n_mic]
    stats: dict
    hit: np.ndarray | None = None   # int32 [n_beams0, depth+1], -2 = not traced
    flag: np.ndarray | None = None  # uint8 same shape
    t_hit: np.ndarray | None = None  # float64 same shape

    @property
    def energy(self):
        return self.e_strict + self.e_flag


class Session:
    """A context on `device` with one mesh built from (xyz, tri, absorption)."""

    def __init__(self, xyz, tri, absorption, tiles_x=1, tiles_y=1, device=0, stream=None, hbm_budget=0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the tracer has no CPU path")
        self.torch = torch
        self.device = device
        # a dedicated stream (torch's default stream has the null handle, which the C ABI
        # reads as "library-owned stream"); torch work for the session goes on it too
        self.stream = stream if stream is not None else torch.cuda.Stream(device)
        self.ctx = bt.bt_create(device, hbm_budget, self.stream)
        self.mesh = bt.bt_build_mesh(self.ctx, xyz, tri, absorption, tiles_x, tiles_y)
        self.beams = None
        self.mics = None
        self._grid = None

    @classmethod
    def from_scene(cls, scene, tiles=None, **kw):
        tx, ty = (scene.tiles_x, scene.tiles_y) if tiles is None else tiles
        return cls(scene.vertices, scene.triangles, scene.absorption, tx, ty, **kw)

    def mesh_info(self):
        return bt.bt_mesh_info(self.mesh)

    def _mics(self, grid):
        if self._grid != grid:
            if self.mics is not None:
                bt.bt_mics_free(self.mics)
            self.mics = bt.bt_mics_grid(self.ctx, *grid) if len(grid) == 7 else bt.bt_mics_grid3d(self.ctx, *grid)
            self._grid = grid
        else:
            bt.bt_mics_reset(self.ctx, self.mics)
        return self.mics

    def params(self, depth, t_min=1e-3, edge_delta=1e-5, air_m=0.0, e_min=0.0, **outs):
        return bt.bt_params_default(max_depth=depth, t_min=t_min, edge_delta=edge_delta, air_m=air_m, e_min=e_min,
                                    **outs)

    def enqueue(self, sources, power, level, depth, grid, params=None):
        """Enqueue one full pass (emit, D+1 x (trace, accumulate)); no synchronisation
        beyond the borrowed-input copy of the emission."""
        mics = self._mics(tuple(grid))
        p = params if params is not None else self.params(depth)
        self.beams = bt.bt_run(self.ctx, self.mesh, sources, power, level, p, mics, self.beams)
        return mics

    def run(self, sources, power, level, depth, grid, *, parity=False, stats=True, **kw) -> RunResult:
        torch = self.torch
        sources = np.asarray(sources, np.float32).reshape(-1, 3)
        n0 = sources.shape[0] * 20 * 4 ** level
        outs = {}
        if parity:
            dev = torch.device("cuda", self.device)
            with torch.cuda.stream(self.stream):
                outs["hit_out"] = torch.full((n0, depth + 1), -2, dtype=torch.int32, device=dev)
                outs["flag_out"] = torch.zeros((n0, depth + 1), dtype=torch.uint8, device=dev)
                outs["t_out"] = torch.full((n0, depth + 1), float("nan"), dtype=torch.float64, device=dev)
        p = self.params(depth, **kw, **outs)
        mics = self.enqueue(sources, power, level, depth, grid, p)
        n_mic = grid_size(grid)
        es = np.empty(n_mic, np.float64)
        ef = np.empty(n_mic, np.float64)
        lv = np.empty(n_mic, np.float64)
        bt.bt_levels(self.ctx, mics, es, ef, lv)
        st = bt.bt_beams_stats(self.ctx, self.beams) if stats else {}
        res = RunResult(es, ef, lv, st)
        if parity:
            self.stream.synchronize()
            res.hit = outs["hit_out"].cpu().numpy()
            res.flag = outs["flag_out"].cpu().numpy()
            res.t_hit = outs["t_out"].cpu().numpy()
        return res

    def close(self):
        if self.ctx is None:
            return
        if self.beams is not None:
            bt.bt_beams_free(self.beams)
        if self.mics is not None:
            bt.bt_mics_free(self.mics)
        bt.bt_mesh_free(self.mesh)
        bt.bt_destroy(self.ctx)
        self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def scene_grid(scene):
    """A scene's microphone grid: (x0, y0, z, dx, dy, nx, ny) when planar, else
    (x0, y0, z0, dx, dy, dz, nx, ny, nz)."""
    if int(getattr(scene, "mic_nz", 1)) == 1:
        return (float(scene.mic_x0), float(scene.mic_y0), float(scene.mic_z), float(scene.mic_dx),
                float(scene.mic_dy), int(scene.mic_nx), int(scene.mic_ny))
    return (float(scene.mic_x0), float(scene.mic_y0), float(scene.mic_z), float(scene.mic_dx), float(scene.mic_dy),
            float(scene.mic_dz), int(scene.mic_nx), int(scene.mic_ny), int(scene.mic_nz))


def grid_size(grid):
    """Microphones in a planar (7-tuple) or volumetric (9-tuple) grid."""
    return grid[5] * grid[6] if len(grid) == 7 else grid[6] * grid[7] * grid[8]
