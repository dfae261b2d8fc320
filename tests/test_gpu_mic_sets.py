"""Microphone sets beyond the full grid, on the GPU: explicit points (bucket-indexed) and
subsets of a grid.  Closed forms, oracle parity, and equality with the grid where the two
describe the same microphones.  Every test prints its case before touching the GPU."""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from scenegen import block_scene, empty_scene, tiny_scene, volumetric_scene
from tests.parity_check import check_mics, strict_share

pytestmark = pytest.mark.gpu
FOUR_PI = 4.0 * math.pi


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def session(scene):
    from paper_1912_03998_amd.tracer import Session
    return Session.from_scene(scene)


def run_set(s, scene, mics, n_out):
    """bt_run into `mics`, then its strict and flag energies (n_out values) and stats."""
    from paper_1912_03998_amd import bt
    p = s.params(scene.depth)
    s.beams = bt.bt_run(s.ctx, s.mesh, scene.sources, scene.power, scene.level, p, mics, s.beams)
    es, ef = np.zeros(n_out), np.zeros(n_out)
    bt.bt_levels(s.ctx, mics, es, ef, None)
    return es, ef, bt.bt_beams_stats(s.ctx, s.beams)


def test_points_free_field(torch_cuda):
    from paper_1912_03998_amd import bt
    rng = np.random.default_rng(3)
    pts = rng.uniform([-20.0, -20.0, -10.0], [20.0, 20.0, 25.0], (2000, 3)).astype(np.float32)
    sc = empty_scene(level=4, src=(0.3, -0.2, 1.0))
    say("points free field")
    with session(sc) as s:
        m = bt.bt_mics_points(s.ctx, pts)
        es, ef, st = run_set(s, sc, m, len(pts))
        bt.bt_mics_free(m)
    ref = 1.0 / (FOUR_PI * ((pts.astype(np.float64) - sc.sources[0].astype(np.float64)) ** 2).sum(1))
    assert np.abs((es + ef) / ref - 1).max() < 1e-6
    assert st["mic_updates"] == len(pts)


def test_points_match_oracle_block(torch_cuda):
    """Random points through the city block's volume (inside buildings too), against the
    oracle's brute force over the same points."""
    from paper_1912_03998_amd import bt
    rng = np.random.default_rng(4)
    pts = rng.uniform([-100.0, -100.0, 0.2], [100.0, 100.0, 65.0], (5000, 3)).astype(np.float32)
    sc = block_scene(0)
    say("points vs oracle, block scene")
    o = O.trace(sc, points=pts, keep_paths=False)
    with session(sc) as s:
        m = bt.bt_mics_points(s.ctx, pts)
        es, ef, st = run_set(s, sc, m, len(pts))
        bt.bt_mics_free(m)
    r = check_mics(o.e_strict, o.e_flag, es, ef)
    assert strict_share(r) >= 0.99 and r["energised"] > 1500, r
    assert abs(st["mic_updates"] - o.counters["mic_updates"]) <= o.flagged.sum() * 20


def test_points_match_oracle_tall_district(torch_cuda):
    """The tall district: receivers scattered around one source up to 150 m high (a few on
    tower walls' sides), level 6, depth 8."""
    from paper_1912_03998_amd import bt
    tall = volumetric_scene(0, level=6)
    k = 20
    sc = tall.with_(sources=tall.sources[k:k + 1], power=tall.power[k:k + 1])
    c = sc.sources[0].astype(np.float64)
    rng = np.random.default_rng(6)
    pts = (c + rng.uniform([-300.0, -300.0, 0.0], [300.0, 300.0, 150.0], (10000, 3))).astype(np.float32)
    say("points vs oracle, tall district, source", k)
    o = O.trace(sc, points=pts, keep_paths=False)
    with session(sc) as s:
        m = bt.bt_mics_points(s.ctx, pts)
        es, ef, st = run_set(s, sc, m, len(pts))
        bt.bt_mics_free(m)
    r = check_mics(o.e_strict, o.e_flag, es, ef)
    assert strict_share(r) >= 0.99 and r["energised"] > 7000, r


@pytest.mark.parametrize("volumetric", [False, True])
def test_points_on_grid_equal_grid(torch_cuda, volumetric):
    """Points on the grid's positions, shuffled, receive the grid's energies."""
    from paper_1912_03998_amd import bt
    from paper_1912_03998_amd.tracer import scene_grid
    sc = block_scene(0)
    if volumetric:
        sc = sc.with_(mic_x0=-98.0, mic_y0=-98.0, mic_dx=4.0, mic_dy=4.0, mic_nx=50, mic_ny=50, mic_z=1.5,
                      mic_nz=8, mic_dz=8.0)
    say("points on grid positions, volumetric", volumetric)
    pos = sc.mic_positions()
    perm = np.random.default_rng(2).permutation(len(pos))
    with session(sc) as s:
        g = s.run(sc.sources, sc.power, sc.level, sc.depth, scene_grid(sc), parity=False)
        m = bt.bt_mics_points(s.ctx, pos[perm].astype(np.float32))
        es, ef, _ = run_set(s, sc, m, len(pos))
        bt.bt_mics_free(m)
    scale = max(g.energy.max(), 1e-300)
    assert np.abs(es - g.e_strict[perm]).max() <= 1e-12 * scale
    assert np.abs(ef - g.e_flag[perm]).max() <= 1e-12 * scale


@pytest.mark.parametrize("volumetric", [False, True])
def test_subset_equals_grid_selection(torch_cuda, volumetric):
    from paper_1912_03998_amd import bt
    from paper_1912_03998_amd.tracer import grid_size, scene_grid
    sc = block_scene(0)
    if volumetric:
        sc = sc.with_(mic_x0=-98.0, mic_y0=-98.0, mic_dx=4.0, mic_dy=4.0, mic_nx=50, mic_ny=50, mic_z=1.5,
                      mic_nz=8, mic_dz=8.0)
    grid = scene_grid(sc)
    n = grid_size(grid)
    idx = np.random.default_rng(8).integers(0, n, 3000).astype(np.int32)   # duplicates too
    say("subset of the grid, volumetric", volumetric)
    with session(sc) as s:
        g = s.run(sc.sources, sc.power, sc.level, sc.depth, grid, parity=False)
        full = bt.bt_mics_grid(s.ctx, *grid) if len(grid) == 7 else bt.bt_mics_grid3d(s.ctx, *grid)
        sub = bt.bt_mics_subset(s.ctx, full, idx)
        bt.bt_mics_free(full)
        es, ef, st = run_set(s, sc, sub, len(idx))
        lv = np.zeros(len(idx))
        bt.bt_levels(s.ctx, sub, None, None, lv)
        bt.bt_mics_free(sub)
    scale = max(g.energy.max(), 1e-300)
    assert np.abs(es - g.e_strict[idx]).max() <= 1e-12 * scale
    assert np.abs(ef - g.e_flag[idx]).max() <= 1e-12 * scale
    e = es + ef
    ok = e > 0
    assert np.abs(lv[ok] - 10 * np.log10(e[ok] / 1e-12)).max() < 1e-9 and np.isneginf(lv[~ok]).all()
    assert st["mic_updates"] < g.stats["mic_updates"]


def test_mic_set_errors(torch_cuda):
    from paper_1912_03998_amd import bt
    say("mic set errors")
    sc = tiny_scene()
    with session(sc) as s:
        grid = bt.bt_mics_grid(s.ctx, -30.0, -30.0, 1.5, 20.0, 20.0, 4, 4)
        pts = bt.bt_mics_points(s.ctx, np.zeros((3, 3), np.float32))
        for bad in (lambda: bt.bt_mics_subset(s.ctx, grid, np.array([16], np.int32)),
                    lambda: bt.bt_mics_subset(s.ctx, grid, np.array([-1], np.int32)),
                    lambda: bt.bt_mics_subset(s.ctx, grid, np.zeros(0, np.int32)),
                    lambda: bt.bt_mics_subset(s.ctx, pts, np.array([0], np.int32)),
                    lambda: bt.bt_mics_points(s.ctx, np.zeros((0, 3), np.float32)),
                    lambda: bt.bt_mics_points(s.ctx, np.array([[0.0, np.inf, 1.0]], np.float32))):
            with pytest.raises(bt.BTError):
                bad()
        sub = bt.bt_mics_subset(s.ctx, grid, np.array([0, 5, 5, 15], np.int32))
        with pytest.raises(bt.BTError):
            bt.bt_mics_subset(s.ctx, sub, np.array([0], np.int32))
        for m in (grid, pts, sub):
            bt.bt_mics_free(m)
