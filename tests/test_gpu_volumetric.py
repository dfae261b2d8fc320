"""Volumetric microphone grids on the GPU (the paper's experiment fills the model's
bounding box with microphones every 4 m): closed forms, oracle parity on small scenes
and on the tall district, and the overflow paths of the per-layer work lists.

Every test prints its case before touching the GPU so that a failing run names it.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from scenegen import block_scene, empty_scene, ground_scene, tiny_scene, volumetric_scene
from tests.parity_check import check_counts, check_flags, check_hits, check_mics, paths_diverge, strict_share

pytestmark = pytest.mark.gpu
FOUR_PI = 4.0 * math.pi


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def session(scene, tiles=None):
    from paper_1912_03998_amd.tracer import Session
    return Session.from_scene(scene, tiles=tiles)


def gpu_run(s, scene, parity=True, **kw):
    from paper_1912_03998_amd.tracer import scene_grid
    return s.run(scene.sources, scene.power, scene.level, scene.depth, scene_grid(scene), parity=parity, **kw)


def verdict(g, o, min_strict_share=0.99):
    n = check_hits(o.hit, o.flag, o.t_hit, g.hit, g.t_hit)
    check_flags(o.hit, o.flag, g.flag)
    div = paths_diverge(o.hit, g.hit)
    check_counts(o.count, o.flagged, g.stats["count"], g.stats["flagged"], diverged=div)
    m = check_mics(o.e_strict, o.e_flag, g.e_strict, g.e_flag, diverged=div)
    say(f"verdict: {m['strict_energised']}/{m['energised']} energised microphones strict, paths diverge: {div}")
    assert strict_share(m) >= min_strict_share, m
    return n, m


def crop(scene, src, nx, ny):
    """The scene's own 3D microphone lattice restricted to nx x ny columns around `src`."""
    i0 = int(np.clip(round((float(src[0]) - scene.mic_x0) / scene.mic_dx) - nx // 2, 0, scene.mic_nx - nx))
    j0 = int(np.clip(round((float(src[1]) - scene.mic_y0) / scene.mic_dy) - ny // 2, 0, scene.mic_ny - ny))
    return scene.with_(mic_x0=scene.mic_x0 + i0 * scene.mic_dx, mic_y0=scene.mic_y0 + j0 * scene.mic_dy,
                       mic_nx=nx, mic_ny=ny)


@pytest.mark.parametrize("level", [1, 3, 5])
def test_free_field_volumetric(torch_cuda, level):
    """Layers below, across and above the source: W / (4 pi d^2) once per microphone."""
    sc = empty_scene(level=level, src=(0.3, -0.2, 1.0), n_mic=9, spacing=3.0, mic_z=-7.5).with_(mic_nz=6,
                                                                                                  mic_dz=3.5)
    say("free field volumetric", level)
    with session(sc) as s:
        g = gpu_run(s, sc)
    m = sc.mic_positions()
    ref = 1.0 / (FOUR_PI * ((m - sc.sources[0].astype(np.float64)) ** 2).sum(1))
    assert np.abs(g.energy / ref - 1).max() < 1e-6
    assert g.stats["mic_updates"] == sc.n_mic


def test_ground_reflection_volumetric(torch_cuda):
    """Direct plus image source above the ground, nothing in the layer below it."""
    alpha = 0.3
    sc = ground_scene(level=5, alpha=alpha, mic_z=-2.5).with_(mic_nz=5, mic_dz=4.0)
    say("ground volumetric")
    with session(sc) as s:
        g = gpu_run(s, sc)
    m = sc.mic_positions()
    src = sc.sources[0].astype(np.float64)
    img = src * np.array([1, 1, -1.0])
    a32 = float(np.float32(alpha))
    ref = (1.0 / ((m - src) ** 2).sum(1) + (1 - a32) / ((m - img) ** 2).sum(1)) / FOUR_PI
    below = m[:, 2] < 0
    assert (g.energy[below] == 0).all()
    elev = np.degrees(np.arctan2(m[:, 2] + src[2], np.hypot(m[:, 0] - src[0], m[:, 1] - src[1])))
    ok = ~below & (elev > 15) & (g.e_flag == 0)
    assert ok.sum() > 200
    assert np.abs(g.energy[ok] / ref[ok] - 1).max() < 1e-6


def test_tiny_scene_volumetric_parity(torch_cuda):
    sc = tiny_scene().with_(mic_z=-2.5, mic_nz=12, mic_dz=2.5)
    say("tiny scene volumetric parity")
    o = O.trace(sc)
    with session(sc) as s:
        g = gpu_run(s, sc)
    # the source sits on the icosphere's vertex ray under the layers above it: 14 % of
    # the energised microphones are ambiguous on both sides
    n, m = verdict(g, o, min_strict_share=0.8)
    assert m["nonzero"] > 100


def test_block_scene_volumetric_parity(torch_cuda):
    """City block with a 3D grid: 50 x 50 columns at 4 m, 16 layers at 4 m up to 61.5 m."""
    sc = block_scene(0).with_(mic_x0=-98.0, mic_y0=-98.0, mic_dx=4.0, mic_dy=4.0, mic_nx=50, mic_ny=50,
                              mic_z=1.5, mic_nz=16, mic_dz=4.0)
    say("block scene volumetric parity")
    o = O.trace(sc)
    with session(sc) as s:
        g = gpu_run(s, sc)
    n, m = verdict(g, o)
    assert m["energised"] > 10_000
    assert g.stats["segments"] == o.counters["segments"]
    assert abs(g.stats["mic_updates"] - o.counters["mic_updates"]) <= o.flagged.sum() * 200


@pytest.mark.parametrize("env,value", [("BT_MIC_LAYER_CAPACITY", "300"), ("BT_MIC_ROW_CAPACITY", "200"),
                                       ("BT_MIC_SPAN_CAPACITY", "100")])
def test_volumetric_work_list_overflow(torch_cuda, monkeypatch, env, value):
    """Tiny (segment, layer), row and span buffers push work onto the fallback paths
    (items, rows and columns done in place); results must not change."""
    sc = block_scene(0).with_(level=4, mic_x0=-98.0, mic_y0=-98.0, mic_dx=4.0, mic_dy=4.0, mic_nx=50, mic_ny=50,
                              mic_z=1.5, mic_nz=16, mic_dz=4.0)
    say("volumetric overflow", env, value)
    o = O.trace(sc)
    monkeypatch.setenv(env, value)
    with session(sc) as s:
        g = gpu_run(s, sc)
    verdict(g, o)
    assert g.stats["mic_layer_visits"] > 0 and g.stats["mic_general"] > 0
    if env == "BT_MIC_LAYER_CAPACITY":
        # the in-place path did run: the buffer holds at most `value` items (its regions
        # of value // 256 items each), the rest were done where they were found
        assert g.stats["mic_general"] > int(value)
        assert g.stats["mic_general"] - int(value) <= g.stats["mic_fallback"] < g.stats["mic_general"]


@pytest.fixture(scope="module")
def tall():
    return volumetric_scene(0, level=6)


def test_tall_district_volumetric_parity(torch_cuda, tall):
    """The 2.5 x 1.5 km district with its towers: the source nearest the tallest tower,
    81,920 beams, depth 8, every layer of the 4 m lattice on 150 x 150 columns around it."""
    sc = tall
    top = sc.vertices[np.argmax(sc.vertices[:, 2])]
    k = int(np.argmin(((sc.sources[:, :2] - top[:2]) ** 2).sum(1)))
    sub = crop(sc.with_(sources=sc.sources[k:k + 1], power=sc.power[k:k + 1]), sc.sources[k], 150, 150)
    say("tall district volumetric parity, source", k, "layers", sub.mic_nz)
    o = O.trace(sub)
    with session(sub) as s:
        g = gpu_run(s, sub)
    n, m = verdict(g, o, min_strict_share=0.98)
    assert n > 200_000
    assert m["energised"] > 1_000_000
    assert g.stats["segments"] == o.counters["segments"] or \
        abs(g.stats["segments"] - o.counters["segments"]) <= o.flagged.sum()


def test_tall_district_full_grid_sample(torch_cuda, tall):
    """Level 7 (327,680 beams) from one street source onto the full 625 x 375 x 58
    lattice (13.6 M microphones), both sides complete; and the volumetric result's layer
    at 2 m equals a planar run at 2 m."""
    from paper_1912_03998_amd.tracer import scene_grid
    sc = tall.with_(level=7, sources=tall.sources[20:21], power=tall.power[20:21])
    say("tall district full grid, level 7, source 20")
    o = O.trace(sc, keep_paths=False)
    with session(sc) as s:
        g = gpu_run(s, sc, parity=False)
        m = check_mics(o.e_strict, o.e_flag, g.e_strict, g.e_flag)
        assert m["energised"] > 8_000_000 and strict_share(m) >= 0.99, m
        say("tall district planar layer 0")
        plane = sc.with_(mic_nz=1)
        p = s.run(plane.sources, plane.power, plane.level, plane.depth, scene_grid(plane), parity=False)
    per = sc.mic_nx * sc.mic_ny
    e0 = g.energy[:per]
    assert np.abs(p.energy - e0).max() <= 1e-9 * max(e0.max(), 1e-300)


def test_tall_district_level8_full_lattice(torch_cuda, tall):
    """The volumetric benchmark's own configuration for one source: level 8 (1,310,720 beams),
    depth 8, every microphone of the 625 x 375 x 58 lattice; both sides complete."""
    sc = tall.with_(level=8, sources=tall.sources[20:21], power=tall.power[20:21])
    say("tall district full lattice, level 8, source 20")
    o = O.trace(sc, keep_paths=False)
    with session(sc) as s:
        g = gpu_run(s, sc, parity=False)
    m = check_mics(o.e_strict, o.e_flag, g.e_strict, g.e_flag)
    say(f"level 8 lattice: {m['strict_energised']}/{m['energised']} energised microphones strict, "
        f"max {m['max_db']:.2e} dB")
    assert m["energised"] > 8_000_000 and strict_share(m) >= 0.99, m
    assert g.stats["segments"] == o.counters["segments"] or \
        abs(g.stats["segments"] - o.counters["segments"]) <= o.flagged.sum()


def test_volumetric_grid_errors(torch_cuda):
    from paper_1912_03998_amd import bt
    say("volumetric grid errors")
    sc = tiny_scene()
    with session(sc) as s:
        for bad in [(0.0, 0.0, 1.5, 1.0, 1.0, 1.0, 4, 4, 0), (0.0, 0.0, 1.5, 1.0, 1.0, 0.0, 4, 4, 3),
                    (0.0, 0.0, 1.5, 1.0, 1.0, float("nan"), 4, 4, 3), (0.0, 0.0, 1.5, 1.0, 1.0, 1.0, 65536, 65536, 2),
                    (0.0, 0.0, 1.5, 1.0, 1.0, 1.0, 1 << 24, 2, 2)]:
            with pytest.raises(bt.BTError):
                bt.bt_mics_grid3d(s.ctx, *bad)
        # nz = 1 ignores dz and is the planar grid
        m = bt.bt_mics_grid3d(s.ctx, -30.0, -30.0, 1.5, 20.0, 20.0, 0.0, 4, 4, 1)
        bt.bt_mics_free(m)
