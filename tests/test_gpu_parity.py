"""GPU parity: the HIP path through the C ABI against the FP64 oracle and closed forms.

Every test prints its case before touching the GPU so that a failing run names it.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from scenegen import (block_scene, corner_scene, district_scene, empty_scene, ground_scene, mirror_scene,
                      sealed_box_scene, tiny_scene, wall_scene)
from tests import closed_forms as CF
from tests.parity_check import (check_counts, check_flags, check_hits, check_mics, paths_diverge,
                                strict_share)

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


def grid(scene):
    from paper_1912_03998_amd.tracer import scene_grid
    return scene_grid(scene)


def gpu_run(s, scene, parity=True, sources=None, power=None, **kw):
    src = scene.sources if sources is None else sources
    pw = scene.power if power is None else power
    return s.run(src, pw, scene.level, scene.depth, grid(scene), parity=parity, **kw)


def full_verdict(scene, g, o, min_strict_share=0.99):
    """Hits, flags, counts and microphones against the oracle; at least min_strict_share of
    the oracle's energised microphones must be strict (compared to 0.01 dB)."""
    n = check_hits(o.hit, o.flag, o.t_hit, g.hit, g.t_hit)
    check_flags(o.hit, o.flag, g.flag)
    div = paths_diverge(o.hit, g.hit)
    check_counts(o.count, o.flagged, g.stats["count"], g.stats["flagged"], diverged=div)
    m = check_mics(o.e_strict, o.e_flag, g.e_strict, g.e_flag, diverged=div)
    say(f"verdict: {n} unflagged segments, {m['strict_energised']}/{m['energised']} energised microphones strict, "
        f"max {m['max_db']:.2e} dB, paths diverge: {div}")
    assert strict_share(m) >= min_strict_share, m
    return n, m


# ---------------------------------------------------------------------------------------
# closed forms on the GPU
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("level", [0, 1, 3, 5])
def test_free_field_direct_path(torch_cuda, level):
    sc = empty_scene(level=level, src=(0.3, -0.2, 1.0))
    say("free field", level)
    with session(sc) as s:
        g = gpu_run(s, sc)
    m = sc.mic_positions()
    ref = 1.0 / (FOUR_PI * ((m - sc.sources[0].astype(np.float64)) ** 2).sum(1))
    assert (g.e_flag == 0).all()
    assert np.abs(g.energy / ref - 1).max() < 1e-6
    assert g.stats["mic_updates"] == sc.n_mic
    assert (g.hit[:, 0] == -1).all()


def test_free_field_fine_grid_staged_boxes(torch_cuda):
    """A 1 cm grid 1 m above the source, level 6: most upward beams hold a few lattice
    points, so many 64-beam batches have more than 32 segments with candidate boxes
    (several staging rounds), and others have such segments at scattered lanes (unused
    staging slots among used ones).  Every microphone is reached once, with the closed-form
    energy."""
    sc = empty_scene(level=6, src=(0.003, -0.002, 0.0), n_mic=201, spacing=0.01, mic_z=1.0)
    say("free field, 1 cm grid, level 6")
    with session(sc) as s:
        g = gpu_run(s, sc, parity=False)
    m = sc.mic_positions()
    ref = 1.0 / (FOUR_PI * ((m - sc.sources[0].astype(np.float64)) ** 2).sum(1))
    assert g.stats["mic_updates"] == sc.n_mic
    assert np.abs(g.energy / ref - 1).max() < 1e-6


@pytest.mark.parametrize("level,alpha", [(3, 0.2), (5, 0.5)])
def test_ground_reflection_image_source(torch_cuda, level, alpha):
    sc = ground_scene(level=level, alpha=alpha)
    say("ground", level, alpha)
    with session(sc) as s:
        g = gpu_run(s, sc)
    m = sc.mic_positions()
    src = sc.sources[0].astype(np.float64)
    img = src * np.array([1, 1, -1.0])
    a32 = float(np.float32(alpha))
    ref = (1.0 / ((m - src) ** 2).sum(1) + (1 - a32) / ((m - img) ** 2).sum(1)) / FOUR_PI
    elev = np.degrees(np.arctan2(m[:, 2] + src[2], np.hypot(m[:, 0] - src[0], m[:, 1] - src[1])))
    ok = (elev > 15) & (g.e_flag == 0)
    assert ok.sum() > 60
    assert np.abs(g.energy[ok] / ref[ok] - 1).max() < 1e-6


@pytest.mark.parametrize("level,alpha,depth", [(2, 0.25, 6), (4, 0.6, 3)])
def test_sealed_box_counts_and_power(torch_cuda, level, alpha, depth):
    sc = sealed_box_scene(level=level, alpha=alpha, depth=depth)
    say("sealed box", level, alpha, depth)
    with session(sc) as s:
        g = gpu_run(s, sc)
    n = 20 * 4 ** level
    st = g.stats
    assert st["generations"] == depth + 1
    assert (st["count"] == n).all()
    assert (st["flagged"] == 0).all()
    a32 = float(np.float32(alpha))
    ref = (1 - a32) ** np.arange(depth + 1)
    assert np.abs(st["power"] / ref - 1).max() < 1e-5
    assert (g.hit >= 0).all()


@pytest.mark.parametrize("ground_z", [3.7, -4.2])
def test_ground_off_origin_image_source(torch_cuda, ground_z):
    """Ground z = h != 0: direct path plus the image at 2h - z_s above it, nothing below."""
    src = (0.25, -0.15, ground_z + 2.0)
    sc = ground_scene(level=4, alpha=0.3, src=src, mic_z=ground_z + 1.5, ground_z=ground_z)
    say("ground off the origin", ground_z)
    ref, ok = CF.ground_offset(sc, ground_z, 0.3)
    with session(sc) as s:
        g = gpu_run(s, sc)
        below = sc.with_(mic_z=ground_z - 1.5)
        gb = gpu_run(s, below)
    ok &= g.e_flag == 0
    assert ok.sum() > 60
    assert np.abs(g.energy[ok] / ref[ok] - 1).max() < 1e-6
    assert (gb.energy == 0.0).all()


def test_wall_off_origin_image_source(torch_cuda):
    """Vertical wall x = c != 0: direct path plus the image at 2c - x_s in front, nothing
    behind."""
    sc = wall_scene(level=4, alpha=0.3, wall_x=7.5)
    say("wall off the origin")
    ref, ok = CF.wall_offset(sc, 7.5, 0.3)
    with session(sc) as s:
        g = gpu_run(s, sc)
        gb = gpu_run(s, wall_scene(level=4, alpha=0.3, wall_x=7.5, behind=True))
    ok &= g.e_flag == 0
    assert ok.sum() > 60
    assert np.abs(g.energy[ok] / ref[ok] - 1).max() < 1e-6
    assert (gb.energy == 0.0).all()


def test_wall_corner_second_order_image(torch_cuda):
    """Wall + ground corner: four images with weights 1, 1 - a_g, 1 - a_w,
    (1 - a_g)(1 - a_w); no third reflection."""
    sc = corner_scene(level=5)
    say("wall + ground corner")
    ref, ok, last_on_wall = CF.corner(sc, 6.0, 0.2, 0.35)
    with session(sc) as s:
        g = gpu_run(s, sc)
    ok &= g.e_flag == 0
    assert ok.sum() > 80
    assert last_on_wall[ok].sum() > 10 and (~last_on_wall[ok]).sum() > 10
    assert np.abs(g.energy[ok] / ref[ok] - 1).max() < 1e-6
    assert g.stats["count"][3] == 0 and g.stats["count"][2] > 0


@pytest.mark.parametrize("eps", [1e-9, -1e-9])
def test_energy_threshold_exact_generation(torch_cuda, eps):
    """e_min within 1e-9 of a generation's beam power in a level-0 sealed box: the run ends
    exactly before or after that generation (the decision is taken in FP64)."""
    e_min, alive = CF.sealed_box_threshold(0.1, 3, eps)
    sc = sealed_box_scene(level=0, alpha=0.1, depth=6)
    say("energy threshold at an exact generation", eps)
    with session(sc) as s:
        g = gpu_run(s, sc, e_min=e_min)
    want = np.array([20 if k < alive else 0 for k in range(7)])
    assert np.array_equal(g.stats["count"], want), g.stats["count"]


def test_sealed_box_maximum_depth(torch_cuda):
    """31 reflections (the maximum): after ~23 bounces a few beams graze a box corner
    within the 1 mm self-intersection guard and leave; both sides must agree."""
    sc = sealed_box_scene(level=2, alpha=0.1, depth=31)
    say("sealed box depth 31")
    o = O.trace(sc)
    with session(sc) as s:
        g = gpu_run(s, sc)
    # after ~23 bounces some beams graze corners: 3 of the 56 energised microphones carry
    # flagged energy on both sides
    full_verdict(sc, g, o, min_strict_share=0.9)
    assert np.array_equal(g.stats["count"], o.count)
    assert np.abs(g.stats["power"] / o.power - 1).max() < 1e-5


# ---------------------------------------------------------------------------------------
# oracle parity on the plain-method workloads
# ---------------------------------------------------------------------------------------

def test_tiny_scene_parity(torch_cuda):
    sc = tiny_scene()
    say("tiny scene parity")
    o = O.trace(sc)
    with session(sc) as s:
        g = gpu_run(s, sc)
    n, m = full_verdict(sc, g, o)
    assert n > 2000
    assert m["nonzero"] >= 12


def test_block_scene_parity(torch_cuda):
    sc = block_scene(0)
    say("block scene parity")
    o = O.trace(sc)
    with session(sc) as s:
        g = gpu_run(s, sc)
    n, m = full_verdict(sc, g, o)
    assert n > 90_000
    assert m["energised"] > 1000
    # the GPU's own work counters agree with the oracle's segment and update counts
    assert g.stats["segments"] == o.counters["segments"]
    assert abs(g.stats["mic_updates"] - o.counters["mic_updates"]) <= o.flagged.sum() * 50


def test_mirror_scene_parity(torch_cuda):
    sc = mirror_scene()
    say("mirror scene parity")
    o = O.trace(sc)
    with session(sc) as s:
        g = gpu_run(s, sc)
    # the source sits on the symmetry plane: its row of microphones lies on shared beam
    # faces, so about 8 % of the energised microphones are ambiguous on both sides
    full_verdict(sc, g, o, min_strict_share=0.9)


@pytest.mark.parametrize("air_m,e_min", [(0.02, 0.0), (0.0, 2e-5)])
def test_physics_variants_parity(torch_cuda, air_m, e_min):
    sc = block_scene(0).with_(level=4)
    say("physics variants", air_m, e_min)
    o = O.trace(sc, m_air=air_m, e_min=e_min)
    with session(sc) as s:
        g = gpu_run(s, sc, air_m=air_m, e_min=e_min)
    full_verdict(sc, g, o)


def test_partition_invariance_block(torch_cuda):
    sc = block_scene(0)
    say("partition invariance block")
    res = []
    for tiles in [(1, 1), (3, 3), (4, 2), (7, 5)]:
        with session(sc, tiles=tiles) as s:
            res.append(gpu_run(s, sc))
    a = res[0]
    for b in res[1:]:
        assert np.array_equal(a.hit, b.hit)
        assert np.array_equal(a.flag, b.flag)
        assert np.array_equal(a.stats["count"], b.stats["count"])
        e = a.energy
        assert np.abs(b.energy - e).max() <= 1e-12 * e.max()


@pytest.mark.parametrize("tiles", [(3, 3), (7, 5)])
def test_tile_queues_equal_in_lane_walk(torch_cuda, tiles):
    """Per-tile beam queues with hand-off between them (1, 2 or 8 queued rounds) give the
    in-lane tile walk's hits, flags, counts and energies exactly."""
    sc = block_scene(0)
    say("tile queues vs in-lane walk, block scene, tiles", tiles)
    with session(sc, tiles=tiles) as s:
        ref = gpu_run(s, sc, queue_rounds=0)
        for rounds in (1, 2, 8):
            g = gpu_run(s, sc, queue_rounds=rounds)
            assert np.array_equal(g.hit, ref.hit) and np.array_equal(g.flag, ref.flag), rounds
            assert np.array_equal(g.t_hit, ref.t_hit, equal_nan=True)
            assert np.array_equal(g.stats["count"], ref.stats["count"])
            assert np.array_equal(g.stats["flagged"], ref.stats["flagged"])
            assert g.stats["mic_updates"] == ref.stats["mic_updates"]
            assert np.abs(g.energy - ref.energy).max() <= 1e-12 * ref.energy.max()


# ---------------------------------------------------------------------------------------
# the district workload (full mesh, 4 x 4 tiles)
# ---------------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def district():
    return district_scene(0)


def test_district_sources_parity(torch_cuda, district):
    """Full district mesh, microphone grid and 4 x 4 tiles; two of the 64 sources traced
    completely by both sides."""
    sc = district
    pick = [5, 40]
    sub = sc.with_(sources=sc.sources[pick], power=sc.power[pick])
    say("district parity, sources", pick)
    o = O.trace(sub)
    with session(sc) as s:
        g = gpu_run(s, sub)
        g1 = None
    n, m = full_verdict(sub, g, o)
    assert n > 300_000
    assert m["energised"] > 30_000
    say("district partition invariance 1x1 vs 4x4")
    with session(sc, tiles=(1, 1)) as s:
        g1 = gpu_run(s, sub)
    assert np.array_equal(g.hit, g1.hit) and np.array_equal(g.flag, g1.flag)
    assert np.abs(g.energy - g1.energy).max() <= 1e-12 * g.energy.max()
    say("district tile queues: 2 and 8 queued rounds against the in-lane walk")
    with session(sc) as s:
        for rounds in (2, 8):
            g2 = gpu_run(s, sub, queue_rounds=rounds)
            assert np.array_equal(g.hit, g2.hit) and np.array_equal(g.flag, g2.flag), rounds
            assert np.array_equal(g.stats["count"], g2.stats["count"])
            assert np.abs(g.energy - g2.energy).max() <= 1e-12 * g.energy.max()


def test_district_full_size(torch_cuda, district):
    """All 64 sources (5,242,880 initial beams, depth 8) in the benchmark's configuration:
    the full verdict against the complete oracle run, and linearity over sources."""
    sc = district
    say("district full size")
    with session(sc) as s:
        g = gpu_run(s, sc)
        st = g.stats
        assert st["count"][0] == sc.n_beams0
        assert (np.diff(st["count"]) <= 0).all()
        # the oracle traces the whole workload too (a few seconds on 16 threads)
        say("district full oracle")
        o = O.trace(sc)
        n, m = full_verdict(sc, g, o)
        assert n > 13_000_000
        assert m["energised"] > 190_000

        assert st["segments"] == o.counters["segments"] or \
            abs(st["segments"] - o.counters["segments"]) <= o.flagged.sum()
        del o
        # linearity: the sum of four 16-source runs equals the 64-source run
        say("district linearity")
        acc = np.zeros(sc.n_mic)
        for k in range(4):
            idx = slice(16 * k, 16 * (k + 1))
            r = s.run(sc.sources[idx], sc.power[idx], sc.level, sc.depth, grid(sc), parity=False)
            acc += r.energy
        e = g.energy
        assert np.abs(acc - e).max() <= 1e-9 * e.max()
        assert (e > 0).sum() > 100_000
    # bt_run with a record budget below the workload's: two generation slots, a microphone
    # pass per generation, the same energies, under 4 GB of device memory
    from paper_1912_03998_amd import bt
    say("district through bt_run with two generation slots")
    with session(sc) as s2:
        g2 = s2.run(sc.sources, sc.power, sc.level, sc.depth, grid(sc), parity=False, run_records=1 << 24)
        used = bt.bt_memory_used(s2.ctx)
    say(f"district device memory with two generation slots: {used / 1e9:.2f} GB")
    assert used < 4e9
    assert np.abs(g2.energy - e).max() <= 1e-12 * e.max()
    assert np.array_equal(g2.stats["count"], st["count"])


def test_run_chunks_sources_beyond_the_index_range(torch_cuda):
    """49 sources at level 9 (256,901,120 generation-0 beams) with depth 8: n_beams0 (depth + 1)
    exceeds 2^31 - 1, yet one bt_run call traces them (source chunks, two generation slots
    each); the energies equal the sum of the 49 single-source runs to 1e-12, the statistics
    add up, and the free-field closed form holds."""
    from paper_1912_03998_amd import bt
    sc = empty_scene(level=9, src=(0.0, 0.0, 1.0), n_mic=21, spacing=5.0, mic_z=6.0)
    rng = np.random.default_rng(9)
    src = rng.uniform([-8.0, -8.0, 0.5], [8.0, 8.0, 3.0], (49, 3)).astype(np.float32)
    pw = rng.uniform(0.5, 2.0, 49).astype(np.float32)
    depth, level = 8, 9
    n0 = 49 * 20 * 4 ** level
    assert n0 * (depth + 1) > 2 ** 31 - 1
    say("bt_run over 49 level-9 sources, depth 8")
    with session(sc) as s:
        g = s.run(src, pw, level, depth, grid(sc), parity=False)
        used = bt.bt_memory_used(s.ctx)
        acc = np.zeros(sc.n_mic)
        for k in range(49):
            r = s.run(src[k:k + 1], pw[k:k + 1], level, depth, grid(sc), parity=False)
            acc += r.energy
    e = g.energy
    assert np.abs(acc - e).max() <= 1e-12 * e.max()
    assert g.stats["segments"] == n0 and g.stats["count"][0] == n0 and g.stats["mic_updates"] == 49 * sc.n_mic
    m = sc.mic_positions()
    ref = sum(float(w) / (FOUR_PI * ((m - p.astype(np.float64)) ** 2).sum(1)) for p, w in zip(src, pw))
    assert np.abs(e / ref - 1).max() < 1e-6
    assert used < 8e9, used


# ---------------------------------------------------------------------------------------
# boundary behaviour
# ---------------------------------------------------------------------------------------

def test_error_paths(torch_cuda):
    from paper_1912_03998_amd import bt
    say("error paths")
    ctx = bt.bt_create(0, 0, None)
    try:
        v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
        t = np.array([[0, 1, 2]], np.int32)
        a = np.array([0.1], np.float32)
        with pytest.raises(bt.BTError) as e:
            bt.bt_build_mesh(ctx, v, np.array([[0, 1, 3]], np.int32), a)
        assert e.value.status == -1
        with pytest.raises(bt.BTError):
            bt.bt_build_mesh(ctx, np.array([[0, 0, np.nan], [1, 0, 0], [0, 1, 0]], np.float32), t, a)
        with pytest.raises(bt.BTError):
            bt.bt_build_mesh(ctx, v, t, np.array([1.5], np.float32))
        with pytest.raises(bt.BTError):
            bt.bt_build_mesh(ctx, np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0]], np.float32), t, a)
        with pytest.raises(bt.BTError):
            bt.bt_build_mesh(ctx, v, t, a, 0, 1)
        mesh = bt.bt_build_mesh(ctx, v, t, a)
        with pytest.raises(bt.BTError):
            bt.bt_emit_beams(ctx, [[0, 0, 1]], [1.0], 10)
        with pytest.raises(bt.BTError):
            bt.bt_mics_grid(ctx, 0, 0, 1, 0, 1, 4, 4)
        beams = bt.bt_emit_beams(ctx, [[0.2, 0.2, 1]], [1.0], 1)
        mics = bt.bt_mics_grid(ctx, 0, 0, 0.5, 0.25, 0.25, 4, 4)
        p = bt.bt_params_default(max_depth=1)
        # a set created by binding and never emitted: nothing to trace or accumulate, and
        # its statistics are zeros
        unemitted = bt.bt_beams_bind_mics(ctx, None, mics)
        for call in (lambda: bt.bt_trace(ctx, mesh, unemitted, p), lambda: bt.bt_trace_all(ctx, mesh, unemitted, p),
                     lambda: bt.bt_accumulate_mics(ctx, mesh, unemitted, p, mics)):
            with pytest.raises(bt.BTError) as e:
                call()
            assert e.value.status == -6
        st0 = bt.bt_beams_stats(ctx, unemitted)
        assert st0["segments"] == 0 and st0["generations"] == 0 and st0["node_visits"] == 0
        bt.bt_beams_free(unemitted)
        with pytest.raises(bt.BTError) as e:
            bt.bt_accumulate_mics(ctx, mesh, beams, p, mics)
        assert e.value.status == -6
        with pytest.raises(bt.BTError):
            bt.bt_trace(ctx, mesh, beams, bt.bt_params_default(max_depth=40))
        assert bt.bt_trace(ctx, mesh, beams, p, want_next=True) >= 0
        # the emission's generations belong to the mesh they were traced with
        other = bt.bt_build_mesh(ctx, v * 2.0, t, a)
        with pytest.raises(bt.BTError) as e:
            bt.bt_trace(ctx, other, beams, p)
        assert e.value.status == -1
        with pytest.raises(bt.BTError) as e:
            bt.bt_accumulate_mics(ctx, other, beams, p, mics)
        assert e.value.status == -1
        bt.bt_mesh_free(other)
        bt.bt_accumulate_mics(ctx, mesh, beams, p, mics)
        with pytest.raises(bt.BTError):
            bt.bt_trace(ctx, mesh, beams, bt.bt_params_default(max_depth=2))
        bt.bt_trace(ctx, mesh, beams, p)
        with pytest.raises(bt.BTError) as e:
            bt.bt_trace(ctx, mesh, beams, p)
        assert e.value.status == -6
        with pytest.raises(bt.BTError) as e:
            bt.bt_poll(ctx, 12345, 16)
        assert e.value.status == -5
        bt.bt_beams_free(beams)
        bt.bt_mics_free(mics)
        bt.bt_mesh_free(mesh)
    finally:
        bt.bt_destroy(ctx)
    small = bt.bt_create(0, 4096, None)
    try:
        with pytest.raises(bt.BTError) as e:
            bt.bt_mics_grid(small, 0, 0, 0, 1, 1, 1000, 1000)
        assert e.value.status == -2
    finally:
        bt.bt_destroy(small)


def test_degenerate_inputs(torch_cuda):
    """No sources, a single microphone, a mesh without triangles."""
    from paper_1912_03998_amd.tracer import Session
    say("degenerate inputs")
    sc = tiny_scene()
    with Session.from_scene(sc) as s:
        r = s.run(np.zeros((0, 3), np.float32), np.zeros(0, np.float32), 3, 3, grid(sc), parity=True)
        assert (r.energy == 0).all() and r.stats["segments"] == 0
        r = s.run(sc.sources, sc.power, 3, 3, (10.0, -10.0, 1.5, 1.0, 1.0, 1, 1), parity=False)
        o = O.trace(sc.with_(mic_x0=10.0, mic_y0=-10.0, mic_nx=1, mic_ny=1, mic_dx=1.0, mic_dy=1.0))
        check_mics(o.e_strict, o.e_flag, r.e_strict, r.e_flag)


def test_submit_poll_matches_plain_run(torch_cuda):
    from paper_1912_03998_amd import bt
    say("submit / poll")
    sc = block_scene(0).with_(level=3, depth=4)
    with session(sc) as s:
        ref = gpu_run(s, sc, parity=False)
        tickets = [bt.bt_submit(s.ctx, s.mesh, sc.sources, sc.power, sc.level, sc.depth, grid(sc)) for _ in range(3)]
        out = {}
        for _ in range(100000):
            for tk in tickets:
                if tk not in out:
                    r = bt.bt_poll(s.ctx, tk, sc.n_mic)
                    if r is not None:
                        out[tk] = r
            if len(out) == len(tickets):
                break
        assert len(out) == 3
        for tk in tickets:
            e, f, segs, upd = out[tk]
            assert segs == ref.stats["segments"]
            assert np.abs(e - ref.energy).max() <= 1e-12 * ref.energy.max()
        tk = bt.bt_submit(s.ctx, s.mesh, sc.sources, sc.power, sc.level, sc.depth, grid(sc))
        bt.bt_cancel(s.ctx, tk)
        with pytest.raises(bt.BTError):
            bt.bt_poll(s.ctx, tk, sc.n_mic)


@pytest.mark.parametrize("every", [1, 3])
def test_microphone_passes_between_generations(torch_cuda, every):
    """However the generations are grouped into microphone passes (each pass reuses the
    work buffers of the previous one), the energies equal one pass at the end (up to
    FP64 atomic ordering) and the oracle's."""
    from paper_1912_03998_amd import bt
    sc = block_scene(0)
    say("microphone passes every", every, "generations")
    o = O.trace(sc)
    with session(sc) as s:
        ref = gpu_run(s, sc, parity=False)
        mics = s._mics(grid(sc))
        p = s.params(sc.depth)
        s.beams = bt.bt_emit_beams(s.ctx, sc.sources, sc.power, sc.level, s.beams)
        bt.bt_mics_reset(s.ctx, mics)
        for g in range(sc.depth + 1):
            bt.bt_trace(s.ctx, s.mesh, s.beams, p)
            if (g + 1) % every == 0:
                bt.bt_accumulate_mics(s.ctx, s.mesh, s.beams, p, mics)
        bt.bt_accumulate_mics(s.ctx, s.mesh, s.beams, p, mics)
        n = sc.n_mic
        es, ef = np.zeros(n), np.zeros(n)
        bt.bt_levels(s.ctx, mics, es, ef, None)
        st = bt.bt_beams_stats(s.ctx, s.beams)
    assert st["mic_updates"] == ref.stats["mic_updates"]
    assert np.abs(es - ref.e_strict).max() <= 1e-12 * ref.e_strict.max()
    assert np.abs(ef - ref.e_flag).max() <= 1e-12 * max(ref.e_flag.max(), 1e-300)
    check_mics(o.e_strict, o.e_flag, es, ef)


@pytest.mark.parametrize("env,value", [("BT_MIC_ROW_CAPACITY", "1000"), ("BT_MIC_ROW_CAPACITY", "50000"),
                                       ("BT_MIC_SPAN_CAPACITY", "1000")])
def test_mic_work_buffer_overflow(torch_cuda, monkeypatch, env, value):
    """Small work-item buffers force wide footprints onto the one-wave-per-segment path
    (every one of them when the row buffer's per-wave regions hold nothing, some when they
    hold a few rows each) and long rows onto in-place processing; results must not change."""
    sc = block_scene(0)
    say("mic work buffer overflow", env, value)
    o = O.trace(sc)
    monkeypatch.setenv(env, value)
    with session(sc) as s:
        g = gpu_run(s, sc)
    full_verdict(sc, g, o)


def test_directional_sources_parity(torch_cuda):
    """Directional sources (a smooth per-face intensity pattern): energies against the
    oracle with the same weights, and generation-0 power equal to the sources' power."""
    from paper_1912_03998_amd import bt
    sc = block_scene(0).with_(level=4, depth=4)
    say("directional sources, block scene")
    c = O.icosphere(sc.level).sum(1)
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    axis = np.array([1.0, 0.5, 0.2]) / np.linalg.norm([1.0, 0.5, 0.2])
    w = np.tile((1.0 + 0.8 * (c @ axis)) ** 2, (sc.n_src, 1)).astype(np.float32)
    o = O.trace(sc, weights=w, keep_paths=False)
    with session(sc) as s:
        p = s.params(sc.depth)
        mics = s._mics(grid(sc))
        s.beams = bt.bt_emit_beams_directional(s.ctx, sc.sources, sc.power, w, sc.level, s.beams)
        for _ in range(sc.depth + 1):
            bt.bt_trace(s.ctx, s.mesh, s.beams, p)
        bt.bt_accumulate_mics(s.ctx, s.mesh, s.beams, p, mics)
        es, ef = np.zeros(sc.n_mic), np.zeros(sc.n_mic)
        bt.bt_levels(s.ctx, mics, es, ef, None)
        st = bt.bt_beams_stats(s.ctx, s.beams)
        with pytest.raises(bt.BTError):
            bt.bt_emit_beams_directional(s.ctx, sc.sources, sc.power, -w, sc.level, s.beams)
    check_mics(o.e_strict, o.e_flag, es, ef)
    assert abs(st["power"][0] - float(sc.power.sum())) < 1e-6 * float(sc.power.sum())
    assert abs(st["power"][1] - o.power[1]) < 1e-5 * o.power[1]
