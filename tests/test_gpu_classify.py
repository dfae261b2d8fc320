"""Beams classified for a planar microphone grid as they are created
(bt_beams_bind_mics), against the microphone pass that decides from each frustum.

The decision (no microphone possible, a lattice box of candidates, or the clipped
footprint) depends on the frustum alone, so taking it at emission and reflection must
give the same candidates, tests and energies as taking it in the microphone pass.  The
pass uses the stored decisions only when every generation it covers was classified for
its grid's plane and lattice; otherwise it decides from the frustums, with the same
result.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from scenegen import block_scene, district_scene
from tests.parity_check import check_mics

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def manual_run(s, sc, mics, bind=None, bind_after_emit=None, subset=None):
    """Emit, trace every generation and accumulate once into `mics` on a fresh beam set;
    `bind` (a microphone set) is bound before emission, `bind_after_emit` after it."""
    from paper_1912_03998_amd import bt
    p = s.params(sc.depth)
    beams = None
    if bind is not None:
        beams = bt.bt_beams_bind_mics(s.ctx, beams, bind)
    beams = bt.bt_emit_beams(s.ctx, sc.sources, sc.power, sc.level, beams)
    if bind_after_emit is not None:
        bt.bt_beams_bind_mics(s.ctx, beams, bind_after_emit)
    for _ in range(sc.depth + 1):
        bt.bt_trace(s.ctx, s.mesh, beams, p)
    bt.bt_mics_reset(s.ctx, mics)
    bt.bt_accumulate_mics(s.ctx, s.mesh, beams, p, mics)
    n = subset if subset is not None else sc.n_mic
    es, ef = np.zeros(n), np.zeros(n)
    bt.bt_levels(s.ctx, mics, es, ef, None)
    st = bt.bt_beams_stats(s.ctx, beams)
    bt.bt_beams_free(beams)
    return es, ef, st


def same(a, b):
    scale = max(np.abs(a).max(), 1e-300)
    return np.abs(a - b).max() <= 1e-12 * scale


def test_bound_equals_unbound_block(torch_cuda):
    """Block scene: classified at creation or in the pass, the same tests, updates and
    energies; every segment's class is read from its creation; the parity contract holds."""
    from paper_1912_03998_amd import bt
    from paper_1912_03998_amd.tracer import Session, scene_grid
    sc = block_scene(0)
    with Session.from_scene(sc) as s:
        mics = bt.bt_mics_grid(s.ctx, *scene_grid(sc))
        say("block scene: unbound, then bound before emission")
        es0, ef0, st0 = manual_run(s, sc, mics)
        es1, ef1, st1 = manual_run(s, sc, mics, bind=mics)
        bt.bt_mics_free(mics)
    assert st0["mic_classified"] == 0
    assert st1["mic_classified"] == st1["segments"] > 0
    assert st0["mic_tests"] == st1["mic_tests"] and st0["mic_updates"] == st1["mic_updates"]
    assert same(es0, es1) and same(ef0, ef1)
    o = O.trace(sc, keep_paths=False)
    check_mics(o.e_strict, o.e_flag, es1, ef1)


def test_classes_used_only_when_they_cover_the_pass(torch_cuda):
    """Bound after emission (generation 0 unclassified), bound to another grid, or bound
    and accumulated into a subset of the bound grid: the pass reads stored classes only in
    the last case, and every result equals the unbound pass."""
    from paper_1912_03998_amd import bt
    from paper_1912_03998_amd.tracer import Session, scene_grid
    sc = block_scene(0).with_(level=4, depth=4)
    grid = scene_grid(sc)
    with Session.from_scene(sc) as s:
        mics = bt.bt_mics_grid(s.ctx, *grid)
        other = bt.bt_mics_grid(s.ctx, grid[0] + 1.0, *grid[1:])
        rng = np.random.default_rng(3)
        idx = np.sort(rng.choice(sc.n_mic, 2000, replace=False)).astype(np.int32)
        sub = bt.bt_mics_subset(s.ctx, mics, idx)
        say("block scene level 4: unbound")
        es0, ef0, st0 = manual_run(s, sc, mics)
        say("bound after emission")
        es1, ef1, st1 = manual_run(s, sc, mics, bind_after_emit=mics)
        say("bound to a shifted grid")
        es2, ef2, st2 = manual_run(s, sc, mics, bind=other)
        say("bound to the grid, accumulated into a subset of it")
        es3, ef3, st3 = manual_run(s, sc, sub, bind=mics, subset=len(idx))
        for m in (sub, other, mics):
            bt.bt_mics_free(m)
    assert st1["mic_classified"] == 0 and st2["mic_classified"] == 0
    assert st3["mic_classified"] == st3["segments"] > 0
    for es, ef, st in ((es1, ef1, st1), (es2, ef2, st2)):
        assert same(es0, es) and same(ef0, ef)
        assert st["mic_tests"] == st0["mic_tests"] and st["mic_updates"] == st0["mic_updates"]
    assert same(es0[idx], es3) and same(ef0[idx], ef3)


def test_sealed_box_every_beam_reflects(torch_cuda):
    """A sealed box around the source: every beam reflects at every generation (depth 7,
    so the queue holds 8 n0 segments), and the microphone plane inside is crossed from
    both sides.  Classified at creation or in the pass, resident or with two generation
    slots: the same tests, updates and energies, which meet the oracle."""
    from paper_1912_03998_amd import bt
    from paper_1912_03998_amd.tracer import Session, scene_grid
    from scenegen import sealed_box_scene
    sc = sealed_box_scene(level=3, depth=7)
    with Session.from_scene(sc) as s:
        mics = bt.bt_mics_grid(s.ctx, *scene_grid(sc))
        say("sealed box level 3 depth 7: unbound, then bound before emission")
        es0, ef0, st0 = manual_run(s, sc, mics)
        es1, ef1, st1 = manual_run(s, sc, mics, bind=mics)
        bt.bt_mics_free(mics)
        n0 = 20 * 4 ** sc.level
        assert list(st1["count"]) == [n0] * (sc.depth + 1)   # every beam reflects
        assert st1["mic_classified"] == st1["segments"] == (sc.depth + 1) * n0
        assert st0["mic_tests"] == st1["mic_tests"] > 0 and st0["mic_updates"] == st1["mic_updates"] > 0
        assert same(es0, es1) and same(ef0, ef1)
        for records in (0, 1):
            say("sealed box through bt_run, run_records", records)
            r = s.run(sc.sources, sc.power, sc.level, sc.depth, scene_grid(sc), run_records=records)
            assert r.stats["mic_classified"] == r.stats["segments"] == st0["segments"]
            assert r.stats["mic_tests"] == st0["mic_tests"] and r.stats["mic_updates"] == st0["mic_updates"]
            assert same(es0, r.e_strict) and same(ef0, r.e_flag)
    o = O.trace(sc, keep_paths=False)
    check_mics(o.e_strict, o.e_flag, es1, ef1)


def test_bt_run_classifies_district(torch_cuda):
    """bt_run binds its set to a planar grid: on the full district (64 sources, depth 8)
    every segment's class comes from its creation, in the resident layout and with two
    generation slots, and both equal the unbound pass."""
    from paper_1912_03998_amd import bt
    from paper_1912_03998_amd.tracer import Session, scene_grid
    sc = district_scene()
    with Session.from_scene(sc) as s:
        mics = bt.bt_mics_grid(s.ctx, *scene_grid(sc))
        say("district: unbound manual pass")
        es0, ef0, st0 = manual_run(s, sc, mics)
        bt.bt_mics_free(mics)
        for records in (0, 1 << 24):
            say("district through bt_run, run_records", records)
            r = s.run(sc.sources, sc.power, sc.level, sc.depth, scene_grid(sc), run_records=records)
            assert r.stats["mic_classified"] == r.stats["segments"] == st0["segments"]
            assert r.stats["mic_tests"] == st0["mic_tests"] and r.stats["mic_updates"] == st0["mic_updates"]
            assert same(es0, r.e_strict) and same(ef0, r.e_flag)


def test_bind_rejects_non_planar_sets(torch_cuda):
    """Explicit points and volumetric grids have no planar class: binding them is
    refused (BT_EINVAL) and leaves the set as it was; unbinding always succeeds."""
    from paper_1912_03998_amd import bt
    from paper_1912_03998_amd.tracer import Session, scene_grid
    sc = block_scene(0).with_(level=3, depth=2)
    with Session.from_scene(sc) as s:
        grid = bt.bt_mics_grid(s.ctx, *scene_grid(sc))
        pts = bt.bt_mics_points(s.ctx, np.array([[1.0, 2.0, 1.5], [3.0, -4.0, 2.0]], np.float32))
        vol = bt.bt_mics_grid3d(s.ctx, -98.0, -98.0, 1.5, 4.0, 4.0, 4.0, 50, 50, 4)
        beams = bt.bt_beams_bind_mics(s.ctx, None, grid)
        for m in (pts, vol):
            with pytest.raises(bt.BTError) as e:
                bt.bt_beams_bind_mics(s.ctx, beams, m)
            assert e.value.status == -1
        # still bound to the grid: a run classifies every segment
        p = s.params(sc.depth)
        beams = bt.bt_emit_beams(s.ctx, sc.sources, sc.power, sc.level, beams)
        for _ in range(sc.depth + 1):
            bt.bt_trace(s.ctx, s.mesh, beams, p)
        bt.bt_accumulate_mics(s.ctx, s.mesh, beams, p, grid)
        st = bt.bt_beams_stats(s.ctx, beams)
        assert st["mic_classified"] == st["segments"] > 0
        bt.bt_beams_bind_mics(s.ctx, beams, None)
        bt.bt_beams_free(beams)
        for m in (vol, pts, grid):
            bt.bt_mics_free(m)
