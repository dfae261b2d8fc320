"""The allocation-free microphone pass (bt_accumulate_mics_static) against the allocating
one (bt_accumulate_mics) and the oracle, through the C ABI.

Both passes run the same kernels; only where their work lists live differs (a static
device array against the beam set's buffers), so the energies agree up to the order of
FP64 atomic additions.  Consecutive calls share the static array, so the second call
with a smaller input must not see the first one's leftovers.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from scenegen import block_scene, district_scene, tiny_scene
from tests.parity_check import check_mics

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def run_pass(s, sc, static, every_generation=False):
    """Emit, trace every generation, accumulate (after each generation or once at the
    end) with the chosen entry point; returns strict and flag energies and the stats."""
    from paper_1912_03998_amd import bt
    from paper_1912_03998_amd.tracer import grid_size, scene_grid
    grid = scene_grid(sc)
    mics = bt.bt_mics_grid(s.ctx, *grid) if len(grid) == 7 else bt.bt_mics_grid3d(s.ctx, *grid)
    acc = bt.bt_accumulate_mics_static if static else bt.bt_accumulate_mics
    p = s.params(sc.depth)
    s.beams = bt.bt_emit_beams(s.ctx, sc.sources, sc.power, sc.level, s.beams)
    for _ in range(sc.depth + 1):
        bt.bt_trace(s.ctx, s.mesh, s.beams, p)
        if every_generation:
            acc(s.ctx, s.mesh, s.beams, p, mics)
    acc(s.ctx, s.mesh, s.beams, p, mics)
    n = grid_size(grid)
    es, ef = np.zeros(n), np.zeros(n)
    bt.bt_levels(s.ctx, mics, es, ef, None)
    st = bt.bt_beams_stats(s.ctx, s.beams)
    bt.bt_mics_free(mics)
    return es, ef, st


def same(a, b):
    scale = max(np.abs(a).max(), 1e-300)
    return np.abs(a - b).max() <= 1e-12 * scale


def test_static_pass_two_calls_then_smaller(torch_cuda):
    """Block scene at level 5, then a smaller input (level 3, depth 3, a quarter of the
    grid) on the same context: each equals the allocating pass and meets the parity
    contract against the oracle."""
    from paper_1912_03998_amd.tracer import Session
    big = block_scene(0)
    small = big.with_(level=3, depth=3, mic_nx=50, mic_ny=50)
    with Session.from_scene(big) as s:
        for sc in (big, small):
            say("static pass vs allocating pass, level", sc.level, "depth", sc.depth, "mics", sc.n_mic)
            es0, ef0, st0 = run_pass(s, sc, static=False)
            es1, ef1, st1 = run_pass(s, sc, static=True)
            assert same(es0, es1) and same(ef0, ef1)
            assert st0["mic_updates"] == st1["mic_updates"] and st0["mic_tests"] == st1["mic_tests"]
            o = O.trace(sc, keep_paths=False)
            check_mics(o.e_strict, o.e_flag, es1, ef1)


def test_static_pass_volumetric(torch_cuda):
    """A volumetric grid (the (segment, layer) items live in the static array too)."""
    from paper_1912_03998_amd.tracer import Session
    sc = tiny_scene().with_(mic_z=-2.5, mic_nz=12, mic_dz=2.5)
    with Session.from_scene(sc) as s:
        say("static pass, volumetric tiny scene")
        es0, ef0, _ = run_pass(s, sc, static=False)
        es1, ef1, _ = run_pass(s, sc, static=True)
    assert same(es0, es1) and same(ef0, ef1)
    o = O.trace(sc, keep_paths=False)
    check_mics(o.e_strict, o.e_flag, es1, ef1)


def test_static_pass_limit_and_district_per_generation(torch_cuda):
    """The full district (5,242,880 generation-0 beams, 9 generations): one pass over
    every generation exceeds the static array and is refused with nothing enqueued;
    a pass after every generation fits and equals the allocating single pass."""
    from paper_1912_03998_amd import bt
    from paper_1912_03998_amd.tracer import Session, scene_grid
    sc = district_scene(0)
    with Session.from_scene(sc) as s:
        say("static pass, district, refused when too large")
        mics = bt.bt_mics_grid(s.ctx, *scene_grid(sc))
        p = s.params(sc.depth)
        s.beams = bt.bt_emit_beams(s.ctx, sc.sources, sc.power, sc.level, s.beams)
        for _ in range(sc.depth + 1):
            bt.bt_trace(s.ctx, s.mesh, s.beams, p)
        with pytest.raises(bt.BTError) as e:
            bt.bt_accumulate_mics_static(s.ctx, s.mesh, s.beams, p, mics)
        assert e.value.status == -1
        bt.bt_mics_free(mics)
        say("static pass, district, every generation")
        es0, ef0, st0 = run_pass(s, sc, static=False)
        es1, ef1, st1 = run_pass(s, sc, static=True, every_generation=True)
    assert same(es0, es1) and same(ef0, ef1)
    assert st0["mic_updates"] == st1["mic_updates"]
