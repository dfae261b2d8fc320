"""GPU batches of independent scenarios: each scenario's energies in a batch equal those of
the same scenario run alone, whatever the chunking, with or without a captured graph, and
the oracle's.  Every test prints its case before touching the GPU."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from scenegen import batch_scenarios, block_scene, district_scene
from tests.parity_check import check_mics

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def make_scenarios(seed=1, n=7):
    """Uneven scenarios on the block scene: 0-3 sources inside the building-free disc around
    the origin, levels 1-4, depths 0-6, sub-rectangles of the 2 m microphone grid, some with
    a random subset of their grid."""
    from paper_1912_03998_amd import bt
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        ns = [1, 2, 3, 0, 1, 2, 3][k % 7]
        ang = rng.uniform(0, 2 * np.pi, ns)
        rad = rng.uniform(0.5, 5.0, ns)
        src = np.stack([rad * np.cos(ang), rad * np.sin(ang), rng.uniform(0.5, 2.0, ns)], 1).astype(np.float32)
        pw = rng.uniform(0.5, 2.0, ns).astype(np.float32)
        nx, ny = int(rng.integers(10, 60)), int(rng.integers(10, 60))
        i0, j0 = int(rng.integers(0, 100 - nx)), int(rng.integers(0, 100 - ny))
        grid = (np.float32(-99 + 2 * i0), np.float32(-99 + 2 * j0), np.float32(1.5), np.float32(2.0), np.float32(2.0),
                nx, ny)
        subset = None
        if k % 3 == 1:
            subset = rng.choice(nx * ny, size=max(1, nx * ny // 5), replace=True).astype(np.int32)
        out.append(bt.Scenario(src, pw, int(rng.integers(1, 5)), int(rng.integers(0, 7)), grid, subset))
    return out


def alone(s, sc):
    """The scenario run by itself with bt_run: (strict + flag, flag) over its outputs."""
    g = tuple(float(v) for v in sc.grid[:5]) + tuple(int(v) for v in sc.grid[5:])
    r = s.run(sc.src, sc.power, sc.level, sc.max_depth, g, parity=False)
    e, f = r.e_strict + r.e_flag, r.e_flag
    if sc.subset is not None:
        e, f = e[sc.subset], f[sc.subset]
    return e, f, r.stats["segments"]


def assert_same(a, b, rel=1e-12):
    scale = max(float(np.abs(b).max()), 1e-300)
    assert np.abs(a - b).max() <= rel * scale, (np.abs(a - b).max(), scale)


def session():
    from paper_1912_03998_amd.tracer import Session
    sc = block_scene(0)
    return Session.from_scene(sc)


def test_batch_equals_scenarios_alone(torch_cuda):
    from paper_1912_03998_amd import bt
    say("batch vs alone, one chunk")
    scs = make_scenarios()
    with session() as s:
        st = bt.bt_batch_run(s.ctx, s.mesh, scs)
        assert st["chunks"] == 1
        total = 0
        for sc in scs:
            e, f, segs = alone(s, sc)
            assert_same(sc.energy, e)
            assert_same(sc.flag, f)
            total += segs
        assert st["beams0"] == sum(len(sc.src) * 20 * 4 ** sc.level for sc in scs)
        assert st["segments"] == total


@pytest.mark.parametrize("k", [0, 2, 5])
def test_batch_scenario_matches_oracle(torch_cuda, k):
    from paper_1912_03998_amd import bt
    say("batch vs oracle, scenario", k)
    scs = make_scenarios()
    base = block_scene(0)
    sc = scs[k]
    x0, y0, z, dx, dy, nx, ny = sc.grid
    o = O.trace(base.with_(sources=sc.src, power=sc.power, level=sc.level, depth=sc.max_depth, mic_x0=x0, mic_y0=y0,
                           mic_z=z, mic_dx=dx, mic_dy=dy, mic_nx=nx, mic_ny=ny))
    with session() as s:
        bt.bt_batch_run(s.ctx, s.mesh, scs)
    es, ef = o.e_strict, o.e_flag
    if sc.subset is not None:
        es, ef = es[sc.subset], ef[sc.subset]
    check_mics(es, ef, sc.energy - sc.flag, sc.flag)


@pytest.mark.parametrize("use_graph", [0, 1])
def test_batch_chunking_and_graph(torch_cuda, use_graph):
    """Small chunks (several per batch, so a captured graph is replayed for each, with host
    work and synchronisation between replays) give the one-chunk results; a second call
    gives them again."""
    from paper_1912_03998_amd import bt
    say("batch chunks, graph", use_graph)
    ref = make_scenarios()
    with session() as s:
        bt.bt_batch_run(s.ctx, s.mesh, ref)
        for rep in range(2):
            scs = make_scenarios()
            st = bt.bt_batch_run(s.ctx, s.mesh, scs, opts={"chunk_beams": 6000, "blocks_per_cu": 4,
                                                           "use_graph": use_graph})
            assert st["chunks"] >= 3
            for a, b in zip(scs, ref):
                assert_same(a.energy, b.energy)
                assert_same(a.flag, b.flag)


@pytest.mark.parametrize("env,value", [("BT_MIC_ROW_CAPACITY", "40"), ("BT_MIC_SPAN_CAPACITY", "20")])
def test_batch_mic_work_overflow(torch_cuda, monkeypatch, env, value):
    """Scenario sets use the planar row, span and one-wave-per-segment kernels of the
    microphone stage: tiny row and span buffers push wide footprints onto the one-wave path
    and long rows onto in-place processing; every scenario keeps its result."""
    from paper_1912_03998_amd import bt
    say("batch mic work overflow", env, value)
    ref = make_scenarios()
    with session() as s:
        bt.bt_batch_run(s.ctx, s.mesh, ref)
    monkeypatch.setenv(env, value)
    scs = make_scenarios()
    with session() as s:
        bt.bt_batch_run(s.ctx, s.mesh, scs)
    for a, b in zip(scs, ref):
        assert_same(a.energy, b.energy)
        assert_same(a.flag, b.flag)


def test_batch_rejects_bad_scenarios(torch_cuda):
    from paper_1912_03998_amd import bt
    say("batch validation")
    with session() as s:
        good = make_scenarios(n=2)
        bad = make_scenarios(n=2)
        bad[1].max_depth = 40
        with pytest.raises(bt.BTError) as e:
            bt.bt_batch_run(s.ctx, s.mesh, bad)
        assert e.value.status == -1
        bad = make_scenarios(n=2)
        bad[0].subset = np.array([0, 10 ** 7], np.int32)
        bad[0].energy = np.zeros(2)
        bad[0].flag = np.zeros(2)
        with pytest.raises(bt.BTError):
            bt.bt_batch_run(s.ctx, s.mesh, bad)
        bad = make_scenarios(n=2)
        bad[0].src = np.array([[1e6, 0, 1]], np.float32)
        bad[0].power = np.ones(1, np.float32)
        with pytest.raises(bt.BTError):
            bt.bt_batch_run(s.ctx, s.mesh, bad)
        with pytest.raises(bt.BTError):
            bt.bt_batch_run(s.ctx, s.mesh, good, opts={"chunk_beams": -1, "blocks_per_cu": 0, "use_graph": 0})
        st = bt.bt_batch_run(s.ctx, s.mesh, [])
        assert st["chunks"] == 0


def test_batch_autotune(torch_cuda):
    from paper_1912_03998_amd import bt
    say("batch autotune")
    scs = make_scenarios(seed=3, n=14)
    with session() as s:
        opts, secs = bt.bt_batch_autotune(s.ctx, s.mesh, scs)
        assert opts["chunk_beams"] > 0 and opts["blocks_per_cu"] in (4, 8) and opts["use_graph"] in (0, 1)
        assert len(secs) >= 4 and all(t > 0 for t in secs)
        ref = make_scenarios(seed=3, n=14)
        bt.bt_batch_run(s.ctx, s.mesh, ref)
        bt.bt_batch_run(s.ctx, s.mesh, scs, opts=opts)
        for a, b in zip(scs, ref):
            assert_same(a.energy, b.energy)


def test_full_batch_workload_sampled_against_oracle(torch_cuda):
    """The batched workload at full size (256 district scenarios, 96.7 M generation-0
    beams, several chunks): 24 scenarios, the three cheapest, the one with the most
    sources and 20 drawn at random over every chunk, checked against the oracle over
    their microphone subsets."""
    from paper_1912_03998_amd import bt
    from paper_1912_03998_amd.tracer import Session
    base = district_scene(0)
    specs = batch_scenarios(0, 256)
    say("full batch workload:", sum(q.n_beams0 for q in specs), "generation-0 beams")
    with Session.from_scene(base) as s:
        scs = [bt.Scenario(q.sources, q.power, q.level, q.depth, q.grid, q.subset) for q in specs]
        st = bt.bt_batch_run(s.ctx, s.mesh, scs)
    assert st["beams0"] == sum(q.n_beams0 for q in specs) and st["chunks"] > 1
    cost = [q.n_beams0 * (q.depth + 1) for q in specs]
    picks = sorted(range(len(specs)), key=lambda k: cost[k])[:3]
    picks.append(max(range(len(specs)), key=lambda k: (len(specs[k].sources), -cost[k])))
    rest = [k for k in range(len(specs)) if k not in picks]
    picks += sorted(np.random.default_rng(5).choice(rest, 20, replace=False).tolist())
    for k in picks:
        q = specs[k]
        say("oracle for scenario", k, len(q.sources), "sources, level", q.level, "depth", q.depth)
        x0, y0, z, dx, dy, nx, ny = q.grid
        o = O.trace(base.with_(sources=q.sources, power=q.power, level=q.level, depth=q.depth, mic_x0=x0, mic_y0=y0,
                               mic_z=z, mic_dx=dx, mic_dy=dy, mic_nx=nx, mic_ny=ny), keep_paths=False)
        sc = scs[k]
        check_mics(o.e_strict[q.subset], o.e_flag[q.subset], sc.energy - sc.flag, sc.flag)
