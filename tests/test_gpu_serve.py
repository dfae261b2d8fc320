"""GPU request server: every request's result is the same alone (bt_run) and in the mix of
a continuously batched server, whatever arrives while it runs, across session changes,
and in the plain one-at-a-time mode.  Every test prints its case before touching the GPU."""
import sys
import time

import numpy as np
import pytest

from oracle import oracle as O
from scenegen import block_scene, district_scene, serving_requests
from tests.parity_check import check_mics
from tests.test_gpu_batch import alone, assert_same, make_scenarios

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def session():
    from paper_1912_03998_amd.tracer import Session
    return Session.from_scene(block_scene(0))


def wait_all(srv, tickets, timeout=60.0):
    out = {}
    t_end = time.time() + timeout
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() < t_end, "requests did not finish"
        time.sleep(0.0005)
    return out


def expected(s, scs):
    return [alone(s, sc)[:2] for sc in scs]


@pytest.mark.parametrize("mode", [0, 1])
def test_served_equals_alone(torch_cuda, mode):
    """All requests submitted at once: each result equals the request run alone."""
    from paper_1912_03998_amd import bt
    say("served at once, mode", mode)
    with session() as s:
        want = expected(s, make_scenarios(seed=5, n=14))
        scs = make_scenarios(seed=5, n=14)
        with bt.Server(s.ctx, s.mesh, mode=mode) as srv:
            tickets = [srv.submit(sc) for sc in scs]
            res = wait_all(srv, tickets)
        for sc, (e, f) in zip(scs, want):
            assert_same(sc.energy, e)
            assert_same(sc.flag, f)
        for t in tickets:
            t_sub, t_adm, t_done = res[t]
            assert 0 <= t_sub <= t_adm <= t_done


def test_continuous_batching_mix(torch_cuda):
    """Requests arriving while others are on the GPU join them (their admission falls
    inside earlier requests' lifetimes) and still get their alone results."""
    from paper_1912_03998_amd import bt
    say("served with staggered arrivals")
    with session() as s:
        want = expected(s, make_scenarios(seed=6, n=21))
        scs = make_scenarios(seed=6, n=21)
        with bt.Server(s.ctx, s.mesh) as srv:
            tickets = []
            for k, sc in enumerate(scs):
                tickets.append(srv.submit(sc))
                time.sleep(0.0003 * (k % 4))
            res = wait_all(srv, tickets)
        for sc, (e, f) in zip(scs, want):
            assert_same(sc.energy, e)
            assert_same(sc.flag, f)
        spans = [res[t] for t in tickets]
        overlapped = sum(1 for i in range(1, len(spans))
                         if any(spans[j][1] <= spans[i][1] < spans[j][2] for j in range(i)))
        assert overlapped >= 1


def test_session_rotation(torch_cuda):
    """Small sessions force closing, draining and reopening sessions many times."""
    from paper_1912_03998_amd import bt
    say("served with small sessions")
    with session() as s:
        scs0 = make_scenarios(seed=7, n=28)
        want = expected(s, scs0)
        biggest = max(len(sc.src) * 20 * 4 ** sc.level * (sc.max_depth + 1) for sc in scs0)
        scs = make_scenarios(seed=7, n=28)
        with bt.Server(s.ctx, s.mesh, max_records=max(biggest, 2 * 20 * 4 ** 4), arena_bytes=1 << 22) as srv:
            tickets = [srv.submit(sc) for sc in scs]
            wait_all(srv, tickets)
        for sc, (e, f) in zip(scs, want):
            assert_same(sc.energy, e)
            assert_same(sc.flag, f)


def test_server_errors(torch_cuda):
    from paper_1912_03998_amd import bt
    say("server errors")
    with session() as s:
        with bt.Server(s.ctx, s.mesh, max_records=1000) as srv:
            big = make_scenarios(seed=8, n=1)[0]
            big.level = 4
            with pytest.raises(bt.BTError) as e:
                srv.submit(big)
            assert e.value.status == -2
            bad = make_scenarios(seed=8, n=1)[0]
            bad.max_depth = 99
            with pytest.raises(bt.BTError) as e:
                srv.submit(bad)
            assert e.value.status == -1
            with pytest.raises(bt.BTError) as e:
                srv.poll(12345)
            assert e.value.status == -5
        with pytest.raises(bt.BTError):
            bt.Server(s.ctx, s.mesh, mode=7)


def test_district_stream_sampled_against_oracle(torch_cuda):
    """The serving workload on the district at 800 requests/s (300 requests submitted at
    their Poisson arrival times, continuously batched): 20 requests (the cheapest, the
    median, the costliest and 17 drawn at random) checked against the oracle over their
    microphone rectangles."""
    from paper_1912_03998_amd import bt
    from paper_1912_03998_amd.tracer import Session
    base = district_scene(0)
    reqs = serving_requests(0, n=300, rate=800.0)
    say("district stream: 300 requests at 800 req/s")
    with Session.from_scene(base) as s:
        scs = [bt.Scenario(q.sources, q.power, q.level, q.depth, q.grid) for q in reqs]
        with bt.Server(s.ctx, s.mesh) as srv:
            tickets = []
            t0 = time.perf_counter()
            for q, sc in zip(reqs, scs):
                while time.perf_counter() - t0 < q.arrival:
                    time.sleep(0.0001)
                tickets.append(srv.submit(sc))
            wait_all(srv, tickets, timeout=120.0)
    cost = [q.n_beams0 * (q.depth + 1) for q in reqs]
    order = sorted(range(len(reqs)), key=lambda k: cost[k])
    picks = [order[0], order[len(order) // 2], order[-1]]
    rest = [k for k in range(len(reqs)) if k not in picks]
    picks += sorted(np.random.default_rng(6).choice(rest, 17, replace=False).tolist())
    for k in picks:
        q = reqs[k]
        say("oracle for request", k, len(q.sources), "sources, level", q.level, "depth", q.depth,
            "mics", q.grid[5], "x", q.grid[6])
        x0, y0, z, dx, dy, nx, ny = q.grid
        o = O.trace(base.with_(sources=q.sources, power=q.power, level=q.level, depth=q.depth, mic_x0=x0, mic_y0=y0,
                               mic_z=z, mic_dx=dx, mic_dy=dy, mic_nx=nx, mic_ny=ny), keep_paths=False)
        sc = scs[k]
        check_mics(o.e_strict, o.e_flag, sc.energy - sc.flag, sc.flag)
