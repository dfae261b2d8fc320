"""The seeded batch and serving workloads on the district: sizes and distributions as
specified, every source on a street centre line, every microphone inside the grid."""
import numpy as np

from scenegen import batch_scenarios, serving_requests


def on_street(p):
    x, y = p[:, 0].astype(np.float64), p[:, 1].astype(np.float64)
    lx = np.abs((x + 1000.0) / 200.0 - np.round((x + 1000.0) / 200.0)) < 1e-4
    ly = np.abs((y + 1000.0) / 200.0 - np.round((y + 1000.0) / 200.0)) < 1e-4
    return (lx | ly) & (np.abs(x) <= 1000) & (np.abs(y) <= 1000) & (p[:, 2] == np.float32(0.5))


def test_batch_scenarios():
    b = batch_scenarios(0, 256)
    assert len(b) == 256
    ns = np.array([len(s.sources) for s in b])
    assert ns.min() >= 1 and ns.max() <= 64 and 10 < ns.mean() < 20      # E = 64 / ln 65 ~ 15.3
    assert {s.level for s in b} <= {3, 4, 5, 6} and len({s.level for s in b}) == 4
    d = np.array([s.depth for s in b])
    assert d.min() >= 2 and d.max() <= 10
    for s in b:
        assert on_street(s.sources).all()
        assert len(s.subset) == 10_000 and len(np.unique(s.subset)) == 10_000
        assert s.subset.min() >= 0 and s.subset.max() < 250_000
    total = sum(s.n_beams0 for s in b)
    assert 60e6 < total < 160e6
    assert batch_scenarios(0, 4)[2].subset.tolist() == batch_scenarios(0, 4)[2].subset.tolist()


def test_serving_requests():
    r = serving_requests(0, 2000, rate=200.0)
    t = np.array([q.arrival for q in r])
    assert t[0] == 0.0 and (np.diff(t) >= 0).all()
    assert abs(np.diff(t).mean() - 1 / 200.0) < 0.1 / 200.0
    for q in r:
        assert 1 <= len(q.sources) <= 32 and 3 <= q.depth <= 8 and q.level in (4, 5)
        assert on_street(q.sources).all()
        x0, y0, z, dx, dy, nx, ny = q.grid
        i0, j0 = (float(x0) + 998.0) / 4.0, (float(y0) + 998.0) / 4.0
        assert i0 == int(i0) and j0 == int(j0) and i0 + nx <= 500 and j0 + ny <= 500 and i0 >= 0 and j0 >= 0
    n = np.array([q.n_mic for q in r])
    assert n.min() >= 500 and n.max() <= 51_000 and 8_000 < n.mean() < 18_000
    beams = np.mean([q.n_beams0 for q in r])
    assert 80e3 < beams < 150e3                                              # ~111 k expected
