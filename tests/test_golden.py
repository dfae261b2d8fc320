"""Stored oracle results (tests/golden/*.txt, written from the oracle alone by
tests/golden/write_golden.py) against the oracle as it stands (CPU) and against the HIP
path through the C ABI (GPU, with the parity contract of tests/parity_check.py).

The paper prints no worked example, so these fixtures are the oracle's own results on
three small scenes (paper Section 2: beams, one specular child per hit, contributions
inside each frustum; Section 4: a regular microphone grid).  The CPU test catches any
change of the oracle's results; the GPU test compares the HIP path with them."""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from tests.golden.write_golden import cases
from tests.parity_check import check_counts, check_mics

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
NAMES = [name for name, _ in cases()]


def load(name):
    out = {}
    with open(os.path.join(HERE, name + ".txt")) as f:
        lines = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    k = 0
    while lines[k][0] != "mics":
        key, vals = lines[k][0], lines[k][1:]
        out[key] = np.array([float(v) if key == "power" else int(v) for v in vals])
        k += 1
    n = int(lines[k][1])
    rows = lines[k + 1:k + 1 + n]
    assert [int(r[0]) for r in rows] == list(range(n))
    out["e_strict"] = np.array([float(r[1]) for r in rows])
    out["e_flag"] = np.array([float(r[2]) for r in rows])
    return out


@pytest.mark.parametrize("name", NAMES)
def test_oracle_reproduces_golden(name):
    """The oracle's counts and counters equal the stored ones; its power sums and
    energies agree to 1e-12 relative (the order of its FP64 additions may change with
    the thread count)."""
    sc = dict(cases())[name]
    g = load(name)
    r = O.trace(sc, keep_paths=False)
    assert np.array_equal(r.count, g["count"]) and np.array_equal(r.flagged, g["flagged"])
    for k in ("segments", "hits", "children", "mic_updates"):
        assert r.counters[k] == int(g[k][0]), k
    assert np.allclose(r.power, g["power"], rtol=1e-12, atol=0.0)
    scale = max(np.abs(g["e_strict"] + g["e_flag"]).max(), 1e-300)
    assert np.abs(r.e_strict - g["e_strict"]).max() <= 1e-12 * scale
    assert np.abs(r.e_flag - g["e_flag"]).max() <= 1e-12 * scale


@pytest.mark.gpu
@pytest.mark.parametrize("name", NAMES)
def test_hip_path_meets_golden(name):
    """The HIP path (bt_run through the C ABI) against the stored results: per-generation
    counts and flags, the segment and update totals, and every microphone under the
    parity contract."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1912_03998_amd.tracer import Session, scene_grid
    sc = dict(cases())[name]
    g = load(name)
    print("[case] golden", name, file=sys.stderr, flush=True)
    with Session.from_scene(sc) as s:
        r = s.run(sc.sources, sc.power, sc.level, sc.depth, scene_grid(sc))
    check_counts(g["count"], g["flagged"], r.stats["count"], r.stats["flagged"], diverged=False)
    assert r.stats["segments"] == int(g["segments"][0])
    assert r.stats["mic_updates"] == int(g["mic_updates"][0])
    assert np.allclose(r.stats["power"], g["power"], rtol=1e-9, atol=0.0)
    check_mics(g["e_strict"], g["e_flag"], r.e_strict, r.e_flag)
