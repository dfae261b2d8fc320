"""Write the oracle's work counts for the plain-method workloads (test/benchmark data).

The benchmark's algorithmic-byte numerator is fixed by the oracle's reference
traversal (binary binned-SAH hierarchy, nearer child first, closest-hit pruning), so
that a better or worse GPU hierarchy cannot change it.  This script runs only the
oracle and writes reference_work.json next to itself.

    python oracle/reference_work.py [--configs 0 1 2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import oracle as O  # noqa: E402
from scenegen import config_scene  # noqa: E402

OUT = os.path.join(HERE, "reference_work.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", type=int, nargs="+", default=[0, 1, 2])
    args = ap.parse_args()
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for c in args.configs:
        sc = config_scene(c)
        t0 = time.time()
        r = O.trace(sc, keep_paths=False)
        dt = time.time() - t0
        data[sc.name] = {
            "config": c, "n_tri": sc.n_tri, "n_src": sc.n_src, "level": sc.level, "depth": sc.depth,
            "n_mic": sc.n_mic, "count": r.count.tolist(), "flagged": r.flagged.tolist(),
            "power": r.power.tolist(), **r.counters,
            "oracle_seconds": round(dt, 3), "oracle_threads": O.default_threads(),
        }
        print(sc.name, json.dumps(data[sc.name]), flush=True)
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
