"""Write the stored oracle results under tests/golden/ (run from the repository root:
`python tests/golden/write_golden.py`).

The paper prints no worked example: no value of a beam, a hit or a microphone level for a
stated input.  The fixtures here are therefore the FP64 oracle's own results on three
small synthetic scenes, written by this script, which calls nothing but the oracle.  The
oracle itself is pinned by closed forms and invariants (tests/test_oracle_pins.py); the
fixtures freeze its results so that a later change to its arithmetic shows up as a
changed fixture, and they give the GPU tests expected values that need no oracle run.

What each fixture holds (paper Section 2: beams from point sources, one specular child
per hit that loses energy at the surface, contributions of every beam to the microphones
inside its frustum; Section 4: microphones on a regular grid):
  per generation: segments, flagged segments, power carried by the generation's beams;
  totals: segments, hits, children, microphone updates;
  per microphone (row-major over the grid): strict and flag energy (W/m^2).
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from scenegen import corner_scene, sealed_box_scene, tiny_scene  # noqa: E402


def cases():
    """(fixture name, scene): small enough for a stored text file."""
    return [("tiny", tiny_scene()),
            ("sealed_box", sealed_box_scene(level=2, depth=4)),
            ("corner", corner_scene(level=4, depth=3))]


def write(name, sc):
    r = O.trace(sc, keep_paths=False, n_threads=1)
    path = os.path.join(HERE, name + ".txt")
    with open(path, "w") as f:
        f.write(f"# oracle results for scene {sc.name}: level {sc.level}, depth {sc.depth}, "
                f"t_min {O.T_MIN}, delta {O.DELTA}, no air absorption, no energy threshold\n")
        f.write("# written by tests/golden/write_golden.py (oracle only)\n")
        f.write("count " + " ".join(str(int(x)) for x in r.count) + "\n")
        f.write("flagged " + " ".join(str(int(x)) for x in r.flagged) + "\n")
        f.write("power " + " ".join(repr(float(x)) for x in r.power) + "\n")
        for k in ("segments", "hits", "children", "mic_updates"):
            f.write(f"{k} {r.counters[k]}\n")
        f.write(f"mics {sc.n_mic}\n")
        for i in range(sc.n_mic):
            f.write(f"{i} {float(r.e_strict[i])!r} {float(r.e_flag[i])!r}\n")
    return path


if __name__ == "__main__":
    O.build(force=False)
    for name, sc in cases():
        print(write(name, sc))
