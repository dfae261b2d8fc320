"""The oracle's pins catch plausible mistakes: each case below plants one mistake in a
copy of the oracle's source (on the CPU, in a temporary directory), builds it, runs the
pin that should notice it, and expects that pin to fail.  The oracle itself is not
touched.

Mistakes planted: the reflecting plane's offset dropped from the mirrored apex, from
the near cap, from the far cap or from the far cap's footprint on the microphone plane
(Section 2: a reflection mirrors the beam in the surface; only planes through the
origin hide these); the energy threshold compared before absorption (Section 2: a beam loses energy when it reflects, and weak beams are
deleted); the edge directions mirrored without restoring their orientation; the child
placed on the wrong side of its reflector.
"""
import os

import pytest

from oracle import oracle as O
from tests import test_oracle_pins as P

SRC = os.path.join(os.path.dirname(O.__file__), "bt_oracle.c")

MUTATIONS = {
    "apex mirror without the plane offset": (
        "v_sub(bm->A, P, q);", "v_copy(bm->A, q);",
        [lambda: P.pin_ground_off_origin(3.7), lambda: P.pin_wall_off_origin(),
         lambda: P.pin_corner_second_order()]),
    "near cap without the plane offset": (
        "v_sub(m, f->Pn, q);", "v_copy(m, q);",
        [lambda: P.pin_ground_off_origin(3.7)]),
    "far cap without the plane offset": (
        "v_sub(m, f->Pf, q);", "v_copy(m, q);",
        [lambda: P.pin_ground_off_origin(3.7), lambda: P.pin_ground_off_origin(-4.2),
         lambda: P.pin_wall_off_origin()]),
    "far cap footprint without the plane offset": (
        "hp[nh++] = make_hplane(g, f->Pf, z, eps);", "hp[nh++] = make_hplane(g, (double[3]){0, 0, 0}, z, eps);",
        [lambda: P.pin_ground_off_origin(-4.2), lambda: P.pin_wall_off_origin()]),
    "threshold before absorption": (
        "bm.K * bm.omega * (1.0 - (double)s->alpha[hr.hit]) <= p->e_min",
        "bm.K * bm.omega <= p->e_min",
        [lambda: P.pin_threshold_generation(1e-9), lambda: P.pin_threshold_generation(-1e-9)]),
    "mirrored edges keep the parent's order": (
        "mirror_dir(bm->d[2], n, ch->d[1]);\n    mirror_dir(bm->d[1], n, ch->d[2]);",
        "mirror_dir(bm->d[1], n, ch->d[1]);\n    mirror_dir(bm->d[2], n, ch->d[2]);",
        [lambda: P.pin_wall_off_origin(), lambda: P.pin_corner_second_order()]),
    "child on the wrong side of its reflector": (
        "ch->near_sign = v_dot(bm->c, N) > 0.0 ? -1 : 1;",
        "ch->near_sign = v_dot(bm->c, N) > 0.0 ? 1 : -1;",
        [lambda: P.pin_ground_off_origin(-4.2), lambda: P.pin_corner_second_order()]),
}


@pytest.fixture(scope="module")
def oracle_source():
    with open(SRC) as f:
        return f.read()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, oracle_source, tmp_path, monkeypatch):
    find, replace, pins = MUTATIONS[name]
    assert oracle_source.count(find) == 1, f"mutation site not unique: {find!r}"
    mutant = tmp_path / "mutant.c"
    mutant.write_text(oracle_source.replace(find, replace))
    lib = O.load(O.compile_to(str(mutant), str(tmp_path / "libmutant.so")))
    monkeypatch.setattr(O, "_lib", lib)
    for pin in pins:
        with pytest.raises(AssertionError):
            pin()
    # and the unbroken oracle passes the same pins
    monkeypatch.setattr(O, "_lib", None)
    for pin in pins:
        pin()
