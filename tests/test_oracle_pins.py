"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Closed forms (direct path, image source, sealed box power), textbook geometry
(icosahedron, solid angles), brute force on tiny inputs (an independent numpy
linear solve for ray/triangle hits, all-microphone membership), and invariants
(energy bookkeeping, mirror symmetry).  A plausible mistake in the oracle (a
dropped term, a wrong sign or index, a transposed operand) fails one of these.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from scenegen import (block_scene, corner_scene, district_scene, empty_scene, ground_scene, mirror_scene,
                      sealed_box_scene, tiny_scene, wall_scene)
from tests import closed_forms as CF

FOUR_PI = 4.0 * math.pi


# ----------------------------------------------------------------------------
# Icosphere (beam directions)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("level", range(0, 6))
def test_icosphere_counts_orientation_unit(level):
    d = O.icosphere(level)
    assert d.shape == (20 * 4 ** level, 3, 3)
    norms = np.linalg.norm(d, axis=2)
    assert np.abs(norms - 1.0).max() < 4e-16
    det = np.einsum("fi,fi->f", d[:, 0], np.cross(d[:, 1], d[:, 2]))
    assert (det > 0).all()


@pytest.mark.parametrize("level", range(0, 5))
def test_icosphere_closed_oriented_surface(level):
    """Every directed edge appears once and its reverse once: a closed, consistently
    oriented triangulation of the sphere (V - E + F = 2), with shared vertices bit-identical."""
    d = O.icosphere(level)
    keys = {}
    faces = []
    for f in range(d.shape[0]):
        ids = []
        for k in range(3):
            key = d[f, k].tobytes()
            ids.append(keys.setdefault(key, len(keys)))
        faces.append(ids)
    edges = {}
    for (a, b, c) in faces:
        for (u, v) in ((a, b), (b, c), (c, a)):
            edges[(u, v)] = edges.get((u, v), 0) + 1
    assert all(n == 1 for n in edges.values())
    assert all((v, u) in edges for (u, v) in edges)
    V, E, F = len(keys), len(edges) // 2, len(faces)
    assert V - E + F == 2
    assert V == 10 * 4 ** level + 2


def test_icosahedron_textbook_geometry():
    """Level 0 is the regular icosahedron inscribed in the unit sphere: 12 vertices, each
    of degree 5, edge length 4 / sqrt(10 + 2 sqrt 5)."""
    d = O.icosphere(0)
    verts = np.unique(d.reshape(-1, 3), axis=0)
    assert verts.shape[0] == 12
    edge = 4.0 / math.sqrt(10.0 + 2.0 * math.sqrt(5.0))
    for f in range(20):
        for k in range(3):
            assert abs(np.linalg.norm(d[f, k] - d[f, (k + 1) % 3]) - edge) < 1e-14
    deg = [sum(1 for f in range(20) if any((d[f, k] == v).all() for k in range(3))) for v in verts]
    assert deg == [5] * 12


def test_solid_angle_closed_forms():
    ex, ey, ez = np.eye(3)
    assert abs(O.solid_angle(ex, ey, ez) - math.pi / 2) < 1e-15  # one octant
    # a thin cone: area / r^2 of a small flat triangle at unit distance
    e = 1e-4
    a, b, c = np.array([0, 0, 1.0]), np.array([e, 0, 1.0]), np.array([0, e, 1.0])
    a, b, c = (v / np.linalg.norm(v) for v in (a, b, c))
    assert abs(O.solid_angle(a, b, c) / (0.5 * e * e) - 1) < 1e-3


@pytest.mark.parametrize("level", range(0, 6))
def test_solid_angles_tile_the_sphere(level):
    d = O.icosphere(level)
    om = np.array([O.solid_angle(*d[f]) for f in range(d.shape[0])]) if level < 5 else None
    if om is None:
        # vectorised Van Oosterom-Strackee for the big level (independent of the oracle's C)
        num = np.abs(np.einsum("fi,fi->f", d[:, 0], np.cross(d[:, 1], d[:, 2])))
        den = 1 + np.einsum("fi,fi->f", d[:, 0], d[:, 1]) + np.einsum("fi,fi->f", d[:, 1], d[:, 2]) \
            + np.einsum("fi,fi->f", d[:, 2], d[:, 0])
        om = 2 * np.arctan2(num, den)
    assert abs(om.sum() - FOUR_PI) < 1e-12
    if level >= 5:
        ratio = om.max() / om.min()
        assert 1.25 < ratio < 1.35


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_icosphere_mirror_symmetric(axis):
    d = O.icosphere(3)
    c = d.sum(axis=1)
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    m = c.copy()
    m[:, axis] *= -1
    a = np.round(c, 12)
    b = np.round(m, 12)
    a = a[np.lexsort(a.T[::-1])]
    b = b[np.lexsort(b.T[::-1])]
    assert np.abs(a - b).max() < 1e-11


# ----------------------------------------------------------------------------
# Closest hit: brute force vs BVH vs an independent linear solve
# ----------------------------------------------------------------------------

def _random_soup(seed, n_tri=150, span=20.0):
    rng = np.random.default_rng(seed)
    cen = rng.uniform(-span, span, size=(n_tri, 3))
    v = (cen[:, None, :] + rng.normal(scale=2.0, size=(n_tri, 3, 3))).reshape(-1, 3).astype(np.float32)
    t = np.arange(3 * n_tri, dtype=np.int32).reshape(-1, 3)
    sc = empty_scene().with_(vertices=v, triangles=t, absorption=np.full(n_tri, 0.1, np.float32))
    return sc


def _solve_hits(scene, o, c, start, t_min):
    """Independent closest hit: solve o + t c = v0 + u e1 + v e2 with numpy per triangle."""
    V = scene.vertices.astype(np.float64)
    T = scene.triangles
    best_t, best = np.inf, -1
    for k in range(T.shape[0]):
        if k == start:
            continue
        v0, v1, v2 = V[T[k]]
        M = np.stack([-c, v1 - v0, v2 - v0], axis=1)
        if abs(np.linalg.det(M)) < 1e-12:
            continue
        t, u, v = np.linalg.solve(M, o - v0)
        if u >= -1e-9 and v >= -1e-9 and u + v <= 1 + 1e-9 and t > t_min:
            if t < best_t - 1e-9:
                best_t, best = t, k
    return best, best_t


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_closest_hit_bvh_equals_brute_and_linear_solve(seed):
    sc = _random_soup(seed)
    rng = np.random.default_rng(100 + seed)
    n = 400
    o = rng.uniform(-25, 25, size=(n, 3))
    # half the rays aim at (jittered) triangle centroids so that many of them hit
    V = sc.vertices.astype(np.float64)[sc.triangles].mean(axis=1)
    aim = V[rng.integers(0, sc.n_tri, size=n)] + rng.normal(scale=1.0, size=(n, 3))
    c = np.where(np.arange(n)[:, None] % 2 == 0, aim - o, rng.normal(size=(n, 3)))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    hb, tb, fb, _, _ = O.closest_hits(sc, o, c, use_bvh=False)
    hv, tv, fv, nv, tt = O.closest_hits(sc, o, c, use_bvh=True)
    assert np.array_equal(hb, hv) and np.array_equal(fb, fv)
    assert np.array_equal(tb[hb >= 0], tv[hv >= 0])
    assert (hb >= 0).sum() > 80  # the check is not vacuous
    assert tt.sum() < 0.5 * n * sc.n_tri  # the BVH culls
    for r in range(n):
        if fb[r]:
            continue
        h, t = _solve_hits(sc, o[r], c[r], -1, O.T_MIN)
        assert h == hb[r], r
        if h >= 0:
            assert abs(t - tb[r]) < 1e-9 * max(1.0, t)


def test_tie_and_edge_rules():
    """Two coplanar triangles sharing a diagonal; a duplicate triangle; start exclusion."""
    v = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3], [0, 1, 2]], np.int32)  # tri 2 duplicates tri 0
    sc = empty_scene().with_(vertices=v, triangles=t, absorption=np.full(3, 0.1, np.float32))
    down = np.array([[0, 0, -1.0]])
    # interior of tri 0 (x > y): tri 0 and its duplicate tie -> lowest id 0, flagged (tie)
    h, th, f, _, _ = O.closest_hits(sc, np.array([[0.7, 0.2, 1.0]]), down)
    assert h[0] == 0 and th[0] == 1.0 and f[0] == 1
    # interior of tri 1, far from every edge: clean hit, not flagged
    h, th, f, _, _ = O.closest_hits(sc, np.array([[0.25, 0.7, 1.0]]), down)
    assert h[0] == 1 and f[0] == 0
    # exactly on the shared diagonal: both contain the point -> lowest id, flagged
    h, th, f, _, _ = O.closest_hits(sc, np.array([[0.5, 0.5, 1.0]]), down)
    assert h[0] == 0 and f[0] == 1
    # within 1e-6 m of the diagonal (inside tri 1): flagged as near-edge
    h, th, f, _, _ = O.closest_hits(sc, np.array([[0.4, 0.400001, 1.0]]), down)
    assert h[0] == 1 and f[0] == 1
    # near miss just outside the square by 5e-6 m: no hit, flagged
    h, th, f, _, _ = O.closest_hits(sc, np.array([[1.000005, 0.3, 1.0]]), down)
    assert h[0] == -1 and f[0] == 1
    # 1e-3 m outside: clean miss
    h, th, f, _, _ = O.closest_hits(sc, np.array([[1.001, 0.3, 1.0]]), down)
    assert h[0] == -1 and f[0] == 0
    # start triangle excluded: starting on tri 1 the ray sees nothing else
    h, th, f, _, _ = O.closest_hits(sc, np.array([[0.25, 0.7, 1.0]]), down, start=np.array([1]))
    assert h[0] == -1
    # hits at t <= t_min are ignored
    h, th, f, _, _ = O.closest_hits(sc, np.array([[0.25, 0.7, 0.0005]]), down)
    assert h[0] == -1


# ----------------------------------------------------------------------------
# Closed forms for microphone energies
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("level", range(0, 6))
def test_direct_path_free_field(level):
    """No geometry: each microphone gets W / (4 pi d^2) exactly once, at every level."""
    sc = empty_scene(level=level, src=(0.3, -0.2, 1.0))
    r = O.trace(sc, use_bvh=False, mic_mode=0)
    m = sc.mic_positions()
    s = sc.sources[0].astype(np.float64)
    ref = 1.0 / (FOUR_PI * ((m - s) ** 2).sum(1))
    assert (r.e_flag == 0).all()
    assert np.abs(r.energy / ref - 1).max() < 1e-13
    assert r.counters["mic_updates"] == sc.n_mic


@pytest.mark.parametrize("mic_mode", [0, 1])
def test_direct_path_free_field_volumetric(mic_mode):
    """A volumetric grid (layers below, across and above the source): every microphone of
    every layer gets W / (4 pi d^2) exactly once.  (One microphone lies within delta of a
    shared beam face and is reported as ambiguous; its energy is still the closed form.)"""
    sc = empty_scene(level=3, src=(0.3, -0.2, 1.0), n_mic=7, spacing=3.0, mic_z=-5.5).with_(mic_nz=5, mic_dz=4.0)
    r = O.trace(sc, use_bvh=False, mic_mode=mic_mode)
    m = sc.mic_positions()
    assert m.shape == (245, 3) and m[:, 2].min() == -5.5 and m[:, 2].max() == 10.5
    ref = 1.0 / (FOUR_PI * ((m - sc.sources[0].astype(np.float64)) ** 2).sum(1))
    assert (r.e_flag > 0).sum() <= 1
    assert np.abs(r.energy / ref - 1).max() < 1e-13
    assert r.counters["mic_updates"] == sc.n_mic


def test_ground_reflection_volumetric():
    """Ground plane, one reflection, microphones in layers below and above it: layers above
    get the direct plus the image-source term, the layer below the ground gets nothing."""
    alpha = 0.3
    sc = ground_scene(level=4, alpha=alpha, mic_z=-2.5).with_(mic_nz=4, mic_dz=4.0)
    r = O.trace(sc)
    m = sc.mic_positions()
    s = sc.sources[0].astype(np.float64)
    img = s * np.array([1, 1, -1.0])
    a32 = float(np.float32(alpha))
    ref = (1.0 / ((m - s) ** 2).sum(1) + (1 - a32) / ((m - img) ** 2).sum(1)) / FOUR_PI
    below = m[:, 2] < 0
    assert below.sum() == sc.mic_nx * sc.mic_ny
    assert (r.energy[below] == 0).all()
    elev = np.degrees(np.arctan2(m[:, 2] + s[2], np.hypot(m[:, 0] - s[0], m[:, 1] - s[1])))
    ok = ~below & (elev > 15) & (r.e_flag == 0)
    assert ok.sum() > 150
    assert np.abs(r.energy[ok] / ref[ok] - 1).max() < 1e-13


def test_volumetric_layers_equal_planar_runs():
    """Layer k of a volumetric grid holds exactly what a planar grid at height z0 + k dz gets."""
    sc = tiny_scene().with_(mic_z=-2.5, mic_nz=5, mic_dz=4.0)
    r = O.trace(sc, n_threads=1)
    per = sc.mic_nx * sc.mic_ny
    for k in range(sc.mic_nz):
        p = O.trace(sc.with_(mic_z=-2.5 + 4.0 * k, mic_nz=1), n_threads=1)
        assert np.array_equal(r.e_strict[k * per:(k + 1) * per], p.e_strict)
        assert np.array_equal(r.e_flag[k * per:(k + 1) * per], p.e_flag)
    assert (r.energy[:per] == 0).all()   # below the ground
    assert (r.energy[per:] > 0).any()


def test_explicit_points_free_field_and_ground():
    """Explicit microphone points at random positions: W / (4 pi d^2) once each in free
    field, and direct + image source above a ground plane (points below it get nothing)."""
    rng = np.random.default_rng(5)
    pts = rng.uniform([-9.0, -9.0, -6.0], [9.0, 9.0, 12.0], (300, 3)).astype(np.float32)
    sc = empty_scene(level=3, src=(0.3, -0.2, 1.0))
    r = O.trace(sc, points=pts)
    m = pts.astype(np.float64)
    ref = 1.0 / (FOUR_PI * ((m - sc.sources[0].astype(np.float64)) ** 2).sum(1))
    assert np.abs(r.energy / ref - 1).max() < 1e-13
    assert r.counters["mic_updates"] == len(pts)
    alpha = 0.3
    g = ground_scene(level=4, alpha=alpha)
    r = O.trace(g, points=pts)
    s0 = g.sources[0].astype(np.float64)
    img = s0 * np.array([1, 1, -1.0])
    a32 = float(np.float32(alpha))
    ref = (1.0 / ((m - s0) ** 2).sum(1) + (1 - a32) / ((m - img) ** 2).sum(1)) / FOUR_PI
    below = m[:, 2] < 0
    assert below.sum() > 50 and (r.energy[below] == 0).all()
    elev = np.degrees(np.arctan2(m[:, 2] + s0[2], np.hypot(m[:, 0] - s0[0], m[:, 1] - s0[1])))
    ok = ~below & (elev > 15) & (r.e_flag == 0)
    assert ok.sum() > 100
    assert np.abs(r.energy[ok] / ref[ok] - 1).max() < 1e-13


def test_explicit_points_equal_grid():
    """Explicit points placed on the grid's positions (in a shuffled order) get the grid's
    energies bit for bit, planar and volumetric."""
    for sc in (tiny_scene(), tiny_scene().with_(mic_z=-2.5, mic_nz=5, mic_dz=4.0)):
        grid = O.trace(sc, n_threads=1)
        pos = sc.mic_positions()
        perm = np.random.default_rng(1).permutation(len(pos))
        r = O.trace(sc, n_threads=1, points=pos[perm].astype(np.float32))
        assert np.array_equal(r.e_strict, grid.e_strict[perm])
        assert np.array_equal(r.e_flag, grid.e_flag[perm])


def test_directional_source_uniform_weights_is_omni():
    """Equal weights give the omni split (K = W / (4 pi)) up to the rounding of the solid
    angles' sum; any weights conserve the emitted power."""
    sc = empty_scene(level=3, src=(0.3, -0.2, 1.0))
    ref = O.trace(sc)
    r = O.trace(sc, weights=np.full((1, 1280), 3.0, np.float32))
    assert np.abs(r.energy / ref.energy - 1).max() < 1e-12
    w = np.random.default_rng(2).uniform(0.0, 5.0, (1, 1280)).astype(np.float32)
    r = O.trace(sc, weights=w)
    assert abs(r.power[0] - 1.0) < 1e-12


@pytest.mark.parametrize("level", [2, 4])
def test_directional_source_hemisphere_closed_form(level):
    """Weight 1 on the faces whose guiding direction points up, 0 on the others: a
    microphone well above the source receives W / (Omega_up d^2), Omega_up being those
    faces' total solid angle (half of the sphere less the faces whose guiding direction is
    horizontal), and one well below receives nothing."""
    dirs = O.icosphere(level)
    c = dirs.sum(1)
    up = c[:, 2] > 0.0
    flat = c[:, 2] == 0.0
    om = np.array([O.solid_angle(*dirs[f]) for f in range(len(dirs))])
    om_up = om[up].sum()
    assert abs(2.0 * om_up + om[flat].sum() - 4.0 * np.pi) < 1e-11   # mirror symmetry in z
    w = up.astype(np.float32)[None, :]
    src = (0.3, -0.2, 1.0)
    sc = empty_scene(level=level, src=src, n_mic=9, spacing=0.5, mic_z=4.0)   # elevations above 45 degrees
    r = O.trace(sc, weights=w, use_bvh=False, mic_mode=0)
    d2 = ((sc.mic_positions() - np.array(src, np.float32).astype(np.float64)) ** 2).sum(1)
    assert np.abs(r.energy * om_up * d2 - 1.0).max() < 1e-12
    below = O.trace(empty_scene(level=level, src=src, n_mic=9, spacing=0.5, mic_z=-10.0), weights=w, use_bvh=False,
                    mic_mode=0)
    assert (below.energy == 0.0).all()


def test_direct_path_two_sources_and_air_damping():
    sc = empty_scene(level=3, src=(0.3, -0.2, 1.0))
    sc = sc.with_(sources=np.array([[0.3, -0.2, 1.0], [-2.1, 3.3, 0.4]], np.float32),
                  power=np.array([1.0, 2.5], np.float32))
    m_air = 0.01
    r = O.trace(sc, m_air=m_air)
    m = sc.mic_positions()
    ref = np.zeros(sc.n_mic)
    for s, w in zip(sc.sources.astype(np.float64), sc.power.astype(np.float64)):
        d = np.sqrt(((m - s) ** 2).sum(1))
        ref += w * np.exp(-m_air * d) / (FOUR_PI * d * d)
    assert np.abs(r.energy / ref - 1).max() < 1e-13


def test_tie_rule_on_shared_faces_and_vertex_rays():
    """Source on the icosphere's symmetry planes: the microphone row y = 0 lies exactly on
    shared beam faces and the centre microphone on the +z vertex ray.  Every microphone is
    still owned by exactly one beam (total energy equals the closed form), and the ones on
    shared faces are reported as ambiguous (flag energy)."""
    sc = empty_scene(level=2, src=(0.0, 0.0, 1.0), n_mic=9, spacing=3.0, mic_z=2.5)
    r = O.trace(sc, mic_mode=0)
    m = sc.mic_positions()
    ref = 1.0 / (FOUR_PI * ((m - sc.sources[0].astype(np.float64)) ** 2).sum(1))
    assert np.abs(r.energy / ref - 1).max() < 1e-13
    amb = (r.e_flag > 0).reshape(9, 9)
    assert amb[4].all()            # y = 0: on shared faces
    assert amb.sum() == 9          # nowhere else
    assert r.counters["mic_updates"] == sc.n_mic


@pytest.mark.parametrize("level,alpha", [(3, 0.2), (4, 0.5), (5, 0.05)])
def test_single_ground_reflection_is_image_source(level, alpha):
    sc = ground_scene(level=level, alpha=alpha)
    r = O.trace(sc)
    m = sc.mic_positions()
    s = sc.sources[0].astype(np.float64)
    img = s * np.array([1, 1, -1.0])
    a32 = float(np.float32(alpha))
    ref = (1.0 / ((m - s) ** 2).sum(1) + (1 - a32) / ((m - img) ** 2).sum(1)) / FOUR_PI
    # image direction well below the horizon so its beam's guiding ray hits the ground
    elev = np.degrees(np.arctan2(m[:, 2] + s[2], np.hypot(m[:, 0] - s[0], m[:, 1] - s[1])))
    ok = (elev > 15) & (r.e_flag == 0)
    assert ok.sum() > 60
    assert np.abs(r.energy[ok] / ref[ok] - 1).max() < 1e-13
    # depth 0: only the direct path remains
    r0 = O.trace(sc, depth=0)
    ref0 = 1.0 / (FOUR_PI * ((m - s) ** 2).sum(1))
    assert np.abs(r0.energy / ref0 - 1).max() < 1e-13


@pytest.mark.parametrize("level,alpha", [(2, 0.25), (3, 0.1), (4, 0.6)])
def test_sealed_box_counts_and_power(level, alpha):
    sc = sealed_box_scene(level=level, alpha=alpha, depth=6)
    r = O.trace(sc)
    n = 20 * 4 ** level
    assert (r.flagged == 0).all()
    assert (r.count == n).all()
    a32 = float(np.float32(alpha))
    assert np.abs(r.power - (1 - a32) ** np.arange(7)).max() < 1e-13
    assert (r.hit >= 0).all()


def test_energy_bookkeeping_block():
    """P_g = sum over beams alive at g of (W / 4 pi) Omega_b prod_k<g (1 - alpha[hit_k]);
    count_(g+1) = hits at generation g (g < D)."""
    sc = block_scene(0)
    r = O.trace(sc)
    d = O.icosphere(sc.level)
    num = np.abs(np.einsum("fi,fi->f", d[:, 0], np.cross(d[:, 1], d[:, 2])))
    den = 1 + np.einsum("fi,fi->f", d[:, 0], d[:, 1]) + np.einsum("fi,fi->f", d[:, 1], d[:, 2]) \
        + np.einsum("fi,fi->f", d[:, 2], d[:, 0])
    om = 2 * np.arctan2(num, den)
    alpha = sc.absorption.astype(np.float64)
    K = np.full(r.hit.shape[0], 1.0 / FOUR_PI)
    for g in range(sc.depth + 1):
        alive = r.hit[:, g] != -2
        assert alive.sum() == r.count[g]
        assert abs((K[alive] * om[alive]).sum() - r.power[g]) < 1e-12
        if g < sc.depth:
            hit = r.hit[:, g] >= 0
            assert (r.hit[:, g + 1] != -2).sum() == hit.sum()
            K = np.where(hit, K * (1 - alpha[np.maximum(r.hit[:, g], 0)]), K)
    assert (np.diff(r.count) <= 0).all()


# ----------------------------------------------------------------------------
# Reflectors off the origin, a second-order image and the energy threshold.
# Each pin_* function raises AssertionError on a mismatch; the tests below run them
# on the oracle, and tests/test_oracle_mutations.py runs them on deliberately broken
# copies of it to show that each catches a plausible mistake.
# ----------------------------------------------------------------------------

# Microphone modes: 0 tests every microphone against every segment (the membership
# rule alone decides), 1 rasterises the footprint first (a clipping mistake loses
# microphones); a pin runs both.
MODES = (0, 1)


def pin_ground_off_origin(ground_z, level=4, alpha=0.3):
    """Ground z = h: above it, the direct path plus the image at 2h - z_s (a mirror that
    drops the plane's offset puts it at -z_s); below it, exactly nothing (a far or near
    cap that drops the offset lets energy through)."""
    src = (0.25, -0.15, ground_z + 2.0)
    sc = ground_scene(level=level, alpha=alpha, src=src, mic_z=ground_z + 1.5, ground_z=ground_z)
    ref, ok0 = CF.ground_offset(sc, ground_z, alpha)
    for mode in MODES:
        r = O.trace(sc, mic_mode=mode)
        ok = ok0 & (r.e_flag == 0)
        assert ok.sum() > 60, ok.sum()
        err = np.abs(r.energy[ok] / ref[ok] - 1).max()
        assert err < 1e-13, (mode, err)
        below = O.trace(sc.with_(mic_z=ground_z - 1.5), mic_mode=mode)
        assert (below.energy == 0.0).all(), (mode, below.energy.max())


def pin_wall_off_origin(wall_x=7.5, level=4, alpha=0.3):
    """Vertical wall x = c: in front, the direct path plus the image at 2c - x_s; behind
    it, nothing."""
    sc = wall_scene(level=level, alpha=alpha, wall_x=wall_x)
    ref, ok0 = CF.wall_offset(sc, wall_x, alpha)
    for mode in MODES:
        r = O.trace(sc, mic_mode=mode)
        ok = ok0 & (r.e_flag == 0)
        assert ok.sum() > 60, ok.sum()
        err = np.abs(r.energy[ok] / ref[ok] - 1).max()
        assert err < 1e-13, (mode, err)
        behind = O.trace(wall_scene(level=level, alpha=alpha, wall_x=wall_x, behind=True), mic_mode=mode)
        assert (behind.energy == 0.0).all(), (mode, behind.energy.max())


def pin_corner_second_order(level=5):
    """Wall + ground corner: direct, two first-order and one second-order image with
    weights 1, 1 - a_g, 1 - a_w, (1 - a_g)(1 - a_w), reached through either order."""
    sc = corner_scene(level=level)
    ref, ok0, last_on_wall = CF.corner(sc, 6.0, 0.2, 0.35)
    for mode in MODES:
        r = O.trace(sc, mic_mode=mode)
        ok = ok0 & (r.e_flag == 0)
        assert ok.sum() > 80, ok.sum()
        assert last_on_wall[ok].sum() > 10 and (~last_on_wall[ok]).sum() > 10
        err = np.abs(r.energy[ok] / ref[ok] - 1).max()
        assert err < 1e-13, (mode, err)
        assert r.count[3] == 0 and r.count[2] > 0   # no third reflection inside a right angle


def pin_threshold_generation(eps, generation=3, alpha=0.1, depth=6):
    """Level-0 sealed box with e_min at (1 - alpha)^G / 20 (1 +- 1e-9): generations end
    exactly before or after G.  Comparing the power before absorption, or not at all,
    moves the end by one generation."""
    e_min, alive = CF.sealed_box_threshold(alpha, generation, eps)
    r = O.trace(sealed_box_scene(level=0, alpha=alpha, depth=depth), e_min=e_min)
    want = np.array([20 if g < alive else 0 for g in range(depth + 1)])
    assert np.array_equal(r.count, want), (r.count.tolist(), want.tolist())
    a = CF.f32(alpha)
    pw = np.where(want > 0, (1 - a) ** np.arange(depth + 1), 0.0)
    assert np.abs(r.power - pw).max() < 1e-14


@pytest.mark.parametrize("ground_z", [3.7, -4.2])
def test_ground_off_origin_is_image_source(ground_z):
    pin_ground_off_origin(ground_z)


def test_wall_off_origin_is_image_source():
    pin_wall_off_origin()


def test_wall_corner_second_order_image():
    pin_corner_second_order()


@pytest.mark.parametrize("eps", [1e-9, -1e-9])
def test_energy_threshold_ends_at_exact_generation(eps):
    pin_threshold_generation(eps)


# ----------------------------------------------------------------------------
# Microphone enumeration and symmetry
# ----------------------------------------------------------------------------

def _volumetric(sc, nz, dz):
    return sc.with_(mic_nz=nz, mic_dz=dz)


@pytest.mark.parametrize("maker,kw", [(tiny_scene, {}), (mirror_scene, {}), (block_scene, {"beam_end": 3000}),
                                      (lambda: _volumetric(tiny_scene(), 6, 5.0), {}),
                                      (lambda: _volumetric(block_scene().with_(mic_nx=40, mic_ny=40, mic_dx=5.0,
                                                                               mic_dy=5.0), 8, 7.0),
                                       {"beam_end": 3000})])
def test_grid_rasterisation_equals_brute_force(maker, kw):
    sc = maker()
    a = O.trace(sc, mic_mode=1, n_threads=1, **kw)
    b = O.trace(sc, mic_mode=0, n_threads=1, **kw)
    assert np.array_equal(a.e_strict, b.e_strict)
    assert np.array_equal(a.e_flag, b.e_flag)
    assert a.counters["mic_updates"] == b.counters["mic_updates"]
    assert a.counters["mic_updates"] > 0
    assert a.counters["mic_tests"] < b.counters["mic_tests"]


def test_mirror_symmetry():
    sc = mirror_scene()
    r = O.trace(sc)
    E = r.energy.reshape(sc.mic_ny, sc.mic_nx)
    F = (r.e_flag > 0).reshape(sc.mic_ny, sc.mic_nx)
    ok = ~(F | F[:, ::-1])
    assert ok.sum() > 200
    a, b = E[ok], E[:, ::-1][ok]
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    assert (E > 0).sum() > 100


def test_energy_threshold_stops_reflections():
    sc = tiny_scene()
    r = O.trace(sc, e_min=1e9)
    assert r.count[1:].sum() == 0


# ----------------------------------------------------------------------------
# Scene generator shapes (input recipe)
# ----------------------------------------------------------------------------

def test_scene_shapes():
    t = tiny_scene()
    assert t.n_tri == 42 and t.n_mic == 16 and t.n_beams0 == 1280
    b = block_scene(0)
    assert b.n_tri == 1002 and b.n_mic == 10000 and b.n_beams0 == 20480
    b2 = block_scene(0)
    assert np.array_equal(b.vertices, b2.vertices)
    assert not np.array_equal(b.vertices, block_scene(1).vertices)


@pytest.mark.slow
def test_district_shape():
    d = district_scene(0)
    assert 300_000 <= d.n_tri <= 360_000
    assert d.n_src == 64 and d.n_mic == 250_000 and d.n_beams0 == 64 * 81920
    assert len({tuple(s) for s in d.sources.tolist()}) == 64
