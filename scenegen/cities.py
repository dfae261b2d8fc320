"""Seeded synthetic urban scenes for the hybrid beam tracer.

The paper's experiment runs on a CAD model of a city district, with sources at
road crossings and microphones on a regular grid (Section 4).  That model is
not available, so these procedural scenes stand in for it.  They hold only
inputs: vertices, triangles, per-triangle absorption, point sources and a
planar microphone grid.  None of the tracing method's arithmetic lives here;
both the CPU oracle and the GPU library read these arrays as they are.

Every coordinate is rounded to float32 exactly once, here, so that both sides
see bit-identical geometry.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Scene:
    """One tracing problem.

    vertices   float32 [n_v, 3], metres
    triangles  int32 [n_t, 3], indices into vertices
    absorption float32 [n_t], energy fraction lost on reflection, in [0, 1]
    sources    float32 [n_s, 3], point sources
    power      float32 [n_s], watts
    mic grid   x0 + i*dx, y0 + j*dy at height mic_z + k*mic_dz, i < mic_nx, j < mic_ny,
               k < mic_nz (mic_nz = 1: a planar grid); microphone index is
               (k*mic_ny + j)*mic_nx + i
    level      icosphere subdivision level (20*4**level beams per source)
    depth      maximum number of reflections
    tiles      on-device partition of the mesh footprint (tiles_x x tiles_y)
    """

    name: str
    vertices: np.ndarray
    triangles: np.ndarray
    absorption: np.ndarray
    sources: np.ndarray
    power: np.ndarray
    mic_x0: float
    mic_y0: float
    mic_z: float
    mic_dx: float
    mic_dy: float
    mic_nx: int
    mic_ny: int
    level: int
    depth: int
    tiles_x: int = 1
    tiles_y: int = 1
    mic_dz: float = 4.0
    mic_nz: int = 1

    @property
    def n_tri(self) -> int:
        return int(self.triangles.shape[0])

    @property
    def n_src(self) -> int:
        return int(self.sources.shape[0])

    @property
    def n_mic(self) -> int:
        return self.mic_nx * self.mic_ny * self.mic_nz

    @property
    def n_beams0(self) -> int:
        return self.n_src * 20 * 4 ** self.level

    def mic_positions(self) -> np.ndarray:
        """float64 [n_mic, 3] positions of the grid microphones (index (k*ny + j)*nx + i)."""
        i = np.arange(self.mic_nx, dtype=np.float64)
        j = np.arange(self.mic_ny, dtype=np.float64)
        k = np.arange(self.mic_nz, dtype=np.float64)
        x = np.float64(np.float32(self.mic_x0)) + i * np.float64(np.float32(self.mic_dx))
        y = np.float64(np.float32(self.mic_y0)) + j * np.float64(np.float32(self.mic_dy))
        z = np.float64(np.float32(self.mic_z)) + k * np.float64(np.float32(self.mic_dz))
        zz, yy, xx = np.meshgrid(z, y, x, indexing="ij")
        return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)

    def with_(self, **kw) -> "Scene":
        return dataclasses.replace(self, **kw)


class _MeshBuilder:
    """Accumulates float64 vertices and triangles; rounds to float32 at the end."""

    def __init__(self):
        self.v: list[tuple[float, float, float]] = []
        self.t: list[tuple[int, int, int]] = []
        self.a: list[float] = []

    def vert(self, x, y, z) -> int:
        self.v.append((float(x), float(y), float(z)))
        return len(self.v) - 1

    def tri(self, i, j, k, alpha):
        self.t.append((i, j, k))
        self.a.append(float(alpha))

    def quad(self, i, j, k, l, alpha):
        """Planar quad i-j-k-l as two triangles (i,j,k), (i,k,l)."""
        self.tri(i, j, k, alpha)
        self.tri(i, k, l, alpha)

    def arrays(self):
        v = np.asarray(self.v, dtype=np.float64).reshape(-1, 3).astype(np.float32)
        t = np.asarray(self.t, dtype=np.int32).reshape(-1, 3)
        a = np.asarray(self.a, dtype=np.float64).astype(np.float32)
        return v, t, a


def _ground(mb: _MeshBuilder, x0, y0, x1, y1, alpha, cell=None, z=0.0):
    """Ground at height z over [x0,x1]x[y0,y1]; one quad (split along (x0,y0)-(x1,y1)) or a grid."""
    if cell is None:
        a = mb.vert(x0, y0, z)
        b = mb.vert(x1, y0, z)
        c = mb.vert(x1, y1, z)
        d = mb.vert(x0, y1, z)
        mb.quad(a, b, c, d, alpha)
        return
    nx = int(round((x1 - x0) / cell))
    ny = int(round((y1 - y0) / cell))
    base = len(mb.v)
    for j in range(ny + 1):
        for i in range(nx + 1):
            mb.vert(x0 + i * cell, y0 + j * cell, 0.0)
    for j in range(ny):
        for i in range(nx):
            a = base + j * (nx + 1) + i
            mb.quad(a, a + 1, a + nx + 2, a + nx + 1, alpha)


def _box(mb: _MeshBuilder, cx, cy, w, d, h, alphas):
    """Axis-aligned box building without a bottom face: walls -x,+x,-y,+y then roof.

    alphas: 5 absorption values (walls -x, +x, -y, +y, roof).
    """
    xa, xb = cx - w / 2.0, cx + w / 2.0
    ya, yb = cy - d / 2.0, cy + d / 2.0
    b00 = mb.vert(xa, ya, 0.0)
    b10 = mb.vert(xb, ya, 0.0)
    b11 = mb.vert(xb, yb, 0.0)
    b01 = mb.vert(xa, yb, 0.0)
    t00 = mb.vert(xa, ya, h)
    t10 = mb.vert(xb, ya, h)
    t11 = mb.vert(xb, yb, h)
    t01 = mb.vert(xa, yb, h)
    mb.quad(b00, b01, t01, t00, alphas[0])  # -x
    mb.quad(b10, b11, t11, t10, alphas[1])  # +x
    mb.quad(b00, b10, t10, t00, alphas[2])  # -y
    mb.quad(b01, b11, t11, t01, alphas[3])  # +y
    mb.quad(t00, t10, t11, t01, alphas[4])  # roof


def _prism(mb: _MeshBuilder, px, py, h, bands, wall_alpha, roof_alpha):
    """Extruded convex polygon (counter-clockwise px, py), walls split in `bands` bands, roof fan."""
    n = len(px)
    cols = []
    for i in range(n):
        cols.append([mb.vert(px[i], py[i], h * k / bands) for k in range(bands + 1)])
    for i in range(n):
        ii = (i + 1) % n
        for k in range(bands):
            mb.quad(cols[i][k], cols[ii][k], cols[ii][k + 1], cols[i][k + 1], wall_alpha[i])
    for i in range(1, n - 1):
        mb.tri(cols[0][bands], cols[i][bands], cols[i + 1][bands], roof_alpha)


def tiny_scene() -> Scene:
    """2 ground triangles + 4 box buildings (42 triangles), one source, 16 microphones.

    Level 3 (1280 beams), 3 reflections, absorption 0.1 everywhere.
    """
    mb = _MeshBuilder()
    _ground(mb, -50.0, -50.0, 50.0, 50.0, 0.1)
    for (cx, cy, h) in [(20.0, 20.0, 10.0), (-20.0, 20.0, 15.0), (-20.0, -20.0, 20.0), (20.0, -20.0, 25.0)]:
        _box(mb, cx, cy, 10.0, 10.0, h, [0.1] * 5)
    v, t, a = mb.arrays()
    return Scene("tiny", v, t, a,
                 sources=np.array([[0.0, 0.0, 1.0]], np.float32), power=np.ones(1, np.float32),
                 mic_x0=-30.0, mic_y0=-30.0, mic_z=1.5, mic_dx=20.0, mic_dy=20.0, mic_nx=4, mic_ny=4,
                 level=3, depth=3)


def block_scene(seed: int = 0) -> Scene:
    """200 x 200 m ground with 100 seeded box buildings (1002 triangles), one source, 10k mics.

    Footprints 8-25 m, heights U(10, 60) m, per-face absorption U(0.05, 0.3), ground 0.1.
    Each placement attempt redraws the footprint; a candidate is rejected when it comes
    within 1 m of a placed box or within 6 m of the source.  Level 5, 6 reflections.
    """
    rng = np.random.default_rng(seed)
    half = 100.0
    boxes = []
    attempts = 0
    while len(boxes) < 100:
        attempts += 1
        if attempts > 2_000_000:
            raise RuntimeError("block placement did not converge")
        w, d = rng.uniform(8.0, 25.0, size=2)
        cx = rng.uniform(-half + w / 2, half - w / 2)
        cy = rng.uniform(-half + d / 2, half - d / 2)
        # distance from the source column (0,0) to the footprint rectangle
        ddx = max(abs(cx) - w / 2, 0.0)
        ddy = max(abs(cy) - d / 2, 0.0)
        if math.hypot(ddx, ddy) < 6.0:
            continue
        ok = True
        for (bx, by, bw, bd) in boxes:
            if abs(cx - bx) < (w + bw) / 2 + 1.0 and abs(cy - by) < (d + bd) / 2 + 1.0:
                ok = False
                break
        if ok:
            boxes.append((cx, cy, w, d))
    mb = _MeshBuilder()
    _ground(mb, -half, -half, half, half, 0.1)
    for (cx, cy, w, d) in boxes:
        h = rng.uniform(10.0, 60.0)
        alphas = rng.uniform(0.05, 0.3, size=5)
        _box(mb, cx, cy, w, d, h, alphas)
    v, t, a = mb.arrays()
    return Scene(f"block_s{seed}", v, t, a,
                 sources=np.array([[0.0, 0.0, 0.5]], np.float32), power=np.ones(1, np.float32),
                 mic_x0=-99.0, mic_y0=-99.0, mic_z=1.5, mic_dx=2.0, mic_dy=2.0, mic_nx=100, mic_ny=100,
                 level=5, depth=6)


def _fill_block(mb: _MeshBuilder, rng, x0, y0, x1, y1, n_buildings, taken=()):
    """`n_buildings` extruded convex prisms in the block [x0,x1]x[y0,y1]: circumscribed
    disks (radius U(6, 14) m) placed by dart throwing with a 1 m gap to each other and to
    the disks in `taken`, and a 2 m setback; U{6..10} footprint vertices at sorted jittered
    angles; height lognormal (median 20 m, sigma 0.5), walls in ceil(h/10) bands."""
    disks = []
    attempts = 0
    while len(disks) < n_buildings:
        attempts += 1
        if attempts > 200_000:
            raise RuntimeError("block placement did not converge")
        r = rng.uniform(6.0, 14.0)
        cx = rng.uniform(x0 + 2.0 + r, x1 - 2.0 - r)
        cy = rng.uniform(y0 + 2.0 + r, y1 - 2.0 - r)
        ok = True
        for (qx, qy, qr) in list(taken) + disks:
            if (cx - qx) ** 2 + (cy - qy) ** 2 < (r + qr + 1.0) ** 2:
                ok = False
                break
        if ok:
            disks.append((cx, cy, r))
    for (cx, cy, r) in disks:
        _random_prism(mb, rng, cx, cy, r)


def _random_prism(mb: _MeshBuilder, rng, cx, cy, r, h=None):
    """Convex prism on U{6..10} jittered vertices of the circle (cx, cy, r), of height `h`
    or, when None, a lognormal one (median 20 m, sigma 0.5) drawn after the footprint."""
    n = int(rng.integers(6, 11))
    rot = rng.uniform(0.0, 2.0 * math.pi)
    jit = rng.uniform(-0.35, 0.35, size=n)
    ang = rot + 2.0 * math.pi * (np.arange(n) + 0.5 + jit) / n
    px = cx + r * np.cos(ang)
    py = cy + r * np.sin(ang)
    if h is None:
        h = float(rng.lognormal(math.log(20.0), 0.5))
    bands = max(1, int(math.ceil(h / 10.0)))
    wall_alpha = rng.uniform(0.05, 0.3, size=n)
    roof_alpha = float(rng.uniform(0.05, 0.3))
    _prism(mb, px, py, h, bands, wall_alpha, roof_alpha)


def district_scene(seed: int = 0, n_sources: int = 64, level: int = 6, depth: int = 8,
                   tiles: int = 4, buildings_per_block: int = 50) -> Scene:
    """2 x 2 km district: 10 x 10 street grid, 5000 extruded convex-polygon buildings.

    Streets are 20 m wide on the lines x, y = -1000 + 200k (k = 0..10), leaving 100
    blocks of 180 x 180 m.  Each block gets `buildings_per_block` buildings placed by
    dart throwing of their circumscribed disks (radius U(6, 14) m, 1 m gap, 2 m
    setback).  A footprint has U{6..10} vertices on that circle at sorted jittered
    angles, so it is convex.  Heights are lognormal (median 20 m, sigma 0.5); walls are
    split into ceil(h/10) bands.  The ground is a 10 m triangle grid.  Sources sit
    0.5 m above `n_sources` of the 81 interior crossings; microphones form a 4 m grid
    at 1.5 m height (500 x 500).
    """
    rng = np.random.default_rng(seed)
    mb = _MeshBuilder()
    _ground(mb, -1000.0, -1000.0, 1000.0, 1000.0, 0.1, cell=10.0)
    for bj in range(10):
        for bi in range(10):
            x0 = -1000.0 + 200.0 * bi + 10.0
            y0 = -1000.0 + 200.0 * bj + 10.0
            _fill_block(mb, rng, x0, y0, x0 + 180.0, y0 + 180.0, buildings_per_block)
    v, t, a = mb.arrays()
    cross = rng.choice(81, size=n_sources, replace=False)
    src = np.array([[-1000.0 + 200.0 * (1 + c % 9), -1000.0 + 200.0 * (1 + c // 9), 0.5] for c in cross],
                   dtype=np.float32).reshape(-1, 3)
    return Scene(f"district_s{seed}", v, t, a, sources=src, power=np.ones(n_sources, np.float32),
                 mic_x0=-998.0, mic_y0=-998.0, mic_z=1.5, mic_dx=4.0, mic_dy=4.0, mic_nx=500, mic_ny=500,
                 level=level, depth=depth, tiles_x=tiles, tiles_y=tiles)


def volumetric_scene(seed: int = 0, n_sources: int = 49, level: int = 8, depth: int = 8, n_towers: int = 10,
                     buildings_per_block: int = 80) -> Scene:
    """The paper's experiment shape (Section 4): a 2.5 x 1.5 km district with about ten
    towers of 200 m and more, and microphones every 4 m in all three directions filling
    the model's bounding box.

    Streets are 20 m wide on the lines x = -1250 + 250k (k = 0..10) and y = -750 + 250l
    (l = 0..6), leaving 60 blocks of 230 x 230 m.  `n_towers` distinct blocks get one tower
    near their centre: a convex prism of radius U(20, 30) m and height U(200, 235) m.  Each
    block is then filled with `buildings_per_block` buildings as in the district (same
    footprint and height laws, so about the district's density).  The ground is a 10 m
    grid.  Sources sit 0.5 m above the 45 interior crossings and, past those, at random
    points of interior street centre lines.  Microphones form the 4 m grid x = -1248 + 4i,
    y = -748 + 4j, z = 2 + 4k up to the tallest roof (625 x 375 x ceil(h_max / 4)).
    """
    rng = np.random.default_rng(seed)
    mb = _MeshBuilder()
    _ground(mb, -1250.0, -750.0, 1250.0, 750.0, 0.1, cell=10.0)
    blocks = [(bi, bj) for bj in range(6) for bi in range(10)]
    towers = set(int(b) for b in rng.choice(len(blocks), size=n_towers, replace=False))
    for b, (bi, bj) in enumerate(blocks):
        x0 = -1250.0 + 250.0 * bi + 10.0
        y0 = -750.0 + 250.0 * bj + 10.0
        taken = []
        if b in towers:
            r = rng.uniform(20.0, 30.0)
            cx = x0 + 115.0 + rng.uniform(-40.0, 40.0)
            cy = y0 + 115.0 + rng.uniform(-40.0, 40.0)
            h = float(rng.uniform(200.0, 235.0))
            _random_prism(mb, rng, cx, cy, r, h)
            taken.append((cx, cy, r))
        _fill_block(mb, rng, x0, y0, x0 + 230.0, y0 + 230.0, buildings_per_block, taken)
    v, t, a = mb.arrays()
    h_max = float(v[:, 2].max())
    pts = [(-1250.0 + 250.0 * k, -750.0 + 250.0 * l) for l in range(1, 6) for k in range(1, 10)]
    rng_src = np.random.default_rng(seed + 1)
    while len(pts) < n_sources:
        if rng_src.uniform() < 0.5:   # on a line x = const, between two crossings
            pts.append((-1250.0 + 250.0 * int(rng_src.integers(1, 10)), rng_src.uniform(-750.0, 750.0)))
        else:
            pts.append((rng_src.uniform(-1250.0, 1250.0), -750.0 + 250.0 * int(rng_src.integers(1, 6))))
    src = np.array([[x, y, 0.5] for (x, y) in pts[:n_sources]], np.float32).reshape(-1, 3)
    nz = int(math.ceil(h_max / 4.0))
    return Scene(f"volumetric_s{seed}", v, t, a, sources=src, power=np.ones(n_sources, np.float32),
                 mic_x0=-1248.0, mic_y0=-748.0, mic_z=2.0, mic_dx=4.0, mic_dy=4.0, mic_nx=625, mic_ny=375,
                 level=level, depth=depth, tiles_x=5, tiles_y=3, mic_dz=4.0, mic_nz=nz)


# ----------------------------------------------------------------------------------------
# Small analytic scenes used by closed-form and invariant tests
# ----------------------------------------------------------------------------------------

def empty_scene(level=2, src=(0.3, -0.2, 1.0), n_mic=9, spacing=3.0, mic_z=2.5) -> Scene:
    """No geometry at all: every beam escapes after its direct segment."""
    half = (n_mic - 1) / 2.0 * spacing
    return Scene("empty", np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32),
                 np.zeros(0, np.float32), np.array([src], np.float32), np.ones(1, np.float32),
                 mic_x0=-half, mic_y0=-half, mic_z=mic_z, mic_dx=spacing, mic_dy=spacing,
                 mic_nx=n_mic, mic_ny=n_mic, level=level, depth=0)


def ground_scene(level=3, alpha=0.2, half=1000.0, src=(0.25, -0.15, 2.0), n_mic=11, spacing=2.5,
                 mic_z=1.5, depth=1, ground_z=0.0) -> Scene:
    """Single large ground quad at z = ground_z (2 triangles)."""
    mb = _MeshBuilder()
    _ground(mb, -half, -half, half, half, alpha, z=ground_z)
    v, t, a = mb.arrays()
    h = (n_mic - 1) / 2.0 * spacing
    return Scene("ground", v, t, a, np.array([src], np.float32), np.ones(1, np.float32),
                 mic_x0=-h, mic_y0=-h, mic_z=mic_z, mic_dx=spacing, mic_dy=spacing,
                 mic_nx=n_mic, mic_ny=n_mic, level=level, depth=depth)


def wall_scene(level=4, alpha=0.3, wall_x=7.5, half=1000.0, src=(0.25, -0.15, 2.0), nx=9, ny=11, spacing=2.5,
               mic_z=1.5, depth=1, behind=False) -> Scene:
    """Single large vertical wall in the plane x = wall_x (2 triangles, y and z in
    [-half, half]) and nothing else.  The microphone grid's columns lie in front of the wall
    (x < wall_x, the source's side), or behind it when `behind` is set."""
    mb = _MeshBuilder()
    a0 = mb.vert(wall_x, -half, -half)
    a1 = mb.vert(wall_x, half, -half)
    a2 = mb.vert(wall_x, half, half)
    a3 = mb.vert(wall_x, -half, half)
    mb.quad(a0, a1, a2, a3, alpha)
    v, t, a = mb.arrays()
    x0 = wall_x + 1.0 if behind else wall_x - 1.0 - (nx - 1) * spacing
    y0 = -(ny - 1) / 2.0 * spacing
    return Scene("wall", v, t, a, np.array([src], np.float32), np.ones(1, np.float32),
                 mic_x0=x0, mic_y0=y0, mic_z=mic_z, mic_dx=spacing, mic_dy=spacing,
                 mic_nx=nx, mic_ny=ny, level=level, depth=depth)


def corner_scene(level=5, alpha_ground=0.2, alpha_wall=0.35, wall_x=6.0, half=1000.0, src=(-3.0, 0.4, 2.5),
                 nx=10, ny=13, spacing=2.0, mic_z=1.5, depth=3) -> Scene:
    """A ground at z = 0 for x <= wall_x and a vertical wall in the plane x = wall_x above it
    (z in [0, half]): a right-angle corner along the line x = wall_x, z = 0 (4 triangles,
    ground first).  Microphones in front of the wall, above the ground."""
    mb = _MeshBuilder()
    g0 = mb.vert(-half, -half, 0.0)
    g1 = mb.vert(wall_x, -half, 0.0)
    g2 = mb.vert(wall_x, half, 0.0)
    g3 = mb.vert(-half, half, 0.0)
    mb.quad(g0, g1, g2, g3, alpha_ground)
    w2 = mb.vert(wall_x, half, half)
    w3 = mb.vert(wall_x, -half, half)
    mb.quad(g1, g2, w2, w3, alpha_wall)
    v, t, a = mb.arrays()
    x0 = wall_x - 1.0 - (nx - 1) * spacing
    y0 = -(ny - 1) / 2.0 * spacing
    return Scene("corner", v, t, a, np.array([src], np.float32), np.ones(1, np.float32),
                 mic_x0=x0, mic_y0=y0, mic_z=mic_z, mic_dx=spacing, mic_dy=spacing,
                 mic_nx=nx, mic_ny=ny, level=level, depth=depth)


def sealed_box_scene(level=2, alpha=0.25, depth=4, size=(10.0, 8.0, 6.0), src=(0.731, -0.412, 1.137)) -> Scene:
    """Closed axis-aligned box (12 triangles) around the source; every beam hits every time."""
    sx, sy, sz = size
    mb = _MeshBuilder()
    c = [mb.vert(x, y, z) for z in (-sz / 2, sz / 2) for y in (-sy / 2, sy / 2) for x in (-sx / 2, sx / 2)]
    # c index = 4*zi + 2*yi + xi
    faces = [(0, 2, 6, 4), (1, 3, 7, 5), (0, 1, 5, 4), (2, 3, 7, 6), (0, 1, 3, 2), (4, 5, 7, 6)]
    for f in faces:
        mb.quad(c[f[0]], c[f[1]], c[f[2]], c[f[3]], alpha)
    v, t, a = mb.arrays()
    return Scene("sealed_box", v, t, a, np.array([src], np.float32), np.ones(1, np.float32),
                 mic_x0=-3.5, mic_y0=-3.0, mic_z=0.4, mic_dx=1.0, mic_dy=1.0, mic_nx=8, mic_ny=7,
                 level=level, depth=depth)


def mirror_scene(level=3, depth=3) -> Scene:
    """Scene symmetric under x -> -x: ground plus two mirror-image boxes, source on x = 0."""
    mb = _MeshBuilder()
    _ground(mb, -60.0, -60.0, 60.0, 60.0, 0.15)
    _box(mb, 15.0, 10.0, 8.0, 12.0, 12.0, [0.2, 0.1, 0.3, 0.15, 0.05])
    _box(mb, -15.0, 10.0, 8.0, 12.0, 12.0, [0.1, 0.2, 0.3, 0.15, 0.05])  # -x/+x walls swapped
    v, t, a = mb.arrays()
    return Scene("mirror", v, t, a, np.array([[0.0, -5.0, 1.0]], np.float32), np.ones(1, np.float32),
                 mic_x0=-40.0, mic_y0=-40.0, mic_z=1.5, mic_dx=5.0, mic_dy=5.0, mic_nx=17, mic_ny=17,
                 level=level, depth=depth)


def config_scene(index: int, seed: int = 0) -> Scene:
    """The three plain-method workloads: 0 tiny, 1 city block, 2 district."""
    if index == 0:
        return tiny_scene()
    if index == 1:
        return block_scene(seed)
    if index == 2:
        return district_scene(seed)
    raise ValueError(f"no plain-method scene {index}")
