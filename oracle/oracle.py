"""ctypes wrapper of the FP64 CPU oracle (bt_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg.  It shares nothing with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bt_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

N_COUNTERS = 16
COUNTER_NAMES = ["segments", "node_visits", "tri_tests", "mic_updates", "mic_tests", "hits",
                 "flagged_segments", "children"]

# Flag distance of the edge / tie flags, metres (the hit-parity allowance).
DELTA = 1e-5
# Self-intersection guard after a reflection, metres.
T_MIN = 1e-3


def default_threads() -> int:
    """Worker threads: OMP_NUM_THREADS when set, else the CPU count capped at 16."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return max(1, min(os.cpu_count() or 1, 16))


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, no fused multiply-add)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    compile_to(_SRC, tmp)
    os.replace(tmp, _LIB)
    return _LIB


class _Scene(C.Structure):
    _fields_ = [("xyz", C.c_void_p), ("n_vert", C.c_int64), ("tri", C.c_void_p), ("n_tri", C.c_int64),
                ("alpha", C.c_void_p), ("src", C.c_void_p), ("power", C.c_void_p), ("n_src", C.c_int32),
                ("mic_x0", C.c_double), ("mic_y0", C.c_double), ("mic_z", C.c_double),
                ("mic_dx", C.c_double), ("mic_dy", C.c_double), ("mic_nx", C.c_int32), ("mic_ny", C.c_int32),
                ("src_weight", C.c_void_p), ("mic_dz", C.c_double), ("mic_nz", C.c_int32),
                ("mic_xyz", C.c_void_p), ("mic_n", C.c_int64)]


class _Params(C.Structure):
    _fields_ = [("level", C.c_int32), ("depth", C.c_int32), ("t_min", C.c_double), ("delta", C.c_double),
                ("m_air", C.c_double), ("e_min", C.c_double), ("use_bvh", C.c_int32), ("mic_mode", C.c_int32),
                ("n_threads", C.c_int32), ("beam_begin", C.c_int64), ("beam_end", C.c_int64)]


class _Result(C.Structure):
    _fields_ = [("hit", C.c_void_p), ("flag", C.c_void_p), ("t_hit", C.c_void_p), ("count", C.c_void_p),
                ("flagged", C.c_void_p), ("power", C.c_void_p), ("e_strict", C.c_void_p),
                ("e_flag", C.c_void_p), ("counters", C.c_int64 * N_COUNTERS)]


_lib = None


def load(path: str):
    """Load a compiled oracle library from `path` and declare its entry points."""
    L = C.CDLL(path)
    L.orc_ico_nfaces.restype = C.c_int64
    L.orc_ico_nfaces.argtypes = [C.c_int]
    L.orc_icosphere.restype = C.c_int
    L.orc_icosphere.argtypes = [C.c_int, C.c_void_p]
    L.orc_solid_angle.restype = C.c_double
    L.orc_solid_angle.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_trace.restype = C.c_int
    L.orc_trace.argtypes = [C.POINTER(_Scene), C.POINTER(_Params), C.POINTER(_Result)]
    L.orc_closest_hits.restype = C.c_int
    L.orc_closest_hits.argtypes = [C.POINTER(_Scene), C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                   C.c_double, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p]
    L.orc_bvh_depth.restype = C.c_int
    L.orc_bvh_depth.argtypes = [C.POINTER(_Scene), C.c_double]
    return L


def lib():
    global _lib
    if _lib is None:
        path = _LIB if os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC) else build()
        _lib = load(path)
    return _lib


def compile_to(src: str, out: str, extra_flags=()) -> str:
    """Compile an oracle source file (the oracle itself, or a modified copy of it in a
    test) with the oracle's flags into the shared library `out`."""
    subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                           "-shared", "-pthread", "-Wall", "-Wno-unused-function", *extra_flags, "-o", out, src,
                           "-lm"])
    return out


def _ptr(a):
    return None if a is None else a.ctypes.data


def _scene_struct(scene, keep, weights=None, points=None):
    v = np.ascontiguousarray(scene.vertices, np.float32)
    t = np.ascontiguousarray(scene.triangles, np.int32)
    a = np.ascontiguousarray(scene.absorption, np.float32)
    s = np.ascontiguousarray(scene.sources, np.float32)
    w = np.ascontiguousarray(scene.power, np.float32)
    keep.extend([v, t, a, s, w])
    f32 = lambda x: float(np.float32(x))  # noqa: E731  the grid values are float32 inputs
    wt = None
    if weights is not None:
        wt = np.ascontiguousarray(weights, np.float32)
        keep.append(wt)
    pts = None
    if points is not None:
        pts = np.ascontiguousarray(points, np.float32).reshape(-1, 3)
        keep.append(pts)
    return _Scene(_ptr(v), v.shape[0], _ptr(t), t.shape[0], _ptr(a), _ptr(s), _ptr(w), s.shape[0],
                  f32(scene.mic_x0), f32(scene.mic_y0), f32(scene.mic_z), f32(scene.mic_dx), f32(scene.mic_dy),
                  scene.mic_nx, scene.mic_ny, _ptr(wt), f32(scene.mic_dz), scene.mic_nz, _ptr(pts),
                  0 if pts is None else pts.shape[0])


def icosphere(level: int) -> np.ndarray:
    """float64 [20*4**level, 3, 3]: the (d0, d1, d2) unit directions of every beam."""
    n = lib().orc_ico_nfaces(level)
    if n < 0:
        raise ValueError("level out of range")
    out = np.empty((n, 3, 3), np.float64)
    rc = lib().orc_icosphere(level, out.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"orc_icosphere failed ({rc})")
    return out


def solid_angle(d0, d1, d2) -> float:
    a, b, c = (np.ascontiguousarray(x, np.float64) for x in (d0, d1, d2))
    return lib().orc_solid_angle(a.ctypes.data, b.ctypes.data, c.ctypes.data)


@dataclasses.dataclass
class TraceResult:
    hit: np.ndarray | None        # int32 [n_beams0, depth+1]; -2 not traced, -1 escaped
    flag: np.ndarray | None       # uint8 same shape
    t_hit: np.ndarray | None      # float64 same shape
    count: np.ndarray             # int64 [depth+1]
    flagged: np.ndarray           # int64 [depth+1]
    power: np.ndarray             # float64 [depth+1]
    e_strict: np.ndarray          # float64 [n_mic]
    e_flag: np.ndarray            # float64 [n_mic]
    counters: dict

    @property
    def energy(self) -> np.ndarray:
        return self.e_strict + self.e_flag


def trace(scene, *, level=None, depth=None, t_min=T_MIN, delta=DELTA, m_air=0.0, e_min=0.0, use_bvh=True,
          mic_mode=1, n_threads=None, beam_begin=0, beam_end=-1, keep_paths=True, weights=None,
          points=None) -> TraceResult:
    """Trace the whole scene (or the initial beams [beam_begin, beam_end)) in FP64.
    weights: optional float32 [n_src][20 * 4**level] relative intensity of each source per
    icosphere face (a directional source); None = omni.
    points: optional float32 [n][3] explicit microphone points, replacing the grid (each is
    tested against every segment); energies are then per point."""
    level = scene.level if level is None else level
    depth = scene.depth if depth is None else depth
    n_threads = n_threads or default_threads()
    nb = scene.n_src * 20 * 4 ** level
    if weights is not None:
        weights = np.asarray(weights, np.float32)
        assert weights.shape == (scene.n_src, 20 * 4 ** level), weights.shape
    keep = []
    sc = _scene_struct(scene, keep, weights, points)
    pr = _Params(level, depth, t_min, delta, m_air, e_min, int(use_bvh), int(mic_mode), int(n_threads),
                 beam_begin, beam_end)
    hit = flag = th = None
    if keep_paths:
        hit = np.full((nb, depth + 1), -2, np.int32)
        flag = np.zeros((nb, depth + 1), np.uint8)
        th = np.full((nb, depth + 1), np.nan, np.float64)
    count = np.zeros(depth + 1, np.int64)
    flagged = np.zeros(depth + 1, np.int64)
    power = np.zeros(depth + 1, np.float64)
    n_mic = scene.n_mic if points is None else int(np.asarray(points).reshape(-1, 3).shape[0])
    es = np.zeros(n_mic, np.float64)
    ef = np.zeros(n_mic, np.float64)
    res = _Result(_ptr(hit), _ptr(flag), _ptr(th), _ptr(count), _ptr(flagged), _ptr(power), _ptr(es), _ptr(ef))
    rc = lib().orc_trace(C.byref(sc), C.byref(pr), C.byref(res))
    if rc != 0:
        raise RuntimeError(f"orc_trace failed ({rc})")
    counters = {name: int(res.counters[i]) for i, name in enumerate(COUNTER_NAMES)}
    return TraceResult(hit, flag, th, count, flagged, power, es, ef, counters)


def closest_hits(scene, orig, dirs, start=None, *, use_bvh=True, t_min=T_MIN, delta=DELTA):
    """Closest hit of arbitrary rays: (hit id, t, flag, node visits, triangle tests)."""
    orig = np.ascontiguousarray(orig, np.float64)
    dirs = np.ascontiguousarray(dirs, np.float64)
    n = orig.shape[0]
    st = None if start is None else np.ascontiguousarray(start, np.int32)
    keep = []
    sc = _scene_struct(scene, keep)
    hit = np.empty(n, np.int32)
    th = np.empty(n, np.float64)
    fl = np.empty(n, np.uint8)
    nv = np.empty(n, np.int64)
    tt = np.empty(n, np.int64)
    lib().orc_closest_hits(C.byref(sc), int(use_bvh), _ptr(orig), _ptr(dirs), _ptr(st), n, t_min, delta,
                           _ptr(hit), _ptr(th), _ptr(fl), _ptr(nv), _ptr(tt))
    return hit, th, fl, nv, tt


def bvh_depth(scene, margin=DELTA + 1e-6) -> int:
    keep = []
    sc = _scene_struct(scene, keep)
    return lib().orc_bvh_depth(C.byref(sc), margin)


def levels_db(energy, i0=1e-12):
    """Sound level in dB re i0 (W/m^2); zero energy maps to -inf."""
    with np.errstate(divide="ignore"):
        return 10.0 * np.log10(np.asarray(energy, np.float64) / i0)
