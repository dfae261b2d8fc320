"""Thin ctypes binding of libbt.so (include/bt.h), same names as the C ABI.

Argument marshalling only: every step of the tracer runs in the library's kernels.
PyTorch supplies device buffers (for the optional parity outputs) and the stream.
The binding fails loudly when the library is missing or no GPU is visible; there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libbt.so")

BT_OK, BT_PENDING = 0, 1
BT_MAX_LEVEL, BT_MAX_DEPTH = 9, 31
STATUS = {0: "BT_OK", 1: "BT_PENDING", -1: "BT_EINVAL", -2: "BT_ENOMEM", -3: "BT_EDEVICE",
          -4: "BT_EOVERFLOW", -5: "BT_ENOTFOUND", -6: "BT_ESTATE"}

EXPORTED = ["bt_params_default", "bt_status_str", "bt_last_error", "bt_create", "bt_destroy", "bt_memory_used",
            "bt_build_mesh", "bt_mesh_free", "bt_mesh_info", "bt_mics_grid", "bt_mics_grid3d", "bt_mics_subset", "bt_mics_points", "bt_mics_reset", "bt_mics_free",
            "bt_set_partitions",
            "bt_emit_beams", "bt_emit_beams_directional", "bt_beams_free", "bt_beams_stats", "bt_trace", "bt_trace_all",
            "bt_accumulate_mics",
            "bt_accumulate_mics_static", "bt_beams_bind_mics", "bt_levels",
            "bt_run", "bt_submit", "bt_poll", "bt_cancel", "bt_batch_run", "bt_batch_release", "bt_batch_autotune",
            "bt_server_create", "bt_server_submit", "bt_server_poll", "bt_server_destroy",
            "bt_validate_mesh", "bt_validate_sources", "bt_validate_grid", "bt_validate_params"]


class BTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class bt_params(C.Structure):
    _fields_ = [("max_depth", C.c_int32), ("t_min", C.c_double), ("edge_delta", C.c_double),
                ("air_m", C.c_double), ("e_min", C.c_double), ("queue_rounds", C.c_int32),
                ("run_records", C.c_int64), ("hit_out", C.c_void_p),
                ("flag_out", C.c_void_p), ("t_out", C.c_void_p)]


class bt_stats(C.Structure):
    _fields_ = [("generations", C.c_int32), ("count", C.c_int64 * (BT_MAX_DEPTH + 1)),
                ("flagged", C.c_int64 * (BT_MAX_DEPTH + 1)), ("power", C.c_double * (BT_MAX_DEPTH + 1)),
                ("segments", C.c_int64), ("node_visits", C.c_int64), ("tri_tests", C.c_int64),
                ("mic_tests", C.c_int64), ("mic_updates", C.c_int64), ("mic_layer_visits", C.c_int64),
                ("mic_general", C.c_int64), ("mic_fallback", C.c_int64), ("mic_classified", C.c_int64)]


class bt_request(C.Structure):
    _fields_ = [("src_xyz", C.c_void_p), ("src_power", C.c_void_p), ("n_src", C.c_int32), ("level", C.c_int32),
                ("max_depth", C.c_int32), ("mic_x0", C.c_float), ("mic_y0", C.c_float), ("mic_z", C.c_float),
                ("mic_dx", C.c_float), ("mic_dy", C.c_float), ("mic_nx", C.c_int32), ("mic_ny", C.c_int32)]


class bt_result(C.Structure):
    _fields_ = [("energy", C.c_void_p), ("flag_energy", C.c_void_p), ("segments", C.c_int64),
                ("mic_updates", C.c_int64)]


_lib = None


def lib():
    """Load libbt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1912_03998_amd/build.py")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, F32, D = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_double
    sig = {
        "bt_params_default": (None, [P]),
        "bt_status_str": (C.c_char_p, [C.c_int]),
        "bt_last_error": (C.c_char_p, [P]),
        "bt_create": (C.c_int, [C.c_int, C.c_size_t, P, P]),
        "bt_destroy": (C.c_int, [P]),
        "bt_memory_used": (C.c_int, [P, P]),
        "bt_build_mesh": (C.c_int, [P, P, I64, P, P, I64, I32, I32, P]),
        "bt_mesh_free": (C.c_int, [P]),
        "bt_mesh_info": (C.c_int, [P, P, P, P]),
        "bt_mics_grid": (C.c_int, [P, F32, F32, F32, F32, F32, I32, I32, P]),
        "bt_mics_grid3d": (C.c_int, [P, F32, F32, F32, F32, F32, F32, I32, I32, I32, P]),
        "bt_mics_subset": (C.c_int, [P, P, P, I64, P]),
        "bt_mics_points": (C.c_int, [P, P, I64, P]),
        "bt_mics_reset": (C.c_int, [P, P]),
        "bt_mics_free": (C.c_int, [P]),
        "bt_emit_beams": (C.c_int, [P, P, P, I32, I32, P]),
        "bt_emit_beams_directional": (C.c_int, [P, P, P, P, I32, I32, P]),
        "bt_beams_free": (C.c_int, [P]),
        "bt_beams_stats": (C.c_int, [P, P, P]),
        "bt_trace": (C.c_int, [P, P, P, P, P]),
        "bt_trace_all": (C.c_int, [P, P, P, P]),
        "bt_set_partitions": (C.c_int, [P, I32]),
        "bt_accumulate_mics": (C.c_int, [P, P, P, P, P]),
        "bt_accumulate_mics_static": (C.c_int, [P, P, P, P, P]),
        "bt_beams_bind_mics": (C.c_int, [P, P, P]),
        "bt_levels": (C.c_int, [P, P, P, P, P]),
        "bt_run": (C.c_int, [P, P, P, P, I32, I32, P, P, P]),
        "bt_submit": (C.c_int, [P, P, P, P]),
        "bt_poll": (C.c_int, [P, C.c_uint64, P]),
        "bt_cancel": (C.c_int, [P, C.c_uint64]),
        "bt_batch_run": (C.c_int, [P, P, P, I32, P, P, P]),
        "bt_batch_autotune": (C.c_int, [P, P, P, I32, P, P, P, P]),
        "bt_batch_release": (C.c_int, [P]),
        "bt_server_create": (C.c_int, [P, P, P, P, P]),
        "bt_server_submit": (C.c_int, [P, P, P]),
        "bt_server_poll": (C.c_int, [P, C.c_uint64, P]),
        "bt_server_destroy": (C.c_int, [P]),
        "bt_validate_mesh": (C.c_int, [P, C.c_int64, P, P, C.c_int64, I32, I32, P, C.c_size_t]),
        "bt_validate_sources": (C.c_int, [P, P, P, I32, I32, P, C.c_size_t]),
        "bt_validate_grid": (C.c_int, [C.c_float, C.c_float, C.c_float, C.c_float, C.c_float, C.c_float, I32, I32,
                                       I32, P, C.c_size_t]),
        "bt_validate_params": (C.c_int, [P, P, C.c_size_t]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _check(ctx, status, what):
    if status < 0:
        msg = lib().bt_last_error(ctx).decode() if ctx else ""
        raise BTError(status, f"{what}: {msg}")
    return status


# ---------------------------------------------------------------------------------------
# one function per C entry point (ctypes handles are c_void_p values)
# ---------------------------------------------------------------------------------------

def bt_params_default(**kw) -> bt_params:
    p = bt_params()
    lib().bt_params_default(C.byref(p))
    for k, v in kw.items():
        if k in ("hit_out", "flag_out", "t_out"):
            v = _ptr(v)
        setattr(p, k, v)
    return p


def _validated(status, buf):
    return status, buf.value.decode()


def bt_validate_mesh(xyz, tri, absorption, tiles_x=1, tiles_y=1):
    """Host-only check of bt_build_mesh's arguments: (status, reason)."""
    xyz = np.ascontiguousarray(xyz, np.float32).reshape(-1, 3)
    tri = np.ascontiguousarray(tri, np.int32).reshape(-1, 3)
    absorption = np.ascontiguousarray(absorption, np.float32)
    buf = C.create_string_buffer(512)
    return _validated(lib().bt_validate_mesh(_ptr(xyz), xyz.shape[0], _ptr(tri), _ptr(absorption), tri.shape[0],
                                             tiles_x, tiles_y, buf, len(buf)), buf)


def bt_validate_sources(src_xyz, src_power, level, src_weight=None):
    """Host-only check of bt_emit_beams(_directional)'s arguments: (status, reason)."""
    src_xyz = np.ascontiguousarray(src_xyz, np.float32).reshape(-1, 3)
    src_power = np.ascontiguousarray(src_power, np.float32)
    w = None if src_weight is None else np.ascontiguousarray(src_weight, np.float32)
    buf = C.create_string_buffer(512)
    return _validated(lib().bt_validate_sources(_ptr(src_xyz), _ptr(src_power), _ptr(w), src_xyz.shape[0], level,
                                                buf, len(buf)), buf)


def bt_validate_grid(x0, y0, z0, dx, dy, dz, nx, ny, nz):
    """Host-only check of bt_mics_grid3d's arguments: (status, reason)."""
    buf = C.create_string_buffer(512)
    return _validated(lib().bt_validate_grid(x0, y0, z0, dx, dy, dz, nx, ny, nz, buf, len(buf)), buf)


def bt_validate_params(params):
    """Host-only check of tracing parameters: (status, reason)."""
    buf = C.create_string_buffer(512)
    return _validated(lib().bt_validate_params(C.byref(params), buf, len(buf)), buf)


def bt_create(device=0, hbm_budget_bytes=0, stream=None):
    """stream: a torch.cuda.Stream (its HIP handle is passed), a raw handle, or None."""
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    out = C.c_void_p()
    _check(None, lib().bt_create(device, hbm_budget_bytes, stream, C.byref(out)), "bt_create")
    return out


def bt_destroy(ctx):
    _check(ctx, lib().bt_destroy(ctx), "bt_destroy")


def bt_memory_used(ctx) -> int:
    n = C.c_size_t()
    _check(ctx, lib().bt_memory_used(ctx, C.byref(n)), "bt_memory_used")
    return n.value


def bt_build_mesh(ctx, xyz, tri, absorption, tiles_x=1, tiles_y=1):
    xyz = np.ascontiguousarray(xyz, np.float32)
    tri = np.ascontiguousarray(tri, np.int32)
    absorption = np.ascontiguousarray(absorption, np.float32)
    out = C.c_void_p()
    _check(ctx, lib().bt_build_mesh(ctx, _ptr(xyz), xyz.shape[0], _ptr(tri), _ptr(absorption), tri.shape[0],
                                    tiles_x, tiles_y, C.byref(out)), "bt_build_mesh")
    return out


def bt_mesh_free(mesh):
    lib().bt_mesh_free(mesh)


def bt_mesh_info(mesh):
    n, d, r = C.c_int64(), C.c_int32(), C.c_int64()
    _check(None, lib().bt_mesh_info(mesh, C.byref(n), C.byref(d), C.byref(r)), "bt_mesh_info")
    return {"nodes": n.value, "max_depth": d.value, "tri_refs": r.value}


def bt_mics_grid(ctx, x0, y0, z, dx, dy, nx, ny):
    out = C.c_void_p()
    _check(ctx, lib().bt_mics_grid(ctx, x0, y0, z, dx, dy, nx, ny, C.byref(out)), "bt_mics_grid")
    return out


def bt_mics_grid3d(ctx, x0, y0, z0, dx, dy, dz, nx, ny, nz):
    out = C.c_void_p()
    _check(ctx, lib().bt_mics_grid3d(ctx, x0, y0, z0, dx, dy, dz, nx, ny, nz, C.byref(out)), "bt_mics_grid3d")
    return out


def bt_mics_subset(ctx, grid, idx):
    idx = np.ascontiguousarray(idx, np.int32).ravel()
    out = C.c_void_p()
    _check(ctx, lib().bt_mics_subset(ctx, grid, _ptr(idx), idx.size, C.byref(out)), "bt_mics_subset")
    return out


def bt_mics_points(ctx, xyz):
    xyz = np.ascontiguousarray(xyz, np.float32).reshape(-1, 3)
    out = C.c_void_p()
    _check(ctx, lib().bt_mics_points(ctx, _ptr(xyz), xyz.shape[0], C.byref(out)), "bt_mics_points")
    return out


def bt_mics_reset(ctx, mics):
    _check(ctx, lib().bt_mics_reset(ctx, mics), "bt_mics_reset")


def bt_mics_free(mics):
    lib().bt_mics_free(mics)


def bt_emit_beams(ctx, src_xyz, src_power, level, beams=None):
    src_xyz = np.ascontiguousarray(src_xyz, np.float32).reshape(-1, 3)
    src_power = np.ascontiguousarray(src_power, np.float32)
    h = C.c_void_p(beams.value if beams is not None else None)
    _check(ctx, lib().bt_emit_beams(ctx, _ptr(src_xyz), _ptr(src_power), src_xyz.shape[0], level, C.byref(h)),
           "bt_emit_beams")
    return h


def bt_emit_beams_directional(ctx, src_xyz, src_power, src_weight, level, beams=None):
    """src_weight: float32 [n_src][20 * 4**level] relative intensities per face."""
    src_xyz = np.ascontiguousarray(src_xyz, np.float32).reshape(-1, 3)
    src_power = np.ascontiguousarray(src_power, np.float32)
    src_weight = np.ascontiguousarray(src_weight, np.float32)
    if src_weight.shape != (src_xyz.shape[0], 20 * 4 ** level):
        raise ValueError(f"src_weight shape {src_weight.shape}")
    h = C.c_void_p(beams.value if beams is not None else None)
    _check(ctx, lib().bt_emit_beams_directional(ctx, _ptr(src_xyz), _ptr(src_power), _ptr(src_weight),
                                                src_xyz.shape[0], level, C.byref(h)), "bt_emit_beams_directional")
    return h


def bt_beams_free(beams):
    lib().bt_beams_free(beams)


def bt_beams_stats(ctx, beams) -> dict:
    s = bt_stats()
    _check(ctx, lib().bt_beams_stats(ctx, beams, C.byref(s)), "bt_beams_stats")
    g = s.generations
    return {"generations": g, "count": np.array(s.count[:g], np.int64), "flagged": np.array(s.flagged[:g], np.int64),
            "power": np.array(s.power[:g], np.float64), "segments": s.segments, "node_visits": s.node_visits,
            "tri_tests": s.tri_tests, "mic_tests": s.mic_tests, "mic_updates": s.mic_updates,
            "mic_layer_visits": s.mic_layer_visits, "mic_general": s.mic_general, "mic_fallback": s.mic_fallback,
            "mic_classified": s.mic_classified}


def bt_trace(ctx, mesh, beams, params, want_next=False):
    n = C.c_int64(-1)
    _check(ctx, lib().bt_trace(ctx, mesh, beams, C.byref(params), C.byref(n) if want_next else None), "bt_trace")
    return n.value if want_next else None


def bt_trace_all(ctx, mesh, beams, params):
    _check(ctx, lib().bt_trace_all(ctx, mesh, beams, C.byref(params)), "bt_trace_all")


def bt_set_partitions(ctx, k):
    _check(ctx, lib().bt_set_partitions(ctx, k), "bt_set_partitions")


def bt_accumulate_mics(ctx, mesh, beams, params, mics):
    _check(ctx, lib().bt_accumulate_mics(ctx, mesh, beams, C.byref(params), mics), "bt_accumulate_mics")


def bt_accumulate_mics_static(ctx, mesh, beams, params, mics):
    _check(ctx, lib().bt_accumulate_mics_static(ctx, mesh, beams, C.byref(params), mics), "bt_accumulate_mics_static")


def bt_beams_bind_mics(ctx, beams, mics):
    """Classify the set's new beams against a planar grid (mics None: unbind); beams None
    creates an empty set.  Returns the set."""
    h = C.c_void_p(beams.value if beams is not None else None)
    _check(ctx, lib().bt_beams_bind_mics(ctx, C.byref(h), mics), "bt_beams_bind_mics")
    return h


def bt_levels(ctx, mics, strict_out=None, flag_out=None, level_db_out=None):
    """Outputs: numpy float64 arrays or torch float64 tensors (host or device)."""
    _check(ctx, lib().bt_levels(ctx, mics, _ptr(strict_out), _ptr(flag_out), _ptr(level_db_out)), "bt_levels")


def bt_run(ctx, mesh, src_xyz, src_power, level, params, mics, beams=None):
    src_xyz = np.ascontiguousarray(src_xyz, np.float32).reshape(-1, 3)
    src_power = np.ascontiguousarray(src_power, np.float32)
    h = C.c_void_p(beams.value if beams is not None else None)
    _check(ctx, lib().bt_run(ctx, mesh, _ptr(src_xyz), _ptr(src_power), src_xyz.shape[0], level, C.byref(params),
                             mics, C.byref(h)), "bt_run")
    return h


def bt_submit(ctx, mesh, src_xyz, src_power, level, max_depth, grid):
    """grid: (x0, y0, z, dx, dy, nx, ny).  Returns the ticket."""
    src_xyz = np.ascontiguousarray(src_xyz, np.float32).reshape(-1, 3)
    src_power = np.ascontiguousarray(src_power, np.float32)
    x0, y0, z, dx, dy, nx, ny = grid
    req = bt_request(_ptr(src_xyz), _ptr(src_power), src_xyz.shape[0], level, max_depth, x0, y0, z, dx, dy, nx, ny)
    t = C.c_uint64()
    _check(ctx, lib().bt_submit(ctx, mesh, C.byref(req), C.byref(t)), "bt_submit")
    return t.value


def bt_poll(ctx, ticket, n_mic):
    """Returns None while pending, else (energy, flag_energy, segments, mic_updates)."""
    e = np.empty(n_mic, np.float64)
    f = np.empty(n_mic, np.float64)
    r = bt_result(_ptr(e), _ptr(f), 0, 0)
    s = _check(ctx, lib().bt_poll(ctx, ticket, C.byref(r)), "bt_poll")
    if s == BT_PENDING:
        return None
    return e, f, r.segments, r.mic_updates


def bt_cancel(ctx, ticket):
    _check(ctx, lib().bt_cancel(ctx, ticket), "bt_cancel")


class bt_scenario(C.Structure):
    _fields_ = [("src_xyz", C.c_void_p), ("src_power", C.c_void_p), ("n_src", C.c_int32), ("level", C.c_int32),
                ("max_depth", C.c_int32), ("mic_x0", C.c_float), ("mic_y0", C.c_float), ("mic_z", C.c_float),
                ("mic_dx", C.c_float), ("mic_dy", C.c_float), ("mic_nx", C.c_int32), ("mic_ny", C.c_int32),
                ("mic_subset", C.c_void_p), ("n_subset", C.c_int64), ("energy_out", C.c_void_p),
                ("flag_out", C.c_void_p)]


class bt_batch_opts(C.Structure):
    _fields_ = [("chunk_beams", C.c_int64), ("blocks_per_cu", C.c_int32), ("use_graph", C.c_int32)]


class bt_batch_stats(C.Structure):
    _fields_ = [("chunks", C.c_int32), ("beams0", C.c_int64), ("segments", C.c_int64), ("mic_updates", C.c_int64),
                ("seconds", C.c_double)]


BT_TUNE_MAX_CANDIDATES = 32


class Scenario:
    """One scenario of a batch: sources, level, depth, microphone grid (x0, y0, z, dx, dy,
    nx, ny) and an optional subset of grid indices.  After the batch runs, `energy` and
    `flag` hold its outputs."""

    def __init__(self, src_xyz, src_power, level, max_depth, grid, subset=None):
        self.src = np.ascontiguousarray(src_xyz, np.float32).reshape(-1, 3)
        self.power = np.ascontiguousarray(src_power, np.float32)
        self.level, self.max_depth, self.grid = int(level), int(max_depth), tuple(grid)
        self.subset = None if subset is None else np.ascontiguousarray(subset, np.int32)
        nx, ny = int(grid[5]), int(grid[6])
        n_out = len(self.subset) if self.subset is not None else nx * ny
        self.energy = np.zeros(n_out, np.float64)
        self.flag = np.zeros(n_out, np.float64)

    def struct(self) -> bt_scenario:
        x0, y0, z, dx, dy, nx, ny = self.grid
        return bt_scenario(_ptr(self.src), _ptr(self.power), self.src.shape[0], self.level, self.max_depth, x0, y0, z,
                           dx, dy, nx, ny, _ptr(self.subset), 0 if self.subset is None else len(self.subset),
                           _ptr(self.energy), _ptr(self.flag))


def _scenario_array(scenarios):
    arr = (bt_scenario * max(len(scenarios), 1))()
    for k, s in enumerate(scenarios):
        arr[k] = s.struct()
    return arr


def bt_batch_run(ctx, mesh, scenarios, params=None, opts=None) -> dict:
    """Runs the Scenario objects (their energy / flag arrays are filled); returns the stats."""
    arr = _scenario_array(scenarios)
    st = bt_batch_stats()
    o = None if opts is None else (opts if isinstance(opts, bt_batch_opts) else bt_batch_opts(**opts))
    _check(ctx, lib().bt_batch_run(ctx, mesh, arr, len(scenarios), None if params is None else C.byref(params),
                                   None if o is None else C.byref(o), C.byref(st)), "bt_batch_run")
    return {"chunks": st.chunks, "beams0": st.beams0, "segments": st.segments, "mic_updates": st.mic_updates,
            "seconds": st.seconds}


def bt_batch_release(ctx):
    _check(ctx, lib().bt_batch_release(ctx), "bt_batch_release")


def bt_batch_autotune(ctx, mesh, scenarios, params=None):
    """Returns (chosen options as a dict, per-candidate seconds)."""
    arr = _scenario_array(scenarios)
    out = bt_batch_opts()
    secs = (C.c_double * BT_TUNE_MAX_CANDIDATES)()
    nc = C.c_int32()
    _check(ctx, lib().bt_batch_autotune(ctx, mesh, arr, len(scenarios), None if params is None else C.byref(params),
                                        C.byref(out), secs, C.byref(nc)), "bt_batch_autotune")
    return ({"chunk_beams": out.chunk_beams, "blocks_per_cu": out.blocks_per_cu, "use_graph": out.use_graph},
            list(secs[:nc.value]))


BT_SERVE_BATCHED, BT_SERVE_PLAIN = 0, 1


class bt_server_opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("max_records", C.c_int64), ("arena_bytes", C.c_int64),
                ("blocks_per_cu", C.c_int32)]


class bt_serve_result(C.Structure):
    _fields_ = [("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


def bt_server_create(ctx, mesh, params=None, mode=BT_SERVE_BATCHED, max_records=0, arena_bytes=0, blocks_per_cu=0):
    o = bt_server_opts(mode, max_records, arena_bytes, blocks_per_cu)
    out = C.c_void_p()
    _check(ctx, lib().bt_server_create(ctx, mesh, None if params is None else C.byref(params), C.byref(o),
                                       C.byref(out)), "bt_server_create")
    return out


def bt_server_submit(ctx, server, scenario) -> int:
    """scenario: a Scenario; its energy / flag arrays receive the outputs."""
    t = C.c_uint64()
    sc = scenario.struct()
    _check(ctx, lib().bt_server_submit(server, C.byref(sc), C.byref(t)), "bt_server_submit")
    return t.value


def bt_server_poll(ctx, server, ticket):
    """None while pending, else (t_submit, t_admit, t_done) in seconds since the server started."""
    r = bt_serve_result()
    s = _check(ctx, lib().bt_server_poll(server, ticket, C.byref(r)), "bt_server_poll")
    if s == BT_PENDING:
        return None
    return r.t_submit, r.t_admit, r.t_done


def bt_server_destroy(ctx, server):
    _check(ctx, lib().bt_server_destroy(server), "bt_server_destroy")


class Server:
    """A request server on (ctx, mesh): submit Scenario objects, poll their tickets.  The
    submitted Scenario objects are kept alive here until their outputs are written."""

    def __init__(self, ctx, mesh, params=None, mode=BT_SERVE_BATCHED, **opts):
        self.ctx = ctx
        self.h = bt_server_create(ctx, mesh, params, mode, **opts)
        self.live = {}

    def submit(self, scenario) -> int:
        t = bt_server_submit(self.ctx, self.h, scenario)
        self.live[t] = scenario
        return t

    def poll(self, ticket):
        r = bt_server_poll(self.ctx, self.h, ticket)
        if r is not None:
            self.live.pop(ticket, None)
        return r

    def close(self):
        if self.h is not None:
            bt_server_destroy(self.ctx, self.h)
            self.h = None
            self.live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
