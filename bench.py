#!/usr/bin/env python
"""Throughput of the hybrid beam tracer on one MI355X: beam segments/s and microphone
updates/s on the synthetic 2 x 2 km district (331,815 triangles, 64 sources x 81,920
beams, depth 8, 250,000 microphones, 4 x 4 on-device tiles).

A step is one pass of the whole hot path over the workload: emission, then for every
generation the trace (closest hit, tile hand-off, reflection + compaction) and the
microphone accumulation, then the levels.  The mesh and its hierarchy are built once
before timing (reported separately as setup).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_1912_03998_amd", "csrc")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "trace_pmc_district.txt")
REF_WORK = os.path.join(ROOT, "oracle", "reference_work.json")

# algorithmic bytes (canonical record sizes): a beam record 80 B read, a child record
# 80 B written, an 8 B hit record, 64 B per hierarchy node fetched, 36 B per triangle
# tested, 16 B (FP64 read + write) per microphone update
B_BEAM, B_CHILD, B_HIT, B_NODE, B_TRI, B_MIC = 80, 80, 8, 64, 36, 16


DEVICE_HEADERS = ("bt_device.h", "bt_internal.h")   # what the .hip files include besides include/bt.h


def kernel_hash() -> str:
    """Hash of the device code: the kernel sources, the library headers they include and
    the public header (host-only sources such as bt_host.h do not change it)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith(".hip") or name in DEVICE_HEADERS:
            h.update(name.encode())
            h.update(open(os.path.join(CSRC, name), "rb").read())
    h.update(b"bt.h")
    h.update(open(os.path.join(ROOT, "include", "bt.h"), "rb").read())
    return h.hexdigest()[:16]


def pmc_traffic(n_launch_units):
    """HBM bytes per trace launch from the committed rocprofv3 --pmc summary, or None
    when the summary is missing or the kernel source changed since it was taken."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    text = open(PMC_SUMMARY).read()
    m = re.search(r"kernel_sha256_16:\s*([0-9a-f]+)", text)
    b = re.search(r"hbm_bytes_per_step:\s*([0-9.eE+]+)", text)
    if not m or not b or m.group(1) != kernel_hash():
        return None
    return float(b.group(1)) / n_launch_units


def host_facts():
    """The host's logical CPU count and CPU model (from /proc/cpuinfo)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"host_nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(scene, single_sources=16):
    """The FP64 oracle as it stands on the host: every logical CPU (os.cpu_count(), one
    thread each) over the whole workload, and one thread over a bounded sample (the first
    `single_sources` sources, the paper's sequential reference point)."""
    from oracle import oracle as O

    threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    r = O.trace(scene, keep_paths=False, n_threads=threads)
    dt = time.perf_counter() - t0
    k = min(single_sources, scene.n_src)
    one = scene.with_(sources=scene.sources[:k], power=scene.power[:k])
    t0 = time.perf_counter()
    r1 = O.trace(one, keep_paths=False, n_threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": r.counters["segments"] / dt, "unit": "beam-segments/s", "cores": threads, "kind": "oracle",
            "sample": f"whole workload ({r.counters['segments']} segments, {r.counters['mic_updates']} mic updates) "
                      f"in {dt:.2f} s on {threads} threads", "mic_updates_per_s": r.counters["mic_updates"] / dt,
            "single_thread": {"value": r1.counters["segments"] / dt1, "unit": "beam-segments/s", "cores": 1,
                              "sample": f"sources 0-{k - 1} of the workload ({r1.counters['segments']} segments, "
                                        f"{r1.counters['mic_updates']} mic updates) in {dt1:.2f} s",
                              "mic_updates_per_s": r1.counters["mic_updates"] / dt1},
            **host_facts()}


def batch_bench(sess, seed=0, n=256):
    """The batched form: n uneven scenarios on the district (sources on streets, 1280 to
    81920 beams per source, depth 2-10, a random 10 k microphone subset each), autotuned,
    in one call, against the same scenarios run one by one through the plain path."""
    import numpy as np
    from paper_1912_03998_amd import bt
    from scenegen import batch_scenarios

    specs = batch_scenarios(seed, n)

    def scenarios():
        return [bt.Scenario(q.sources, q.power, q.level, q.depth, q.grid, q.subset) for q in specs]

    print(f"[bench] batch: {n} scenarios, {sum(q.n_beams0 for q in specs)} generation-0 beams; autotune ...",
          file=sys.stderr, flush=True)
    opts, cand = bt.bt_batch_autotune(sess.ctx, sess.mesh, scenarios())
    scs = scenarios()
    t0 = time.perf_counter()
    st = bt.bt_batch_run(sess.ctx, sess.mesh, scs, opts=opts)
    batched_s = time.perf_counter() - t0
    print(f"[bench] batch: {batched_s:.3f} s with {opts}; sequential ...", file=sys.stderr, flush=True)
    grid = tuple(float(v) for v in specs[0].grid[:5]) + tuple(int(v) for v in specs[0].grid[5:])
    t0 = time.perf_counter()
    worst = 0.0
    for q, sc in zip(specs, scs):
        r = sess.run(q.sources, q.power, q.level, q.depth, grid, parity=False, stats=False)
        e = (r.e_strict + r.e_flag)[q.subset]
        worst = max(worst, float(np.abs(e - sc.energy).max() / max(np.abs(e).max(), 1e-300)))
    seq_s = time.perf_counter() - t0
    return {"scenarios": n, "beams0": st["beams0"], "segments": st["segments"], "mic_updates": st["mic_updates"],
            "chunks": st["chunks"], "opts": opts, "autotune_candidate_s": [round(x, 4) for x in cand],
            "batched_s": round(batched_s, 4), "batched_segments_per_s": st["segments"] / batched_s,
            "sequential_s": round(seq_s, 4), "sequential_segments_per_s": st["segments"] / seq_s,
            "speedup_vs_sequential": round(seq_s / batched_s, 3), "max_rel_diff_vs_sequential": worst}


def serve_bench(sess, rates, n_of_rate, warm_frac=0.1, seed=0, saturation=400):
    """The serving form: Poisson request streams (1-32 sources on streets, 5120 or 20480
    beams per source, depth 3-8, 1 k-50 k microphone rectangles) at each rate, through the
    continuously batched server and through the plain one-request-at-a-time server; p50 /
    p99 latency (completion minus submission, server clock) over the requests after the
    warm-up ones, and the rate at which a closed burst of requests completes."""
    import numpy as np
    from paper_1912_03998_amd import bt
    from scenegen import serving_requests

    def run(mode, reqs, paced):
        scs = [bt.Scenario(q.sources, q.power, q.level, q.depth, q.grid) for q in reqs]
        with bt.Server(sess.ctx, sess.mesh, mode=mode) as srv:
            out, todo = {}, {}
            t0 = time.perf_counter()
            for k, sc in enumerate(scs):
                while paced and time.perf_counter() - t0 < reqs[k].arrival:
                    for t in list(todo):
                        r = srv.poll(t)
                        if r is not None:
                            out[todo.pop(t)] = r
                    time.sleep(0.0001)
                todo[srv.submit(sc)] = k
            while todo:
                for t in list(todo):
                    r = srv.poll(t)
                    if r is not None:
                        out[todo.pop(t)] = r
                time.sleep(0.0001)
            wall = time.perf_counter() - t0
        return scs, out, wall

    res = {"rates": {}}
    energies = {}
    for rate in rates:
        n = n_of_rate(rate)
        reqs = serving_requests(seed, n, rate)
        w = int(n * warm_frac)
        row = {"requests": n, "warmup": w, "offered_beams0_per_s": rate * float(np.mean([q.n_beams0 for q in reqs]))}
        for mode, name in ((bt.BT_SERVE_BATCHED, "batched"), (bt.BT_SERVE_PLAIN, "plain")):
            print(f"[bench] serve {name} at {rate} req/s, {n} requests ...", file=sys.stderr, flush=True)
            scs, out, wall = run(mode, reqs, True)
            lat = np.array([out[k][2] - out[k][0] for k in range(w, n)])
            span = max(out[k][2] for k in range(w, n)) - min(out[k][0] for k in range(w, n))
            row[name] = {"p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
                         "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
                         "mean_ms": round(1e3 * float(lat.mean()), 3),
                         "completed_per_s": round((n - w) / span, 2)}
            energies[(rate, name)] = [sc.energy for sc in scs]
        a, b = energies[(rate, "batched")], energies[(rate, "plain")]
        row["max_rel_diff_batched_vs_plain"] = max(float(np.abs(x - y).max() / max(np.abs(y).max(), 1e-300))
                                                   for x, y in zip(a, b))
        res["rates"][str(rate)] = row
    # closed burst: every request submitted at once, completion rate of each server
    reqs = serving_requests(seed + 1, saturation, 1e9)
    sat = {"requests": saturation}
    for mode, name in ((bt.BT_SERVE_BATCHED, "batched"), (bt.BT_SERVE_PLAIN, "plain")):
        print(f"[bench] serve {name} burst of {saturation} ...", file=sys.stderr, flush=True)
        _, out, wall = run(mode, reqs, False)
        sat[name + "_req_per_s"] = round(saturation / wall, 2)
        sat[name + "_beams0_per_s"] = sum(q.n_beams0 for q in reqs) / wall
    sat["speedup"] = round(sat["batched_req_per_s"] / sat["plain_req_per_s"], 3)
    res["saturation"] = sat
    return res


def two_slot_bench(scene, steps=5, warmup=2, run_records=1 << 24, partitions=2):
    """The whole step as one bt_run call with a record budget below the workload's
    n_beams0 (depth + 1): two generation slots and a microphone pass per generation, in a
    session of its own (so its device memory is what this form needs)."""
    import numpy as np
    import torch
    from paper_1912_03998_amd import bt
    from paper_1912_03998_amd.tracer import Session, scene_grid

    sess = Session.from_scene(scene)
    ctx, mesh, stream = sess.ctx, sess.mesh, sess.stream
    bt.bt_set_partitions(ctx, partitions)
    mics = sess._mics(scene_grid(scene))
    params = sess.params(scene.depth, run_records=run_records)
    src = np.ascontiguousarray(scene.sources, np.float32)
    pw = np.ascontiguousarray(scene.power, np.float32)
    e = np.zeros(scene.n_mic)

    def step():
        bt.bt_mics_reset(ctx, mics)
        sess.beams = bt.bt_run(ctx, mesh, src, pw, scene.level, params, mics, sess.beams)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    each = []
    for _ in range(steps):
        step()
        torch.cuda.synchronize()
        each.append(time.perf_counter())
    bt.bt_levels(ctx, mics, e, None, None)
    dt = (time.perf_counter() - t0) / steps
    print(f"[bench] two-slot steps (ms): {[round((b - a) * 1e3, 3) for a, b in zip([t0] + each, each)]}",
          file=sys.stderr, flush=True)
    used = bt.bt_memory_used(ctx)
    sess.close()
    return {"step_call": f"bt_run with run_records = {run_records} (two generation slots)", "ms_per_step": round(dt * 1e3, 3),
            "device_memory_bytes": used}


def points_bench(sess, scene, n_points=100_000, steps=3, seed=0):
    """Explicit receivers on the district: n_points uniform over the 2 x 2 km at heights
    U(1.5, 30) m, all sources, against the planar grid pass of the same step."""
    import numpy as np
    import torch
    from paper_1912_03998_amd import bt

    rng = np.random.default_rng(seed)
    pts = rng.uniform([-1000.0, -1000.0, 1.5], [1000.0, 1000.0, 30.0], (n_points, 3)).astype(np.float32)
    ctx, mesh, stream = sess.ctx, sess.mesh, sess.stream
    params = sess.params(scene.depth)
    t0 = time.perf_counter()
    mics = bt.bt_mics_points(ctx, pts)
    torch.cuda.synchronize()
    index_s = time.perf_counter() - t0
    src = np.ascontiguousarray(scene.sources, np.float32)
    pw = np.ascontiguousarray(scene.power, np.float32)
    mic_ms, upd = [], 0
    for k in range(steps + 1):
        sess.beams = bt.bt_emit_beams(ctx, src, pw, scene.level, sess.beams)
        bt.bt_mics_reset(ctx, mics)
        for _ in range(scene.depth + 1):
            bt.bt_trace(ctx, mesh, sess.beams, params)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        bt.bt_accumulate_mics(ctx, mesh, sess.beams, params, mics)
        ev[1].record(stream)
        torch.cuda.synchronize()
        if k > 0:
            mic_ms.append(ev[0].elapsed_time(ev[1]))
        st = bt.bt_beams_stats(ctx, sess.beams)
        upd = st["mic_updates"]
    e = np.zeros(n_points)
    bt.bt_levels(ctx, mics, e, None, None)
    bt.bt_mics_free(mics)
    ms = sorted(mic_ms)[len(mic_ms) // 2]
    return {"workload": f"district, all sources, {n_points} receivers uniform over the district at 1.5-30 m",
            "mic_stage_ms": round(ms, 3), "mic_updates_per_step": upd, "mic_tests_per_step": st["mic_tests"],
            "mic_updates_per_s": upd / (ms * 1e-3), "receivers_reached": int((e > 0).sum()),
            "index_build_s": round(index_s, 3)}


def volumetric_bench(steps, warmup, chunk=7, level=8, oracle_sample=True, partitions=2):
    """The paper's experiment shape: the tall 2.5 x 1.5 km district (towers of 200 m and
    more), 49 street sources x 20 * 4**level beams, depth 8, microphones every 4 m filling
    the bounding box.  A step traces all sources, `chunk` sources per beam set (the queue
    holds every generation of a chunk), into one volumetric grid, then the levels."""
    import numpy as np
    import torch
    from paper_1912_03998_amd import bt
    from paper_1912_03998_amd.tracer import Session, scene_grid
    from scenegen import volumetric_scene

    t0 = time.perf_counter()
    scene = volumetric_scene(0, level=level)
    print(f"[bench] {scene.name}: {scene.n_tri} triangles, {scene.n_src} x {20 * 4 ** level} beams, depth "
          f"{scene.depth}, {scene.mic_nx} x {scene.mic_ny} x {scene.mic_nz} = {scene.n_mic} mics", file=sys.stderr,
          flush=True)
    sess = Session.from_scene(scene)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    ctx, mesh, stream = sess.ctx, sess.mesh, sess.stream
    bt.bt_set_partitions(ctx, partitions)
    mics = sess._mics(scene_grid(scene))
    params = sess.params(scene.depth)
    with torch.cuda.stream(stream):
        level_out = torch.empty(scene.n_mic, dtype=torch.float64, device="cuda")
    src = np.ascontiguousarray(scene.sources, np.float32)
    pw = np.ascontiguousarray(scene.power, np.float32)
    groups = [slice(k, min(k + chunk, scene.n_src)) for k in range(0, scene.n_src, chunk)]
    totals = {"segments": 0, "mic_updates": 0, "mic_tests": 0, "mic_layer_visits": 0, "mic_general": 0,
              "mic_fallback": 0}

    def step(ev=None, count=False):
        bt.bt_mics_reset(ctx, mics)
        for gi, g in enumerate(groups):
            sess.beams = bt.bt_emit_beams(ctx, src[g], pw[g], scene.level, sess.beams)
            if ev is not None:
                ev[gi][0].record(stream)
            bt.bt_trace_all(ctx, mesh, sess.beams, params)
            if ev is not None:
                ev[gi][1].record(stream)
            bt.bt_accumulate_mics(ctx, mesh, sess.beams, params, mics)
            if ev is not None:
                ev[gi][2].record(stream)
            if count:
                st = bt.bt_beams_stats(ctx, sess.beams)
                for k in totals:
                    totals[k] += st[k]
        bt.bt_levels(ctx, mics, None, None, level_out)

    step(count=True)
    for _ in range(max(warmup - 1, 0)):
        step()
    events = [[[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in groups] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(events[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    trace_ms = sum(e[0].elapsed_time(e[1]) for ev in events for e in ev) / steps
    mic_ms = sum(e[1].elapsed_time(e[2]) for ev in events for e in ev) / steps
    e = level_out.cpu().numpy()
    out = {
        "workload": f"{scene.name}: {scene.n_tri} triangles, {scene.n_src} sources x {20 * 4 ** level} beams "
                    f"(icosphere level {level}), depth {scene.depth}, {scene.mic_nx} x {scene.mic_ny} x "
                    f"{scene.mic_nz} = {scene.n_mic} microphones (4 m lattice filling the bounding box), "
                    f"{len(groups)} beam sets of <= {chunk} sources",
        "step_call": f"per beam set: bt_emit_beams ({partitions} partitions), bt_trace_all, bt_accumulate_mics",
        "ms_per_step": round(elapsed * 1000.0 / steps, 2),
        "beam_segments_per_s": totals["segments"] * steps / elapsed,
        "mic_updates_per_s": totals["mic_updates"] * steps / elapsed,
        "segments_per_step": totals["segments"], "mic_updates_per_step": totals["mic_updates"],
        "mic_tests_per_step": totals["mic_tests"],
        "mic_layer_visits_per_step": totals["mic_layer_visits"],
        "mic_general_items_per_step": totals["mic_general"], "mic_general_in_place_per_step": totals["mic_fallback"],
        "kernel_ms_per_step": {"trace": round(trace_ms, 2), "mics": round(mic_ms, 2)},
        "mic_stage_effective_GBps": round(B_MIC * totals["mic_updates"] / (mic_ms * 1e-3) / 1e9, 1),
        "mics_reached": int(np.isfinite(e).sum()),
        "setup_s": round(setup_s, 2),
    }
    # the same step as one bt_run call over all sources: the library takes them in chunks
    # (every generation of a chunk resident) and runs each partition's trace and
    # microphone pass back to back on the partition's stream
    run_params = sess.params(scene.depth, run_records=1 << 28)
    run_beams = [None]

    def run_step():
        bt.bt_mics_reset(ctx, mics)
        run_beams[0] = bt.bt_run(ctx, mesh, src, pw, scene.level, run_params, mics, run_beams[0])
        bt.bt_levels(ctx, mics, None, None, level_out)

    for _ in range(max(warmup, 1)):
        run_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run_step()
    torch.cuda.synchronize()
    run_elapsed = time.perf_counter() - t0
    st = bt.bt_beams_stats(ctx, run_beams[0])
    bt.bt_beams_free(run_beams[0])
    out["one_call"] = {
        "step_call": f"bt_run over all {scene.n_src} sources (run_records = 2^28: the library's source chunks, "
                     "every generation of a chunk resident), then bt_levels",
        "ms_per_step": round(run_elapsed * 1000.0 / steps, 2),
        "segments_per_step": st["segments"], "mic_updates_per_step": st["mic_updates"],
        "same_counts_as_beam_sets": st["segments"] == totals["segments"] and
                                    st["mic_updates"] == totals["mic_updates"],
    }
    sess.close()
    if oracle_sample:
        # the oracle on one whole source of the same workload (bounded CPU time)
        from oracle import oracle as O
        one = scene.with_(sources=scene.sources[20:21], power=scene.power[20:21])
        threads = os.cpu_count() or 1
        print("[bench] volumetric cpu baseline (oracle, one source) ...", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        r = O.trace(one, keep_paths=False, n_threads=threads)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": r.counters["segments"] / dt, "unit": "beam-segments/s", "cores": threads,
                               "kind": "oracle", "mic_updates_per_s": r.counters["mic_updates"] / dt,
                               "sample": f"one source (index 20) of the workload: {r.counters['segments']} "
                                         f"segments, {r.counters['mic_updates']} mic updates in {dt:.2f} s"}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, help="0 tiny, 1 block, 2 district (default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tiles", type=int, default=0, help="override the tile partition (n x n)")
    ap.add_argument("--no-classify", action="store_true",
                    help="leave the beam set unbound (bt_beams_bind_mics not called): the microphone pass decides "
                         "every segment's planar class from its frustum")
    ap.add_argument("--run-call", action="store_true",
                    help="time each step as one bt_run call (source chunks, two generation slots, a microphone "
                         "pass per generation) instead of bt_emit_beams, bt_trace_all and one bt_accumulate_mics")
    ap.add_argument("--partitions", type=int, default=2,
                    help="partitions of the beam set (bt_set_partitions): the sources split into this many groups, "
                         "each traced and accumulated on a stream of its own (1 = one stream)")
    ap.add_argument("--per-generation", action="store_true",
                    help="trace with one bt_trace call per generation (the partitions' streams joined after each) "
                         "instead of one bt_trace_all call")
    ap.add_argument("--queue-rounds", type=int, default=-1,
                    help="per-tile queue rounds of the trace (0 = in-lane tile walk; default: the library's)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-scenario measurement")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--serve-seeds", type=int, default=1,
                    help="request streams per rate (seeds 0 .. N-1; the configured workload names seeds 0-2, "
                         "each adding about two minutes)")
    ap.add_argument("--serve-short", action="store_true",
                    help="serving on short streams (300 / 800 / 2200 requests at 50 / 200 / 800 req/s) instead of "
                         "the configured 200 warm-up + 2000 measured requests per rate")
    ap.add_argument("--no-volumetric", action="store_true", help="skip the volumetric (tall district) measurement")
    ap.add_argument("--no-points", action="store_true", help="skip the explicit-receiver measurement")
    ap.add_argument("--no-two-slot", action="store_true",
                    help="skip the two-generation-slot bt_run measurement (profiles of the default step)")
    ap.add_argument("--volumetric-only", action="store_true",
                    help="only the volumetric measurement (prints its JSON object; for profiling)")
    ap.add_argument("--vol-chunk", type=int, default=7, help="sources per beam set in the volumetric measurement")
    ap.add_argument("--vol-level", type=int, default=8, help="icosphere level of the volumetric measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (HBM counter calibration)")
    ap.add_argument("--gather-calibration", action="store_true",
                    help="only run a gather of one 8-byte value from each of 8 Mi distinct 128-byte lines "
                         "(HBM counter calibration for scattered reads)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the tracer runs on one device)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = 1 << 30
        a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": 3}), flush=True)
        return
    if args.gather_calibration:
        # 8 Mi distinct 128-byte lines of a 1 GiB array, one FP64 value read from each, in a
        # random order: 1 GiB of lines fetched, 64 MiB of values written
        lines = 1 << 23
        src = torch.ones(lines * 16, dtype=torch.float64, device="cuda")
        idx = (torch.randperm(lines, device="cuda") * 16).contiguous()
        for _ in range(3):
            dst = torch.index_select(src, 0, idx)
        torch.cuda.synchronize()
        print(json.dumps({"gather_lines": lines, "line_bytes": 128, "values_written_bytes": lines * 8,
                          "gathers": 3, "checksum": float(dst.sum().item())}), flush=True)
        return

    from paper_1912_03998_amd import bt
    from paper_1912_03998_amd.tracer import Session, scene_grid
    from scenegen import config_scene

    if args.volumetric_only:
        print(json.dumps(volumetric_bench(args.steps, args.warmup, args.vol_chunk, args.vol_level,
                                          oracle_sample=not args.no_cpu_baseline, partitions=args.partitions)),
              flush=True)
        return

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    scene = config_scene(args.config)
    print(f"[bench] {scene.name}: {scene.n_tri} triangles, {scene.n_beams0} beams, depth {scene.depth}, "
          f"{scene.n_mic} mics, tiles {scene.tiles_x}x{scene.tiles_y}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    sess = Session.from_scene(scene, tiles=(args.tiles, args.tiles) if args.tiles > 0 else None)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    ctx, mesh, stream = sess.ctx, sess.mesh, sess.stream
    bt.bt_set_partitions(ctx, args.partitions)
    parts = min(args.partitions, scene.n_src) if scene.n_src >= 2 else 1
    grid = scene_grid(scene)
    mics = sess._mics(grid)
    params = sess.params(scene.depth) if args.queue_rounds < 0 else \
        sess.params(scene.depth, queue_rounds=args.queue_rounds)
    D = scene.depth
    with torch.cuda.stream(stream):
        level_out = torch.empty(scene.n_mic, dtype=torch.float64, device="cuda")
    src = np.ascontiguousarray(scene.sources, np.float32)
    pw = np.ascontiguousarray(scene.power, np.float32)
    if not args.no_classify and not args.run_call:
        # set-up, once: beams are classified for the grid as they are created
        sess.beams = bt.bt_beams_bind_mics(ctx, sess.beams, mics)

    def step(ev=None):
        # ev: [trace start, trace end, microphones end, step start, step end]
        if ev is not None:
            ev[3].record(stream)
        if args.run_call:
            # one call: its stages are not separated (the whole step counts as the trace stage)
            bt.bt_mics_reset(ctx, mics)
            if ev is not None:
                ev[0].record(stream)
            sess.beams = bt.bt_run(ctx, mesh, src, pw, scene.level, params, mics, sess.beams)
            if ev is not None:
                ev[1].record(stream)
                ev[2].record(stream)
            bt.bt_levels(ctx, mics, None, None, level_out)
            if ev is not None:
                ev[4].record(stream)
            return
        # emission, every generation's trace, one microphone pass over all of them, with
        # events between the stages
        sess.beams = bt.bt_emit_beams(ctx, src, pw, scene.level, sess.beams)
        bt.bt_mics_reset(ctx, mics)
        if ev is not None:
            ev[0].record(stream)
        if args.per_generation:
            for g in range(D + 1):
                bt.bt_trace(ctx, mesh, sess.beams, params)
        else:
            bt.bt_trace_all(ctx, mesh, sess.beams, params)
        if ev is not None:
            ev[1].record(stream)
        bt.bt_accumulate_mics(ctx, mesh, sess.beams, params, mics)
        if ev is not None:
            ev[2].record(stream)
        bt.bt_levels(ctx, mics, None, None, level_out)
        if ev is not None:
            ev[4].record(stream)

    for _ in range(args.warmup):
        step()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = bt.bt_beams_stats(ctx, sess.beams)
    trace_ms = sum(events[k][0].elapsed_time(events[k][1]) for k in range(args.steps))
    mic_ms = sum(events[k][1].elapsed_time(events[k][2]) for k in range(args.steps))
    trace_ms /= args.steps
    mic_ms /= args.steps
    ms_per_step = elapsed * 1000.0 / args.steps
    each_ms = sorted(events[k][3].elapsed_time(events[k][4]) for k in range(args.steps))
    segs, upd = st["segments"], st["mic_updates"]

    # algorithmic bytes of the trace kernel, fixed by the oracle's reference traversal
    ref = json.load(open(REF_WORK)).get(scene.name) if os.path.exists(REF_WORK) else None
    roofline = None
    if ref is not None:
        trace_bytes = (B_BEAM + B_HIT) * ref["segments"] + B_CHILD * ref["children"] + \
            B_NODE * ref["node_visits"] + B_TRI * ref["tri_tests"]
        mic_bytes = B_MIC * ref["mic_updates"]
        # the trace stage is what the trace call launches per generation and partition:
        # k_trace, k_tcount, k_reflect (in-lane tile walk), or with per-tile queues k_tbin,
        # (k_tscan, k_tscatter, k_ttrace) per queued round, k_tcount, k_reflect; the
        # microphone stage is the five kernels of one bt_accumulate_mics call per partition
        q = params.queue_rounds
        trace_dominant = trace_ms >= mic_ms
        if trace_dominant:
            dominant = "k_trace+k_tcount+k_reflect" if q == 0 else \
                "k_tbin+k_tscan+k_tscatter+k_ttrace+k_tcount+k_reflect"
        else:
            dominant = "k_mics_plane+k_mics_general+k_mic_rows+k_mics_big+k_mic_spans"
        t_dom = trace_ms if trace_dominant else mic_ms
        b_dom = trace_bytes if trace_dominant else mic_bytes
        # every partition launches the stage's kernels
        launches = ((3 if q == 0 else 3 + 3 * q) * (D + 1) if trace_dominant else 5) * parts
        achieved = b_dom / (t_dom * 1e-3) / 1e9
        traffic = pmc_traffic(launches) if trace_dominant and q == 0 else None
        frac_alg = round(achieved / HBM_PEAK_GBS, 4)
        # measured: the HBM bytes rocprofv3 counted for the stage (FETCH_SIZE + WRITE_SIZE,
        # calibrated) over the stage's time, against the same peak
        frac_meas = round(traffic * launches / (t_dom * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if traffic else None
        roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": frac_alg, "frac_algorithmic": frac_alg, "frac_measured": frac_meas,
                    "traffic": traffic, "traffic_unit": "HBM bytes per launch (stage total / launches)",
                    "algorithmic_bytes_per_step": b_dom, "launches_per_step": launches,
                    "kernel_ms_per_step": round(t_dom, 3),
                    "timing": "HIP events on the context's stream around the stage's call, whose partition "
                              "streams fork from and join to it: the stage's wall-clock span per step (its kernels "
                              "on the two streams overlap; the per-launch duration is that span over the "
                              "launches, the figure the dispatch trace's span line in profiles/ gives)"}
    gpu_bytes = (B_BEAM + B_HIT) * segs + B_NODE * st["node_visits"] + B_TRI * st["tri_tests"]

    out = {
        "metric": "beam-segments/s + mic updates/s on district mesh",
        "value": segs * args.steps / elapsed,
        "unit": "beam-segments/s",
        "mic_updates_per_s": upd * args.steps / elapsed,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 rays / f32 geometry",
        "data": "synthetic",
        "config": {"workload": f"{scene.name}: {scene.n_tri} triangles, {scene.n_src} sources x "
                               f"{20 * 4 ** scene.level} beams (icosphere level {scene.level}), depth {scene.depth}, "
                               f"{scene.n_mic} microphones, "
                               f"{args.tiles or scene.tiles_x}x{args.tiles or scene.tiles_y} tiles",
                   "segments_per_step": segs, "mic_updates_per_step": upd,
                   "mic_tests_per_step": st["mic_tests"],
                   "generation_counts": st["count"].tolist(),
                   "flagged_per_generation": st["flagged"].tolist()},
        "roofline": roofline,
        "kernel_ms_per_step": {"trace": round(trace_ms, 3), "mics": round(mic_ms, 3)},
        "step_ms_events": {"median": round(float(np.median(each_ms)), 3), "min": round(each_ms[0], 3),
                           "max": round(each_ms[-1], 3),
                           "note": "HIP events on the context's stream around each timed step (emission to levels)"},
        "gpu_hierarchy_bytes_per_s": gpu_bytes / (trace_ms * 1e-3) if trace_ms > 0 else None,
        "gpu_node_visits_per_segment": st["node_visits"] / max(segs, 1),
        "gpu_tri_tests_per_segment": st["tri_tests"] / max(segs, 1),
        "setup_s": round(setup_s, 3),
        "step_call": "bt_run (source chunks; every generation resident when the records fit run_records)"
                     if args.run_call else
                     (f"bt_emit_beams ({parts} partitions), " +
                      ("bt_trace per generation" if args.per_generation else "bt_trace_all") +
                      " (every generation resident), bt_accumulate_mics" +
                      ("" if args.no_classify else "; the beam set bound to the grid once at set-up "
                       "(bt_beams_bind_mics: beams classified as they are created)")),
        "partitions": parts,
        "mic_classified_per_step": st["mic_classified"],
        "device_memory_bytes": bt.bt_memory_used(ctx),
        "end_to_end_segments_per_s": segs / (setup_s + ms_per_step * 1e-3),
        "kernel_sha256_16": kernel_hash(),
    }
    if args.config == 2 and not args.no_points:
        out["points"] = points_bench(sess, scene)
    if args.config == 2 and not args.run_call and not args.no_two_slot:
        out["two_slot_run"] = two_slot_bench(scene, partitions=args.partitions)
    if args.config == 2 and not args.no_batch:
        out["batched"] = batch_bench(sess)
    if args.config == 2 and not args.no_serve:
        if args.serve_short:
            n_of_rate, warm = (lambda r: int(min(2200, max(300, 4 * r)))), 0.1
        else:
            n_of_rate, warm = (lambda r: 2200), 200 / 2200
        out["served"] = serve_bench(sess, [50, 200, 800], n_of_rate, warm)
        for seed in range(1, max(args.serve_seeds, 1)):
            # further request streams (another seed each), reported beside seed 0's
            out.setdefault("served_other_seeds", {})[str(seed)] = \
                serve_bench(sess, [50, 200, 800], n_of_rate, warm, seed=seed)
    sess.close()
    if args.config == 2 and not args.no_volumetric:
        out["volumetric"] = volumetric_bench(max(2, min(args.steps, 5)), max(1, min(args.warmup, 2)), args.vol_chunk,
                                             args.vol_level, oracle_sample=not args.no_cpu_baseline,
                                             partitions=args.partitions)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(scene)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
