#!/usr/bin/env python3
"""Benchmark of the per-frame adaptive bisection update on one MI355X.

Modes
  single (default)  one instance, the terrain workload (depth-24 pool, 64x64
                    quad grid, ridged height field): a step is one frame of
                    the update (every stage of the pipeline) along the seeded
                    flythrough.  The first W frames are warm-up (the
                    triangulation grows from the base mesh); the next K are
                    timed between two stream synchronisations.
                    Bisector updates/s = sum over the timed frames of the
                    live count at frame start / elapsed time.
  batch             many instances of uneven size and depth (128 by default),
                    the same frames run one instance per launch sequence and
                    then batched (one launch per stage for all instances,
                    replayed from a HIP graph); both must give identical
                    states.
  serve             Poisson request stream over resident instances through
                    the serving loop (continuous batching, admission by
                    footprint, eviction to host), and the same trace served
                    one request per launch; p50/p99 request latency.

Single-mode protocol (the pipeline is deterministic):
  1. warm up W frames;  2. snapshot the pool;
  3. run the K frames once with per-frame counters (untimed) for the live
     counts and the algorithmic bytes;  4. restore;
  5. run the K frames timed (no events);  6. restore;
  7. run the K frames again with events around every whole frame (p50/p99
     frame latency) and check the final state equals the timed pass's;
  8. once per stage: restore and run the K frames with HIP events around
     that stage's launches on the library's stream; the roofline is
     reported for the longest stage with a byte model (classify, vote,
     fill, resolve);
  9. export the final state's triangles 20 times (HIP events).
Every pass runs the same K frames, so each kernel's dispatches of one pass
([W + jK, W + (j+1)K) in dispatch order) see the same work.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "bisector updates/s per frame (% HBM roofline); p50/p99 update latency"


def algorithmic_bytes(stage: str, st: dict, vb: int = 48) -> float:
    """Bytes a stage must move per launch, from one frame's counters.

    L live bisectors, R merge requests, S bisectors consumed by splits,
    C merge configurations executed, M merged members, P parents (M / 2),
    O split outputs (allocations - P); vb is one vertex record (three world
    positions with depth and parity: 48 bytes in binary32, 96 in binary64)."""
    L = st["live_before"]
    R = st["merge_requests"]
    S = st["split_consumed"]
    C = st["merges_executed"]
    M = st["frees"] - S
    P = M // 2
    O = st["allocations"] - P
    if stage == "classify":
        # rank -> block (4), the vertex record (vb), command write (4); even
        # merge requests are listed (8 for about half of them)
        return (8.0 + vb) * L + 4.0 * R
    if stage == "vote":
        # per listed even member: its list entry (8) and pointer record (16),
        # the commands of the three other members (12) and the Prev pointer
        # of the twin-side member (16); per unanimous configuration the two
        # IDs each of its even members compares (32), its forwarding record
        # and command (20)
        return 52.0 * st["merge_candidates"] + 52.0 * st["merge_configs"]
    if stage == "fill":
        # owner entries (8 + 4); a split bisector's ID (8) and vertex record
        # (vb) read, its fate + forwarding written (20); per split output a
        # free-list entry (4), a vertex record (vb) and the heap ID (8); a
        # merge reads its smallest member's forwarding (16), per parent a
        # member's ID (8), three of the children's six world positions (vb),
        # a free-list entry (4) and writes the parent's record (vb) and heap
        # ID (8); every merged member's fate + forwarding (20).  Flat
        # vertices are decoded from the IDs.
        return (12.0 * (S + C) + (28.0 + vb) * S + (12.0 + vb) * O + 16.0 * C + (20.0 + 2.0 * vb) * P
                + 20.0 * M)
    if stage == "resolve":
        # owner entries (8); a split bisector's pointers (16) and its
        # outputs' free-list entries (16), its three neighbours' pointers
        # (48), its bit (4); per output its pointers (16); per merged parent
        # the smallest member's forwarding (16), the children's pointers
        # (32) and their two outer neighbours' pointers (32), the parent's
        # pointers (16), two bits (8)
        return 8.0 * (S + C) + 84.0 * S + 16.0 * O + 104.0 * P
    if stage == "frame":
        # every stage: rank passes over L (enumerate 4, classify 8 + vb,
        # budget 8, owners 8), the fill and resolve bytes, and the bitfield +
        # tree passes (3/8 byte per pool block, taken as L here)
        return (28.0 + vb) * L + algorithmic_bytes("fill", st, vb) + algorithmic_bytes("resolve", st, vb)
    raise KeyError(stage)


SURVEY_STAGES = ("classify", "vote", "fill", "resolve")          # stages with a byte model
EXTRA_STAGES = ("enumerate", "budget", "chain", "owners", "freelist", "reduce")


def random_calibration() -> dict:
    """The rate at which this GPU serves random line reads, the pattern of
    the pointer passes: gathers of 4-byte elements at uniformly random
    positions of a 2 GiB array (each element its own 128-byte line) and of
    whole 128-byte rows at random, timed with HIP events (torch's gather
    kernel; indices and outputs are sequential and small beside the lines)."""
    import torch
    n = 512 << 20                      # floats: 2 GiB
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    rows = x.view(-1, 32)              # 128-byte rows
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    m = 16 << 20
    idx = torch.randint(0, n, (m,), device="cuda", generator=g)
    ridx = torch.randint(0, rows.shape[0], (m // 4,), device="cuda", generator=g)

    def timed(fn, reps=20):
        for _ in range(3):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps * 1e-3

    t_el = timed(lambda: torch.index_select(x, 0, idx))
    t_row = timed(lambda: torch.index_select(rows, 0, ridx))
    return {"random_element_gather": {"elements": m, "ms": t_el * 1e3, "lines_per_s": m / t_el,
                                      "line_gbs": m * 128 / t_el / 1e9},
            "random_row_gather": {"rows": m // 4, "ms": t_row * 1e3, "lines_per_s": m / 4 / t_row,
                                  "line_gbs": m / 4 * 128 / t_row / 1e9,
                                  "read_plus_write_gbs": m / 4 * 256 / t_row / 1e9}}


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, np.float64), q)) if len(xs) else None


def cpu_baseline(workload: str, budget_s: float, precision: int = 32) -> dict:
    """The CPU reference (single-threaded C) on the first frames of the same
    workload, timed frame by frame until about budget_s seconds of work."""
    from oracle import Oracle
    from paper_2407_02215_amd import inputs as I
    w = I.workload(workload, frames=64)
    o = Oracle(w.mesh, w.depth, w.lod, precision=precision)
    total_l, total_t, frames = 0, 0.0, 0
    lo, hi = None, None
    for cam in w.cameras:
        t0 = time.perf_counter()
        st = o.frame(camera=cam)
        dt = time.perf_counter() - t0
        total_l += st.live_before
        total_t += dt
        frames += 1
        lo = st.live_before if lo is None else lo
        hi = st.live_before
        if total_t >= budget_s:
            break
    return {"value": total_l / total_t, "unit": "bisector updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{workload} frames 0-{frames - 1} from the base mesh (live {lo}..{hi}), "
                      f"{total_t:.1f} s single-threaded on {os.cpu_count()} host cores"}


def run_single(args) -> dict:
    import numpy as np
    import torch
    from paper_2407_02215_amd import cbt
    from paper_2407_02215_amd import inputs as I

    frames = args.warmup + args.steps
    w = I.workload(args.workload, frames=max(frames, 8))
    if len(w.cameras) < frames:
        raise SystemExit(f"workload {args.workload} has {len(w.cameras)} frames, asked for {frames}")
    if args.criterion == "area":
        # the same triangles as the edge thresholds: a bisector with base
        # edge b has area b^2 / 4
        import dataclasses
        w = dataclasses.replace(w, lod=dataclasses.replace(
            w.lod, split_px=w.lod.split_px ** 2 / 4, merge_px=w.lod.merge_px ** 2 / 4, criterion=I.CRIT_AREA))
    inst = cbt.Instance(w.mesh, w.depth, w.lod, tuned=args.schedule is None, precision=args.precision)
    if args.schedule is not None:
        inst.set_schedule(*(int(x) for x in args.schedule.split(",")))
    print(f"# warm-up {args.warmup} frames, schedule {inst.schedule()}", file=sys.stderr, flush=True)
    for cam in w.cameras[:args.warmup]:
        inst.update(cam)
    torch.cuda.synchronize()
    snap = inst.snapshot()
    timed = w.cameras[args.warmup:frames]
    print(f"# counting pass over {len(timed)} frames", file=sys.stderr, flush=True)
    stats = [inst.update(cam, stats=True) for cam in timed]
    inst.restore(*snap)
    print("# timed pass", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for cam in timed:
        inst.update(cam)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    check = [a.copy() for a in inst.pool()]
    print("# latency pass", file=sys.stderr, flush=True)
    inst.restore(*snap)
    inst.time_stage("frame")
    for cam in timed:
        inst.update(cam)
    frame_ms = inst.stage_times()
    inst.time_stage(None)
    again = inst.pool()
    assert all(np.array_equal(a, b) for a, b in zip(check, again)), "non-deterministic frame"
    # stage survey: the same frames once per stage with HIP events around
    # that stage's launches; the roofline is reported for the longest one
    # (or the one --stage names)
    survey = {}
    for stage in (SURVEY_STAGES + EXTRA_STAGES if args.stage == "auto" else (args.stage,)):
        inst.restore(*snap)
        inst.time_stage(stage)
        for cam in timed:
            inst.update(cam)
        n_st, ms_st = inst.stage_time()
        inst.time_stage(None)
        survey[stage] = ms_st / max(1, n_st)
    dominant = max((k for k in survey if k in SURVEY_STAGES or k == args.stage), key=survey.get)
    # triangle export of the final state: live list (4), vertex record, 36
    # bytes written per triangle
    L = inst.live_count()
    tri = torch.empty((L, 3, 3), dtype=torch.float32, device="cuda")
    inst.export_triangles(tri)
    inst.time_stage("export")
    for _ in range(20):
        inst.export_triangles(tri)
    n_exp, exp_ms = inst.stage_time()
    inst.time_stage(None)
    rec = 96 if args.precision == 64 else 48
    exp_bytes = L * (4.0 + rec + 36.0)
    exp_mean = exp_ms / max(1, n_exp)

    updates = sum(s["live_before"] for s in stats)
    value = updates / elapsed
    traffic = args.traffic
    if traffic is None and args.precision == 32 and args.workload == "terrain" and args.criterion == "edge":
        from paper_2407_02215_amd import traffic as T
        traffic = T.lookup(dominant, args.warmup, args.steps, inst.schedule())
    vb = 96 if args.precision == 64 else 48
    alg = sum(algorithmic_bytes(dominant, s, vb) for s in stats) / len(stats)
    mean_ms = survey[dominant]
    achieved = alg / (mean_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "bisector updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 64 else "f32",
        "data": "synthetic (seeded workload generator)",
        "config": {"workload": args.workload, "criterion": args.criterion, "cbt_depth": w.depth,
                   "halfedges": w.mesh.H,
                   "frames": f"{args.warmup}..{frames - 1}", "mean_live": updates / len(stats),
                   "schedule": list(inst.schedule())},
        "latency_ms": {"p50": percentile(frame_ms, 50), "p99": percentile(frame_ms, 99),
                       "what": "GPU time of one whole update, HIP events"},
        "export": {"triangles": L, "ms": exp_mean, "alg_bytes": exp_bytes,
                   "achieved_gbs": exp_bytes / (exp_mean * 1e-3) / 1e9},
        "stage_ms": survey,
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_unit": "HBM bytes per launch",
                     "mean_launch_ms": mean_ms, "alg_bytes_per_launch": alg},
    }
    inst.close()
    return out


def run_converge(args) -> dict:
    """Multi-pass mode from the base mesh at one camera: passes until
    nothing changes, timed as a whole (each pass synchronises to read its
    counters) and pass by pass with HIP events."""
    import torch
    from paper_2407_02215_amd import cbt
    from paper_2407_02215_amd import inputs as I
    w = I.workload(args.workload, frames=256 if args.workload == "planet" else None)
    cam = w.cameras[min(args.camera, len(w.cameras) - 1)]
    runs = []
    for rep in range(3):
        inst = cbt.Instance(w.mesh, w.depth, w.lod, tuned=True, precision=args.precision)
        torch.cuda.synchronize()
        inst.time_stage("frame")
        t0 = time.perf_counter()
        passes, last = inst.update_converge(cam, max_passes=64)
        wall = time.perf_counter() - t0
        pass_ms = inst.stage_times()
        runs.append({"passes": passes, "wall_ms": wall * 1e3, "gpu_ms": float(sum(pass_ms)),
                     "live": inst.live_count(), "converged": last["allocations"] == 0 and last["frees"] == 0})
        inst.close()
    best = min(runs, key=lambda r: r["wall_ms"])
    return {"metric": "multi-pass update to the fixpoint", "value": best["wall_ms"], "unit": "ms",
            "higher_is_better": False, "n_gpus": 1, "runs": runs,
            "dtype": "f64" if args.precision == 64 else "f32", "data": "synthetic (seeded workload generator)",
            "config": {"workload": args.workload, "camera": args.camera, "cbt_depth": w.depth}}


def run_batch(args) -> dict:
    import numpy as np
    import torch
    from paper_2407_02215_amd import cbt
    from paper_2407_02215_amd import inputs as I

    frames = args.warmup + args.steps
    print(f"# building {args.instances} instances", file=sys.stderr, flush=True)
    ws = I.batched_workloads(args.instances, frames=frames, seed=4)
    insts = [cbt.Instance(w.mesh, w.depth, w.lod, tuned=True) for w in ws]
    print(f"# warm-up {args.warmup} frames (one launch sequence per instance)", file=sys.stderr, flush=True)
    for f in range(args.warmup):
        for x, w in zip(insts, ws):
            x.update(w.cameras[f])
    torch.cuda.synchronize()
    snaps = [x.snapshot() for x in insts]
    timed = range(args.warmup, frames)
    print("# counting pass", file=sys.stderr, flush=True)
    updates = 0
    for f in timed:
        for x, w in zip(insts, ws):
            updates += x.update(w.cameras[f], stats=True)["live_before"]
    for x, s in zip(insts, snaps):
        x.restore(*s)
    print("# one instance per launch sequence", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in timed:
        for x, w in zip(insts, ws):
            x.update(w.cameras[f])
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    ref = [[a.copy() for a in x.pool()] for x in insts]
    for x, s in zip(insts, snaps):
        x.restore(*s)
    batch = cbt.Batch(insts, graph=True)
    print("# batched (graph replay)", file=sys.stderr, flush=True)
    batch.update([w.cameras[args.warmup] for w in ws])     # capture (counts as the first frame)
    batch.synchronize()
    t0 = time.perf_counter()
    for f in list(timed)[1:]:
        batch.update([w.cameras[f] for w in ws])
    batch.synchronize()
    t_batch_rest = time.perf_counter() - t0
    same = all(all(np.array_equal(a, b) for a, b in zip(r, x.pool())) for r, x in zip(ref, insts))
    # the graph capture frame is timed separately: replay time per frame
    n = len(timed)
    t_batch = t_batch_rest * n / max(1, n - 1)
    batch.close()
    for x in insts:
        x.close()
    return {
        "metric": "batched bisector updates/s",
        "value": updates / t_batch,
        "unit": "bisector updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_batch * 1e3 / n,
        "higher_is_better": True,
        "vs_one_launch_per_instance": t_single / t_batch,
        "one_launch_per_instance": {"value": updates / t_single, "ms_per_step": t_single * 1e3 / n},
        "identical_states": bool(same),
        "dtype": "f32",
        "data": "synthetic (seeded workload generator)",
        "config": {"workload": "batched", "instances": args.instances,
                   "halfedges": [int(min(w.mesh.H for w in ws)), int(max(w.mesh.H for w in ws))],
                   "depths": [int(min(w.depth for w in ws)), int(max(w.depth for w in ws))],
                   "pool_blocks": int(sum(1 << w.depth for w in ws)), "mean_live_per_frame": updates / n},
    }


def run_serve(args) -> dict:
    import numpy as np
    import torch
    from paper_2407_02215_amd import cbt
    from paper_2407_02215_amd import inputs as I

    rng = np.random.default_rng(11)
    n_req = int(args.rate * args.duration)
    gaps = rng.exponential(1.0 / args.rate, n_req)
    arrivals = np.cumsum(gaps)
    new_frac = 0.10
    base = I.batched_workloads(args.meshes, frames=64, seed=4)
    depth_lo, depth_hi = 14, 22
    specs = []   # (workload, depth, cameras) per instance, resident ones first

    def new_spec():
        w = base[int(rng.integers(len(base)))]
        D = I.depth_for(w.mesh.H, int(rng.integers(depth_lo, depth_hi + 1)))
        cams = I.camera_path_orbit(64, int(rng.integers(1 << 30)))
        specs.append((w, D, cams))
        return len(specs) - 1

    for _ in range(args.instances):
        new_spec()
    trace = []   # (arrival, spec index, camera index)
    counts = {}
    for t in arrivals:
        if rng.random() < new_frac:
            k = new_spec()
        else:
            k = int(rng.integers(len(specs)))
        c = counts.get(k, 0)
        counts[k] = c + 1
        trace.append((float(t), k, c % 64))
    free, total = torch.cuda.mem_get_info()
    arena = int(min(args.budget_gb * (1 << 30), 0.8 * free))
    print(f"# {len(specs)} instances, {n_req} requests at {args.rate}/s, arena {arena / 2**30:.1f} GiB",
          file=sys.stderr, flush=True)

    def serve(max_batch, slots):
        srv = cbt.Server(arena_bytes=arena, memory_budget=arena, max_batch=max_batch, slots=slots,
                         map_capacity=1 << 22)
        ids = {}
        for k in range(args.instances):
            w, D, _ = specs[k]
            ids[k] = srv.open(w.mesh, D, w.lod)
        done = []
        t0 = time.perf_counter()
        last = t0

        def progress():
            nonlocal last
            now = time.perf_counter()
            if now - last > 5.0:
                print(f"#   {len(done)} of {len(trace)} requests done after {now - t0:.1f} s", file=sys.stderr,
                      flush=True)
                last = now

        for t, k, c in trace:
            while time.perf_counter() - t0 < t:
                done += srv.poll()
            if k not in ids:
                w, D, _ = specs[k]
                ids[k] = srv.open(w.mesh, D, w.lod)
            srv.submit(ids[k], specs[k][2][c], len(done))
            progress()
        while len(done) < len(trace):
            got = srv.poll(wait=True)
            done += got
            progress()
            if not got and srv.stats()["in_flight"] == 0:
                break
        done += srv.drain()
        wall = time.perf_counter() - t0
        st = srv.stats()
        lat = [d["latency_ms"] for d in done]
        ok = all(d["status"] == 0 for d in done)
        res = {"p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
               "value": st["bisector_updates"] / wall, "wall_s": wall, "requests": len(done), "all_ok": ok,
               "batches": st["batches"], "mean_batch": len(done) / max(1, st["batches"]),
               "admissions": st["admissions"], "evictions": st["evictions"],
               "host_snapshots": st["host_snapshots"],
               "admit_ms": {"total": st["admit_ms"], "max": st["admit_ms_max"]},
               "evict_ms": {"total": st["evict_ms"], "max": st["evict_ms_max"]}}
        sample = sorted(ids)[:: max(1, len(ids) // 16)]
        states = {k: srv.query(ids[k]) for k in sample}
        srv.close()
        return res, states

    print("# continuous batching", file=sys.stderr, flush=True)
    batched, s1 = serve(args.max_batch, 2)
    print("# one request per launch", file=sys.stderr, flush=True)
    single, s2 = serve(1, 1)
    same = all(all(np.array_equal(s1[k][f], s2[k][f]) for f in ("slot", "heap_id", "twin", "next", "prev"))
               for k in s1)
    return {
        "metric": "served bisector updates/s; p50/p99 request latency",
        "value": batched["value"],
        "unit": "bisector updates/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "latency_ms": {"p50": batched["p50_ms"], "p99": batched["p99_ms"],
                       "what": "submit to completion observed by the host"},
        "served": batched,
        "one_request_per_launch": single,
        "identical_states_sampled": bool(same),
        "dtype": "f32",
        "data": "synthetic (seeded workload generator)",
        "config": {"workload": "served", "rate_per_s": args.rate, "duration_s": args.duration,
                   "resident_instances": args.instances, "new_instance_fraction": new_frac,
                   "distinct_meshes": args.meshes, "arena_gib": arena / 2**30},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--mode", default="single", choices=["single", "batch", "serve", "converge"])
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="terrain", choices=["terrain", "planet", "cube"])
    ap.add_argument("--precision", type=int, default=32, choices=[32, 64],
                    help="vertices, world positions and size test in binary32 or binary64 (single mode)")
    ap.add_argument("--schedule", default=None,
                    help="rank workgroups,reduction levels (single mode; default: the tuned table)")
    ap.add_argument("--criterion", default="edge", choices=["edge", "area"],
                    help="size test of the LOD (single mode): projected base-edge length or triangle area")
    ap.add_argument("--camera", type=int, default=255, help="camera index (converge mode)")
    ap.add_argument("--stage", default="auto", choices=["auto"] + list(SURVEY_STAGES) + ["frame"],
                    help="kernel whose roofline is reported; auto: the longest of the surveyed stages")
    ap.add_argument("--traffic", type=float, default=None,
                    help="HBM bytes per launch of the profiled stage from the byte counters; by default "
                         "the value paper_2407_02215_amd/traffic.py recorded for this kernel source")
    ap.add_argument("--instances", type=int, default=None)
    ap.add_argument("--meshes", type=int, default=32)
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--duration", type=float, default=60.0, help="serve mode: seconds of arrivals")
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--max-batch", type=int, default=128)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain 256 MiB device copies (scale of the HBM byte counters)")
    ap.add_argument("--random-calibration", action="store_true",
                    help="only time gathers at random positions (the rate of random 128-byte line reads)")
    args = ap.parse_args()
    if args.random_calibration:
        print(json.dumps(random_calibration()), flush=True)
        return
    if args.copy_calibration:
        import torch
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel(), "copies": 5}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the update runs on one GPU; --gpus above 1 is not supported"}))
        sys.exit(2)
    if args.mode == "single":
        args.steps = 200 if args.steps is None else args.steps
        args.warmup = 40 if args.warmup is None else args.warmup
        out = run_single(args)
        if not args.no_cpu_baseline:
            print("# CPU reference baseline", file=sys.stderr, flush=True)
            out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_budget, args.precision)
    elif args.mode == "converge":
        out = run_converge(args)
    elif args.mode == "batch":
        args.steps = 48 if args.steps is None else args.steps
        args.warmup = 16 if args.warmup is None else args.warmup
        args.instances = 128 if args.instances is None else args.instances
        out = run_batch(args)
    else:
        args.instances = 512 if args.instances is None else args.instances
        out = run_serve(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
