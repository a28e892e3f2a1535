#!/usr/bin/env python3
"""Benchmark of the per-frame adaptive bisection update on one MI355X.

Modes
  single (default)  one instance, the terrain workload (depth-24 pool, 64x64
                    quad grid, ridged height field): a step is one frame of
                    the update (every stage of the pipeline) along the seeded
                    flythrough.  The first P frames (--preroll, 40) grow the
                    triangulation from the base mesh to its steady state and
                    are not counted; then W warm-up frames, then K timed
                    frames between two stream synchronisations.
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
  1. pre-roll P frames, warm up W frames;  2. snapshot the pool;
  3. run the K frames once with per-frame counters (untimed) for the live
     counts and the byte models;  4. restore;
  5. run the K frames timed (no events), bracketed by two marker kernels
     (torch's spin kernel) outside the timed region, which delimit the
     timed pass in the byte-counter profiles;  6. restore;
  7. run the K frames again with events around every whole frame (frame
     latency percentiles) and check the final state equals the timed pass's;
  8. once per stage: restore and run the K frames with HIP events around
     that stage's launches on the library's stream;
  9. export the final state's triangles 20 times (HIP events);
 10. the CPU reference takes the GPU state at the first timed frame and runs
     the timed frames from there, single-threaded, for about --cpu-budget
     seconds.

Two byte models.  "paper": the minimal state of the paper's method (64-bit
ID, three 32-bit pointers, a 32-bit command, one occupancy bit; the tree
above the 32-bit word): per frame 16 L + 48 S + 24 N + 8 hops + 3/8 2^D
bytes for L live, S consumed by splits (each entered once by a chain: hops
= S), N new bisectors; split by stage in paper_bytes().  "layout": what this
library's layout must move (vertex cache, pointer/forwarding lines, work
lists), per stage in layout_bytes().  Counted bytes come from the rocprofv3
byte counters recorded by paper_2407_02215_amd/traffic.py for the same
command, kernel source and schedule.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# plain VALU issue: 256 CUs x 4 SIMDs, one wave64 instruction per 4 cycles
# each, 2.4 GHz (64 lanes per CU per cycle)
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4
METRIC = "bisector updates/s per frame (% HBM roofline); p50/p99 update latency"
STAGES = ("enumerate", "classify", "vote", "budget", "chain", "owners", "freelist", "fill", "resolve", "reduce")


def frame_counts(st: dict) -> dict:
    """The quantities the byte models use, from one frame's counters."""
    S = st["split_consumed"]
    M = st["frees"] - S             # merged members
    return {"L": st["live_before"], "S": S, "N": st["allocations"], "R": st["merge_requests"],
            "C": st["merges_executed"], "M": M, "P": M // 2, "O": st["allocations"] - M // 2,
            "cand": st["merge_candidates"], "cfg": st["merge_configs"]}


def paper_bytes(stage: str, st: dict, D: int) -> float:
    """Paper-minimal bytes of one stage's launch (the per-frame total
    16 L + 48 S + 24 N + 8 hops + 3/8 2^D split by where each term is
    moved, to the stage of this pipeline that moves it): enumerate reads the
    bitfield (2^D / 8); classify reads the 8-byte ID and writes the 4-byte
    command (12 L); the rank-order scans read the command (4 L, budget); the
    chain walk reads a twin and ORs a mark per hop (8 S); the free list
    updates the bitfield of new blocks (4 N); of a consumed bisector's
    20-byte record the fill reads the ID (8 S) and the pointer pass the three
    pointers (12 S); the fill writes its forwarding (16 S); of a new 20-byte
    record the fill writes the ID (8 N) and the pointer pass the three
    pointers (12 N); the pointer pass patches three neighbour pointers per
    consumed bisector (12 S); the reduction reads the bitfield and writes the
    tree (2^D / 4).  The vote and the owner pass have no term."""
    c = frame_counts(st)
    L, S, N = c["L"], c["S"], c["N"]
    cap = float(1 << D)
    terms = {"enumerate": cap / 8, "classify": 12.0 * L, "vote": 0.0, "budget": 4.0 * L, "chain": 8.0 * S,
             "owners": 0.0, "freelist": 4.0 * N, "fill": 24.0 * S + 8.0 * N, "resolve": 24.0 * S + 12.0 * N,
             "reduce": cap / 4}
    if stage == "frame":
        return sum(terms.values())
    return terms[stage]


def layout_bytes(stage: str, st: dict, D: int, vb: int = 48) -> float:
    """Bytes a stage of this library's layout must move per launch, from one
    frame's counters (vb: one vertex record, 48 bytes in binary32, 96 in
    binary64)."""
    c = frame_counts(st)
    L, R, S, C, M, P, O = c["L"], c["R"], c["S"], c["C"], c["M"], c["P"], c["O"]
    cap = float(1 << D)
    if stage == "enumerate":
        # bitfield word (4 per 32 blocks), rank-list entry per live block
        return cap / 8 + 4.0 * L
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
        return 52.0 * c["cand"] + 52.0 * c["cfg"]
    if stage in ("budget", "owners"):
        # rank entry and command per live bisector; owners write their list
        # entries (12 per owner)
        return 8.0 * L + (12.0 * (S + C) if stage == "owners" else 0.0)
    if stage == "chain":
        # per chain member: pointer record (16) and the mark atomic (4)
        return 20.0 * S
    if stage == "freelist":
        # bitfield read + write, a free-list entry per new block
        return cap / 4 + 4.0 * c["N"]
    if stage == "fill":
        # owner entries (8 + 4); a split bisector's vertex record (vb, its
        # heap ID included) read, its fate + forwarding written (20); per
        # split output a free-list entry (4) and a vertex record (vb); a
        # merge reads its smallest member's forwarding (16), per parent
        # three of the children's six world positions and a member's ID
        # (vb), a free-list entry (4) and writes the parent's record (vb);
        # every merged member's fate + forwarding (20).  Flat vertices are
        # decoded from the IDs.
        return (12.0 * (S + C) + (20.0 + vb) * S + (4.0 + vb) * O + 16.0 * C + (4.0 + 2.0 * vb) * P
                + 20.0 * M)
    if stage == "resolve":
        # owner entries (8); a split bisector's pointers (16) and its
        # outputs' free-list entries (16), its three neighbours' pointers
        # (48), its bit (4); per output its pointers (16); per merged parent
        # the smallest member's forwarding (16), the children's pointers
        # (32) and their two outer neighbours' pointers (32), the parent's
        # pointers (16), two bits (8)
        return 8.0 * (S + C) + 84.0 * S + 16.0 * O + 104.0 * P
    if stage == "reduce":
        return cap / 8 + cap / 8
    if stage == "frame":
        return sum(layout_bytes(k, st, D, vb) for k in STAGES)
    raise KeyError(stage)


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


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown CPU"


def cpu_baseline(w, snap, first: int, last: int, budget_s: float, precision: int = 32) -> dict:
    """The CPU reference (single-threaded C) on the timed frames: it takes
    the GPU's state at frame `first` and runs frames first, first + 1, ...
    (at most through `last`) until about budget_s seconds of frame work."""
    from oracle import Oracle
    o = Oracle(w.mesh, w.depth, w.lod, precision=precision)
    o.set_pool(*snap)
    total_l, total_t, frames = 0, 0.0, 0
    lo = hi = None
    for f in range(first, last + 1):
        t0 = time.perf_counter()
        st = o.frame(camera=w.cameras[f])
        dt = time.perf_counter() - t0
        total_l += st.live_before
        total_t += dt
        frames += 1
        lo = st.live_before if lo is None else lo
        hi = st.live_before
        if total_t >= budget_s:
            break
    return {"value": total_l / total_t, "unit": "bisector updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{w.name} frames {first}-{first + frames - 1} (the first timed frames, live {lo}..{hi}), "
                      f"replayed from the GPU state at frame {first}; {total_t:.1f} s single-threaded on 1 of "
                      f"{os.cpu_count()} host threads, {cpu_model()}"}


def _marker():
    """A kernel dispatch outside the timed region that delimits the timed
    pass in the byte-counter profiles (torch's spin kernel)."""
    import torch
    torch.cuda._sleep(1000)
    torch.cuda.synchronize()


def run_single(args) -> dict:
    import numpy as np
    import torch
    from paper_2407_02215_amd import cbt
    from paper_2407_02215_amd import inputs as I

    P, W, K = args.preroll, args.warmup, args.steps
    frames = P + W + K
    w = I.workload(args.workload, frames=max(frames, 8))
    if len(w.cameras) < frames:
        raise SystemExit(f"workload {args.workload} has {len(w.cameras)} frames, asked for {frames}")
    if args.criterion == "area":
        # the same triangles as the edge thresholds: a bisector with base
        # edge b has area b^2 / 4
        import dataclasses
        w = dataclasses.replace(w, lod=dataclasses.replace(
            w.lod, split_px=w.lod.split_px ** 2 / 4, merge_px=w.lod.merge_px ** 2 / 4, criterion=I.CRIT_AREA))
    elif args.criterion == "distance":
        import dataclasses
        w = dataclasses.replace(w, lod=dataclasses.replace(w.lod, criterion=I.CRIT_DISTANCE))
    inst = cbt.Instance(w.mesh, w.depth, w.lod, tuned=args.schedule is None, precision=args.precision)
    if args.schedule is not None:
        inst.set_schedule(*(int(x) for x in args.schedule.split(",")))
    print(f"# pre-roll {P} + warm-up {W} frames, schedule {inst.schedule()}", file=sys.stderr, flush=True)
    for cam in w.cameras[:P]:
        inst.update(cam)
    if args.schedule is None:
        # the tuned schedule for this depth at the live count the timed
        # window starts from
        inst.apply_tuned()
        print(f"# schedule {inst.schedule()} at {inst.live_count()} live", file=sys.stderr, flush=True)
    for cam in w.cameras[P:P + W]:
        inst.update(cam)
    torch.cuda.synchronize()
    snap = inst.snapshot()
    timed = w.cameras[P + W:frames]
    print(f"# counting pass over frames {P + W}..{frames - 1}", file=sys.stderr, flush=True)
    stats = [inst.update(cam, stats=True) for cam in timed]
    inst.restore(*snap)
    print("# timed pass", file=sys.stderr, flush=True)
    _marker()
    t0 = time.perf_counter()
    for cam in timed:
        inst.update(cam)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    _marker()
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
    print("# per-stage timing pass", file=sys.stderr, flush=True)
    stage_mean = {}
    for stage in STAGES:
        inst.restore(*snap)
        inst.time_stage(stage)
        for cam in timed:
            inst.update(cam)
        n_st, ms_st = inst.stage_time()
        inst.time_stage(None)
        stage_mean[stage] = ms_st / max(1, n_st)
    # triangle export of the final state: live list (4), vertex record, 36
    # bytes written per triangle
    L = inst.live_count()
    tri = torch.empty((max(1, L), 3, 3), dtype=torch.float32, device="cuda")
    inst.export_triangles(tri)
    inst.time_stage("export")
    for _ in range(20):
        inst.export_triangles(tri)
    n_exp, exp_ms = inst.stage_time()
    inst.time_stage(None)
    vb = 96 if args.precision == 64 else 48
    exp_bytes = L * (4.0 + vb + 36.0)
    exp_mean = exp_ms / max(1, n_exp)
    schedule = list(inst.schedule())
    inst.close()

    D = w.depth
    nfr = len(stats)
    mean = lambda f: sum(f(s) for s in stats) / nfr   # noqa: E731
    updates = sum(s["live_before"] for s in stats)
    value = updates / elapsed
    frame_s = elapsed / nfr
    from paper_2407_02215_amd import traffic as T
    rec = T.lookup(args.workload, args.criterion, args.precision, P, W, K, schedule)
    # dominant kernel: the longest stage the paper-minimal model gives bytes
    dominant = max((k for k in STAGES if mean(lambda s, k=k: paper_bytes(k, s, D)) > 0), key=stage_mean.get)
    mean_ms = stage_mean[dominant]
    pb = mean(lambda s: paper_bytes(dominant, s, D))
    lb = mean(lambda s: layout_bytes(dominant, s, D, vb))
    counted = rec["kernels"].get(dominant, {}).get("bytes") if rec else None
    frame_pb = mean(lambda s: paper_bytes("frame", s, D))
    frame_lb = mean(lambda s: layout_bytes("frame", s, D, vb))
    frame_counted = rec["frame_bytes"] if rec else None
    valu = rec.get("frame_valu_insts") if rec else None
    gbs = lambda b, t: b / t / 1e9   # noqa: E731
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "bisector updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": elapsed * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 64 else "f32",
        "data": "synthetic (seeded workload generator)",
        "config": {"workload": args.workload, "criterion": args.criterion, "cbt_depth": D,
                   "halfedges": w.mesh.H, "preroll": P, "frames": f"{P + W}..{frames - 1}",
                   "mean_live": updates / nfr, "schedule": schedule},
        "counters": {"live": mean(lambda s: s["live_before"]),
                     "consumed_by_splits": mean(lambda s: s["split_consumed"]),
                     "new": mean(lambda s: s["allocations"]), "freed": mean(lambda s: s["frees"]),
                     "split_requests": mean(lambda s: s["split_requests"]),
                     "splits_accepted": mean(lambda s: s["split_accepted"]),
                     "merge_requests": mean(lambda s: s["merge_requests"]),
                     "merges_executed": mean(lambda s: s["merges_executed"]),
                     "what": "per-frame means over the timed frames"},
        "rates_per_s": {"splits": mean(lambda s: s["split_consumed"]) / frame_s,
                        "merges": mean(lambda s: s["merges_executed"]) / frame_s,
                        "allocations": mean(lambda s: s["allocations"]) / frame_s,
                        "frees": mean(lambda s: s["frees"]) / frame_s,
                        "what": "bisectors split, configurations merged, blocks allocated and freed per second of the "
                                "timed pass"},
        "latency_ms": {"p10": percentile(frame_ms, 10), "p50": percentile(frame_ms, 50),
                       "p90": percentile(frame_ms, 90), "p99": percentile(frame_ms, 99),
                       "what": "GPU time of one whole update, HIP events"},
        "export": {"triangles": L, "ms": exp_mean, "alg_bytes": exp_bytes,
                   "achieved_gbs": exp_bytes / (exp_mean * 1e-3) / 1e9},
        "stage_ms": stage_mean,
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": gbs(pb, mean_ms * 1e-3), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": gbs(pb, mean_ms * 1e-3) / HBM_PEAK_GBS, "traffic": counted,
                     "traffic_unit": "HBM bytes per launch", "mean_launch_ms": mean_ms,
                     "alg_bytes_per_launch": pb, "bytes": "paper-minimal state"},
        "roofline_layout": {"kernel": dominant, "achieved": gbs(lb, mean_ms * 1e-3),
                            "frac": gbs(lb, mean_ms * 1e-3) / HBM_PEAK_GBS, "alg_bytes_per_launch": lb,
                            "bytes": "this library's layout (vertex cache, pointer and forwarding lines)"},
        "frame": {"ms": frame_s * 1e3,
                  "paper_bytes": frame_pb, "paper_frac": gbs(frame_pb, frame_s) / HBM_PEAK_GBS,
                  "layout_bytes": frame_lb, "layout_frac": gbs(frame_lb, frame_s) / HBM_PEAK_GBS,
                  "counted_bytes": frame_counted,
                  "counted_frac": None if frame_counted is None else gbs(frame_counted, frame_s) / HBM_PEAK_GBS,
                  "valu_frac": None if valu is None else valu / (frame_s * VALU_PEAK_WAVE_INSTS),
                  "what": "whole update per timed frame: bytes over the timed pass's mean frame time against "
                          "8 TB/s; counted = rocprofv3 FETCH_SIZE + WRITE_SIZE of every kernel; VALU = wave64 "
                          "VALU instructions against 256 CUs x 4 SIMDs at 2.4 GHz"},
    }
    if not args.no_cpu_baseline:
        print("# CPU reference baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, snap, P + W, frames - 1, args.cpu_budget, args.precision)
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
    ws = I.batched_workloads(args.instances, frames=frames, seed=4, workers=16)
    insts = [cbt.Instance(w.mesh, w.depth, w.lod, tuned=True) for w in ws]
    print(f"# warm-up {args.warmup} frames (one launch sequence per instance)", file=sys.stderr, flush=True)
    for f in range(args.warmup):
        for x, w in zip(insts, ws):
            x.update(w.cameras[f])
    torch.cuda.synchronize()
    # each member's tuned schedule for the live count it has reached
    for x in insts:
        x.apply_tuned()
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
    n = len(timed)

    def batched(persistent: bool):
        """The timed frames as one batch (graph replay; one launch per stage,
        or one persistent launch per frame): seconds per frame, whether every
        member ends in the one-launch-sequence state."""
        for x, s in zip(insts, snaps):
            x.restore(*s)
        batch = cbt.Batch(insts, graph=True, persistent=persistent)
        kind = "persistent" if persistent else "one launch per stage"
        print(f"# batched, {kind} (graph replay)", file=sys.stderr, flush=True)
        batch.update([w.cameras[args.warmup] for w in ws])     # capture (counts as the first frame)
        batch.synchronize()
        t0 = time.perf_counter()
        for f in list(timed)[1:]:
            batch.update([w.cameras[f] for w in ws])
        batch.synchronize()
        t_rest = time.perf_counter() - t0
        same = all(all(np.array_equal(a, b) for a, b in zip(r, x.pool())) for r, x in zip(ref, insts))
        batch.close()
        # the graph capture frame is timed separately: replay time per frame
        return t_rest * n / max(1, n - 1), bool(same)

    t_stage, same_stage = batched(False)
    t_persist, same_persist = batched(True)
    for x in insts:
        x.close()
    t_batch = min(t_stage, t_persist)
    return {
        "metric": "batched bisector updates/s",
        "value": updates / t_batch,
        "unit": "bisector updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_batch * 1e3 / n,
        "higher_is_better": True,
        "launch": "persistent" if t_persist <= t_stage else "one launch per stage",
        "vs_one_launch_per_instance": t_single / t_batch,
        "one_launch_per_instance": {"value": updates / t_single, "ms_per_step": t_single * 1e3 / n},
        "persistent": {"value": updates / t_persist, "ms_per_step": t_persist * 1e3 / n,
                       "identical_states": same_persist},
        "launch_per_stage": {"value": updates / t_stage, "ms_per_step": t_stage * 1e3 / n,
                             "identical_states": same_stage},
        "identical_states": bool(same_stage and same_persist),
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
    depth_lo, depth_hi = 14, 22
    # resident instances: members 0 .. n-1 of a batched configuration (each
    # its own mesh, depth and camera path); arriving instances: the next
    # new_pool members, in turn, then the same meshes again with a fresh
    # depth and camera path
    print(f"# building {args.instances} + {args.new_pool} instances", file=sys.stderr, flush=True)
    resident = I.batched_workloads(args.instances, frames=64, seed=1000, workers=16)
    pool = I.batched_workloads(args.new_pool, frames=64, seed=1000, first=args.instances, workers=16)
    specs = [(w, w.depth, w.cameras) for w in resident]   # (workload, depth, cameras) per instance
    n_new = 0

    def new_spec():
        nonlocal n_new
        w = pool[n_new % len(pool)]
        if n_new < len(pool):
            D, cams = w.depth, w.cameras
        else:
            D = I.depth_for(w.mesh.H, int(rng.integers(depth_lo, depth_hi + 1)))
            cams = I.camera_path_orbit(64, int(rng.integers(1 << 30)))
        n_new += 1
        specs.append((w, D, cams))
        return len(specs) - 1

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
                         map_capacity=1 << 22, tuned=True)
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
                   "instances_opened": len(specs), "distinct_meshes": args.instances + min(n_new, args.new_pool),
                   "arena_gib": arena / 2**30,
                   "admission_footprint": "workspace bytes per instance (about 112 per pool block)"},
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
    ap.add_argument("--preroll", type=int, default=40,
                    help="single mode: untimed frames from the base mesh to the steady state, before the warm-up")
    ap.add_argument("--criterion", default="edge", choices=["edge", "area", "distance"],
                    help="size test of the LOD (single mode): projected base-edge length, triangle area, or "
                         "the cull-free distance-only variant")
    ap.add_argument("--camera", type=int, default=255, help="camera index (converge mode)")
    ap.add_argument("--instances", type=int, default=None)
    ap.add_argument("--new-pool", type=int, default=1024,
                    help="serve mode: distinct meshes for arriving instances (reused in turn after that)")
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
        # without arguments: the steady window past the pre-roll (terrain
        # frames 40..239)
        args.steps = 200 if args.steps is None else args.steps
        args.warmup = 0 if args.warmup is None else args.warmup
        out = run_single(args)
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
