#!/usr/bin/env python3
"""Benchmark of the per-frame adaptive bisection update on one MI355X.

A step is one frame of the update (every stage of the pipeline) along the
seeded camera path of the workload.  The first W frames are warm-up (the
triangulation grows from the base mesh to its steady size); the next K frames
are timed between two stream synchronisations.  Bisector updates/s =
sum over the timed frames of the live count at frame start / elapsed time.

Measurement protocol (deterministic pipeline):
  1. warm up W frames;  2. snapshot the pool;
  3. run the K frames once with per-frame counters (untimed) to get the live
     counts;  4. restore the snapshot;
  5. run the same K frames again, timed, with HIP events around the profiled
     stage on the library's stream.
The roofline object reports that stage: algorithmic bytes per launch over
its mean event-timed duration, against the 8 TB/s HBM peak.
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


def algorithmic_bytes(stage: str, st: dict, cap: int) -> float:
    """Bytes a stage must move per launch, from the frame's counters.

    L live bisectors, R merge requests, S bisectors consumed by splits,
    M merged configurations, N new bisectors."""
    L = st["live_before"]
    R = st["merge_requests"]
    S = st["split_consumed"]
    N = st["allocations"]
    consumed = st["frees"]
    if stage == "classify":
        # heap ID read (8 B) + command write (4 B) per bisector; a merge
        # request also reads its pointers (12 B) and three neighbour IDs (24 B)
        return 12.0 * L + 36.0 * R
    if stage == "frame":
        # per bisector: ID read and command write/read (16 B); per consumed
        # bisector: record read (20 B), forwarding write (16 B), neighbour
        # fix-ups (12 B); per new bisector: record write (20 B) and bit (4 B);
        # bitfield read twice and the tree levels above the word (3/8 B/slot)
        return 16.0 * L + 48.0 * consumed + 24.0 * N + 0.375 * cap
    raise KeyError(stage)


def cpu_baseline(workload: str, budget_s: float) -> dict:
    """The CPU reference (single-threaded C) on the first frames of the same
    workload, timed frame by frame until about budget_s seconds of work."""
    from oracle import Oracle
    from paper_2407_02215_amd import inputs as I
    w = I.workload(workload, frames=64)
    o = Oracle(w.mesh, w.depth, w.lod)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="terrain", choices=["terrain", "planet", "cube"])
    ap.add_argument("--stage", default="classify", choices=["classify", "frame"])
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain 256 MiB device copies (scale of the HBM byte counters)")
    args = ap.parse_args()
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
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU runs are not part of this build"}))
        sys.exit(2)

    import torch
    from paper_2407_02215_amd import cbt
    from paper_2407_02215_amd import inputs as I

    frames = args.warmup + args.steps
    w = I.workload(args.workload, frames=max(frames, 8))
    if len(w.cameras) < frames:
        raise SystemExit(f"workload {args.workload} has {len(w.cameras)} frames, asked for {frames}")
    inst = cbt.Instance(w.mesh, w.depth, w.lod)
    stream = inst.stream
    print(f"# warm-up {args.warmup} frames", file=sys.stderr, flush=True)
    for cam in w.cameras[:args.warmup]:
        inst.update(cam)
    torch.cuda.synchronize()
    snap = inst.snapshot()
    timed = w.cameras[args.warmup:frames]
    print(f"# counting pass over {len(timed)} frames", file=sys.stderr, flush=True)
    stats = [inst.update(cam, stats=True) for cam in timed]
    inst.restore(*snap)
    print("# timed pass", file=sys.stderr, flush=True)
    inst.time_stage(args.stage)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for cam in timed:
        inst.update(cam)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launches, stage_ms = inst.stage_time()
    inst.time_stage(None)
    # the timed pass must reproduce the counted one
    check = inst.pool()
    inst.restore(*snap)
    for cam in timed:
        inst.update(cam)
    again = inst.pool()
    import numpy as np
    assert all(np.array_equal(a, b) for a, b in zip(check, again)), "non-deterministic frame"

    updates = sum(s["live_before"] for s in stats)
    value = updates / elapsed
    alg = sum(algorithmic_bytes(args.stage, s, inst.cap) for s in stats) / len(stats)
    mean_ms = stage_ms / max(1, launches)
    achieved = alg / (mean_ms * 1e-3) / 1e9
    out = {
        "metric": "bisector updates/s per frame (% HBM roofline); p50/p99 update latency",
        "value": value,
        "unit": "bisector updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded workload generator)",
        "config": {"workload": args.workload, "cbt_depth": w.depth, "halfedges": w.mesh.H,
                   "frames": f"{args.warmup}..{frames - 1}", "mean_live": updates / len(stats)},
        "roofline": {"bound": "hbm", "kernel": args.stage, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "mean_launch_ms": mean_ms, "alg_bytes_per_launch": alg},
    }
    if not args.no_cpu_baseline:
        print("# CPU reference baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_budget)
    print(json.dumps(out), flush=True)
    inst.close()


if __name__ == "__main__":
    main()
