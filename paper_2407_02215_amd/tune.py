"""Launch-schedule autotuner (run on the GPU).

For each CBT depth it builds a busy instance (a seeded closed sphere mesh
whose halfedge count grows with the depth, sphere projection with fBm
displacement, an orbit camera path run until the pool is well used),
snapshots it, and then times the same frames under every candidate
schedule -- rank workgroups G (each owns a contiguous chunk of ceil(L/G)
ranks) and tree levels per reduction workgroup -- restoring the snapshot
before each candidate.  Frame time is read from HIP events around the whole
update.  The fastest schedule per depth is written to a JSON table that
``cbt.Instance`` applies when it is created (``tuned=True``).

Schedules change only how work is cut into workgroups, never results (the
GPU tests check several schedules against the CPU reference).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "schedule.json")

GROUPS = [16, 32, 64, 128, 256, 512, 1024, 2048]
LEVELS = [5, 7, 10]


def _busy_instance(D: int, seed: int, frames: int):
    from . import cbt
    from . import inputs as I
    H = max(24, min(50000, (1 << D) >> 8))
    w = I.batched_workloads(1, frames=frames, seed=seed, h_range=(H, H), d_range=(D, D), table_res=128)[0]
    inst = cbt.Instance(w.mesh, w.depth, w.lod)
    return inst, w


def _time_frames(inst, cams) -> float:
    inst.time_stage("frame")
    for c in cams:
        inst.update(c)
    n, ms = inst.stage_time()
    inst.time_stage(None)
    return ms / max(1, n)


def tune_depth(D: int, seed: int = 17, warm: int = 40, timed: int = 8, verbose: bool = True) -> dict:
    inst, w = _busy_instance(D, seed, warm + timed)
    for c in w.cameras[:warm]:
        inst.update(c)
    snap = inst.snapshot()
    live = inst.live_count()
    cams = w.cameras[warm:warm + timed]
    results = []
    best = None
    for g in GROUPS:
        if g > max(16, inst.cap // 32):
            continue
        inst.restore(*snap)
        inst.set_schedule(g, 10)
        _time_frames(inst, cams[:2])          # warm the code path
        inst.restore(*snap)
        t = _time_frames(inst, cams)
        results.append({"rank_groups": g, "reduce_levels": 10, "frame_ms": t})
        if best is None or t < best[2]:
            best = (g, 10, t)
    for lv in LEVELS:
        if lv == 10:
            continue
        inst.restore(*snap)
        inst.set_schedule(best[0], lv)
        t = _time_frames(inst, cams)
        results.append({"rank_groups": best[0], "reduce_levels": lv, "frame_ms": t})
        if t < best[2]:
            best = (best[0], lv, t)
    inst.close()
    out = {"D": D, "live": live, "rank_groups": best[0], "reduce_levels": best[1], "frame_ms": best[2],
           "candidates": results}
    if verbose:
        print(json.dumps({k: v for k, v in out.items() if k != "candidates"}), flush=True)
    return out


def load_table(path: str = TABLE) -> dict:
    """depth -> (rank_groups, reduce_levels), empty when no table exists."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        t = json.load(f)
    return {int(e["D"]): (int(e["rank_groups"]), int(e["reduce_levels"])) for e in t["entries"]}


def lookup(D: int, table: dict) -> tuple | None:
    """The entry of the nearest tuned depth (None when the table is empty)."""
    if not table:
        return None
    d = min(table, key=lambda x: (abs(x - D), -x))
    return table[d]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--depths", default="12,14,16,18,20,22,24")
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args()
    import torch
    entries = []
    t0 = time.time()
    for D in [int(x) for x in args.depths.split(",")]:
        entries.append(tune_depth(D))
    table = {"device": torch.cuda.get_device_name(0), "seconds": time.time() - t0, "entries": entries}
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(f"wrote {args.out}", file=sys.stderr)


if __name__ == "__main__":
    main()
