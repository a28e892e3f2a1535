"""Launch-schedule autotuner (run on the GPU).

For each CBT depth it builds a busy instance (a seeded closed sphere mesh
whose halfedge count grows with the depth, sphere projection with fBm
displacement, an orbit camera path that refines it frame by frame) and
snapshots it at several live counts on the way (when the live count first
passes 1/256, 1/32 and 1/8 of the pool, and at the end of the path).  At
each snapshot it times the same frames under every candidate schedule --
rank workgroups G (each owns a contiguous chunk of ceil(L/G) ranks) and
tree levels per reduction workgroup -- restoring the snapshot before each
candidate.  Frame time is read from HIP events around the whole update.
The fastest schedule per (depth, live count) is written to a JSON table;
``cbt.Instance`` applies the entry of the nearest depth and live count
(``tuned=True`` at creation, the busiest entry of the depth;
``Instance.apply_tuned()`` for its current live count).  The workgroup
size is a build-time constant, not a candidate here: whole-library builds
at 128 and 512 threads per workgroup measured slower on the depth-24
terrain than 256 (four wave64).

Schedules change only how work is cut into workgroups, never results (the
GPU tests check several schedules against the CPU reference).
"""
from __future__ import annotations

import argparse
import json
import math
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


LIVE_FRACS = (1 / 256, 1 / 32, 1 / 8)


def _tune_snapshot(inst, snap, cams) -> dict:
    """Every candidate schedule timed over cams from snap; the fastest."""
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
    return {"rank_groups": best[0], "reduce_levels": best[1], "frame_ms": best[2], "candidates": results}


def tune_depth(D: int, seed: int = 17, warm: int = 40, timed: int = 8, verbose: bool = True) -> list:
    inst, w = _busy_instance(D, seed, warm + timed)
    cap = inst.cap
    marks = [int(f * cap) for f in LIVE_FRACS]
    snaps = []
    for f, c in enumerate(w.cameras[:warm]):
        inst.update(c)
        live = inst.live_count()
        while marks and live >= marks[0]:
            marks.pop(0)
            snaps.append((f + 1, live, inst.snapshot()))
    if not snaps or snaps[-1][0] != warm:
        snaps.append((warm, inst.live_count(), inst.snapshot()))
    out = []
    for f, live, snap in snaps:
        cams = w.cameras[f:f + timed]
        if len(cams) < timed:
            continue
        e = {"D": D, "live": live}
        e.update(_tune_snapshot(inst, snap, cams))
        out.append(e)
        if verbose:
            print(json.dumps({k: v for k, v in e.items() if k != "candidates"}), flush=True)
    inst.close()
    return out


def load_table(path: str = TABLE) -> dict:
    """depth -> [(live, rank_groups, reduce_levels), ...] by live count,
    empty when no table exists."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        t = json.load(f)
    out = {}
    for e in t["entries"]:
        out.setdefault(int(e["D"]), []).append((int(e["live"]), int(e["rank_groups"]), int(e["reduce_levels"])))
    return {d: sorted(v) for d, v in out.items()}


def lookup(D: int, table: dict, live: int | None = None) -> tuple | None:
    """(rank_groups, reduce_levels) of the nearest tuned depth, and within it
    of the live count nearest to live (ratio-wise; the busiest entry when
    live is None).  None when the table is empty."""
    if not table:
        return None
    d = min(table, key=lambda x: (abs(x - D), -x))
    entries = table[d]
    if live is None:
        e = entries[-1]
    else:
        x = math.log(max(1, int(live)))
        e = min(entries, key=lambda t: abs(math.log(max(1, t[0])) - x))
    return e[1], e[2]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--depths", default="12,14,16,18,20,22,24")
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args()
    import torch
    entries = []
    t0 = time.time()
    for D in [int(x) for x in args.depths.split(",")]:
        entries += tune_depth(D)
    table = {"device": torch.cuda.get_device_name(0), "seconds": time.time() - t0, "entries": entries}
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(f"wrote {args.out}", file=sys.stderr)


if __name__ == "__main__":
    main()
