"""HBM traffic and VALU instructions of the benchmark's timed frames, from
rocprofv3 counter runs.

Counter runs of the benchmark (``--pmc FETCH_SIZE``, ``--pmc WRITE_SIZE``
and, optionally, ``--pmc SQ_INSTS_VALU``) give values per dispatch; two runs
of a plain device copy of known size (``bench.py --copy-calibration``) give
the scale of each byte counter (bytes moved / bytes the counter reports).
The benchmark brackets its timed pass with two marker kernels (torch's spin
kernel) outside the timed region; every frame kernel dispatched between the
two markers belongs to the timed pass.  Per stage, the counters summed over
those dispatches and divided by the number of timed frames give bytes per
launch; summed over every kernel, bytes per frame.

The record is added to ``traffic.json`` beside this file, keyed by the
workload, criterion, precision, pre-roll, warm-up and timed frame counts,
the launch schedule (read from the benchmark line of the counter run) and a
digest of the kernel source; the benchmark reports counted traffic only
while all of them match.

    python -m paper_2407_02215_amd.traffic --fetch F.csv --write W.csv [--valu V.csv] \\
        --copy-fetch CF.csv --copy-write CW.csv --bench-log F.log

A kernel trace of the same command (``rocprofv3 --kernel-trace``) gives the
timed pass's launch durations per stage:

    python -m paper_2407_02215_amd.traffic trace --trace T_kernel_trace.csv --steps K
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "traffic.json")
KERNEL_SOURCE = os.path.join(HERE, "csrc", "cbt_kernels.hip")
COPY_BYTES = 256 << 20   # bench.py --copy-calibration copies this many bytes

# kernel name tag -> pipeline stage
KERNEL_STAGE = {"k_enumerate<": "enumerate", "k_classify<": "classify", "k_vote<": "vote", "k_budget<": "budget",
                "k_walk<": "chain", "k_owners<": "owners", "k_freelist<": "freelist", "k_fill<": "fill",
                "k_resolve<": "resolve", "k_reduce_sub<": "reduce", "k_reduce_top<": "reduce"}
MARKER = "spin"


def source_digest() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def stage_of(name: str):
    for tag, stage in KERNEL_STAGE.items():
        if tag in name:
            return stage
    return None


def dispatches(path: str, counter: str) -> dict:
    """{dispatch id: (kernel name, counter summed over the dispatch's rows)}."""
    acc = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        d = int(r["Dispatch_Id"])
        name, v = acc.get(d, (r["Kernel_Name"], 0.0))
        acc[d] = (name, v + float(r["Counter_Value"]))
    return acc


def timed_window(acc: dict):
    """Dispatch ids strictly between the first two marker kernels."""
    marks = sorted(d for d, (name, _) in acc.items() if MARKER in name)
    if len(marks) < 2:
        raise SystemExit(f"expected two marker dispatches, found {len(marks)}")
    return marks[0], marks[1]


def per_stage(acc: dict, steps: int) -> tuple:
    """Counter per launch of each stage and per frame over every kernel, in
    the timed window."""
    lo, hi = timed_window(acc)
    stage, total, other = {}, 0.0, []
    for d, (name, v) in acc.items():
        if not lo < d < hi:
            continue
        st = stage_of(name)
        if st is None:
            other.append(name)
            continue
        stage[st] = stage.get(st, 0.0) + v / steps
        total += v / steps
    if other:
        raise SystemExit(f"unexpected kernels in the timed window: {sorted(set(other))[:3]}")
    return stage, total


def _copy_match(name: str) -> bool:
    return "copyBuffer" in name or "elementwise" in name


def scale(path: str, counter: str) -> float:
    """Bytes per counter unit: the copy's bytes over its counter reading
    (the largest dispatch of the copy run, the 256 MiB copies)."""
    v = [x for name, x in dispatches(path, counter).values() if _copy_match(name)]
    return COPY_BYTES / (max(v) * 1024.0)


def bench_line(path: str) -> dict:
    """The benchmark line (the last JSON line with a "metric" key) of a log."""
    line_ = None
    for line in open(path, errors="replace"):
        line = line.strip()
        if line.startswith('{"metric"'):
            line_ = json.loads(line)
    if line_ is None:
        raise SystemExit(f"no benchmark line in {path}")
    return line_


def key_of(workload, criterion, precision, preroll, warmup, steps, schedule) -> dict:
    return {"workload": workload, "criterion": criterion, "precision": int(precision), "preroll": int(preroll),
            "warmup": int(warmup), "steps": int(steps), "schedule": [int(x) for x in schedule]}


def measure(fetch, write, copy_fetch, copy_write, key: dict, valu=None) -> dict:
    steps = key["steps"]
    sf, sw = scale(copy_fetch, "FETCH_SIZE"), scale(copy_write, "WRITE_SIZE")
    f_stage, f_total = per_stage(dispatches(fetch, "FETCH_SIZE"), steps)
    w_stage, w_total = per_stage(dispatches(write, "WRITE_SIZE"), steps)
    kernels = {}
    for st in sorted(set(f_stage) | set(w_stage)):
        fb = f_stage.get(st, 0.0) * 1024.0 * sf
        wb = w_stage.get(st, 0.0) * 1024.0 * sw
        kernels[st] = {"fetch_bytes": fb, "write_bytes": wb, "bytes": fb + wb}
    rec = dict(key)
    rec.update({"kernels": kernels, "frame_bytes": f_total * 1024.0 * sf + w_total * 1024.0 * sw,
                "fetch_scale": sf, "write_scale": sw, "source_sha256": source_digest()})
    if valu:
        v_stage, v_total = per_stage(dispatches(valu, "SQ_INSTS_VALU"), steps)
        for st, v in v_stage.items():
            kernels.setdefault(st, {})["valu_insts"] = v
        rec["frame_valu_insts"] = v_total
    return rec


def _load(path: str = None):
    path = path or TABLE
    if not os.path.exists(path):
        return []
    with open(path) as f:
        t = json.load(f)
    return t if isinstance(t, list) else []


def record(rec: dict, path: str = None):
    """Adds rec to the table, replacing an entry with the same key."""
    path = path or TABLE
    keys = ("workload", "criterion", "precision", "preroll", "warmup", "steps", "schedule")
    rows = [r for r in _load(path) if any(r.get(k) != rec.get(k) for k in keys)]
    rows.append(rec)
    with open(path, "w") as f:
        json.dump(rows, f, indent=1)


def lookup(workload, criterion, precision, preroll, warmup, steps, schedule):
    """The record for this command, kernel source and launch schedule, or
    None."""
    want = key_of(workload, criterion, precision, preroll, warmup, steps, schedule)
    digest = source_digest()
    for r in _load():
        if all(r.get(k) == v for k, v in want.items()) and r.get("source_sha256") == digest:
            return r
    return None


def trace_window(path: str, steps: int) -> dict:
    """From a rocprofv3 kernel trace of the benchmark: per stage, the mean
    duration (microseconds) of its launches in the timed pass (between the
    two marker kernels) and their number per frame."""
    rows = []
    for r in csv.DictReader(open(path)):
        rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    marks = sorted(d for d, name, _ in rows if MARKER in name)
    if len(marks) < 2:
        raise SystemExit(f"expected two marker dispatches, found {len(marks)}")
    lo, hi = marks[0], marks[1]
    acc = {}
    for d, name, ns in rows:
        if not lo < d < hi:
            continue
        st = stage_of(name)
        if st is None:
            raise SystemExit(f"unexpected kernel in the timed window: {name}")
        n, t = acc.get(st, (0, 0))
        acc[st] = (n + 1, t + ns)
    return {st: {"launches_per_frame": n / steps, "mean_us": t / n / 1e3, "us_per_frame": t / steps / 1e3}
            for st, (n, t) in sorted(acc.items())}


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "trace":
        tp = argparse.ArgumentParser(description="timed-window kernel durations from a kernel trace")
        tp.add_argument("cmd")
        tp.add_argument("--trace", required=True)
        tp.add_argument("--steps", type=int, required=True)
        t = tp.parse_args()
        print(json.dumps(trace_window(t.trace, t.steps), indent=1))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--valu", default=None, help="SQ_INSTS_VALU counter run (optional)")
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--bench-log", required=True, help="output of one of the counter runs (its benchmark line)")
    ap.add_argument("--out", default=TABLE)
    a = ap.parse_args()
    b = bench_line(a.bench_log)
    c = b["config"]
    key = key_of(c["workload"], c["criterion"], 64 if b["dtype"] == "f64" else 32, c["preroll"], b["warmup"],
                 b["steps"], c["schedule"])
    rec = measure(a.fetch, a.write, a.copy_fetch, a.copy_write, key, a.valu)
    record(rec, a.out)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
