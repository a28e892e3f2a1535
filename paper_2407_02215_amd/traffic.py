"""HBM traffic of one kernel per launch, from rocprofv3 byte counters.

Two counter runs of the benchmark (``--pmc FETCH_SIZE``, then
``--pmc WRITE_SIZE``) give KiB per dispatch; two runs of a plain device copy
of known size (``bench.py --copy-calibration``) give the scale of each
counter (bytes moved / bytes the counter reports).  The benchmark's kernel
dispatches come in its protocol order: W warm-up frames, then passes over
the same K frames (counting, timed, latency, stage survey); the timed pass
is dispatches [W + K, W + 2K) of the kernel.  The kernel is the one whose
roofline the benchmark line reports (``--kernel auto``) or a named stage.
The result is written to ``traffic.json`` beside this file together with a
digest of the kernel source and the launch schedule the counter run used
(read from its benchmark line); the benchmark reports it only while both
still match.

    python -m paper_2407_02215_amd.traffic --fetch F.csv --write W.csv \\
        --copy-fetch CF.csv --copy-write CW.csv --bench-log F.log --kernel auto --warmup 40 --steps 200
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "traffic.json")
KERNEL_SOURCE = os.path.join(HERE, "csrc", "cbt_kernels.hip")
COPY_BYTES = 256 << 20   # bench.py --copy-calibration copies this many bytes


def source_digest() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def per_dispatch(path: str, counter: str, match) -> list:
    """Counter values (summed over the rows of one dispatch) of the kernels
    whose name satisfies match, in dispatch order."""
    acc = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter or not match(r["Kernel_Name"]):
            continue
        d = int(r["Dispatch_Id"])
        acc[d] = acc.get(d, 0.0) + float(r["Counter_Value"])
    return [acc[d] for d in sorted(acc)]


def _kernel_match(stage: str):
    tag = f"k_{stage}<"
    return lambda name: tag in name


def _copy_match(name: str) -> bool:
    return "copyBuffer" in name or "elementwise" in name


def scale(path: str, counter: str) -> float:
    """Bytes per counter unit: the copy's bytes over its counter reading
    (the largest dispatch of the copy run, the 256 MiB copies)."""
    v = per_dispatch(path, counter, _copy_match)
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


def measure(fetch, write, copy_fetch, copy_write, stage, warmup, steps, schedule) -> dict:
    m = _kernel_match(stage)
    f = per_dispatch(fetch, "FETCH_SIZE", m)
    w = per_dispatch(write, "WRITE_SIZE", m)
    need = warmup + 2 * steps
    if len(f) < need or len(w) < need:
        raise SystemExit(f"expected {need} dispatches of k_{stage}, found {len(f)} / {len(w)}")
    lo, hi = warmup + steps, warmup + 2 * steps
    sf, sw = scale(copy_fetch, "FETCH_SIZE"), scale(copy_write, "WRITE_SIZE")
    fb = sum(f[lo:hi]) / steps * 1024.0 * sf
    wb = sum(w[lo:hi]) / steps * 1024.0 * sw
    return {"kernel": stage, "bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
            "fetch_scale": sf, "write_scale": sw, "warmup": warmup, "steps": steps, "schedule": schedule,
            "source_sha256": source_digest()}


def lookup(stage: str, warmup: int, steps: int, schedule):
    """Bytes per launch of the stage's kernel if measured on this kernel
    source, frame range and launch schedule, else None."""
    if not os.path.exists(TABLE):
        return None
    with open(TABLE) as f:
        t = json.load(f)
    if (t.get("kernel") != stage or t.get("warmup") != warmup or t.get("steps") != steps
            or t.get("schedule") != [int(x) for x in schedule] or t.get("source_sha256") != source_digest()):
        return None
    return float(t["bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--bench-log", required=True, help="output of the FETCH_SIZE run (its benchmark line)")
    ap.add_argument("--kernel", default="auto", help="stage name, or auto: the benchmark line's roofline kernel")
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--out", default=TABLE)
    a = ap.parse_args()
    b = bench_line(a.bench_log)
    kernel = b["roofline"]["kernel"] if a.kernel == "auto" else a.kernel
    t = measure(a.fetch, a.write, a.copy_fetch, a.copy_write, kernel, a.warmup, a.steps,
                [int(x) for x in b["config"]["schedule"]])
    with open(a.out, "w") as f:
        json.dump(t, f, indent=1)
    print(json.dumps(t))


if __name__ == "__main__":
    main()
