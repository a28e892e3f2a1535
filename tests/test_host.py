"""Host-side logic that needs no GPU: the benchmark's refusal of several
GPUs, the HBM traffic computation from byte-counter CSVs, and the seeded
input generators' determinism."""
import csv
import json
import os
import subprocess
import sys

import numpy as np

from paper_2407_02215_amd import inputs as I
from paper_2407_02215_amd import traffic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def _write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, name, v in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_traffic_from_counter_csvs(tmp_path):
    """Dispatches of the stage's kernel in protocol order: W warm-up, then
    the K counted and the K timed ones; the timed pass's mean KiB, scaled by
    the copy calibration (copy bytes / the copy's counter reading), is the
    result.  Rows of one dispatch are summed (one per XCD)."""
    W, K = 2, 3
    kern = "void cbtk::k_resolve<false>(cbtk::Batch, cbtk::Inst)"
    other = "void cbtk::k_fill<false, float>(cbtk::Batch, cbtk::Inst)"
    fetch, write = [], []
    d = 0
    for i in range(W + 2 * K + 1):
        d += 1
        fetch += [(d, kern, 100.0 * (i + 1)), (d, kern, 100.0 * (i + 1))]   # two rows: 200 (i+1) KiB
        write += [(d, kern, 50.0)]
        d += 1
        fetch += [(d, other, 1e6)]
        write += [(d, other, 1e6)]
    _write_counters(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _write_counters(tmp_path / "w.csv", "WRITE_SIZE", write)
    copy_kib = traffic.COPY_BYTES / 1024.0
    _write_counters(tmp_path / "cf.csv", "FETCH_SIZE", [(1, "copyBuffer", copy_kib / 2), (2, "copyBuffer", 1.0)])
    _write_counters(tmp_path / "cw.csv", "WRITE_SIZE", [(1, "copyBuffer", copy_kib)])
    t = traffic.measure(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "cf.csv"),
                        str(tmp_path / "cw.csv"), "resolve", W, K, [1024, 10])
    timed = [200.0 * (i + 1) for i in range(W + K, W + 2 * K)]
    assert t["fetch_scale"] == 2.0 and t["write_scale"] == 1.0
    assert t["fetch_bytes"] == sum(timed) / K * 1024.0 * 2.0
    assert t["write_bytes"] == 50.0 * 1024.0
    assert t["bytes_per_launch"] == t["fetch_bytes"] + t["write_bytes"]
    assert t["source_sha256"] == traffic.source_digest()


def test_traffic_lookup_requires_same_source_and_schedule(tmp_path, monkeypatch):
    table = tmp_path / "traffic.json"
    rec = {"kernel": "resolve", "bytes_per_launch": 123.0, "warmup": 40, "steps": 200, "schedule": [1024, 10],
           "source_sha256": traffic.source_digest()}
    table.write_text(json.dumps(rec))
    monkeypatch.setattr(traffic, "TABLE", str(table))
    assert traffic.lookup("resolve", 40, 200, [1024, 10]) == 123.0
    assert traffic.lookup("resolve", 40, 200, [512, 10]) is None
    assert traffic.lookup("fill", 40, 200, [1024, 10]) is None
    assert traffic.lookup("resolve", 40, 100, [1024, 10]) is None
    rec["source_sha256"] = "0" * 64
    table.write_text(json.dumps(rec))
    assert traffic.lookup("resolve", 40, 200, [1024, 10]) is None


def test_input_generators_are_seeded():
    a = I.batched_workloads(3, frames=4, seed=9, h_range=(24, 400), d_range=(12, 14), table_res=32)
    b = I.batched_workloads(3, frames=4, seed=9, h_range=(24, 400), d_range=(12, 14), table_res=32)
    for x, y in zip(a, b):
        assert x.depth == y.depth
        assert np.array_equal(x.mesh.twin, y.mesh.twin) and np.array_equal(x.mesh.pos, y.mesh.pos)
        for c, e in zip(x.cameras, y.cameras):
            assert np.array_equal(np.asarray(c.pos), np.asarray(e.pos))
    d1 = I.random_decisions(1000, 5, 0.3, 0.2)
    assert np.array_equal(d1, I.random_decisions(1000, 5, 0.3, 0.2))
    assert not np.array_equal(d1, I.random_decisions(1000, 6, 0.3, 0.2))
    assert set(np.unique(d1).tolist()) <= {0, 1, 2}
