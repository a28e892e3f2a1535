"""Host-side logic that needs no GPU: the benchmark's refusal of several
GPUs, the HBM traffic computation from byte-counter CSVs, and the seeded
input generators' determinism."""
import csv
import json
import os
import subprocess
import sys

import numpy as np
import pytest

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
    """Every frame kernel dispatched between the two marker kernels belongs
    to the timed pass: per stage the counters summed over those dispatches
    and divided by the timed frames, scaled by the copy calibration (copy
    bytes / the copy's counter reading); rows of one dispatch (one per XCD)
    are summed; dispatches outside the markers do not count."""
    K = 3
    res = "void cbtk::k_resolve<false>(cbtk::Batch, cbtk::Inst)"
    fill = "void cbtk::k_fill<false, float>(cbtk::Batch, cbtk::Inst)"
    red = "void cbtk::k_reduce_top<false>(cbtk::Batch, cbtk::Inst)"
    spin = "spin_kernel(long)"
    fetch, write, valu = [], [], []
    d = 0

    def frame(scale_):
        nonlocal d
        for name, f, w in ((res, 100.0, 50.0), (fill, 30.0, 20.0), (red, 1.0, 1.0)):
            d += 1
            fetch.extend([(d, name, f * scale_ / 2), (d, name, f * scale_ / 2)])
            write.append((d, name, w * scale_))
            valu.append((d, name, 10.0))

    frame(99.0)                      # before the timed pass
    d += 1
    fetch.append((d, spin, 5.0)); write.append((d, spin, 5.0)); valu.append((d, spin, 1.0))
    for _ in range(K):
        frame(1.0)
    d += 1
    fetch.append((d, spin, 5.0)); write.append((d, spin, 5.0)); valu.append((d, spin, 1.0))
    frame(77.0)                      # after it
    for n, c, rows in (("f", "FETCH_SIZE", fetch), ("w", "WRITE_SIZE", write), ("v", "SQ_INSTS_VALU", valu)):
        _write_counters(tmp_path / f"{n}.csv", c, rows)
    copy_kib = traffic.COPY_BYTES / 1024.0
    _write_counters(tmp_path / "cf.csv", "FETCH_SIZE", [(1, "copyBuffer", copy_kib / 2), (2, "copyBuffer", 1.0)])
    _write_counters(tmp_path / "cw.csv", "WRITE_SIZE", [(1, "copyBuffer", copy_kib)])
    key = traffic.key_of("terrain", "edge", 32, 40, 5, K, [1024, 10])
    t = traffic.measure(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "cf.csv"),
                        str(tmp_path / "cw.csv"), key, valu=str(tmp_path / "v.csv"))
    assert t["fetch_scale"] == 2.0 and t["write_scale"] == 1.0
    assert t["kernels"]["resolve"]["fetch_bytes"] == 100.0 * 1024.0 * 2.0
    assert t["kernels"]["resolve"]["write_bytes"] == 50.0 * 1024.0
    assert t["kernels"]["fill"]["bytes"] == (30.0 * 2.0 + 20.0) * 1024.0
    assert t["kernels"]["reduce"]["valu_insts"] == pytest.approx(10.0)
    assert t["frame_bytes"] == pytest.approx(((100 + 30 + 1) * 2.0 + (50 + 20 + 1)) * 1024.0)
    assert t["frame_valu_insts"] == pytest.approx(30.0)
    assert t["source_sha256"] == traffic.source_digest()


def test_traffic_lookup_requires_same_command_source_and_schedule(tmp_path, monkeypatch):
    table = tmp_path / "traffic.json"
    monkeypatch.setattr(traffic, "TABLE", str(table))
    key = traffic.key_of("terrain", "edge", 32, 40, 5, 20, [1024, 10])
    rec = dict(key, kernels={"resolve": {"bytes": 123.0}}, frame_bytes=456.0, source_sha256=traffic.source_digest())
    traffic.record(rec)
    traffic.record(dict(rec, steps=200, frame_bytes=789.0))
    assert traffic.lookup("terrain", "edge", 32, 40, 5, 20, [1024, 10])["frame_bytes"] == 456.0
    assert traffic.lookup("terrain", "edge", 32, 40, 5, 200, [1024, 10])["frame_bytes"] == 789.0
    assert traffic.lookup("terrain", "edge", 32, 40, 5, 20, [512, 10]) is None
    assert traffic.lookup("terrain", "area", 32, 40, 5, 20, [1024, 10]) is None
    assert traffic.lookup("terrain", "edge", 32, 0, 5, 20, [1024, 10]) is None
    traffic.record(dict(rec, frame_bytes=1.0))                # same key: replaced
    assert len(json.loads(table.read_text())) == 2
    traffic.record(dict(rec, source_sha256="0" * 64))
    assert traffic.lookup("terrain", "edge", 32, 40, 5, 20, [1024, 10]) is None


def test_byte_models_follow_the_paper_minimal_total():
    """The paper-minimal per-stage bytes add up to 16 L + 48 S + 24 N +
    8 hops + 3/8 2^D with hops = S."""
    sys.path.insert(0, ROOT)
    import bench
    st = {"live_before": 1000, "split_consumed": 70, "allocations": 150, "frees": 90, "merge_requests": 300,
          "merges_executed": 5, "merge_candidates": 120, "merge_configs": 12}
    D = 14
    assert bench.paper_bytes("frame", st, D) == 16 * 1000 + 48 * 70 + 24 * 150 + 8 * 70 + 3 / 8 * (1 << D)
    assert bench.layout_bytes("frame", st, D) > bench.paper_bytes("frame", st, D)


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


def test_tuned_schedule_lookup_by_depth_and_live_count(tmp_path):
    """The tuned table holds several live counts per depth; the lookup takes
    the nearest depth (the deeper one on a tie), then the live count nearest
    by ratio, or the busiest entry when no live count is given."""
    import json
    from paper_2407_02215_amd import tune
    entries = [{"D": 16, "live": 1000, "rank_groups": 32, "reduce_levels": 10},
               {"D": 16, "live": 100000, "rank_groups": 256, "reduce_levels": 7},
               {"D": 20, "live": 30000, "rank_groups": 64, "reduce_levels": 10},
               {"D": 20, "live": 700000, "rank_groups": 512, "reduce_levels": 5}]
    p = tmp_path / "schedule.json"
    p.write_text(json.dumps({"device": "test", "seconds": 0.0, "entries": entries}))
    t = tune.load_table(str(p))
    assert t[16] == [(1000, 32, 10), (100000, 256, 7)]
    assert tune.lookup(16, t) == (256, 7)
    assert tune.lookup(16, t, 2000) == (32, 10)
    assert tune.lookup(16, t, 50000) == (256, 7)      # log-nearer to 1e5 than to 1e3
    assert tune.lookup(18, t, 800000) == (512, 5)     # tie between 16 and 20: the deeper table
    assert tune.lookup(24, t, 40000) == (64, 10)
    assert tune.lookup(16, {}, 5) is None


def test_trace_window_means_between_markers(tmp_path):
    """Kernel-trace durations: only the launches strictly between the two
    marker kernels count; per stage the mean launch duration and the
    launches per timed frame (two reduction launches per frame)."""
    from paper_2407_02215_amd import traffic as T
    rows = []
    d = 0

    def add(name, ns):
        nonlocal d
        d += 1
        rows.append({"Dispatch_Id": d, "Kernel_Name": name, "Start_Timestamp": 1000 * d,
                     "End_Timestamp": 1000 * d + ns})

    fill = "void cbtk::k_fill<false, float>(cbtk::Batch, cbtk::Inst)"
    sub = "void cbtk::k_reduce_sub<false>(cbtk::Batch, cbtk::Inst)"
    top = "void cbtk::k_reduce_top<false>(cbtk::Batch, cbtk::Inst)"
    add(fill, 999_000)                   # before the timed pass
    add("spin_kernel(long)", 5)
    for k in range(4):
        add(fill, 100_000 + 1000 * k)
        add(sub, 4000)
        add(top, 2000)
    add("spin_kernel(long)", 5)
    add(fill, 999_000)                   # after it
    p = tmp_path / "trace_kernel_trace.csv"
    with open(p, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    tw = T.trace_window(str(p), 4)
    assert tw["fill"]["launches_per_frame"] == 1.0
    assert abs(tw["fill"]["mean_us"] - 101.5) < 1e-9
    assert tw["reduce"]["launches_per_frame"] == 2.0
    assert abs(tw["reduce"]["mean_us"] - 3.0) < 1e-9
    assert abs(tw["reduce"]["us_per_frame"] - 6.0) < 1e-9
