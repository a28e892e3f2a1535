"""Serving loop (cbt_server_*): requests for many instances arrive in an
interleaved order, are batched continuously (batches of varying membership,
two launch slots in flight), with a memory budget small enough that idle
instances are evicted (their live records kept in the arena or on the host)
and re-admitted.  Every instance
must end in exactly the state it reaches alone with the same cameras, and
in the CPU reference's state for those cameras."""
import numpy as np
import pytest
import torch  # noqa: F401

from oracle import Oracle
from paper_2407_02215_amd import cbt
from paper_2407_02215_amd import inputs as I
from tests.gpu_checks import log

pytestmark = pytest.mark.gpu


def _alone(w, frames):
    inst = cbt.Instance(w.mesh, w.depth, w.lod)
    for cam in w.cameras[:frames]:
        inst.update(cam)
    q = inst.query(tree=True)
    inst.close()
    return q


def _reference(w, frames):
    """The CPU reference's state after the same cameras, in query form."""
    orc = Oracle(w.mesh, w.depth, w.lod)
    for cam in w.cameras[:frames]:
        orc.frame(camera=cam)
    ids, tw, nx, pv = orc.pool()
    live = np.nonzero(ids)[0]
    return {"slot": live.astype(np.int32), "heap_id": ids[live], "twin": tw[live], "next": nx[live],
            "prev": pv[live], "tree": orc.heap()}


@pytest.mark.parametrize("room", ["three", "one"])
def test_served_results_equal_alone(room):
    """room: the budget holds about three workspaces (evicted instances'
    records stay in the arena), or one (records go to host memory)."""
    ws = I.batched_workloads(6, frames=10, seed=31, h_range=(24, 2000), d_range=(12, 14), table_res=64)
    sizes = [cbt.workspace_bytes(w.mesh.H, w.depth) for w in ws]
    budget = sum(sorted(sizes)[-3:]) + (1 << 20) if room == "three" else max(sizes) + (1 << 12)
    log(f"[server] H={[w.mesh.H for w in ws]} D={[w.depth for w in ws]} budget={budget}")
    # the tuned schedule table (per depth and live count) in one of the two runs
    srv = cbt.Server(arena_bytes=budget, memory_budget=budget, max_batch=4, slots=2, map_capacity=1 << 16,
                     tuned=(room == "three"))
    ids = [srv.open(w.mesh, w.depth, w.lod) for w in ws]
    rng = np.random.default_rng(5)
    nxt = [0] * len(ws)
    order = []
    for i, w in enumerate(ws):
        order += [i] * len(w.cameras)
    rng.shuffle(order)
    done = []
    tag = 0
    for i in order:
        srv.submit(ids[i], ws[i].cameras[nxt[i]], tag)
        nxt[i] += 1
        tag += 1
        if rng.random() < 0.4:
            done += srv.poll(wait=bool(rng.random() < 0.5))
    done += srv.drain()
    assert len(done) == tag
    assert all(c["status"] == 0 for c in done), [c for c in done if c["status"] != 0][:3]
    st = srv.stats()
    log(f"[server] stats {st}")
    assert st["evictions"] > 0 and st["admissions"] > len(ws)
    if room == "one":
        assert st["host_snapshots"] > 0
    assert st["frames"] == tag
    sizes_seen = {c["batch_size"] for c in done}
    if room == "three":
        assert max(sizes_seen) > 1
    for i, w in enumerate(ws):
        ref = _alone(w, len(w.cameras))
        orc = _reference(w, len(w.cameras))
        got = srv.query(ids[i], tree=True)
        for key in ("slot", "heap_id", "twin", "next", "prev", "tree"):
            assert np.array_equal(got[key], ref[key]), f"instance {i}: {key} differs from the instance alone"
            assert np.array_equal(got[key], orc[key]), f"instance {i}: {key} differs from the reference"
    srv.close()


def test_server_refuses_instance_over_budget():
    w = I.workload("cube")
    small = cbt.workspace_bytes(w.mesh.H, 12)
    srv = cbt.Server(arena_bytes=small + (1 << 16), memory_budget=small + (1 << 16), max_batch=2, slots=1,
                     map_capacity=1 << 12)
    srv.open(w.mesh, 12, w.lod)
    with pytest.raises(cbt.CbtError) as e:
        srv.open(w.mesh, 16, w.lod)
    assert e.value.status == -6
    srv.close()
