"""Batched update (cbt_batch_*): many instances of uneven mesh size and
depth advanced by shared launches (one per stage, or one persistent launch
per frame), eagerly or from a captured HIP graph, must give every member
exactly the state it gets alone (and the CPU reference's state)."""
import numpy as np
import pytest
import torch  # noqa: F401

from oracle import Oracle
from paper_2407_02215_amd import cbt
from paper_2407_02215_amd import inputs as I
from tests.gpu_checks import assert_same_state, assert_same_tree, log

pytestmark = pytest.mark.gpu


def _same_pool(a, b, label):
    for name, x, y in zip(("heap_id", "twin", "next", "prev"), a.pool(), b.pool()):
        bad = np.nonzero(x != y)[0]
        assert bad.size == 0, f"{label} {name}: {bad.size} mismatches, first {bad[:5].tolist()}"
    ta = a.query(tree=True)["tree"]
    tb = b.query(tree=True)["tree"]
    assert np.array_equal(ta, tb), f"{label}: trees differ"


@pytest.mark.parametrize("graph,persistent", [(True, False), (False, False), (True, True), (False, True)])
def test_batched_matches_single_instances(graph, persistent):
    ws = I.batched_workloads(10, frames=14, seed=5, h_range=(24, 4000), d_range=(12, 16), table_res=64)
    log(f"[batch graph={graph} persistent={persistent}] H={[w.mesh.H for w in ws]} D={[w.depth for w in ws]}")
    alone = [cbt.Instance(w.mesh, w.depth, w.lod) for w in ws]
    members = [cbt.Instance(w.mesh, w.depth, w.lod) for w in ws]
    # uneven schedules inside one batch: the smallest grid, and the default
    for i, m in enumerate(members):
        if i % 3 == 0:
            m.set_schedule(16, 5)
    batch = cbt.Batch(members, graph=graph, persistent=persistent)
    for f in range(len(ws[0].cameras)):
        for a, w in zip(alone, ws):
            a.update(w.cameras[f])
        st = batch.update([w.cameras[f] for w in ws], stats=(f % 4 == 3))
        if st:
            assert all(s["live_after"] > 0 for s in st)
    batch.synchronize()
    torch.cuda.synchronize()
    grew = 0
    for i, (a, m) in enumerate(zip(alone, members)):
        _same_pool(a, m, f"member {i}")
        grew += a.live_count() > ws[i].mesh.H
    assert grew >= len(ws) // 2
    batch.close()
    for x in alone + members:
        x.close()


@pytest.mark.parametrize("persistent", [False, True])
def test_batched_members_match_reference(persistent):
    ws = I.batched_workloads(4, frames=10, seed=9, h_range=(24, 600), d_range=(12, 14), table_res=64)
    members = [cbt.Instance(w.mesh, w.depth, w.lod) for w in ws]
    orcs = [Oracle(w.mesh, w.depth, w.lod) for w in ws]
    log(f"[batch reference persistent={persistent}]")
    batch = cbt.Batch(members, graph=True, persistent=persistent)
    for f in range(len(ws[0].cameras)):
        stats = batch.update([w.cameras[f] for w in ws], stats=True)
        for i, (o, w) in enumerate(zip(orcs, ws)):
            st = o.frame(camera=w.cameras[f])
            assert stats[i]["live_before"] == st.live_before
            assert stats[i]["allocations"] == st.allocations, f"member {i} frame {f}"
            assert stats[i]["frees"] == st.frees
    for i, (m, o) in enumerate(zip(members, orcs)):
        assert_same_state(m, o, f"member {i}")
        assert_same_tree(m, o, f"member {i}")
    batch.close()


@pytest.mark.parametrize("persistent", [False, True])
def test_batched_injected_decisions_match_reference(persistent):
    meshes = [(I.mesh_cube(), 10), (I.mesh_icosahedron(), 12), (I.mesh_quad_sphere(3, 0.5, 11), 11),
              (I.mesh_two_triangles(False), 8), (I.mesh_two_triangles(True), 3)]
    members = [cbt.Instance(m, D) for m, D in meshes]
    orcs = [Oracle(m, D) for m, D in meshes]
    log(f"[batch injected persistent={persistent}]")
    batch = cbt.Batch(members, graph=True, persistent=persistent)
    rng = np.random.default_rng(21)
    for f in range(12):
        ps, pm = (0.5, 0.1) if f < 6 else (0.1, 0.6)
        decs = [I.random_decisions(o.cap, int(rng.integers(1 << 30)), ps, pm) for o in orcs]
        batch.update_with_decisions(decs)
        for o, d in zip(orcs, decs):
            o.frame(decisions=d)
    batch.synchronize()
    for i, (m, o) in enumerate(zip(members, orcs)):
        assert_same_state(m, o, f"member {i}")
        assert_same_tree(m, o, f"member {i}")
    batch.close()


def test_persistent_spans_match_single_instances():
    """Pools large enough that the persistent frame runs several workgroups
    per work item (the depth-20 planet: 2048 rank workgroups, 128 bitfield
    workgroups) beside small ones, against the same instances alone."""
    planet = I.workload("planet", frames=24, table_res=128)
    cube = I.workload("cube", frames=8)
    ws = [planet, cube, planet]
    alone = [cbt.Instance(w.mesh, w.depth, w.lod) for w in ws]
    members = [cbt.Instance(w.mesh, w.depth, w.lod) for w in ws]
    members[2].set_schedule(100, 7)
    alone[2].set_schedule(100, 7)
    log("[batch spans] planet D=20 x2, cube D=16")
    batch = cbt.Batch(members, graph=True, persistent=True)
    for f in range(20):
        cams = [w.cameras[min(f, len(w.cameras) - 1)] for w in ws]
        for a, c in zip(alone, cams):
            a.update(c)
        st = batch.update(cams, stats=(f % 5 == 4))
        if st:
            assert all(s["live_after"] > 0 for s in st)
    batch.synchronize()
    torch.cuda.synchronize()
    for i, (a, m) in enumerate(zip(alone, members)):
        _same_pool(a, m, f"member {i}")
    assert alone[0].live_count() > 10_000
    batch.close()
    for x in alone + members:
        x.close()


def test_persistent_wait_failure_is_reported():
    """The failure path of the persistent frame, forced from the host: the
    budget stage's waits give up at once (as a wait that ran out of its
    bound would), the later stages are skipped, the update reports a device
    error and the members refuse further work; the device itself stays
    usable (a new instance then matches the CPU reference)."""
    ws = I.batched_workloads(3, frames=6, seed=7, h_range=(24, 800), d_range=(12, 14), table_res=64)
    members = [cbt.Instance(w.mesh, w.depth, w.lod) for w in ws]
    log("[batch failure path] persistent, budget stage forced to give up")
    batch = cbt.Batch(members, graph=True, persistent=True)
    batch.update([w.cameras[0] for w in ws], stats=True)
    batch.fail_stage(3)
    with pytest.raises(cbt.CbtError) as e:
        batch.update([w.cameras[1] for w in ws], stats=True)
    assert e.value.status == -5 and "0x20" in str(e.value)
    with pytest.raises(cbt.CbtError):
        members[0].update(ws[0].cameras[2])
    batch.close()
    for m in members:
        m.close()
    w = ws[1]
    inst = cbt.Instance(w.mesh, w.depth, w.lod)
    orc = Oracle(w.mesh, w.depth, w.lod)
    for cam in w.cameras[:4]:
        inst.update(cam)
        orc.frame(camera=cam)
    assert_same_state(inst, orc, "after the failure")
    inst.close()


def test_batched_configuration_sampled_against_reference():
    """The batched configuration at its full size and seed (128 closed sphere
    meshes of 24 to 50,000 halfedges, depths 14-22, tuned schedules, a HIP
    graph), 20 frames from the base meshes with one launch per stage and
    with one persistent launch per frame; sampled members (the smallest and
    deepest, the largest mesh, and three more) replayed on the CPU
    reference with the same cameras and compared slot by slot."""
    frames = 20
    log("[batched configuration] building 128 workloads")
    ws = I.batched_workloads(128, frames=64, seed=4, workers=1)
    H = [w.mesh.H for w in ws]
    sample = sorted({int(np.argmin(H)), int(np.argmax(H)), 0, 64, 127})
    refs = {}
    for i in sample:
        w = ws[i]
        o = Oracle(w.mesh, w.depth, w.lod)
        for f in range(frames):
            o.frame(camera=w.cameras[f])
        refs[i] = o
        log(f"[batched configuration] reference member {i}: H={w.mesh.H} D={w.depth} live {o.live_count}")
    for persistent in (False, True):
        members = [cbt.Instance(w.mesh, w.depth, w.lod, tuned=True) for w in ws]
        batch = cbt.Batch(members, graph=True, persistent=persistent)
        for f in range(frames):
            batch.update([w.cameras[f] for w in ws])
        batch.synchronize()
        log(f"[batched configuration] persistent={persistent}: {frames} frames done")
        for i in sample:
            assert_same_state(members[i], refs[i], f"member {i} persistent={persistent}")
            assert_same_tree(members[i], refs[i], f"member {i} persistent={persistent}")
        batch.close()
        for m in members:
            m.close()
        del members
        torch.cuda.empty_cache()
