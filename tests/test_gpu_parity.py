"""Parity of the HIP path (through the C ABI) with the CPU reference:
initialisation, injected-decision frames, the paper's chain example, the
LOD-driven workloads frame by frame, determinism and snapshot/restore.

Every comparison is element by element on the same seeded inputs: heap IDs
and neighbour slots of every pool block, the full CBT heap, the per-block
decisions, and flat-domain vertices (bit-exact; the tolerance the vertices
are allowed is 1e-5 relative, but both sides evaluate the same binary32
operations in the same order)."""
import zlib

import numpy as np
import pytest
import torch  # noqa: F401  (first import can be slow on a fresh box: pay it at collection)

from oracle import Oracle
from paper_2407_02215_amd import cbt
from paper_2407_02215_amd import inputs as I
from tests.gpu_checks import assert_same_state, assert_same_tree, check_properties, log
from tests.helpers import decisions_for, paper_j_to_heap, we1_mesh

pytestmark = pytest.mark.gpu


def _meshes():
    return {
        "we1": (we1_mesh(4), 8),
        "cube": (I.mesh_cube(), 10),
        "ico": (I.mesh_icosahedron(), 10),
        "open2": (I.mesh_two_triangles(False), 8),
        "pillow": (I.mesh_two_triangles(True), 8),
        "qsphere": (I.mesh_quad_sphere(3, 0.5, 11), 12),
        "grid64": (I.mesh_grid(64), 16),
    }


def _vertices_match(inst, orc, label):
    q = inst.query(vertices=True)
    ov = orc.vertices()
    gv = q["vertices"]
    ref = ov[q["slot"]]
    assert np.array_equal(gv.view(np.uint32), ref.view(np.uint32)), f"{label}: vertices differ"


@pytest.mark.parametrize("name", list(_meshes()))
def test_init_matches_reference(name):
    mesh, D = _meshes()[name]
    log(f"[init] {name} H={mesh.H} D={D}")
    inst = cbt.Instance(mesh, D)
    orc = Oracle(mesh, D)
    assert inst.live_count() == mesh.H
    assert_same_state(inst, orc, name)
    assert_same_tree(inst, orc, name)
    _vertices_match(inst, orc, name)
    inst.close()


@pytest.mark.parametrize("name", list(_meshes()))
def test_injected_frames_match_reference(name):
    mesh, D = _meshes()[name]
    inst = cbt.Instance(mesh, D)
    orc = Oracle(mesh, D)
    rng = np.random.default_rng(zlib.crc32(name.encode()) % 9973)
    for f in range(14):
        p_split = [0.5, 0.3, 0.1, 0.05][f % 4]
        p_merge = [0.1, 0.4, 0.7, 0.9][f % 4]
        dec = I.random_decisions(orc.cap, int(rng.integers(1 << 30)), p_split, p_merge)
        label = f"{name} frame {f}"
        log(f"[injected] {label} L={orc.live_count}")
        gst = inst.update_with_decisions(dec, stats=True)
        ost = orc.frame(decisions=dec)
        for key in ("live_before", "split_requests", "split_accepted", "merge_requests", "merge_configs",
                    "merge_accepted", "merges_executed", "split_consumed", "allocations", "frees", "live_after"):
            assert gst[key] == getattr(ost, key), f"{label}: {key} gpu={gst[key]} ref={getattr(ost, key)}"
        gdec = inst.decisions()
        odec = orc.decisions()[0]
        was_live = gdec != 255
        assert was_live.sum() == ost.live_before
        assert np.array_equal(gdec[was_live], odec[was_live]), f"{label}: decisions differ"
        assert_same_state(inst, orc, label)
    assert_same_tree(inst, orc, name)
    _vertices_match(inst, orc, name)
    inst.close()


def test_saturated_pool_matches_reference():
    """A pool close to full: the rank-order reservation cut decides."""
    mesh = I.mesh_cube()
    D = 7
    inst = cbt.Instance(mesh, D)
    orc = Oracle(mesh, D)
    rng = np.random.default_rng(4)
    rejected = 0
    for f in range(30):
        dec = I.random_decisions(orc.cap, int(rng.integers(1 << 30)), 0.6, 0.3)
        log(f"[saturated] frame {f} L={orc.live_count}")
        gst = inst.update_with_decisions(dec, stats=True)
        ost = orc.frame(decisions=dec)
        assert gst["split_accepted"] == ost.split_accepted
        rejected += ost.split_requests - ost.split_accepted
        assert_same_state(inst, orc, f"saturated frame {f}")
    assert rejected > 0


def test_we3_chain_example_on_gpu():
    mesh = we1_mesh(seed=1)
    inst = cbt.Instance(mesh, 6)
    orc = Oracle(mesh, 6)
    k = orc.k

    def step(hids, code):
        dec = decisions_for(orc, hids, code)
        g = inst.update_with_decisions(dec, stats=True)
        o = orc.frame(decisions=dec)
        assert_same_state(inst, orc, f"we3 {hids}")
        return g, o

    step([paper_j_to_heap(7, 0, k)], I.DEC_SPLIT)
    g, _ = step([paper_j_to_heap(14, 1, k)], I.DEC_SPLIT)
    assert g["allocations"] == 5
    g, _ = step([paper_j_to_heap(j, 2, k) for j in (28, 29, 46, 47)], I.DEC_MERGE)
    assert g["merges_executed"] == 1
    g, _ = step([paper_j_to_heap(j, 1, k) for j in (22, 23)], I.DEC_MERGE)
    assert g["merges_executed"] == 1
    assert_same_tree(inst, orc, "we3")


def test_frame_constants_match_reference():
    w = I.workload("cube")
    inst = cbt.Instance(w.mesh, w.depth, w.lod)
    orc = Oracle(w.mesh, w.depth, w.lod)
    for cam in w.cameras:
        g = inst.frame_constants(cam)
        o = orc.frame_constants(cam)
        assert np.array_equal(g.view(np.uint32), o.view(np.uint32))


def _lockstep(w, frames, label, check_vertices_every=0, tree_every=1):
    inst = cbt.Instance(w.mesh, w.depth, w.lod)
    orc = Oracle(w.mesh, w.depth, w.lod)
    for f, cam in enumerate(w.cameras[:frames]):
        log(f"[lockstep] {label} frame {f} L={orc.live_count}")
        gst = inst.update(cam, stats=True)
        ost = orc.frame(camera=cam)
        gdec = inst.decisions()
        odec = orc.decisions()[0]
        live_before = gdec != 255
        assert live_before.sum() == ost.live_before
        mism = np.nonzero(gdec[live_before] != odec[live_before])[0]
        assert mism.size == 0, f"{label} frame {f}: {mism.size} decisions differ"
        assert gst["allocations"] == ost.allocations and gst["live_after"] == ost.live_after
        assert_same_state(inst, orc, f"{label} frame {f}")
        if tree_every and f % tree_every == 0:
            assert_same_tree(inst, orc, f"{label} frame {f}")
        if check_vertices_every and f % check_vertices_every == 0:
            _vertices_match(inst, orc, f"{label} frame {f}")
    return inst, orc


def test_cube_workload_lockstep():
    w = I.workload("cube")
    inst, orc = _lockstep(w, 8, "cube", check_vertices_every=1)
    assert orc.live_count > 1000
    inst.close()


def test_planet_workload_lockstep_first_frames():
    w = I.workload("planet", frames=256, table_res=128)
    inst, orc = _lockstep(w, 40, "planet", check_vertices_every=13, tree_every=10)
    assert orc.live_count > 100000
    inst.close()


def test_terrain_full_depth_lockstep_first_frames():
    """Depth-24 pool (16M blocks), the launch configuration of the
    benchmark; lock-step with the reference while the reference is fast."""
    w = I.workload("terrain", frames=16, table_res=513)
    inst, orc = _lockstep(w, 12, "terrain", check_vertices_every=0, tree_every=6)
    ids, tw, nx, pv = inst.pool()
    heap = inst.query(tree=True)["tree"]
    check_properties(ids, tw, nx, pv, heap, orc.k, w.mesh.H, w.depth)
    inst.close()


def test_determinism_run_twice():
    w = I.workload("planet", frames=24, table_res=64)
    states = []
    for rep in range(2):
        inst = cbt.Instance(w.mesh, w.depth, w.lod)
        for cam in w.cameras:
            inst.update(cam)
        states.append([a.copy() for a in inst.pool()])
        inst.close()
    for a, b in zip(*states):
        assert np.array_equal(a, b)


def test_snapshot_restore_continues_identically():
    w = I.workload("cube")
    a = cbt.Instance(w.mesh, w.depth, w.lod)
    for cam in w.cameras[:5]:
        a.update(cam)
    snap = a.snapshot()
    b = cbt.Instance(w.mesh, w.depth, w.lod)
    b.restore(*snap)
    for cam in w.cameras[5:]:
        a.update(cam)
        b.update(cam)
    for x, y in zip(a.pool(), b.pool()):
        assert np.array_equal(x, y)
    a.close()
    b.close()


def test_restore_from_reference_state():
    """A state built by the reference (a valid input to the HIP path) and
    then advanced on both sides stays identical."""
    mesh = I.mesh_icosahedron()
    D = 12
    orc = Oracle(mesh, D)
    rng = np.random.default_rng(8)
    for f in range(6):
        orc.frame(decisions=I.random_decisions(orc.cap, int(rng.integers(1 << 30)), 0.4, 0.2))
    inst = cbt.Instance(mesh, D)
    inst.restore(*orc.pool())
    assert_same_state(inst, orc, "restored")
    assert_same_tree(inst, orc, "restored")
    for f in range(4):
        dec = I.random_decisions(orc.cap, int(rng.integers(1 << 30)), 0.3, 0.4)
        inst.update_with_decisions(dec)
        orc.frame(decisions=dec)
        assert_same_state(inst, orc, f"after restore frame {f}")
    inst.close()


@pytest.mark.parametrize("groups,levels", [(16, 5), (17, 6), (45, 8), (64, 7), (2048, 10)])
def test_schedule_does_not_change_results(groups, levels):
    """Launch schedules (rank workgroups, reduction levels per workgroup)
    change only how the work is cut: every schedule gives the reference's
    state, including ragged last chunks, many empty workgroups and odd
    workgroup counts (the LOD pass takes two rank chunks per workgroup, so
    its last workgroup then holds one)."""
    w = I.workload("planet", frames=256, table_res=64)
    inst = cbt.Instance(w.mesh, w.depth, w.lod)
    inst.set_schedule(groups, levels)
    assert inst.schedule() == (groups, levels)
    orc = Oracle(w.mesh, w.depth, w.lod)
    log(f"[schedule] groups={groups} levels={levels}")
    for f, cam in enumerate(w.cameras[:20]):
        inst.update(cam)
        orc.frame(camera=cam)
    assert_same_state(inst, orc, f"schedule {groups}/{levels}")
    assert_same_tree(inst, orc, f"schedule {groups}/{levels}")
    inst.close()


def test_live_records_roundtrip():
    """cbt_export_live gives the reference's live bisectors in ascending
    block order; importing them (from device or host memory) into fresh
    instances reproduces the state, and the update continues identically."""
    w = I.workload("planet", frames=24, table_res=64)
    a = cbt.Instance(w.mesh, w.depth, w.lod)
    orc = Oracle(w.mesh, w.depth, w.lod)
    for cam in w.cameras[:12]:
        a.update(cam)
        orc.frame(camera=cam)
    rec = a.export_live()
    r = rec.cpu().numpy().view(np.uint32)
    ids, tw, nx, pv = orc.pool()
    live = np.nonzero(ids)[0]
    assert r.shape == (live.size, 6)
    assert np.array_equal(r[:, 0], live)
    assert np.array_equal(r[:, 1].astype(np.uint64) | (r[:, 2].astype(np.uint64) << np.uint64(32)), ids[live])
    for col, ref in ((3, tw), (4, nx), (5, pv)):
        assert np.array_equal(r[:, col].view(np.int32), ref[live])
    b = cbt.Instance(w.mesh, w.depth, w.lod)
    b.import_live(rec)
    c = cbt.Instance(w.mesh, w.depth, w.lod)
    c.import_live(r.copy())
    for x in (b, c):
        assert_same_state(x, orc, "imported")
        assert_same_tree(x, orc, "imported")
    for f, cam in enumerate(w.cameras[12:24]):
        orc.frame(camera=cam)
        for x in (a, b, c):
            x.update(cam)
    for x in (a, b, c):
        assert_same_state(x, orc, "after import")
        x.close()


@pytest.mark.parametrize("name,D", [("we1", 4), ("open2", 3), ("open2", 4), ("pillow", 3), ("cube", 5)])
def test_small_pools_match_reference(name, D):
    """Pools of fewer than 32 blocks (one partial bitfield word, whose count
    is the tree root) down to D = ceil(log2 H): injected frames until the
    pool saturates, state, tree and canonical pairs against the reference."""
    mesh = {"we1": we1_mesh(4), "open2": I.mesh_two_triangles(False), "pillow": I.mesh_two_triangles(True),
            "cube": I.mesh_cube()}[name]
    inst = cbt.Instance(mesh, D)
    orc = Oracle(mesh, D)
    assert_same_state(inst, orc, f"{name} D={D} init")
    assert_same_tree(inst, orc, f"{name} D={D} init")
    rng = np.random.default_rng(zlib.crc32(f"{name}{D}".encode()))
    for f in range(10):
        dec = I.random_decisions(orc.cap, int(rng.integers(1 << 30)), [0.6, 0.2, 0.4][f % 3], [0.2, 0.7, 0.4][f % 3])
        log(f"[small] {name} D={D} frame {f} L={orc.live_count}")
        gst = inst.update_with_decisions(dec, stats=True)
        ost = orc.frame(decisions=dec)
        assert (gst["allocations"], gst["frees"], gst["live_after"]) == (ost.allocations, ost.frees, ost.live_after)
        assert_same_state(inst, orc, f"{name} D={D} frame {f}")
        assert_same_tree(inst, orc, f"{name} D={D} frame {f}")
    assert sorted(inst.canonical()) == orc.canonical()
    inst.close()


def test_canonical_pairs_match_reference():
    """cbt_query's root halfedge and subdivision code per bisector (the
    paper's b_j^d, computed by the library) against the reference's pool."""
    w = I.workload("planet", frames=256, table_res=64)
    inst = cbt.Instance(w.mesh, w.depth, w.lod)
    orc = Oracle(w.mesh, w.depth, w.lod)
    for cam in w.cameras[:30]:
        inst.update(cam)
        orc.frame(camera=cam)
    q = inst.query()
    ids = orc.pool()[0]
    live = np.nonzero(ids)[0]
    assert np.array_equal(q["slot"], live)
    k = orc.k
    for s_i, (x, h, c) in enumerate(zip(ids[live].tolist(), q["root_h"].tolist(), q["subdiv_id"].tolist())):
        d = x.bit_length() - 1 - k
        assert h == (x >> d) - (1 << k) and c == (1 << d) | (x & ((1 << d) - 1)), (s_i, x, h, c)
    assert inst.canonical() == orc.canonical()
    assert len(set(inst.canonical())) == live.size
    inst.close()


def test_new_world_parameters_between_frames():
    """A displacement amplitude that changes between frames: the cached world
    positions are rebuilt from the heap IDs the vertex records carry (the
    frames write no other copy), and the frames after it follow the
    reference, for a single instance and for a batch member."""
    import dataclasses
    w = I.workload("planet", frames=40, table_res=64)
    inst = cbt.Instance(w.mesh, w.depth, w.lod)
    member = cbt.Instance(w.mesh, w.depth, w.lod)
    batch = cbt.Batch([member], graph=False)
    orc = Oracle(w.mesh, w.depth, w.lod)
    steeper = dataclasses.replace(w.lod, amplitude=w.lod.amplitude * 4.0)
    for f, cam in enumerate(w.cameras[:24]):
        if f == 12:
            for x in (inst, member, orc):
                x.set_lod(steeper)
        log(f"[new world] frame {f} L={orc.live_count}")
        inst.update(cam)
        batch.update([cam])
        orc.frame(camera=cam)
        assert_same_state(inst, orc, f"frame {f}")
        if f in (12, 13, 23):
            _vertices_match(inst, orc, f"frame {f}")
            _vertices_match(member, orc, f"member, frame {f}")
            assert_same_state(member, orc, f"member, frame {f}")
    assert orc.live_count > 10000
    batch.close()
    inst.close()
    member.close()


def test_maximum_depth_pool_matches_reference():
    """The deepest pool the library accepts (D = 30: 2^30 blocks, a 120 GB
    workspace) against the reference at D = 20.  While the budget cuts
    nothing (checked on the reference every frame), a frame does not depend
    on the pool's size: the same decisions give the same owners, the same
    first free blocks (all below 2^20) and the same records, so the live
    records must agree exactly."""
    import torch
    mesh = I.mesh_grid(64)
    small, big = 20, 30
    need = cbt.workspace_bytes(mesh.H, big) + (1 << big) + (2 << 30)   # workspace, decisions, headroom
    if torch.cuda.mem_get_info()[0] < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory")
    orc = Oracle(mesh, small)
    inst = cbt.Instance(mesh, big)
    log(f"[max depth] D={big} workspace {inst.cap} blocks")
    dev = torch.zeros(1 << big, dtype=torch.uint8, device="cuda")
    rng = np.random.default_rng(30)
    for f in range(8):
        ps, pm = (0.3, 0.1) if f < 5 else (0.05, 0.85)
        dec = I.random_decisions(1 << small, int(rng.integers(1 << 30)), ps, pm)
        dev[: 1 << small].copy_(torch.from_numpy(dec))
        gst = inst.update_with_decisions(dev, stats=True)
        ost = orc.frame(decisions=dec)
        log(f"[max depth] frame {f} L={ost.live_before} -> {ost.live_after}")
        assert ost.split_accepted == ost.split_requests and ost.merge_accepted == ost.merge_configs
        for k in ("live_before", "split_requests", "split_accepted", "merge_configs", "merges_executed",
                  "allocations", "live_after"):
            assert gst[k] == getattr(ost, k), (f, k, gst[k], getattr(ost, k))
    assert orc.live_count > 200000
    assert inst.live_count() == orc.live_count
    r = inst.export_live().cpu().numpy().view(np.uint32)
    ids, tw, nx, pv = orc.pool()
    live = np.nonzero(ids)[0]
    assert np.array_equal(r[:, 0], live)
    assert np.array_equal(r[:, 1].astype(np.uint64) | (r[:, 2].astype(np.uint64) << np.uint64(32)), ids[live])
    for col, ref in ((3, tw), (4, nx), (5, pv)):
        assert np.array_equal(r[:, col].view(np.int32), ref[live])
    inst.close()
    del dev, inst
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", ["cube", "qsphere", "open2"])
def test_degenerate_frames_match_reference(name):
    """Frames that change nothing and the round trip: every block KEEP
    (no allocation, no free, the same pool), every block MERGE on the base
    mesh (roots never merge: the same pool), four frames of SPLIT everywhere,
    then MERGE everywhere until no merge executes, which returns the roots
    (Section 2.3).  The GPU matches the reference slot by slot after every
    frame."""
    mesh = {"cube": I.mesh_cube(), "qsphere": I.mesh_quad_sphere(2, 0.5, 9),
            "open2": I.mesh_two_triangles(False)}[name]
    D = 12
    inst = cbt.Instance(mesh, D)
    orc = Oracle(mesh, D)
    base = [a.copy() for a in inst.pool()]
    roots = sorted(int(x) for x in base[0] if x)
    for label, code in (("keep", 0), ("merge at the roots", 2)):
        gst = inst.update_with_decisions(np.full(inst.cap, code, np.uint8), stats=True)
        ost = orc.frame(decisions=np.full(orc.cap, code, np.uint8))
        assert gst["allocations"] == ost.allocations == 0 and gst["frees"] == 0, label
        for a, b in zip(inst.pool(), base):
            assert np.array_equal(a, b), label
        assert_same_state(inst, orc, label)
    for f in range(4):
        inst.update_with_decisions(np.ones(inst.cap, np.uint8))
        orc.frame(decisions=np.ones(orc.cap, np.uint8))
        assert_same_state(inst, orc, f"split {f}")
        assert_same_tree(inst, orc, f"split {f}")
    assert orc.live_count > 8 * mesh.H
    for f in range(40):
        gst = inst.update_with_decisions(np.full(inst.cap, 2, np.uint8), stats=True)
        ost = orc.frame(decisions=np.full(orc.cap, 2, np.uint8))
        assert gst["merges_executed"] == ost.merges_executed, f"merge {f}"
        assert_same_state(inst, orc, f"merge {f}")
        if ost.merges_executed == 0:
            break
    assert_same_tree(inst, orc, "after the round trip")
    assert sorted(int(x) for x in inst.pool()[0] if x) == roots
    assert inst.live_count() == mesh.H
    inst.close()
