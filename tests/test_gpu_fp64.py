"""Binary64 instances (CBT_INIT_FP64; the paper evaluates planet vertices in
double precision, Section 4.2) against the reference's binary64 path: the
decoded vertices, the decisions and the pool state bit for bit, at the
planet's deep levels where binary32 and binary64 part ways."""
import numpy as np
import pytest
import torch  # noqa: F401

from oracle import Oracle
from paper_2407_02215_amd import cbt
from paper_2407_02215_amd import inputs as I
from tests.gpu_checks import assert_same_state, assert_same_tree, log
from tests.helpers import we1_mesh

pytestmark = pytest.mark.gpu


def _meshes():
    return {
        "we1": (we1_mesh(4), 8),
        "cube": (I.mesh_cube(), 10),
        "ico": (I.mesh_icosahedron(), 10),
        "qsphere": (I.mesh_quad_sphere(3, 0.5, 11), 12),
        "grid64": (I.mesh_grid(64), 16),
    }


def _vertices64_match(inst, orc, label):
    q = inst.query(vertices64=True)
    ref = orc.vertices64()[q["slot"]]
    got = q["vertices64"]
    bad = np.nonzero((got.view(np.uint64) != ref.view(np.uint64)).any(axis=1))[0]
    assert bad.size == 0, f"{label}: {bad.size} bisectors' binary64 vertices differ, first {bad[:4].tolist()}"


@pytest.mark.parametrize("name", list(_meshes()))
def test_fp64_init_and_injected_frames(name):
    mesh, D = _meshes()[name]
    inst = cbt.Instance(mesh, D, precision=64)
    orc = Oracle(mesh, D, precision=64)
    assert_same_state(inst, orc, f"{name} init")
    _vertices64_match(inst, orc, f"{name} init")
    rng = np.random.default_rng(31 + len(name))
    for f in range(8):
        dec = I.random_decisions(orc.cap, int(rng.integers(1 << 30)), [0.5, 0.2, 0.05, 0.3][f % 4],
                                 [0.1, 0.5, 0.8, 0.3][f % 4])
        log(f"[fp64 injected] {name} frame {f} L={orc.live_count}")
        gst = inst.update_with_decisions(dec, stats=True)
        ost = orc.frame(decisions=dec)
        assert gst["live_after"] == ost.live_after and gst["allocations"] == ost.allocations
        assert_same_state(inst, orc, f"{name} frame {f}")
    assert_same_tree(inst, orc, name)
    _vertices64_match(inst, orc, name)
    # the binary32 view of a binary64 instance is its binary64 decode rounded
    q = inst.query(vertices=True, vertices64=True)
    assert np.array_equal(q["vertices"], q["vertices64"].astype(np.float32))
    inst.close()


def test_fp64_planet_lockstep_first_frames():
    w = I.workload("planet", frames=256, table_res=64)
    inst = cbt.Instance(w.mesh, w.depth, w.lod, precision=64)
    orc = Oracle(w.mesh, w.depth, w.lod, precision=64)
    for f, cam in enumerate(w.cameras[:24]):
        log(f"[fp64 lockstep] planet frame {f} L={orc.live_count}")
        gst = inst.update(cam, stats=True)
        ost = orc.frame(camera=cam)
        gdec = inst.decisions()
        odec = orc.decisions()[0]
        was_live = gdec != 255
        assert was_live.sum() == ost.live_before
        assert np.array_equal(gdec[was_live], odec[was_live]), f"fp64 planet frame {f}: decisions differ"
        assert gst["live_after"] == ost.live_after
        assert_same_state(inst, orc, f"fp64 planet frame {f}")
    assert_same_tree(inst, orc, "fp64 planet")
    _vertices64_match(inst, orc, "fp64 planet")
    inst.close()


@pytest.mark.parametrize("criterion", [I.CRIT_EDGE, I.CRIT_AREA])
def test_fp64_deep_planet_descent(criterion):
    """The last camera of the descent (about 1e-5 radii above the ground):
    60 passes of the multi-pass mode from the base mesh reach some forty
    levels below the roots.  Binary64 instance and binary64 reference agree
    bit for bit (state, tree, vertices, exported triangles); the binary32
    instance ends elsewhere."""
    import dataclasses
    w = I.workload("planet", frames=256, table_res=64)
    lod = w.lod if criterion == I.CRIT_EDGE else dataclasses.replace(w.lod, split_px=49.0, merge_px=12.25,
                                                                     criterion=I.CRIT_AREA)
    D = 19
    cam = w.cameras[255]
    inst = cbt.Instance(w.mesh, D, lod, precision=64)
    orc = Oracle(w.mesh, D, lod, precision=64)
    passes, _ = inst.update_converge(cam, max_passes=60)
    ref_passes = 0
    for _ in range(60):
        st = orc.frame(camera=cam)
        ref_passes += 1
        if st.allocations == 0 and st.frees == 0:
            break
    log(f"[fp64 descent crit={criterion}] {passes} passes, live {inst.live_count()}")
    assert passes == ref_passes
    assert_same_state(inst, orc, "fp64 descent")
    assert_same_tree(inst, orc, "fp64 descent")
    _vertices64_match(inst, orc, "fp64 descent")
    ids = orc.pool()[0]
    live = np.nonzero(ids)[0]
    depth = max(int(x).bit_length() - 1 - orc.k for x in ids[live].tolist())
    assert depth >= 35
    # exported triangles: the reference's binary64 world positions, rounded
    # once to binary32, on a sample of the live bisectors
    tri = inst.export_triangles().cpu().numpy()
    assert tri.shape[0] == live.size
    v64 = orc.vertices64()
    rng = np.random.default_rng(2)
    for r in rng.choice(live.size, size=min(3000, live.size), replace=False).tolist():
        ref = np.stack([orc.world_position64(v64[live[r]][3 * i:3 * i + 3]) for i in range(3)]).astype(np.float32)
        assert np.array_equal(tri[r].view(np.uint32), ref.view(np.uint32)), f"triangle {r}"
    # the binary32 instance, same camera and passes, ends in another state
    inst32 = cbt.Instance(w.mesh, D, lod)
    inst32.update_converge(cam, max_passes=60)
    a = inst.pool()[0]
    b = inst32.pool()[0]
    assert not np.array_equal(a, b)
    inst32.close()
    inst.close()


@pytest.mark.parametrize("persistent", [False, True])
def test_fp64_batch_matches_single_instances(persistent):
    ws = I.batched_workloads(4, frames=10, seed=21, h_range=(24, 800), d_range=(12, 14), table_res=64)
    alone = [cbt.Instance(w.mesh, w.depth, w.lod, precision=64) for w in ws]
    members = [cbt.Instance(w.mesh, w.depth, w.lod, precision=64) for w in ws]
    log(f"[fp64 batch persistent={persistent}]")
    batch = cbt.Batch(members, graph=True, persistent=persistent)
    for f in range(len(ws[0].cameras)):
        for a, w in zip(alone, ws):
            a.update(w.cameras[f])
        batch.update([w.cameras[f] for w in ws])
    batch.synchronize()
    torch.cuda.synchronize()
    for i, (a, m) in enumerate(zip(alone, members)):
        for name, x, y in zip(("heap_id", "twin", "next", "prev"), a.pool(), m.pool()):
            assert np.array_equal(x, y), f"member {i} {name}"
        qa = a.query(vertices64=True)
        qm = m.query(vertices64=True)
        assert np.array_equal(qa["vertices64"].view(np.uint64), qm["vertices64"].view(np.uint64))
    batch.close()
    # one batch holds one precision
    mixed = [alone[0], cbt.Instance(ws[1].mesh, ws[1].depth, ws[1].lod)]
    with pytest.raises(cbt.CbtError):
        cbt.Batch(mixed, graph=False)
    for x in alone + members + mixed[1:]:
        x.close()
