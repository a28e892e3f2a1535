"""Whole-frame properties of the reference: structural invariants after every
frame, exact area, split-all/merge-all round trip, the memory budget and the
root rule (Section 3.3; Section 2.3)."""
import zlib

import numpy as np
import pytest

from oracle import Oracle
from paper_2407_02215_amd import inputs as I
from tests.helpers import decisions_for, neighbour_ids, triangle_area64, we1_mesh


def _meshes():
    return {
        "we1": we1_mesh(2),
        "cube": I.mesh_cube(),
        "ico": I.mesh_icosahedron(),
        "grid4": I.mesh_grid(4),
        "pillow": I.mesh_two_triangles(True),
        "open2": I.mesh_two_triangles(False),
        "qsphere": I.mesh_quad_sphere(2, 0.5, 9),
    }


def _area(o):
    ids = o.pool()[0]
    v = o.vertices()
    return sum(triangle_area64(v[s]) for s in np.nonzero(ids)[0])


@pytest.mark.parametrize("name", list(_meshes()))
def test_invariants_under_random_decisions(name):
    mesh = _meshes()[name]
    D = max(10, I.depth_for(mesh.H, 10))
    o = Oracle(mesh, D)
    a0 = _area(o)
    rng = np.random.default_rng(zlib.crc32(name.encode()) % 1000)
    for f in range(12):
        p_split = 0.35 if f < 6 else 0.1
        dec = I.random_decisions(o.cap, int(rng.integers(1 << 30)), p_split, 0.5)
        st = o.frame(decisions=dec)
        o.check()
        assert st.allocations <= st.free_before
        assert st.live_after == st.live_before + st.allocations - st.frees
        assert st.live_after == o.live_count == o.heap()[1]
        assert abs(_area(o) - a0) <= 1e-6 * a0


@pytest.mark.parametrize("name", ["we1", "cube", "open2", "pillow"])
def test_split_all_then_merge_all_round_trip(name):
    mesh = _meshes()[name]
    o = Oracle(mesh, 12)
    roots = sorted(int(x) for x in o.pool()[0] if x)
    for f in range(4):
        o.frame(decisions=np.ones(o.cap, np.uint8))
        o.check()
    assert o.live_count > 8 * mesh.H
    for f in range(40):
        st = o.frame(decisions=np.full(o.cap, 2, np.uint8))
        o.check()
        if st.merges_executed == 0:
            break
    assert sorted(int(x) for x in o.pool()[0] if x) == roots
    assert o.heap()[1] == mesh.H
    # the roots may sit in other blocks now; compare neighbours by ID
    base = 1 << o.k
    nb = neighbour_ids(o)
    for h in range(mesh.H):
        t, n, p = (int(a[h]) for a in (mesh.twin, mesh.next, mesh.prev))
        assert nb[base + h] == (None if t < 0 else base + t, base + n, base + p)


def test_roots_never_merge():
    """Alg. 4 has no parent for a root: with every bisector requesting a
    merge, the root triangulation is unchanged (including roots whose
    indices 2i, 2i+1 are Next-adjacent, as in every quad of the cube)."""
    mesh = I.mesh_cube()
    o = Oracle(mesh, 8)
    before = [a.copy() for a in o.pool()]
    st = o.frame(decisions=np.full(o.cap, 2, np.uint8))
    assert st.merge_requests == 0 and st.merges_executed == 0 and st.allocations == 0
    for a, b in zip(before, o.pool()):
        assert (a == b).all()


def test_budget_saturation():
    """At a nearly full pool the reservations are cut in rank order: merges
    first, then splits of 3d+4 blocks each; no frame allocates more blocks
    than are free and the pool never overflows."""
    mesh = I.mesh_cube()     # 24 roots
    D = 7                    # 128 blocks
    o = Oracle(mesh, D)
    rng = np.random.default_rng(4)
    saw_reject = False
    for f in range(30):
        dec = I.random_decisions(o.cap, int(rng.integers(1 << 30)), 0.6, 0.3)
        st = o.frame(decisions=dec)
        o.check()
        assert st.allocations <= st.free_before
        assert st.live_after <= o.cap
        if st.split_accepted < st.split_requests:
            saw_reject = True
    assert saw_reject


def test_budget_prefix_rule_against_brute_force():
    """Accepted splits are exactly the rank-order prefix of split requests
    whose cumulative 3d+4 cost (after all merge reservations) fits in F."""
    mesh = I.mesh_cube()
    o = Oracle(mesh, 7)
    rng = np.random.default_rng(5)
    for f in range(3):
        o.frame(decisions=I.random_decisions(o.cap, int(rng.integers(1 << 30)), 0.5, 0.0))
    ids = o.pool()[0]
    live = np.nonzero(ids)[0]
    F = o.cap - live.size
    dec = np.zeros(o.cap, np.uint8)
    dec[live] = I.DEC_SPLIT   # no merges -> no merge reservations
    costs = [3 * (int(ids[s]).bit_length() - 1 - o.k) + 4 for s in live]
    want = int(np.searchsorted(np.cumsum(costs), F, side="right"))
    st = o.frame(decisions=dec)
    assert st.split_accepted == want
    o.check()


def test_depth_limit_of_64bit_ids():
    """No bisector is split past the 64-bit index width (d + 1 <= 63 - k)."""
    mesh = I.mesh_two_triangles(False)   # k = 3 -> depth limit 60
    o = Oracle(mesh, 12)
    for f in range(70):
        st = o.frame(decisions=decisions_for(o, [max(int(x) for x in o.pool()[0] if x)], I.DEC_SPLIT))
    o.check()
    assert st.max_depth == 63 - o.k


@pytest.mark.slow
def test_cube_workload_frames():
    w = I.workload("cube")
    o = Oracle(w.mesh, w.depth, w.lod)
    for cam in w.cameras:
        st = o.frame(camera=cam)
        o.check()
    assert st.live_after > 1000


def test_property_checker_accepts_reference_states_and_rejects_corruption():
    """The vectorised property checker used on GPU outputs accepts valid
    states and rejects planted mistakes (on CPU arrays)."""
    from tests.gpu_checks import check_properties
    mesh = I.mesh_icosahedron()
    o = Oracle(mesh, 12)
    rng = np.random.default_rng(12)
    for f in range(8):
        o.frame(decisions=I.random_decisions(o.cap, int(rng.integers(1 << 30)), 0.4, 0.3))
    ids, tw, nx, pv = o.pool()
    heap = o.heap()
    check_properties(ids, tw, nx, pv, heap, o.k, mesh.H, o.D)
    s = np.nonzero(ids)[0]
    bad = [ids.copy(), tw.copy(), nx.copy(), pv.copy(), heap.copy()]
    bad[1][s[3]] = nx[s[3]]                 # a wrong twin pointer
    with pytest.raises(AssertionError):
        check_properties(*bad, o.k, mesh.H, o.D)
    bad = [ids.copy(), tw, nx, pv, heap]
    bad[0][s[5]] = ids[s[5]] * 2            # a bisector replaced by its child
    with pytest.raises(AssertionError):
        check_properties(*bad, o.k, mesh.H, o.D)
    h2 = heap.copy()
    h2[3] += 1
    with pytest.raises(AssertionError):
        check_properties(ids, tw, nx, pv, h2, o.k, mesh.H, o.D)
