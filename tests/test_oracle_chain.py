"""Pins of the reference's refinement and decimation: the paper's
compatibility-chain example (Fig. 3, Section 2.3), the allocation count of
Section 3.3 and an exact textbook newest-vertex-bisection model."""
import numpy as np
import pytest

from oracle import Oracle
from paper_2407_02215_amd import inputs as I
from tests.helpers import (NVBModel, decisions_for, model_neighbour_ids, neighbour_ids, paper_j_to_heap,
                           read_golden, slot_of_id, we1_mesh)


def _parse_b(tok):
    j, d = tok[1:].split("^")
    return int(j), int(d)


def test_we3_compatibility_chain_and_merges():
    g = read_golden("we3_chain.txt")
    mesh = we1_mesh(seed=1)
    o = Oracle(mesh, 6)
    k = o.k
    hid = lambda tok: paper_j_to_heap(*_parse_b(tok), k)  # noqa: E731

    # b_14^1 exists once root 7 is split (its twin root 1 splits with it)
    st = o.frame(decisions=decisions_for(o, [hid("b7^0")], I.DEC_SPLIT))
    assert st.allocations == 4 and st.split_consumed == 2
    o.check()

    lhs, rhs = g["split"].split("->")
    outs, consumed = rhs.split("consumed")
    before = set(int(x) for x in o.pool()[0] if x)
    st = o.frame(decisions=decisions_for(o, [hid(lhs.split()[0])], I.DEC_SPLIT))
    o.check()
    after = set(int(x) for x in o.pool()[0] if x)
    want_new = {hid(t) for t in outs.split()}
    want_gone = {hid(t) for t in consumed.split()}
    assert after - before == want_new
    assert before - after == want_gone
    assert st.allocations == len(want_new) == 5
    d14 = 1
    assert st.allocations <= 3 * d14 + 4            # maxAllocation bound, Section 3.3
    # pointer consequences of Table 1 + Alg. 5 derived by hand for this case
    nb = neighbour_ids(o)
    assert nb[hid("b29^2")][1] == hid("b46^2")      # Next(b_29) borders b_46
    assert nb[hid("b46^2")][2] == hid("b29^2")
    assert nb[hid("b22^1")][2] is None              # b_11 was a border root

    lhs, rhs = g["merge4"].split("->")
    st = o.frame(decisions=decisions_for(o, [hid(t) for t in lhs.split()], I.DEC_MERGE))
    o.check()
    assert st.merges_executed == 1 and st.allocations == 2 and st.frees == 4
    ids = set(int(x) for x in o.pool()[0] if x)
    assert {hid(t) for t in rhs.split()} <= ids
    assert not ({hid(t) for t in lhs.split()} & ids)

    lhs, rhs = g["merge2"].split("->")
    st = o.frame(decisions=decisions_for(o, [hid(t) for t in lhs.split()], I.DEC_MERGE))
    o.check()
    assert st.merges_executed == 1 and st.allocations == 1
    ids = set(int(x) for x in o.pool()[0] if x)
    assert hid(rhs.split()[0]) in ids
    # back to the state after the first frame
    assert len(ids) == 14


def _state_copy(mesh, D, o):
    c = Oracle(mesh, D)
    c.set_pool(*o.pool())
    return c


def _model_from(o, mesh):
    m = NVBModel(mesh, o.k)
    ids = sorted(int(x) for x in o.pool()[0] if x)
    # rebuild the model's leaves by refining the roots along the live IDs
    want = set(ids)
    changed = True
    while changed:
        changed = False
        for x in list(m.tri):
            if x not in want:
                m.bisect(x)
                changed = True
    assert set(m.tri) == want
    return m


@pytest.mark.parametrize("closed", [False, True])
def test_single_refinements_match_textbook_nvb(closed):
    """Exhaustive split sequences on the two-triangle meshes: after splitting
    any one bisector, the reference's bisector set and every neighbour
    pointer equal the exact geometric newest-vertex-bisection model."""
    mesh = I.mesh_two_triangles(closed)
    D = 10
    start = Oracle(mesh, D)
    frontier = [start]
    seen = set()
    visited = 0
    for level in range(3):
        nxt = []
        for o in frontier:
            ids = [int(x) for x in o.pool()[0] if x]
            for x in ids:
                c = _state_copy(mesh, D, o)
                model = _model_from(c, mesh)
                c.frame(decisions=decisions_for(c, [x], I.DEC_SPLIT))
                c.check()
                model.refine(x)
                got = set(int(y) for y in c.pool()[0] if y)
                assert got == set(model.tri), (level, x)
                assert neighbour_ids(c) == model_neighbour_ids(model), (level, x)
                key = tuple(sorted(got))
                visited += 1
                if key not in seen:
                    seen.add(key)
                    nxt.append(c)
        frontier = nxt[:40]
    assert visited > 50


@pytest.mark.parametrize("seed", range(4))
def test_multi_initiator_frames_match_sequential_nvb(seed):
    """Several initiators in one frame give the same triangulation as
    refining them one after the other (in any order) in the exact model."""
    mesh = we1_mesh(seed=seed)
    D = 9
    o = Oracle(mesh, D)
    rng = np.random.default_rng(seed)
    for frame in range(4):
        ids = [int(x) for x in o.pool()[0] if x]
        pick = [x for x in ids if rng.random() < 0.3]
        model = _model_from(o, mesh)
        o.frame(decisions=decisions_for(o, pick, I.DEC_SPLIT))
        o.check()
        for x in reversed(pick):
            if x in model.tri:
                model.refine(x)
        assert set(int(y) for y in o.pool()[0] if y) == set(model.tri)
        assert neighbour_ids(o) == model_neighbour_ids(model)


@pytest.mark.parametrize("seed", range(3))
def test_merges_match_geometric_configurations(seed):
    """Alg. 4: with every leaf voting to merge, exactly the configurations
    found from geometry alone (a refinement-edge midpoint surrounded by the
    children of one border parent, or of two parents sharing that edge)
    are merged, and pointers match the exact model."""
    mesh = I.mesh_two_triangles(seed % 2 == 1) if seed < 2 else we1_mesh(seed)
    D = 10
    o = Oracle(mesh, D)
    rng = np.random.default_rng(50 + seed)
    for frame in range(5):
        ids = [int(x) for x in o.pool()[0] if x]
        o.frame(decisions=decisions_for(o, [x for x in ids if rng.random() < 0.5], I.DEC_SPLIT))
    o.check()
    for rnd in range(6):
        model = _model_from(o, mesh)
        configs = model.mergeable_parents()
        ids = [int(x) for x in o.pool()[0] if x]
        st = o.frame(decisions=decisions_for(o, ids, I.DEC_MERGE))
        o.check()
        for p in sorted(set(configs)):
            if p in configs and all(c in model.tri for c in configs[p]):
                grp = configs[p]
                parents = sorted({c >> 1 for c in grp})
                for q in parents:
                    model.merge(q)
        assert set(int(y) for y in o.pool()[0] if y) == set(model.tri), rnd
        assert neighbour_ids(o) == model_neighbour_ids(model)
        assert st.merges_executed == len({tuple(sorted(v)) for v in configs.values()})


def test_confluence_over_initiator_orders():
    """The frame result does not depend on the order in which the literal
    recursive refinement visits the initiators (every order also agrees with
    the closure of split marks, which the reference checks internally)."""
    mesh = I.mesh_cube()
    D = 10
    base = Oracle(mesh, D)
    rng = np.random.default_rng(3)
    for frame in range(3):
        ids = [int(x) for x in base.pool()[0] if x]
        base.frame(decisions=decisions_for(base, [x for x in ids if rng.random() < 0.4], I.DEC_SPLIT))
    ids = [int(x) for x in base.pool()[0] if x]
    pick = [x for x in ids if rng.random() < 0.5]
    results = set()
    for seed in range(25):
        c = _state_copy(mesh, D, base)
        c.set_initiator_shuffle(seed)
        c.frame(decisions=decisions_for(c, pick, I.DEC_SPLIT))
        c.check()
        ids2, tw, nx, pv = c.pool()
        results.add((ids2.tobytes(), tw.tobytes(), nx.tobytes(), pv.tobytes()))
    assert len(results) == 1


def test_small_chain_all_orders():
    """Forty seeded orders of four initiators give one result."""
    mesh = I.mesh_two_triangles(True)
    D = 8
    base = Oracle(mesh, D)
    base.frame(decisions=np.ones(base.cap, np.uint8))
    ids = [int(x) for x in base.pool()[0] if x]
    pick = ids[:4]
    results = set()
    for seed in range(40):
        c = _state_copy(mesh, D, base)
        c.set_initiator_shuffle(seed + 1)
        c.frame(decisions=decisions_for(c, pick, I.DEC_SPLIT))
        results.add(c.pool()[0].tobytes())
    assert len(results) == 1
