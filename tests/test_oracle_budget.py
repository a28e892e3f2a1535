"""Brute-force pins of the reference's memory budget and slot policy
(Section 3.3 kernels 4-5, Alg. 8-9, and the readings of the reservation
rule the paper leaves open).

Each frame's expected result is rebuilt here without the reference's frame
code: merge configurations come from geometry (the exact newest-vertex
bisection model of tests/helpers.py: refinement-edge midpoints with two or
four incident leaves), splits from the textbook recursive refinement of
that model, free blocks from a plain scan of the pre-frame bitfield.  The
rules restated on those independent inputs:

  * a merge configuration is unanimous when every member decided MERGE; its
    reservation (one block per parent: 1 for a border pair, 2 for a cycle
    of four) is charged at its smallest-ID member's rank, and accepted when
    the inclusive rank-order prefix of unanimous reservations is within
    F = 2^D - L;
  * a SPLIT of depth d reserves 3d + 4 blocks; it is accepted when the
    total of ALL unanimous merge reservations (accepted or not) plus the
    inclusive rank-order prefix of split reservations is within F;
  * accepted splits run first; an accepted merge executes unless one of its
    members was consumed by a split;
  * the new blocks are the first N zero bits of the pre-frame bitfield,
    taken in rank order of their owners (a split bisector, or the smallest
    member of an executed merge), each owner's outputs in ascending heap ID.

Random states and decisions on small meshes at pool sizes where the budget
binds (including F < 2, which starves cycles of four)."""
import zlib

import numpy as np
import pytest

from oracle import Oracle
from paper_2407_02215_amd import inputs as I
from tests.helpers import NVBModel, exact_decode_matrix, exact_root_triangles, we1_mesh


def _model_of(ids_live, mesh, k):
    roots = exact_root_triangles(mesh, lift=True)
    m = NVBModel.__new__(NVBModel)
    m.k = k
    m.tri = {int(x): exact_decode_matrix(int(x), k, roots) for x in ids_live}
    m._index()
    return m


def _depth(x, k):
    return int(x).bit_length() - 1 - k


def expected_frame(ids_pre, dec, mesh, k, D):
    """The frame's result from the rules above: (ids per slot, pointer ids
    per slot, counters)."""
    cap = 1 << D
    live = np.nonzero(ids_pre)[0]                  # rank order = ascending slot
    L = live.size
    F = cap - L
    rank_of = {int(ids_pre[s]): r for r, s in enumerate(live.tolist())}
    slot_of = {int(ids_pre[s]): int(s) for s in live.tolist()}
    ids = [int(ids_pre[s]) for s in live.tolist()]
    eff = {}
    for x in ids:
        d = int(dec[slot_of[x]])
        if d == I.DEC_MERGE and _depth(x, k) == 0:
            d = I.DEC_KEEP                              # roots never merge
        eff[x] = d
    model = _model_of(ids, mesh, k)
    cfgs = {tuple(sorted(v)) for v in model.mergeable_parents().values()}
    unan = sorted((c for c in cfgs if all(eff[x] == I.DEC_MERGE for x in c)), key=lambda c: rank_of[min(c)])
    Tm = sum(len(c) // 2 for c in unan)
    acc_m, run = [], 0
    for c in unan:
        run += len(c) // 2
        if run <= F:
            acc_m.append(c)
    acc_s, run = [], 0
    for x in ids:                                       # rank order
        if eff[x] == I.DEC_SPLIT:
            run += 3 * _depth(x, k) + 4
            if Tm + run <= F:
                acc_s.append(x)
    for x in acc_s:                                     # splits first, in rank order
        if x in model.tri:
            model.refine(x)
    split_consumed = [x for x in ids if x not in model.tri]
    consumed = set(split_consumed)
    executed = [c for c in acc_m if not any(x in consumed for x in c)]
    for c in executed:
        for p in sorted({x >> 1 for x in c}):
            model.merge(p)
        consumed.update(c)
    exec_min = {min(c): c for c in executed}
    outputs = []                                        # owners in rank order
    for x in ids:
        if x in consumed and x in split_consumed:
            sh = lambda y: y >> (int(y).bit_length() - int(x).bit_length())   # noqa: E731
            outputs += sorted(y for y in model.tri if y > x and sh(y) == x)
        elif x in exec_min:
            outputs += sorted({y >> 1 for y in exec_min[x]})
    free = np.nonzero(ids_pre == 0)[0][:len(outputs)]
    assert free.size == len(outputs) <= F
    post = ids_pre.copy()
    for x in consumed:
        post[slot_of[x]] = 0
    new_slot = {}
    for y, s in zip(outputs, free.tolist()):
        post[s] = y
        new_slot[y] = s
    # pointers: neighbours in the final model, as heap IDs per slot
    nb = {}
    for y in model.tri:
        s = new_slot.get(y, slot_of.get(y))
        nb[s] = tuple(model.neighbour(y, e) for e in range(3))
    stats = dict(live_before=L, free_before=F,
                 split_requests=sum(1 for x in ids if eff[x] == I.DEC_SPLIT),
                 split_accepted=len(acc_s),
                 merge_requests=sum(1 for x in ids if eff[x] == I.DEC_MERGE),
                 merge_configs=len(unan), merge_accepted=len(acc_m), merges_executed=len(executed),
                 split_consumed=len(split_consumed), allocations=len(outputs), frees=len(consumed),
                 live_after=L + len(outputs) - len(consumed))
    return post, nb, stats


CASES = {
    # mesh, depth (slots just above the roots, so the budget binds), frames
    "we1": (lambda: we1_mesh(3), 6, 14),
    "open2": (lambda: I.mesh_two_triangles(False), 5, 14),
    "pillow": (lambda: I.mesh_two_triangles(True), 5, 14),
    "cube": (lambda: I.mesh_cube(), 7, 12),
    "ico": (lambda: I.mesh_icosahedron(), 8, 10),
}


@pytest.mark.parametrize("name", list(CASES))
def test_budget_and_slots_against_brute_force(name):
    make, D, frames = CASES[name]
    mesh = make()
    o = Oracle(mesh, D)
    k = o.k
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    seen = {"merge_rejected": 0, "split_rejected": 0, "executed": 0, "vetoed": 0, "quad": 0}
    for f in range(frames):
        p_split, p_merge = [(0.3, 0.5), (0.6, 0.3), (0.15, 0.8), (0.5, 0.5)][f % 4]
        dec = I.random_decisions(o.cap, int(rng.integers(1 << 30)), p_split, p_merge)
        ids_pre = o.pool()[0]
        post, nb, want = expected_frame(ids_pre, dec, mesh, k, D)
        st = o.frame(decisions=dec)
        for key, v in want.items():
            assert getattr(st, key) == v, f"{name} frame {f}: {key} ref={getattr(st, key)} brute={v}"
        ids, tw, nx, pv = o.pool()
        assert np.array_equal(ids, post), f"{name} frame {f}: slot assignment differs"
        for s, (t, n, p) in nb.items():
            got = tuple(None if q < 0 else int(ids[q]) for q in (tw[s], nx[s], pv[s]))
            assert got == (t, n, p), f"{name} frame {f}: pointers of slot {s}"
        seen["merge_rejected"] += want["merge_configs"] - want["merge_accepted"]
        seen["split_rejected"] += want["split_requests"] - want["split_accepted"]
        seen["executed"] += want["merges_executed"]
        seen["vetoed"] += want["merge_accepted"] - want["merges_executed"]
    # the frames exercised every branch of the rules
    assert seen["split_rejected"] > 0 and seen["executed"] > 0, seen


def test_budget_merge_cut_on_saturated_pools():
    """Pools filled by splits until no split fits any more (F below the
    smallest 3d + 4), then merge-heavy frames: the unanimous reservations
    exceed F, so the merge cut itself rejects configurations; mixed frames
    after that let splits veto accepted merges."""
    tot = {"merge_rejected": 0, "vetoed": 0, "executed": 0}
    for name, (make, D, _) in CASES.items():
        mesh = make()
        o = Oracle(mesh, D)
        rng = np.random.default_rng(zlib.crc32(("sat-" + name).encode()))
        for f in range(40):
            st = o.frame(decisions=I.random_decisions(o.cap, int(rng.integers(1 << 30)), 0.9, 0.0))
            if st.split_accepted == 0:
                break
        for f in range(6):
            p_split, p_merge = [(0.0, 0.97), (0.3, 0.65), (0.02, 0.95)][f % 3]
            dec = I.random_decisions(o.cap, int(rng.integers(1 << 30)), p_split, p_merge)
            ids_pre = o.pool()[0]
            post, _, want = expected_frame(ids_pre, dec, mesh, o.k, D)
            st = o.frame(decisions=dec)
            for key, v in want.items():
                assert getattr(st, key) == v, f"{name} saturated frame {f}: {key} ref={getattr(st, key)} brute={v}"
            assert np.array_equal(o.pool()[0], post), f"{name} saturated frame {f}: slots differ"
            tot["merge_rejected"] += want["merge_configs"] - want["merge_accepted"]
            tot["vetoed"] += want["merge_accepted"] - want["merges_executed"]
            tot["executed"] += want["merges_executed"]
    assert tot["merge_rejected"] > 0 and tot["vetoed"] > 0 and tot["executed"] > 0, tot
