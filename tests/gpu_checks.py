"""Comparison and property checks used by the GPU tests.

``assert_same_state`` compares the HIP path's pool with the CPU reference
slot by slot.  ``check_properties`` verifies, with vectorised numpy written
independently of the reference, the structural properties any valid state
has at any size: the tree is the sum reduction of the bitfield, neighbour
pointers are mutual with one of the allowed edge pairings, and the live
bisectors of every root form a complete prefix code (exact area).
"""
from __future__ import annotations

import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _diff(name, a, b, k=5):
    bad = np.nonzero(a != b)[0]
    return f"{name}: {bad.size} mismatches, first slots {bad[:k].tolist()} gpu={a[bad[:k]].tolist()} ref={b[bad[:k]].tolist()}"


def assert_same_state(inst, orc, label=""):
    gi, gt, gn, gp = inst.pool()
    oi, ot, on, op = orc.pool()
    errs = []
    for name, a, b in (("heap_id", gi, oi), ("twin", gt, ot), ("next", gn, on), ("prev", gp, op)):
        if not np.array_equal(a, b):
            errs.append(_diff(name, a, b))
    assert not errs, f"{label}: " + "; ".join(errs)


def assert_same_tree(inst, orc, label=""):
    g = inst.query(tree=True)["tree"]
    o = orc.heap()
    assert np.array_equal(g, o), f"{label}: " + _diff("tree", g, o)


def _depth(ids, k):
    # floor(log2(id)) - k for uint64 ids > 0
    x = ids.astype(np.uint64)
    d = np.zeros(x.shape, np.int64)
    for sh in (32, 16, 8, 4, 2, 1):
        big = x >= (np.uint64(1) << np.uint64(sh))
        d[big] += sh
        x = np.where(big, x >> np.uint64(sh), x)
    return d - k


def check_properties(ids, tw, nx, pv, heap, k, H, D):
    cap = 1 << D
    live = ids != 0
    L = int(live.sum())
    assert heap[1] == L
    assert np.array_equal(heap[cap:], live.astype(np.uint32))
    inner = np.arange(1, cap)
    assert np.array_equal(heap[inner], heap[2 * inner] + heap[2 * inner + 1])
    s = np.nonzero(live)[0]
    d = _depth(ids[s], k)
    depth = np.full(cap, -1, np.int64)
    depth[s] = d
    ptr = [tw, nx, pv]
    for e in range(3):
        p = ptr[e][s]
        has = p >= 0
        src, dst = s[has], p[has]
        assert (dst < cap).all() and live[dst].all(), f"edge {e}: pointer to a free block"
        back = [(ptr[f][dst] == src) for f in range(3)]
        cnt = back[0].astype(int) + back[1] + back[2]
        assert (cnt == 1).all(), f"edge {e}: {(cnt != 1).sum()} pointers not mutual"
        f = np.argmax(np.stack(back), axis=0)
        ds, dd = depth[src], depth[dst]
        if e == 0:
            ok = ((f == 0) & (ds == dd)) | ((f != 0) & (ds == dd + 1))
        else:
            ok = ((f == 3 - e) & (ds == dd)) | ((f == 0) & (dd == ds + 1))
        assert ok.all(), f"edge {e}: {(~ok).sum()} pointer pairs of an invalid type"
    # complete prefix code per root: sum of 2^(61-d) is 2^61, no live ancestor
    h = (ids[s] >> d.astype(np.uint64)).astype(np.int64) - (1 << k)
    assert ((h >= 0) & (h < H)).all()
    w = np.left_shift(np.uint64(1), (61 - d).astype(np.uint64))
    tot = np.zeros(H, np.uint64)
    np.add.at(tot, h, w)
    assert (tot == np.uint64(1) << np.uint64(61)).all(), "bisectors do not tile every root exactly"
    srt = np.sort(ids[s])
    assert (np.diff(srt) > 0).all(), "duplicate bisector"
    anc = ids[s].copy()
    for lvl in range(1, int(d.max()) + 1 if d.size else 1):
        anc = anc >> np.uint64(1)
        valid = d >= lvl
        pos = np.searchsorted(srt, anc[valid])
        pos = np.minimum(pos, srt.size - 1)
        assert not (srt[pos] == anc[valid]).any(), "a bisector and its ancestor are both live"
    return L
