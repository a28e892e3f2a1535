"""Shared test helpers: golden-fixture parsing and an exact-arithmetic
geometric model of newest-vertex bisection used to pin the CPU reference.

The geometric model is written independently of the reference: it works on
explicit triangles with rational (Fraction) vertices, finds neighbours by
matching edge endpoints, and refines with the textbook recursive
newest-vertex-bisection procedure (the reference's Alg. 3 works on stored
neighbour pointers instead).
"""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np

from paper_2407_02215_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name: str) -> dict:
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(" ")
            out[key] = rest.strip()
    return out


def we1_mesh(seed: int = 0) -> I.HalfedgeMesh:
    g = read_golden("we1_halfedge_table.txt")
    arr = {k: np.array([int(x) for x in g[k].split()], np.int32) for k in ("twin", "next", "prev", "vert", "edge", "face")}
    V = int(arr["vert"].max()) + 1
    pos = np.random.default_rng(seed).normal(size=(V, 3)).astype(np.float32)
    return I.HalfedgeMesh(arr["twin"], arr["next"], arr["prev"], arr["vert"], arr["edge"], arr["face"], pos)


def paper_j_to_heap(j: int, d: int, k: int) -> int:
    """b_j^d of the paper -> heap ID 2^(k+d) + j."""
    return (1 << (k + d)) + j


# --------------------------------------------------------------------------
# exact geometric model
# --------------------------------------------------------------------------

def F3(p):
    return tuple(Fraction(float(c)) for c in p)


def mid(a, b):
    return tuple((x + y) / 2 for x, y in zip(a, b))


def exact_root_triangles(mesh, lift: bool = False):
    """Root bisector of halfedge h: (Vert(h), Vert(Next(h)), mean of the
    face's vertices), exact.  With lift=True every face's mean is moved off
    the surface by a face-dependent amount, so that faces glued along all
    their edges (a pillow) still have distinct interior vertices; newest
    vertex bisection is combinatorial, so the lift changes no adjacency."""
    out = []
    face_of = {}
    for h in range(mesh.H):
        ring = [h]
        g = int(mesh.next[h])
        while g != h:
            ring.append(g)
            g = int(mesh.next[g])
        pts = [F3(mesh.pos[mesh.vert[x]]) for x in ring]
        c = tuple(sum(p[i] for p in pts) / len(pts) for i in range(3))
        if lift:
            # an offset in all three coordinates with coprime denominators,
            # so that no lifted mean lands on a point of another face
            f = face_of.setdefault(min(ring), len(face_of) + 1)
            c = (c[0] + Fraction(f, 101), c[1] + Fraction(2 * f, 103), c[2] + Fraction(3 * f, 107))
        out.append((F3(mesh.pos[mesh.vert[h]]), F3(mesh.pos[mesh.vert[mesh.next[h]]]), c))
    return out


M0 = ((1, 0, 0), (0, 0, 1), (Fraction(1, 2), Fraction(1, 2), 0))
M1 = ((0, 0, 1), (0, 1, 0), (Fraction(1, 2), Fraction(1, 2), 0))


def matmul3(A, B):
    return tuple(tuple(sum(A[i][k] * B[k][j] for k in range(3)) for j in range(3)) for i in range(3))


def exact_decode_matrix(hid: int, k: int, roots):
    """Vertices of a bisector from its subdivision matrix, exactly as a
    product of splitting matrices taken from the least significant path bit
    upwards, applied to the root triangle."""
    d = hid.bit_length() - 1 - k
    h = (hid >> d) - (1 << k)
    M = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
    x = hid
    for _ in range(d):
        M = matmul3(M, M1 if (x & 1) else M0)
        x >>= 1
    V = roots[h]
    return tuple(tuple(sum(M[i][j] * V[j][c] for j in range(3)) for c in range(3)) for i in range(3))


def _edges(tri):
    a, b, c = tri
    return [(a, b), (b, c), (c, a)]  # Twin, Next, Prev edges


class NVBModel:
    """Triangulation of exact triangles keyed by heap ID; the refinement edge
    of triangle (a, b, c) is (a, b) and its newest vertex is c."""

    def __init__(self, mesh, k):
        self.k = k
        self.tri = {}
        for h, t in enumerate(exact_root_triangles(mesh, lift=True)):
            self.tri[(1 << k) + h] = t
        self._index()

    def _index(self):
        self.edge_map = {}
        for x, t in self.tri.items():
            for e in _edges(t):
                self.edge_map.setdefault(frozenset(e), set()).add(x)

    def neighbour(self, x, e_index):
        e = frozenset(_edges(self.tri[x])[e_index])
        others = self.edge_map.get(e, set()) - {x}
        assert len(others) <= 1
        return next(iter(others)) if others else None

    def bisect(self, x):
        a, b, c = self.tri.pop(x)
        m = mid(a, b)
        self.tri[2 * x] = (a, c, m)
        self.tri[2 * x + 1] = (c, b, m)
        self._index()

    def refine(self, x, guard=0):
        """Textbook recursive newest-vertex bisection of triangle x."""
        assert guard < 200
        n = self.neighbour(x, 0)
        if n is None:
            self.bisect(x)
            return
        if frozenset(_edges(self.tri[n])[0]) != frozenset(_edges(self.tri[x])[0]):
            self.refine(n, guard + 1)
            n = self.neighbour(x, 0)
            assert n is not None and frozenset(_edges(self.tri[n])[0]) == frozenset(_edges(self.tri[x])[0])
        self.bisect(x)
        self.bisect(n)

    def mergeable_parents(self):
        """Parents whose children may be merged, from geometry alone: the
        midpoint m of the parent's refinement edge has exactly the parent's
        two children around it (border), or exactly four leaves that are the
        children of two triangles sharing that refinement edge."""
        fan = {}
        for x, t in self.tri.items():
            for v in t:
                fan.setdefault(v, []).append(x)
        out = {}
        for x in self.tri:
            if (x >> 1).bit_length() - 1 < self.k:
                continue  # roots have no parent
            p = x >> 1
            if p in out:
                continue
            if (x ^ 1) not in self.tri:
                continue
            a, _, m = self.tri[2 * p]
            _, b, _ = self.tri[2 * p + 1]
            around = fan.get(m, [])
            if sorted(around) == sorted([2 * p, 2 * p + 1]):
                out[p] = (2 * p, 2 * p + 1)
            elif len(around) == 4:
                rest = [y for y in around if y not in (2 * p, 2 * p + 1)]
                if len(rest) == 2 and rest[0] ^ 1 == rest[1]:
                    q = rest[0] >> 1
                    if q not in out and frozenset(_edges(self.parent_tri(q))[0]) == frozenset((a, b)):
                        out[p] = (2 * p, 2 * p + 1, 2 * q, 2 * q + 1)
                        out[q] = out[p]
        return out

    def parent_tri(self, q):
        a, c, _ = self.tri[2 * q]
        _, b, _ = self.tri[2 * q + 1]
        return (a, b, c)

    def merge(self, p):
        t = self.parent_tri(p)
        del self.tri[2 * p]
        del self.tri[2 * p + 1]
        self.tri[p] = t
        self._index()


def pool_ids(oracle_obj):
    ids, tw, nx, pv = oracle_obj.pool()
    return ids, tw, nx, pv


def neighbour_ids(oracle_obj):
    """{heap id: (twin id, next id, prev id)} with None for border."""
    ids, tw, nx, pv = oracle_obj.pool()
    out = {}
    for s in np.nonzero(ids)[0].tolist():
        def nid(p):
            return None if p < 0 else int(ids[p])
        out[int(ids[s])] = (nid(int(tw[s])), nid(int(nx[s])), nid(int(pv[s])))
    return out


def model_neighbour_ids(model: NVBModel):
    return {x: tuple(model.neighbour(x, e) for e in range(3)) for x in model.tri}


def slot_of_id(oracle_obj, hid):
    ids = oracle_obj.pool()[0]
    w = np.nonzero(ids == np.uint64(hid))[0]
    assert w.size == 1, hid
    return int(w[0])


def decisions_for(oracle_obj, heap_ids, code):
    dec = np.zeros(oracle_obj.cap, np.uint8)
    for x in heap_ids:
        dec[slot_of_id(oracle_obj, x)] = code
    return dec


def triangle_area64(v):
    a = v[0:3].astype(np.float64)
    b = v[3:6].astype(np.float64)
    c = v[6:9].astype(np.float64)
    return 0.5 * np.linalg.norm(np.cross(b - a, c - a))
