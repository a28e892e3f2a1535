"""Pins of the reference's initialisation: the paper's halfedge table
(Section 2.1 figure), the root-bisector example b_7^0 (Section 2.2) and the
pool initialisation rules (Section 3.3)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import Oracle, OracleError
from paper_2407_02215_amd import inputs as I
from tests.helpers import F3, exact_decode_matrix, exact_root_triangles, read_golden, we1_mesh


def test_we1_roots_in_first_blocks():
    mesh = we1_mesh()
    o = Oracle(mesh, 6)
    k = 4  # ceil(log2 12)
    assert o.k == k
    ids, tw, nx, pv = o.pool()
    assert o.live_count == 12
    for h in range(12):
        assert ids[h] == (1 << k) + h
        assert tw[h] == mesh.twin[h] and nx[h] == mesh.next[h] and pv[h] == mesh.prev[h]
    assert not ids[12:].any()
    heap = o.heap()
    assert heap[1] == 12
    assert heap[64:76].tolist() == [1] * 12 and not heap[76:].any()
    o.check()


def test_we1_root7_example():
    g = read_golden("we1_halfedge_table.txt")
    want = dict(kv.split("=") for kv in g["root7_neighbours"].split())
    mesh = we1_mesh(seed=3)
    o = Oracle(mesh, 6)
    ids, tw, nx, pv = o.pool()
    assert (nx[7], pv[7], tw[7]) == (int(want["next"]), int(want["prev"]), int(want["twin"]))
    tri = o.root_triangle(7)
    assert tri[0].tobytes() == mesh.pos[1].tobytes()   # Vert(h7) = 1
    assert tri[1].tobytes() == mesh.pos[2].tobytes()   # Vert(h8) = 2
    face = [1, 2, 4, 5, 6]                              # vertices of h7's face
    mean = np.mean(mesh.pos[face].astype(np.float64), axis=0)
    assert np.allclose(tri[2], mean, rtol=0, atol=1e-6)


def test_root_centroid_shared_within_face():
    mesh = we1_mesh(seed=5)
    o = Oracle(mesh, 6)
    for f in range(3):
        hs = np.nonzero(mesh.face == f)[0]
        v2 = {o.root_triangle(int(h))[2].tobytes() for h in hs}
        assert len(v2) == 1


def test_depth_bounds():
    g = read_golden("we1_halfedge_table.txt")
    mesh = we1_mesh()
    dmin = int(g["min_depth"])
    with pytest.raises(OracleError):
        Oracle(mesh, dmin - 1)
    Oracle(mesh, dmin).check()


@pytest.mark.parametrize("bad", ["twin_not_involution", "next_prev", "digon", "vert_range"])
def test_invalid_meshes_rejected(bad):
    m = I.mesh_cube()
    tw, nx, pv, vt = m.twin.copy(), m.next.copy(), m.prev.copy(), m.vert.copy()
    if bad == "twin_not_involution":
        tw[0], tw[1] = tw[1], tw[0]
    elif bad == "next_prev":
        pv[0] = 5
    elif bad == "vert_range":
        vt[3] = 99
    elif bad == "digon":
        two = I.HalfedgeMesh(np.array([-1, -1, -1, -1], np.int32), np.array([1, 0, 3, 2], np.int32),
                             np.array([1, 0, 3, 2], np.int32), np.array([0, 1, 1, 0], np.int32),
                             np.zeros(4, np.int32), np.zeros(4, np.int32), np.zeros((2, 3), np.float32))
        with pytest.raises(OracleError):
            Oracle(two, 4)
        return
    bm = I.HalfedgeMesh(tw, nx, pv, vt, m.edge, m.face, m.pos)
    with pytest.raises(OracleError):
        Oracle(bm, 8)


def test_decode_matches_subdivision_matrix_exactly_on_dyadic_mesh():
    """Eq. 1 / Alg. 2: the reference's level-by-level decode equals the
    exact product of splitting matrices whenever all values are dyadic
    (cube: corners +-1, quad centroids on the axes)."""
    mesh = I.mesh_cube()
    o = Oracle(mesh, 10)
    k = o.k
    roots = exact_root_triangles(mesh)
    rng = np.random.default_rng(7)
    for _ in range(300):
        h = int(rng.integers(0, mesh.H))
        d = int(rng.integers(0, 40))
        path = int(rng.integers(0, 1 << d)) if d else 0
        hid = (1 << (k + d)) + (h << d) + path
        want = exact_decode_matrix(hid, k, roots)
        got = o.decode(hid)
        for i in range(3):
            assert tuple(Fraction(float(c)) for c in got[i]) == want[i], (hid, i)


def test_decode_close_to_exact_on_generic_mesh():
    """Non-dyadic positions: binary32 decode within its error bound of the
    exact subdivision-matrix vertices."""
    mesh = we1_mesh(seed=11)
    o = Oracle(mesh, 6)
    k = o.k
    roots = exact_root_triangles(mesh)
    rng = np.random.default_rng(8)
    for _ in range(200):
        h = int(rng.integers(0, mesh.H))
        d = int(rng.integers(0, 24))
        hid = (1 << (k + d)) + (h << d) + (int(rng.integers(0, 1 << d)) if d else 0)
        want = np.array([[float(c) for c in v] for v in exact_decode_matrix(hid, k, roots)])
        got = o.decode(hid).astype(np.float64)
        scale = np.max(np.abs(mesh.pos))
        assert np.max(np.abs(got - want)) <= 4e-7 * scale * (1 + d / 4)


def test_decode_of_created_bisector_matches_walk():
    """A bisector reached by splitting frame after frame decodes to the same
    vertices as the direct decode of its ID."""
    mesh = I.mesh_cube()
    o = Oracle(mesh, 10)
    k = o.k
    target = (1 << (k + 6)) + (5 << 6) + 0b101101
    for lvl in range(6):
        cur = target >> (6 - lvl)
        ids = o.pool()[0]
        s = int(np.nonzero(ids == np.uint64(cur))[0][0])
        dec = np.zeros(o.cap, np.uint8)
        dec[s] = 1
        o.frame(decisions=dec)
        o.check()
    ids = o.pool()[0]
    s = int(np.nonzero(ids == np.uint64(target))[0][0])
    assert o.vertices()[s].tobytes() == o.decode(target).tobytes()
