"""Pins of the reference's binary64 variant (the paper evaluates planet
vertex positions in double precision, Section 4.2): the Alg. 2 decode
against the exact product of splitting matrices, world positions against
closed forms, the size test against a float64 projection, and the reason
for the variant -- at planet scale the binary32 decode collapses
vertices, the binary64 one does not."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import Oracle
from paper_2407_02215_amd import inputs as I
from tests.helpers import exact_decode_matrix, exact_root_triangles, we1_mesh


def test_decode64_exact_on_dyadic_mesh_deep():
    """Cube (dyadic positions): the binary64 decode equals the exact
    splitting-matrix product down to depth 48."""
    mesh = I.mesh_cube()
    o = Oracle(mesh, 10, precision=64)
    k = o.k
    roots = exact_root_triangles(mesh)
    rng = np.random.default_rng(17)
    for _ in range(300):
        h = int(rng.integers(0, mesh.H))
        d = int(rng.integers(0, 49))
        path = int(rng.integers(0, 1 << d)) if d else 0
        hid = (1 << (k + d)) + (h << d) + path
        want = exact_decode_matrix(hid, k, roots)
        got = o.decode64(hid)
        for i in range(3):
            assert tuple(Fraction(c) for c in got[i].tolist()) == want[i], (hid, i)


def test_decode64_close_to_exact_on_generic_mesh():
    mesh = we1_mesh(seed=11)
    o = Oracle(mesh, 6, precision=64)
    k = o.k
    roots = exact_root_triangles(mesh)
    rng = np.random.default_rng(18)
    scale = float(np.max(np.abs(mesh.pos)))
    for _ in range(200):
        h = int(rng.integers(0, mesh.H))
        d = int(rng.integers(0, 50))
        hid = (1 << (k + d)) + (h << d) + (int(rng.integers(0, 1 << d)) if d else 0)
        want = [[float(c) for c in v] for v in exact_decode_matrix(hid, k, roots)]
        got = o.decode64(hid)
        # the root centroid is rounded once in binary64, then every level
        # adds at most half an ulp
        assert np.max(np.abs(got - np.array(want))) <= 2e-15 * scale * (1 + d), (hid, d)


def test_world_position64_closed_forms():
    m = I.mesh_icosahedron()
    c, amp = 0.625, 0.125
    table = np.full((6, 16, 16), c, np.float32)
    o = Oracle(m, 8, I.LodParams(I.MODE_SPHERE, 4.0, 2.0, table, amp), precision=64)
    rng = np.random.default_rng(3)
    for _ in range(50):
        v = rng.normal(size=3)
        p = o.world_position64(v)
        n = v / np.linalg.norm(v)
        assert np.allclose(p, n * (1 + amp * c), rtol=0, atol=1e-15)
    res = 65
    t = np.arange(res, dtype=np.float64)
    jj, ii = np.meshgrid(t, t, indexing="ij")
    grid = (0.003 * ii - 0.002 * jj + 0.1).astype(np.float32)
    o = Oracle(I.mesh_grid(2), 8, I.LodParams(I.MODE_HEIGHTFIELD, 2.0, 1.0, grid, 0.5), precision=64)
    for _ in range(100):
        v = np.array([rng.random(), rng.random(), 0.25])
        # bilinear interpolation of the float32 texels, in binary64
        s, tt = v[0] * (res - 1), v[1] * (res - 1)
        i0, j0 = min(int(s), res - 2), min(int(tt), res - 2)
        fx, fy = s - i0, tt - j0
        T = grid.astype(np.float64)
        a, b, cc, e = T[j0, i0], T[j0, i0 + 1], T[j0 + 1, i0], T[j0 + 1, i0 + 1]
        h = (a + fx * (b - a)) + fy * ((cc + fx * (e - cc)) - (a + fx * (b - a)))
        p = o.world_position64(v)
        assert p[0] == v[0] and p[1] == v[1]
        assert abs(p[2] - (0.25 + 0.5 * h)) < 1e-15


def _flat_mesh_in_front(seed, z0=2.0):
    m = I.mesh_grid(3)
    rng = np.random.default_rng(seed)
    pos = m.pos.astype(np.float64).copy()
    pos = (pos - 0.5) * 2.0
    pos[:, 2] = z0 + 0.3 * rng.random(pos.shape[0])
    m.pos = pos.astype(np.float32)
    return m


@pytest.mark.parametrize("criterion", [I.CRIT_EDGE, I.CRIT_AREA])
def test_decisions64_match_float64_projection(criterion):
    """The binary64 size test agrees with the float64 pinhole projection
    (explicit division) everywhere outside a 1e-9 relative band."""
    m = _flat_mesh_in_front(4)
    lod = I.LodParams(I.MODE_FLAT, 30.0, 12.0, criterion=criterion)
    o = Oracle(m, 12, lod, precision=64)
    for _ in range(4):
        o.frame(decisions=np.ones(o.cap, np.uint8))
    cam = I.Camera(np.array((0.1, -0.2, -0.5), np.float32), np.array((0.1, 0.05, 1.0), np.float32),
                   np.array((0.0, 1.0, 0.1), np.float32), math.radians(70.0), 640, 480, 0.05)
    # exact double frame: the camera inputs are binary32 values
    c = cam.pos.astype(np.float64)
    fw = cam.fwd.astype(np.float64) / np.linalg.norm(cam.fwd.astype(np.float64))
    r = np.cross(fw, cam.up.astype(np.float64))
    r /= np.linalg.norm(r)
    up = np.cross(r, fw)
    th = math.tan(0.5 * float(np.float32(cam.fovy)))
    f = 0.5 * cam.height / th
    ids = o.pool()[0]
    live = np.nonzero(ids)[0]
    verts = o.vertices64()
    sizes = []
    proj = {}
    for s in live:
        q = verts[s].reshape(3, 3) - c
        x, y, z = q @ r, q @ up, q @ fw
        proj[s] = (x, y, z)
        if (z > cam.znear).all():
            sx, sy = f * x / z, f * y / z
            if criterion == I.CRIT_AREA:
                sizes.append(0.5 * abs((sx[1] - sx[0]) * (sy[2] - sy[0]) - (sx[2] - sx[0]) * (sy[1] - sy[0])))
            else:
                sizes.append(math.hypot(sx[1] - sx[0], sy[1] - sy[0]))
    split, merge = float(np.float32(np.quantile(sizes, 0.7))), float(np.float32(np.quantile(sizes, 0.3)))
    o.set_lod(I.LodParams(I.MODE_FLAT, split, merge, criterion=criterion))
    o.frame(camera=cam)
    dec = o.decisions()[0]
    tanx, tany = th * cam.width / cam.height, th
    kinds, checked = set(), 0
    for s in live:
        x, y, z = proj[s]
        culled = any(cond.all() for cond in (z < cam.znear, x > tanx * z, x < -tanx * z, y > tany * z,
                                              y < -tany * z))
        if culled:
            want = I.DEC_MERGE
        elif (z[:2] < cam.znear).any() or (criterion == I.CRIT_AREA and (z < cam.znear).any()):
            want = I.DEC_SPLIT
        else:
            sx, sy = f * x / z, f * y / z
            if criterion == I.CRIT_AREA:
                size = 0.5 * abs((sx[1] - sx[0]) * (sy[2] - sy[0]) - (sx[2] - sx[0]) * (sy[1] - sy[0]))
            else:
                size = math.hypot(sx[1] - sx[0], sy[1] - sy[0])
            if min(abs(size - split) / split, abs(size - merge) / merge) < 1e-9:
                continue
            want = I.DEC_SPLIT if size > split else (I.DEC_MERGE if size < merge else I.DEC_KEEP)
        assert dec[s] == want, (s, dec[s], want)
        kinds.add(want)
        checked += 1
    assert checked > 0.99 * live.size
    assert kinds == {I.DEC_SPLIT, I.DEC_MERGE, I.DEC_KEEP}


def test_binary64_keeps_planet_scale_triangles_apart():
    """Near the surface of a unit planet (the last frames of the descent,
    1e-5 radius altitude), 4-pixel edges are about 4e-8 radii long, which a
    bisector reaches about 50 levels deep -- below the binary32 spacing at
    radius 1 (6e-8): the binary32 decode collapses vertices (zero-length
    edges), the binary64 decode of the same IDs does not."""
    w = I.workload("planet", frames=256, table_res=64)
    o = Oracle(w.mesh, 16, w.lod, precision=64)
    rng = np.random.default_rng(5)
    k = o.k
    collapsed32 = collapsed64 = 0
    for _ in range(200):
        h = int(rng.integers(0, w.mesh.H))
        d = 52
        hid = (1 << (k + d)) + (h << d) + int(rng.integers(0, 1 << d))
        v32 = o.decode(hid).astype(np.float64)
        v64 = o.decode64(hid)
        collapsed32 += int(np.all(v32[0] == v32[1]) or np.all(v32[0] == v32[2]) or np.all(v32[1] == v32[2]))
        collapsed64 += int(np.all(v64[0] == v64[1]) or np.all(v64[0] == v64[2]) or np.all(v64[1] == v64[2]))
    assert collapsed32 > 100
    assert collapsed64 == 0
