"""Pins of the reference's LOD step: frame constants, world positions
(sphere projection with cube-map displacement, height-map displacement,
Section 4.1) and the screen-space decision against a float64 projection."""
import math

import numpy as np
import pytest

from oracle import Oracle
from paper_2407_02215_amd import inputs as I


def _flat_mesh_in_front(seed, z0=2.0):
    """A small open mesh (a 3x3 grid) placed in front of a camera at the
    origin that looks along +z."""
    m = I.mesh_grid(3)
    rng = np.random.default_rng(seed)
    pos = m.pos.astype(np.float64).copy()
    pos = (pos - 0.5) * 2.0
    pos[:, 2] = z0 + 0.3 * rng.random(pos.shape[0])
    m.pos = pos.astype(np.float32)
    return m


def _cam(fovy_deg=60.0, w=800, h=600, znear=0.05, pos=(0, 0, 0), fwd=(0, 0, 1), up=(0, 1, 0)):
    return I.Camera(np.array(pos, np.float32), np.array(fwd, np.float32), np.array(up, np.float32),
                    math.radians(fovy_deg), w, h, znear)


def test_frame_constants_closed_form():
    m = _flat_mesh_in_front(0)
    o = Oracle(m, 8, I.LodParams(I.MODE_FLAT, 6.0, 3.0))
    cam = _cam(90.0, 1000, 500, 0.25)
    K = o.frame_constants(cam)
    assert K[0:3].tolist() == [0, 0, 0]
    assert K[3:6].tolist() == [-1, 0, 0]           # right = fwd x up
    assert K[6:9].tolist() == [0, 1, 0]
    assert K[9:12].tolist() == [0, 0, 1]
    assert abs(K[12] / 250.0 ** 2 - 1) < 1e-6         # (h/2 / tan(45deg))^2
    assert K[13] == 36.0 and K[14] == 9.0
    assert abs(K[15] - 2.0) < 1e-6 and abs(K[16] - 1.0) < 1e-6
    assert K[17] == np.float32(0.25)


def _decide64(p, K, split_px, merge_px, tanx, tany, znear, f):
    """Decision from a float64 pinhole projection of the base edge."""
    q = p - K[0:3].astype(np.float64)
    x = q @ K[3:6].astype(np.float64)
    y = q @ K[6:9].astype(np.float64)
    z = q @ K[9:12].astype(np.float64)
    for cond in (z < znear, x > tanx * z, x < -tanx * z, y > tany * z, y < -tany * z):
        if cond.all():
            return I.DEC_MERGE, None
    if z[0] < znear or z[1] < znear:
        return I.DEC_SPLIT, None
    sx = f * x[:2] / z[:2]
    sy = f * y[:2] / z[:2]
    L = math.hypot(sx[1] - sx[0], sy[1] - sy[0])
    margin = min(abs(L - split_px) / split_px, abs(L - merge_px) / merge_px)
    if L > split_px:
        return I.DEC_SPLIT, margin
    if L < merge_px:
        return I.DEC_MERGE, margin
    return I.DEC_KEEP, margin


@pytest.mark.parametrize("seed", range(3))
def test_decisions_match_float64_projection(seed):
    m = _flat_mesh_in_front(seed)
    split_px, merge_px = 30.0, 12.0
    o = Oracle(m, 12, I.LodParams(I.MODE_FLAT, split_px, merge_px))
    for _ in range(4):   # depth >= 2 everywhere: no root overrides
        o.frame(decisions=np.ones(o.cap, np.uint8))
    cam = _cam(70.0, 640, 480, 0.05, pos=(0.1, -0.2, -0.5), fwd=(0.1, 0.05, 1.0), up=(0.0, 1.0, 0.1))
    K = o.frame_constants(cam)
    ids = o.pool()[0]
    verts = o.vertices()
    live = np.nonzero(ids)[0]
    th = math.tan(0.5 * cam.fovy)
    f = 0.5 * cam.height / th
    # thresholds at quantiles of the projected base-edge lengths, so that all
    # three decisions occur
    lens = []
    for s in live:
        v = verts[s].reshape(3, 3).astype(np.float64)
        q = v - K[0:3].astype(np.float64)
        x, y, z = q @ K[3:6].astype(np.float64), q @ K[6:9].astype(np.float64), q @ K[9:12].astype(np.float64)
        if z[0] > cam.znear and z[1] > cam.znear:
            lens.append(math.hypot(f * (x[1] / z[1] - x[0] / z[0]), f * (y[1] / z[1] - y[0] / z[0])))
    split_px, merge_px = float(np.quantile(lens, 0.7)), float(np.quantile(lens, 0.3))
    o.set_lod(I.LodParams(I.MODE_FLAT, split_px, merge_px))
    o.frame(camera=cam)
    dec = o.decisions()[0]
    split_px, merge_px = float(np.float32(split_px)), float(np.float32(merge_px))
    n_checked = 0
    kinds = set()
    for s in live:
        v = verts[s].reshape(3, 3).astype(np.float64)
        want, margin = _decide64(v, K, split_px, merge_px, th * cam.width / cam.height, th, cam.znear, f)
        if margin is not None and margin < 1e-4:
            continue
        assert dec[s] == want, (s, dec[s], want)
        kinds.add(want)
        n_checked += 1
    assert n_checked > 0.9 * live.size
    assert kinds == {I.DEC_SPLIT, I.DEC_MERGE, I.DEC_KEEP}


def test_culled_bisectors_merge():
    m = _flat_mesh_in_front(1)
    o = Oracle(m, 10, I.LodParams(I.MODE_FLAT, 1e6, 0.0))   # nothing splits by size
    for _ in range(3):
        o.frame(decisions=np.ones(o.cap, np.uint8))
    cam = _cam(30.0, 100, 100, 0.05, pos=(0, 0, 0), fwd=(1, 0, 0.3), up=(0, 1, 0))
    o.frame(camera=cam)
    dec = o.decisions()[0]
    ids = o.pool()[0]
    # looking mostly sideways: most of the mesh is outside the frustum
    assert (dec[np.nonzero(ids)[0]] == I.DEC_MERGE).sum() > 0


def test_sphere_projection_constant_table():
    m = I.mesh_icosahedron()
    c = 0.625
    table = np.full((6, 16, 16), c, np.float32)
    amp = 0.125
    o = Oracle(m, 8, I.LodParams(I.MODE_SPHERE, 4.0, 2.0, table, amp))
    rng = np.random.default_rng(0)
    for _ in range(50):
        v = rng.normal(size=3).astype(np.float32) * 0.7
        p = o.world_position(v)
        n = v.astype(np.float64) / np.linalg.norm(v.astype(np.float64))
        assert np.allclose(p, n * (1 + amp * c), rtol=0, atol=3e-7)


def _linear_cubemap(res, a, b, e):
    t = np.arange(res, dtype=np.float64)
    jj, ii = np.meshgrid(t, t, indexing="ij")
    face = np.arange(6)[:, None, None]
    return (a * ii[None] + b * jj[None] + e * face).astype(np.float32)


def test_sphere_bilinear_reproduces_linear_table():
    res = 33
    a, b, e = 0.01, 0.02, 0.5
    table = _linear_cubemap(res, a, b, e)
    amp = 0.25
    o = Oracle(I.mesh_icosahedron(), 8, I.LodParams(I.MODE_SPHERE, 4.0, 2.0, table, amp))
    rng = np.random.default_rng(1)
    for _ in range(200):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        v = (n * 0.8).astype(np.float32)
        nn = v.astype(np.float64) / np.linalg.norm(v.astype(np.float64))
        ax = np.abs(nn)
        if ax[0] >= ax[1] and ax[0] >= ax[2]:
            f, u, w = (0 if nn[0] >= 0 else 1), nn[1] / ax[0], nn[2] / ax[0]
        elif ax[1] >= ax[2]:
            f, u, w = (2 if nn[1] >= 0 else 3), nn[0] / ax[1], nn[2] / ax[1]
        else:
            f, u, w = (4 if nn[2] >= 0 else 5), nn[0] / ax[2], nn[1] / ax[2]
        h = a * (u + 1) * 0.5 * (res - 1) + b * (w + 1) * 0.5 * (res - 1) + e * f
        p = o.world_position(v)
        assert np.allclose(p, nn * (1 + amp * h), rtol=0, atol=2e-6)


def test_heightfield_bilinear_reproduces_linear_table():
    res = 65
    t = np.arange(res, dtype=np.float64)
    jj, ii = np.meshgrid(t, t, indexing="ij")
    table = (0.003 * ii - 0.002 * jj + 0.1).astype(np.float32)
    amp = 0.5
    o = Oracle(I.mesh_grid(2), 8, I.LodParams(I.MODE_HEIGHTFIELD, 2.0, 1.0, table, amp))
    rng = np.random.default_rng(2)
    for _ in range(200):
        v = np.array([rng.random(), rng.random(), 0.25], np.float32)
        x, y = float(v[0]), float(v[1])
        h = 0.003 * x * (res - 1) - 0.002 * y * (res - 1) + 0.1
        p = o.world_position(v)
        assert p[0] == v[0] and p[1] == v[1]
        assert abs(p[2] - (0.25 + amp * h)) < 2e-6


def _area_decide64(p, K, split_a, merge_a, tanx, tany, znear, f):
    """Decision from the float64 shoelace area of the pinhole-projected
    triangle (explicit division by depth)."""
    q = p - K[0:3].astype(np.float64)
    x = q @ K[3:6].astype(np.float64)
    y = q @ K[6:9].astype(np.float64)
    z = q @ K[9:12].astype(np.float64)
    for cond in (z < znear, x > tanx * z, x < -tanx * z, y > tany * z, y < -tany * z):
        if cond.all():
            return I.DEC_MERGE, None
    if (z < znear).any():
        return I.DEC_SPLIT, None
    sx, sy = f * x / z, f * y / z
    area = 0.5 * abs((sx[1] - sx[0]) * (sy[2] - sy[0]) - (sx[2] - sx[0]) * (sy[1] - sy[0]))
    margin = min(abs(area - split_a) / split_a, abs(area - merge_a) / merge_a)
    if area > split_a:
        return I.DEC_SPLIT, margin
    if area < merge_a:
        return I.DEC_MERGE, margin
    return I.DEC_KEEP, margin


@pytest.mark.parametrize("seed", range(3))
def test_area_decisions_match_float64_projection(seed):
    """The projected-area criterion (the paper's screen-space area target):
    the division-free binary32 test agrees with the area of the projected
    triangle computed in float64 outside a 1e-4 relative band."""
    m = _flat_mesh_in_front(seed)
    o = Oracle(m, 12, I.LodParams(I.MODE_FLAT, 400.0, 100.0, criterion=I.CRIT_AREA))
    for _ in range(4):
        o.frame(decisions=np.ones(o.cap, np.uint8))
    cam = _cam(70.0, 640, 480, 0.05, pos=(0.1, -0.2, -0.5), fwd=(0.1, 0.05, 1.0), up=(0.0, 1.0, 0.1))
    K = o.frame_constants(cam)
    ids = o.pool()[0]
    verts = o.vertices()
    live = np.nonzero(ids)[0]
    th = math.tan(0.5 * cam.fovy)
    f = 0.5 * cam.height / th
    areas = []
    for s in live:
        v = verts[s].reshape(3, 3).astype(np.float64)
        q = v - K[0:3].astype(np.float64)
        x, y, z = q @ K[3:6].astype(np.float64), q @ K[6:9].astype(np.float64), q @ K[9:12].astype(np.float64)
        if (z > cam.znear).all():
            sx, sy = f * x / z, f * y / z
            areas.append(0.5 * abs((sx[1] - sx[0]) * (sy[2] - sy[0]) - (sx[2] - sx[0]) * (sy[1] - sy[0])))
    split_a, merge_a = float(np.quantile(areas, 0.7)), float(np.quantile(areas, 0.3))
    o.set_lod(I.LodParams(I.MODE_FLAT, split_a, merge_a, criterion=I.CRIT_AREA))
    K2 = o.frame_constants(cam)
    assert K2[13] == np.float32(2.0 * split_a) and K2[14] == np.float32(2.0 * merge_a)
    o.frame(camera=cam)
    dec = o.decisions()[0]
    split_a, merge_a = float(np.float32(split_a)), float(np.float32(merge_a))
    n_checked = 0
    kinds = set()
    for s in live:
        v = verts[s].reshape(3, 3).astype(np.float64)
        want, margin = _area_decide64(v, K, split_a, merge_a, th * cam.width / cam.height, th, cam.znear, f)
        if margin is not None and margin < 1e-4:
            continue
        assert dec[s] == want, (s, dec[s], want)
        kinds.add(want)
        n_checked += 1
    assert n_checked > 0.9 * live.size
    assert kinds == {I.DEC_SPLIT, I.DEC_MERGE, I.DEC_KEEP}


def test_area_criterion_closed_form():
    """A triangle facing the camera at depth z with legs a, b has projected
    area f^2 a b / (2 z^2); each of its three root bisectors (fanned around
    the face centroid, Alg. 1) covers a third of it.  Just below and above a
    threshold set from that closed form the root splits or keeps."""
    pos = np.array([[0.0, 0.0, 2.0], [0.3, 0.0, 2.0], [0.0, 0.2, 2.0]], np.float32)
    m = I.halfedge_from_faces([[0, 1, 2]], pos)
    cam = _cam(60.0, 800, 600, 0.05, pos=(0.05, 0.05, 0.0), fwd=(0, 0, 1), up=(0, 1, 0))
    f = 0.5 * 600 / math.tan(math.radians(30.0))
    area = f * f * 0.3 * 0.2 / (2 * 2.0 * 2.0) / 3.0
    for thr, want in ((area * 0.999, I.DEC_SPLIT), (area * 1.001, I.DEC_KEEP)):
        o = Oracle(m, 4, I.LodParams(I.MODE_FLAT, thr, thr / 4, criterion=I.CRIT_AREA))
        o.frame(camera=cam)
        dec, A, Bs, _ = o.decisions()
        # root 0 sits in block 0 (roots never merge; a split is not overridden)
        assert dec[0] == want
        assert abs(float(A[0]) / (2.0 * area * float(Bs[0]) / (2.0 * np.float32(thr))) - 1.0) < 1e-5


def _distance_decide64(p, cam_pos, split_px, merge_px, f):
    """Cull-free distance-only decision in float64: the base edge's length
    over its midpoint's distance, in pixels (f e / r)."""
    e = np.linalg.norm(p[1] - p[0])
    r = np.linalg.norm(0.5 * (p[0] + p[1]) - cam_pos)
    px = f * e / r
    margin = min(abs(px - split_px) / split_px, abs(px - merge_px) / merge_px)
    if px > split_px:
        return I.DEC_SPLIT, margin
    if px < merge_px:
        return I.DEC_MERGE, margin
    return I.DEC_KEEP, margin


def test_distance_criterion_closed_form():
    """Base edge of length e whose midpoint is at distance r from the camera
    subtends f e / r pixels whatever the view direction: with the camera
    looking away from the mesh (every vertex behind it, which the frustum
    criteria would merge) the root still splits just below that threshold
    and keeps just above it."""
    pos = np.array([[-0.25, 0.0, 4.0], [0.25, 0.0, 4.0], [0.0, 0.5, 4.0]], np.float32)
    m = I.halfedge_from_faces([[0, 1, 2]], pos)
    f = 0.5 * 600 / math.tan(math.radians(30.0))
    e, r = 0.5, 4.0                      # root 0: v0 = (-0.25, 0, 4), v1 = (0.25, 0, 4)
    px = f * e / r
    for fwd in ((0, 0, 1), (0, 0, -1), (1, 0, 0)):
        cam = _cam(60.0, 800, 600, 0.05, pos=(0, 0, 0), fwd=fwd, up=(0, 1, 0))
        for thr, want in ((px * 0.999, I.DEC_SPLIT), (px * 1.001, I.DEC_KEEP)):
            o = Oracle(m, 4, I.LodParams(I.MODE_FLAT, thr, thr / 4, criterion=I.CRIT_DISTANCE))
            o.frame(camera=cam)
            dec, A, Bs, _ = o.decisions()
            assert dec[0] == want, (fwd, thr)
            # A / Bs = (f e)^2 / (thr r)^2
            assert abs(float(A[0]) / float(Bs[0]) / (px / float(np.float32(thr))) ** 2 - 1.0) < 1e-5


@pytest.mark.parametrize("seed", range(2))
def test_distance_decisions_match_float64(seed):
    """The distance-only criterion agrees with a float64 evaluation of
    f |p1 - p0| / |m - c| outside a 1e-4 relative band, for bisectors in
    front of and behind the camera alike (no frustum merge)."""
    m = _flat_mesh_in_front(seed)
    o = Oracle(m, 12, I.LodParams(I.MODE_FLAT, 30.0, 12.0, criterion=I.CRIT_DISTANCE))
    for _ in range(4):
        o.frame(decisions=np.ones(o.cap, np.uint8))
    cam = _cam(70.0, 640, 480, 0.05, pos=(0.1, -0.2, 2.1), fwd=(0.3, 0.05, 1.0), up=(0.0, 1.0, 0.1))
    th = math.tan(0.5 * cam.fovy)
    f = 0.5 * cam.height / th
    ids = o.pool()[0]
    verts = o.vertices()
    live = np.nonzero(ids)[0]
    cpos = cam.pos.astype(np.float64)
    px = []
    for s in live:
        v = verts[s].reshape(3, 3).astype(np.float64)
        px.append(f * np.linalg.norm(v[1] - v[0]) / np.linalg.norm(0.5 * (v[0] + v[1]) - cpos))
    split_px, merge_px = float(np.quantile(px, 0.7)), float(np.quantile(px, 0.3))
    o.set_lod(I.LodParams(I.MODE_FLAT, split_px, merge_px, criterion=I.CRIT_DISTANCE))
    o.frame(camera=cam)
    dec = o.decisions()[0]
    split_px, merge_px = float(np.float32(split_px)), float(np.float32(merge_px))
    behind = 0
    kinds = set()
    n_checked = 0
    K = o.frame_constants(cam)
    for s in live:
        v = verts[s].reshape(3, 3).astype(np.float64)
        want, margin = _distance_decide64(v, cpos, split_px, merge_px, f)
        if margin < 1e-4:
            continue
        assert dec[s] == want, (s, dec[s], want)
        kinds.add(want)
        n_checked += 1
        behind += int(((v - K[0:3].astype(np.float64)) @ K[9:12].astype(np.float64) < 0).all())
    assert n_checked > 0.9 * live.size
    assert kinds == {I.DEC_SPLIT, I.DEC_MERGE, I.DEC_KEEP}
    assert behind > 0          # bisectors behind the camera are decided by size, not culled
