"""Seeded synthetic inputs: halfedge meshes, displacement tables, camera paths
and injected decision vectors.

This module is shared by the HIP path and by the CPU reference used in tests.
It builds *inputs only*: it holds none of the bisection method's arithmetic
(no bisector decoding, no LOD test, no table sampling used by either side).
Everything is a pure function of its seed.

Mesh convention (paper Section 2.1, halfedge table of the halfedge figure):
each halfedge h has Twin (-1 on a border), Next, Prev, Vert (its origin
vertex), Edge and Face.  Faces are listed counter-clockwise seen from outside,
so twin halfedges run in opposite directions.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

# LOD modes understood by both sides (world-position recipe applied to the
# flat-domain vertices before the screen-space test).
MODE_FLAT = 0        # p = v
MODE_SPHERE = 1      # p = normalize(v) * (1 + amp * cubemap(normalize(v)))
MODE_HEIGHTFIELD = 2  # p = v + (0, 0, amp * grid(v.x, v.y))

DEC_KEEP, DEC_SPLIT, DEC_MERGE = 0, 1, 2

# size criteria of the screen-space test: projected base-edge length
# (thresholds in pixels), projected triangle area (thresholds in pixels^2), or
# the cull-free distance-only variant (base edge over its midpoint's
# distance, in pixels, no frustum test)
CRIT_EDGE, CRIT_AREA, CRIT_DISTANCE = 0, 1, 2


@dataclasses.dataclass
class HalfedgeMesh:
    twin: np.ndarray
    next: np.ndarray
    prev: np.ndarray
    vert: np.ndarray
    edge: np.ndarray
    face: np.ndarray
    pos: np.ndarray  # (V, 3) float32

    @property
    def H(self) -> int:
        return int(self.twin.shape[0])

    @property
    def V(self) -> int:
        return int(self.pos.shape[0])


def halfedge_from_faces(faces: Sequence[Sequence[int]], pos) -> HalfedgeMesh:
    """Build the halfedge operators of a polygon mesh given as vertex cycles."""
    pos = np.ascontiguousarray(np.asarray(pos, dtype=np.float32).reshape(-1, 3))
    H = sum(len(f) for f in faces)
    twin = np.full(H, -1, np.int32)
    nxt = np.zeros(H, np.int32)
    prv = np.zeros(H, np.int32)
    vert = np.zeros(H, np.int32)
    face = np.zeros(H, np.int32)
    edge = np.zeros(H, np.int32)
    directed = {}
    h0 = 0
    for fi, f in enumerate(faces):
        n = len(f)
        if n < 3:
            raise ValueError("faces need at least 3 vertices")
        for i in range(n):
            h = h0 + i
            vert[h] = f[i]
            nxt[h] = h0 + (i + 1) % n
            prv[h] = h0 + (i - 1) % n
            face[h] = fi
            key = (int(f[i]), int(f[(i + 1) % n]))
            if key in directed:
                raise ValueError(f"non-manifold or inconsistently oriented edge {key}")
            directed[key] = h
        h0 += n
    eid = 0
    for (a, b), h in sorted(directed.items(), key=lambda kv: kv[1]):
        t = directed.get((b, a), -1)
        twin[h] = t
        if t == -1 or t > h:
            edge[h] = eid
            if t != -1:
                edge[t] = eid
            eid += 1
    return HalfedgeMesh(twin, nxt, prv, vert, edge, face, pos)


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------

def mesh_cube() -> HalfedgeMesh:
    """Cube with corners at (+-1, +-1, +-1): 6 quads, 24 halfedges, closed."""
    p = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], np.float32)

    def vid(x, y, z):
        return ((x > 0) << 2) | ((y > 0) << 1) | int(z > 0)
    faces = [
        [vid(1, -1, -1), vid(1, 1, -1), vid(1, 1, 1), vid(1, -1, 1)],      # +x
        [vid(-1, -1, -1), vid(-1, -1, 1), vid(-1, 1, 1), vid(-1, 1, -1)],  # -x
        [vid(-1, 1, -1), vid(-1, 1, 1), vid(1, 1, 1), vid(1, 1, -1)],      # +y
        [vid(-1, -1, -1), vid(1, -1, -1), vid(1, -1, 1), vid(-1, -1, 1)],  # -y
        [vid(-1, -1, 1), vid(1, -1, 1), vid(1, 1, 1), vid(-1, 1, 1)],      # +z
        [vid(-1, -1, -1), vid(-1, 1, -1), vid(1, 1, -1), vid(1, -1, -1)],  # -z
    ]
    return _orient_outward(faces, p)


def _orient_outward(faces, p):
    """Flip any face whose normal points towards the origin (convex shapes)."""
    out = []
    for f in faces:
        a, b, c = (p[f[0]].astype(np.float64), p[f[1]].astype(np.float64), p[f[2]].astype(np.float64))
        n = np.cross(b - a, c - a)
        cen = np.mean([p[i] for i in f], axis=0)
        out.append(list(f) if np.dot(n, cen) > 0 else list(reversed(f)))
    return halfedge_from_faces(out, p)


def mesh_icosahedron() -> HalfedgeMesh:
    """Regular icosahedron on the unit sphere: 20 triangles, 60 halfedges."""
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for a in (-1.0, 1.0):
        for b in (-phi, phi):
            v += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    v = np.array(v, np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    # faces = triples of mutually nearest vertices (edge length is the minimum)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    emin = np.min(d[d > 1e-9])
    adj = np.abs(d - emin) < 1e-6
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            for k in range(j + 1, 12):
                if adj[i, j] and adj[j, k] and adj[i, k]:
                    faces.append([i, j, k])
    assert len(faces) == 20
    return _orient_outward(faces, v.astype(np.float32))


def mesh_grid(n: int) -> HalfedgeMesh:
    """n x n quads over [0,1]^2 in the z=0 plane ((n+1)^2 vertices, 4n^2 halfedges)."""
    xs = np.arange(n + 1, dtype=np.float64) / n
    pos = np.zeros(((n + 1) * (n + 1), 3), np.float32)
    for j in range(n + 1):
        for i in range(n + 1):
            pos[j * (n + 1) + i] = (xs[i], xs[j], 0.0)
    faces = []
    for j in range(n):
        for i in range(n):
            a = j * (n + 1) + i
            faces.append([a, a + 1, a + n + 2, a + n + 1])
    return halfedge_from_faces(faces, pos)


def mesh_two_triangles(closed: bool) -> HalfedgeMesh:
    """Smallest test meshes: two triangles sharing one edge (open, 4 border
    halfedges) or glued along all three edges (a closed 'pillow')."""
    if closed:
        pos = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
        # the second face is the first with reversed orientation; the pillow is
        # closed and every halfedge has a twin.
        return halfedge_from_faces([[0, 1, 2], [0, 2, 1]], pos)
    pos = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], np.float32)
    return halfedge_from_faces([[0, 1, 2], [0, 2, 3]], pos)


def mesh_quad_sphere(n: int, split_prob: float, seed: int) -> HalfedgeMesh:
    """Closed quad-sphere: an n x n grid on every cube face projected to the
    unit sphere; each quad is split into two triangles with probability
    split_prob (seeded), giving a mixed tri/quad closed mesh."""
    rng = np.random.default_rng(seed)
    verts = {}
    pos = []

    def vid(p):
        key = tuple(int(round(c * 2 * n)) for c in p)
        if key not in verts:
            verts[key] = len(pos)
            q = np.array(p, np.float64)
            pos.append(q / np.linalg.norm(q))
        return verts[key]
    faces = []
    for axis in range(3):
        for sgn in (-1.0, 1.0):
            for j in range(n):
                for i in range(n):
                    quad = []
                    for (di, dj) in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        u = -1.0 + 2.0 * (i + di) / n
                        v = -1.0 + 2.0 * (j + dj) / n
                        p = [0.0, 0.0, 0.0]
                        p[axis] = sgn
                        p[(axis + 1) % 3] = u
                        p[(axis + 2) % 3] = v
                        quad.append(vid(p))
                    if rng.random() < split_prob:
                        if rng.random() < 0.5:
                            faces += [[quad[0], quad[1], quad[2]], [quad[0], quad[2], quad[3]]]
                        else:
                            faces += [[quad[0], quad[1], quad[3]], [quad[1], quad[2], quad[3]]]
                    else:
                        faces.append(quad)
    p = np.array(pos, np.float32)
    return _orient_outward_sphere(faces, p)


def _orient_outward_sphere(faces, p):
    out = []
    for f in faces:
        a, b, c = (p[f[0]].astype(np.float64), p[f[1]].astype(np.float64), p[f[2]].astype(np.float64))
        n = np.cross(b - a, c - a)
        cen = np.mean([p[i] for i in f], axis=0)
        out.append(list(f) if np.dot(n, cen) > 0 else list(reversed(f)))
    return halfedge_from_faces(out, p)


def random_mesh_of_size(target_h: int, seed: int) -> HalfedgeMesh:
    """Closed tri/quad sphere mesh with roughly target_h halfedges (>= 24)."""
    rng = np.random.default_rng(seed)
    split_prob = float(rng.uniform(0.0, 1.0))
    # H ~= 24 n^2 (1 + split_prob / 2)
    n = max(1, int(round(math.sqrt(target_h / (24.0 * (1.0 + 0.5 * split_prob))))))
    return mesh_quad_sphere(n, split_prob, seed + 7919)


def depth_for(H: int, D: int) -> int:
    """Smallest valid CBT depth >= D for a mesh with H halfedges."""
    k = max(0, int(math.ceil(math.log2(H))))
    return max(D, k)


# --------------------------------------------------------------------------
# noise tables (inputs sampled by the LOD's world-position step)
# --------------------------------------------------------------------------

def _perm_grad(seed: int, dim: int):
    rng = np.random.default_rng(seed)
    perm = rng.permutation(256).astype(np.int64)
    perm = np.concatenate([perm, perm])
    g = rng.normal(size=(256, dim))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return perm, g


def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def gradient_noise3(p: np.ndarray, perm, grad) -> np.ndarray:
    """Classic lattice gradient noise in 3D (float64), value range about [-1,1]."""
    pi = np.floor(p).astype(np.int64)
    pf = p - pi
    pi &= 255
    u = _fade(pf)
    gx, gy, gz = grad[:, 0].copy(), grad[:, 1].copy(), grad[:, 2].copy()
    acc = []
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                h = perm[perm[perm[pi[:, 0] + dx] + pi[:, 1] + dy] + pi[:, 2] + dz]
                acc.append(gx[h] * (pf[:, 0] - dx) + gy[h] * (pf[:, 1] - dy) + gz[h] * (pf[:, 2] - dz))
    # trilinear blend with fade weights
    x00 = acc[0] + u[:, 0] * (acc[1] - acc[0])
    x10 = acc[2] + u[:, 0] * (acc[3] - acc[2])
    x01 = acc[4] + u[:, 0] * (acc[5] - acc[4])
    x11 = acc[6] + u[:, 0] * (acc[7] - acc[6])
    y0 = x00 + u[:, 1] * (x10 - x00)
    y1 = x01 + u[:, 1] * (x11 - x01)
    out = y0 + u[:, 2] * (y1 - y0)
    return out * 1.5


def gradient_noise2(p: np.ndarray, perm, grad) -> np.ndarray:
    pi = np.floor(p).astype(np.int64)
    pf = p - pi
    pi &= 255
    u = _fade(pf)
    gx, gy = grad[:, 0].copy(), grad[:, 1].copy()
    acc = []
    for dy in (0, 1):
        for dx in (0, 1):
            h = perm[perm[pi[:, 0] + dx] + pi[:, 1] + dy]
            acc.append(gx[h] * (pf[:, 0] - dx) + gy[h] * (pf[:, 1] - dy))
    x0 = acc[0] + u[:, 0] * (acc[1] - acc[0])
    x1 = acc[2] + u[:, 0] * (acc[3] - acc[2])
    return (x0 + u[:, 1] * (x1 - x0)) * 1.4


def cubemap_directions(res: int) -> np.ndarray:
    """Unit directions of every texel of a 6 x res x res cube map, layout
    [face][j][i]; face order +x,-x,+y,-y,+z,-z; texel (i, j) sits at
    u = -1 + 2 i/(res-1), v = -1 + 2 j/(res-1), where (u, v) are the (y, z),
    (x, z) and (x, y) components for the x, y and z faces respectively."""
    t = -1.0 + 2.0 * np.arange(res, dtype=np.float64) / (res - 1)
    uu, vv = np.meshgrid(t, t, indexing="xy")  # uu varies with i (columns)
    dirs = np.zeros((6, res, res, 3))
    for f in range(6):
        axis, sgn = f // 2, (1.0 if f % 2 == 0 else -1.0)
        others = [a for a in range(3) if a != axis]
        dirs[f, :, :, axis] = sgn
        dirs[f, :, :, others[0]] = uu
        dirs[f, :, :, others[1]] = vv
    dirs /= np.linalg.norm(dirs, axis=3, keepdims=True)
    return dirs


def fbm_cubemap(res: int, seed: int, octaves: int = 8, lacunarity: float = 2.0,
                gain: float = 0.5, base_freq: float = 2.0) -> np.ndarray:
    """8-octave fBm of 3D gradient noise baked on a cube map, scaled to [-1, 1]."""
    perm, grad = _perm_grad(seed, 3)
    d = cubemap_directions(res).reshape(-1, 3)
    acc = np.zeros(d.shape[0])
    amp, freq = 1.0, base_freq
    for o in range(octaves):
        acc += amp * gradient_noise3(d * freq + 17.0 * o, perm, grad)
        amp *= gain
        freq *= lacunarity
    acc /= max(1e-12, np.max(np.abs(acc)))
    return acc.reshape(6, res, res).astype(np.float32)


def ridged_grid(res: int, seed: int, octaves: int = 8, lacunarity: float = 2.0,
                gain: float = 0.5, base_freq: float = 4.0) -> np.ndarray:
    """Ridged multifractal heightfield over [0,1]^2, layout [j][i] (j along y),
    texel (i, j) at (i/(res-1), j/(res-1)); values scaled to [0, 1]."""
    perm, grad = _perm_grad(seed, 2)
    t = np.arange(res, dtype=np.float64) / (res - 1)
    xx, yy = np.meshgrid(t, t, indexing="xy")
    p = np.stack([xx.ravel(), yy.ravel()], axis=1)
    acc = np.zeros(p.shape[0])
    amp, freq, wsum = 1.0, base_freq, 0.0
    for o in range(octaves):
        n = gradient_noise2(p * freq + 31.0 * o, perm, grad)
        r = (1.0 - np.abs(n)) ** 2
        acc += amp * r
        wsum += amp
        amp *= gain
        freq *= lacunarity
    acc -= acc.min()
    acc /= max(1e-12, acc.max())
    return acc.reshape(res, res).astype(np.float32)


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Camera:
    pos: np.ndarray   # float32[3]
    fwd: np.ndarray   # float32[3]
    up: np.ndarray    # float32[3]
    fovy: float       # radians
    width: int
    height: int
    znear: float

    def as_array(self) -> np.ndarray:
        """float32[13]: pos, fwd, up, fovy, width, height, znear."""
        return np.concatenate([self.pos, self.fwd, self.up,
                               [self.fovy, self.width, self.height, self.znear]]).astype(np.float32)


@dataclasses.dataclass
class LodParams:
    mode: int
    split_px: float
    merge_px: float
    table: np.ndarray | None = None  # float32, cube map (6,res,res) or grid (res,res)
    amplitude: float = 0.0
    criterion: int = CRIT_EDGE

    @property
    def table_res(self) -> int:
        return 0 if self.table is None else int(self.table.shape[-1])


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def camera_path_cube(frames: int = 8, seed: int = 1) -> List[Camera]:
    rng = np.random.default_rng(seed)
    u = _unit(rng.normal(size=3))
    c0 = np.array([0.0, 0.0, 3.0])
    out = []
    for t in range(frames):
        c = c0 + 0.1 * t * u
        out.append(Camera(c.astype(np.float32), (-c).astype(np.float32),
                          np.array([0, 1, 0], np.float32), math.radians(60.0),
                          1024, 1024, float(1e-3 * np.linalg.norm(c))))
    return out


def camera_path_planet(frames: int, seed: int, table: np.ndarray, amplitude: float) -> List[Camera]:
    """Descent along a seeded radial direction, altitude 10 -> 1e-5 radii
    (log-spaced), looking at the planet centre.  The camera stays above the
    displaced surface: its radius is 1 + amplitude * (max of the 2x2 texels
    around the direction) + altitude."""
    rng = np.random.default_rng(seed)
    u = _unit(rng.normal(size=3))
    w = rng.normal(size=3)
    up = _unit(w - np.dot(w, u) * u)
    hmax = _cubemap_local_max(table, u)
    out = []
    for t in range(frames):
        a = 10.0 ** (1.0 - 6.0 * t / max(1, frames - 1))
        r = 1.0 + amplitude * hmax + a
        c = r * u
        out.append(Camera(c.astype(np.float32), (-u).astype(np.float32), up.astype(np.float32),
                          math.radians(60.0), 1920, 1080, float(0.1 * a)))
    return out


def _cubemap_local_max(table, n):
    res = table.shape[-1]
    a = np.abs(n)
    if a[0] >= a[1] and a[0] >= a[2]:
        f, uu, vv = (0 if n[0] >= 0 else 1), n[1] / a[0], n[2] / a[0]
    elif a[1] >= a[2]:
        f, uu, vv = (2 if n[1] >= 0 else 3), n[0] / a[1], n[2] / a[1]
    else:
        f, uu, vv = (4 if n[2] >= 0 else 5), n[0] / a[2], n[1] / a[2]
    i = min(res - 2, int((uu + 1) * 0.5 * (res - 1)))
    j = min(res - 2, int((vv + 1) * 0.5 * (res - 1)))
    return float(np.max(table[f, j:j + 2, i:i + 2]))


def camera_path_terrain(frames: int, seed: int, table: np.ndarray, amplitude: float) -> List[Camera]:
    """Seeded random-walk flythrough over [0,1]^2: 1% of the extent per frame,
    heading drift N(0, 0.2 rad) per frame, reflection at [0.05, 0.95],
    altitude 0.02 above the local terrain maximum, pitched 30 degrees down."""
    rng = np.random.default_rng(seed)
    res = table.shape[-1]
    x, y = 0.5, 0.5
    th = float(rng.uniform(0, 2 * math.pi))
    out = []
    for t in range(frames):
        i = min(res - 2, int(x * (res - 1)))
        j = min(res - 2, int(y * (res - 1)))
        hz = amplitude * float(np.max(table[j:j + 2, i:i + 2]))
        c = np.array([x, y, hz + 0.02])
        pitch = math.radians(-30.0)
        fwd = np.array([math.cos(th) * math.cos(pitch), math.sin(th) * math.cos(pitch), math.sin(pitch)])
        out.append(Camera(c.astype(np.float32), fwd.astype(np.float32), np.array([0, 0, 1], np.float32),
                          math.radians(60.0), 3840, 2160, 1e-3))
        th += float(rng.normal(0.0, 0.2))
        x += 0.01 * math.cos(th)
        y += 0.01 * math.sin(th)
        if x < 0.05 or x > 0.95:
            x = min(0.95, max(0.05, x))
            th = math.pi - th
        if y < 0.05 or y > 0.95:
            y = min(0.95, max(0.05, y))
            th = -th
    return out


def camera_path_orbit(frames: int, seed: int, d0: float = 4.0, d1: float = 1.05) -> List[Camera]:
    """Sphere instance path: distance log-spaced d0 -> d1 radii along a seeded
    direction with seeded angular drift, looking at the centre."""
    rng = np.random.default_rng(seed)
    u = _unit(rng.normal(size=3))
    drift = _unit(rng.normal(size=3))
    out = []
    for t in range(frames):
        s = t / max(1, frames - 1)
        dist = d0 * (d1 / d0) ** s
        dirn = _unit(u + 0.3 * s * (drift - np.dot(drift, u) * u))
        c = dist * dirn
        w = np.array([0.0, 0.0, 1.0]) if abs(dirn[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
        up = _unit(w - np.dot(w, dirn) * dirn)
        out.append(Camera(c.astype(np.float32), (-dirn).astype(np.float32), up.astype(np.float32),
                          math.radians(60.0), 1920, 1080, float(0.1 * (dist - 1.0) + 1e-6)))
    return out


# --------------------------------------------------------------------------
# injected decisions (test hook) and workload bundles
# --------------------------------------------------------------------------

def random_decisions(capacity: int, seed: int, p_split: float, p_merge: float) -> np.ndarray:
    """One decision code per pool slot (KEEP=0, SPLIT=1, MERGE=2)."""
    rng = np.random.default_rng(seed)
    r = rng.random(capacity)
    out = np.zeros(capacity, np.uint8)
    out[r < p_split] = DEC_SPLIT
    out[(r >= p_split) & (r < p_split + p_merge)] = DEC_MERGE
    return out


@dataclasses.dataclass
class Workload:
    name: str
    mesh: HalfedgeMesh
    depth: int
    lod: LodParams
    cameras: List[Camera]


def workload(name: str, frames: int | None = None, table_res: int | None = None) -> Workload:
    """The synthetic stand-ins for the paper's scenes (sizes in the docstrings
    of the individual builders)."""
    if name == "cube":
        cams = camera_path_cube(frames or 8, seed=1)
        return Workload(name, mesh_cube(), 16, LodParams(MODE_FLAT, 8.0, 4.0), cams)
    if name == "planet":
        res = table_res or 512
        table = fbm_cubemap(res, seed=2)
        amp = 1e-3
        cams = camera_path_planet(frames or 256, seed=2, table=table, amplitude=amp)
        return Workload(name, mesh_icosahedron(), 20, LodParams(MODE_SPHERE, 4.0, 2.0, table, amp), cams)
    if name == "terrain":
        res = table_res or 2049
        table = ridged_grid(res, seed=3)
        amp = 0.05
        cams = camera_path_terrain(frames or 512, seed=3, table=table, amplitude=amp)
        return Workload(name, mesh_grid(64), 24, LodParams(MODE_HEIGHTFIELD, 2.0, 1.0, table, amp), cams)
    raise KeyError(name)


def _batched_member(args) -> tuple:
    """Mesh, depth and camera path of member i of a batched configuration,
    drawn from a generator seeded by (seed, i) alone, so that members can be
    built in any order or in parallel."""
    i, seed, frames, h_range, d_range = args
    rng = np.random.default_rng([seed, i])
    lo, hi = math.log(h_range[0]), math.log(h_range[1])
    target = int(round(math.exp(rng.uniform(lo, hi))))
    mesh = random_mesh_of_size(max(24, target), int(rng.integers(1 << 30)))
    D = depth_for(mesh.H, int(rng.integers(d_range[0], d_range[1] + 1)))
    cams = camera_path_orbit(frames, int(rng.integers(1 << 30)))
    return mesh, D, cams


def batched_workloads(n: int, frames: int = 64, seed: int = 4, h_range=(24, 50000), d_range=(14, 22),
                      table_res: int = 256, first: int = 0, workers: int = 1) -> List[Workload]:
    """Independent instances for the batched configuration: closed tri/quad
    sphere meshes with a log-uniform halfedge count in h_range, CBT depth
    uniform in d_range (raised to ceil(log2 H) where needed), sphere
    projection with one shared seeded fBm cube map (amplitude 1e-3 radius),
    and a seeded orbit camera path of its own per instance (4 -> 1.05 radii,
    split above 4 px, merge below 2 px at 1920x1080).  Members first ..
    first + n - 1 of the configuration seeded by seed; workers > 1 builds
    them in that many processes."""
    table = fbm_cubemap(table_res, seed=seed + 101)
    lod = LodParams(MODE_SPHERE, 4.0, 2.0, table, 1e-3)
    jobs = [(i, seed, frames, tuple(h_range), tuple(d_range)) for i in range(first, first + n)]
    if workers > 1 and n > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(workers, n)) as pool:
            members = pool.map(_batched_member, jobs, chunksize=max(1, n // (4 * workers)))
    else:
        members = [_batched_member(j) for j in jobs]
    return [Workload(f"batched-{i}", mesh, D, lod, cams) for (i, *_), (mesh, D, cams) in zip(jobs, members)]
