"""Python binding of the gfx950 bisection-update library (include/cbt.h).

Argument marshalling only: every step of the update runs in the HIP kernels
of ``libcbt_hip.so``.  PyTorch provides the device workspace, the device copy
of displacement tables and decision vectors, and the stream.  There is no
fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcbt_hip.so")
_LIB = None

CBT_OK = 0
STATUS = {0: "ok", -1: "invalid argument", -2: "invalid mesh", -3: "invalid depth", -4: "capacity",
          -5: "device error", -6: "workspace too small", -7: "failed handle"}

EXPORTED = ["cbt_workspace_bytes", "cbt_init", "cbt_update", "cbt_update_with_decisions", "cbt_query",
            "cbt_query_decisions", "cbt_snapshot", "cbt_restore", "cbt_frame_constants", "cbt_live_count",
            "cbt_destroy", "cbt_status_string", "cbt_last_error", "cbt_time_stage", "cbt_stage_time"]

STAGES = {"enumerate": 1, "classify": 2, "vote": 3, "budget": 4, "chain": 5, "owners": 6, "offsets": 7,
          "freelist": 8, "fill": 9, "resolve": 10, "reduce": 11, "frame": 12}


class CbtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Mesh(C.Structure):
    _fields_ = [("H", C.c_int32), ("twin", C.c_void_p), ("next", C.c_void_p), ("prev", C.c_void_p),
                ("vert", C.c_void_p), ("V", C.c_int32), ("pos", C.c_void_p)]


class Camera(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("fwd", C.c_float * 3), ("up", C.c_float * 3), ("fovy", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32), ("znear", C.c_float)]


class LodParams(C.Structure):
    _fields_ = [("mode", C.c_int32), ("split_px", C.c_float), ("merge_px", C.c_float), ("table", C.c_void_p),
                ("table_res", C.c_int32), ("amplitude", C.c_float)]


class FrameStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "live_before", "free_before", "split_requests", "split_accepted", "merge_requests", "merge_configs",
        "merge_accepted", "merges_executed", "split_consumed", "allocations", "frees", "live_after", "max_depth")]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class Bisectors(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("count", C.c_int64), ("slot", C.c_void_p), ("heap_id", C.c_void_p),
                ("twin", C.c_void_p), ("next", C.c_void_p), ("prev", C.c_void_p), ("vertices", C.c_void_p),
                ("tree", C.c_void_p)]


def load_library():
    """Loads libcbt_hip.so; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2407_02215_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.cbt_workspace_bytes.argtypes = [C.c_int32, C.c_int32]
    lib.cbt_workspace_bytes.restype = C.c_size_t
    lib.cbt_init.argtypes = [C.POINTER(Mesh), C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.cbt_update.argtypes = [vp, C.POINTER(Camera), C.POINTER(LodParams), C.POINTER(FrameStats)]
    lib.cbt_update_with_decisions.argtypes = [vp, vp, C.POINTER(FrameStats)]
    lib.cbt_query.argtypes = [vp, C.POINTER(Bisectors)]
    lib.cbt_query_decisions.argtypes = [vp, vp]
    lib.cbt_snapshot.argtypes = [vp, vp, vp, vp, vp]
    lib.cbt_restore.argtypes = [vp, vp, vp, vp, vp]
    lib.cbt_frame_constants.argtypes = [vp, C.POINTER(Camera), C.POINTER(LodParams), vp]
    lib.cbt_live_count.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.cbt_destroy.argtypes = [vp]
    lib.cbt_time_stage.argtypes = [vp, C.c_int32]
    lib.cbt_stage_time.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    lib.cbt_status_string.argtypes = [C.c_int32]
    lib.cbt_status_string.restype = C.c_char_p
    lib.cbt_last_error.argtypes = [vp]
    lib.cbt_last_error.restype = C.c_char_p
    for f in ("cbt_init", "cbt_update", "cbt_update_with_decisions", "cbt_query", "cbt_query_decisions",
              "cbt_snapshot", "cbt_restore", "cbt_frame_constants", "cbt_live_count", "cbt_destroy",
              "cbt_time_stage", "cbt_stage_time"):
        getattr(lib, f).restype = C.c_int32
    _LIB = lib
    return lib


def workspace_bytes(H: int, D: int) -> int:
    return int(load_library().cbt_workspace_bytes(H, D))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def make_camera(cam) -> Camera:
    c = Camera()
    for i in range(3):
        c.pos[i] = float(cam.pos[i])
        c.fwd[i] = float(cam.fwd[i])
        c.up[i] = float(cam.up[i])
    c.fovy = float(np.float32(cam.fovy))
    c.width = int(cam.width)
    c.height = int(cam.height)
    c.znear = float(np.float32(cam.znear))
    return c


def canonical(heap_ids, k: int):
    """Sorted (root halfedge, 1 followed by the path bits) pairs."""
    out = []
    for x in np.asarray(heap_ids, np.uint64).tolist():
        d = int(x).bit_length() - 1 - k
        out.append(((x >> d) - (1 << k), (1 << d) | (x & ((1 << d) - 1))))
    return sorted(out)


class Instance:
    """One bisection-update instance resident on the GPU."""

    def __init__(self, mesh, depth: int, lod=None, device: str = "cuda", stream=None):
        import torch
        self._torch = torch
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("the bisection update needs a HIP device")
        self.device = torch.device(device)
        self.D = int(depth)
        self.cap = 1 << self.D
        self.H = int(mesh.H)
        self.k = (self.H - 1).bit_length()   # ceil(log2 H)
        nbytes = workspace_bytes(self.H, self.D)
        if nbytes == 0:
            raise CbtError(-3, f"invalid H={self.H} / D={self.D}")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._arrays = [np.ascontiguousarray(a, np.int32) for a in (mesh.twin, mesh.next, mesh.prev, mesh.vert)]
        pos = np.ascontiguousarray(mesh.pos, np.float32)
        m = Mesh(self.H, *(_ptr(a) for a in self._arrays), int(pos.shape[0]), _ptr(pos))
        h = C.c_void_p()
        st = self.lib.cbt_init(C.byref(m), self.D, C.c_void_p(self.workspace.data_ptr()), nbytes,
                               C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != CBT_OK:
            raise CbtError(st, self.lib.cbt_last_error(None).decode())
        self.h = h
        self.lod = None
        self._table = None
        if lod is not None:
            self.set_lod(lod)

    # -- lifecycle --------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.cbt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != CBT_OK:
            raise CbtError(st, self.lib.cbt_last_error(self.h).decode())

    # -- LOD --------------------------------------------------------------
    def set_lod(self, lod):
        torch = self._torch
        self.lod = lod
        if lod.table is not None:
            self._table = torch.from_numpy(np.ascontiguousarray(lod.table, np.float32)).to(self.device)
        else:
            self._table = None
        self._lodp = LodParams(int(lod.mode), float(lod.split_px), float(lod.merge_px),
                               C.c_void_p(self._table.data_ptr()) if self._table is not None else None,
                               int(lod.table_res), float(lod.amplitude))

    # -- frames -------------------------------------------------------------
    def update(self, camera, stats: bool = False):
        if self.lod is None:
            raise CbtError(-1, "no LOD parameters")
        cam = make_camera(camera)
        st = FrameStats() if stats else None
        self._check(self.lib.cbt_update(self.h, C.byref(cam), C.byref(self._lodp), C.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def update_with_decisions(self, decisions, stats: bool = False):
        torch = self._torch
        if isinstance(decisions, np.ndarray):
            dec = torch.from_numpy(np.ascontiguousarray(decisions, np.uint8)).to(self.device)
        else:
            dec = decisions.to(self.device, torch.uint8).contiguous()
        assert dec.numel() == self.cap
        self._dec_keep = dec
        st = FrameStats() if stats else None
        self._check(self.lib.cbt_update_with_decisions(self.h, C.c_void_p(dec.data_ptr()),
                                                       C.byref(st) if stats else None))
        return st.as_dict() if stats else None

    # -- queries ------------------------------------------------------------
    def live_count(self) -> int:
        n = C.c_int64()
        self._check(self.lib.cbt_live_count(self.h, C.byref(n)))
        return int(n.value)

    def query(self, vertices: bool = False, tree: bool = False):
        b = Bisectors()
        b.capacity = 0
        if tree:
            heap = np.zeros(2 * self.cap, np.uint32)
            b.tree = _ptr(heap)
        self._check(self.lib.cbt_query(self.h, C.byref(b)))
        L = int(b.count)
        out = {"count": L}
        slot = np.zeros(L, np.int32)
        ids = np.zeros(L, np.uint64)
        tw = np.zeros(L, np.int32)
        nx = np.zeros(L, np.int32)
        pv = np.zeros(L, np.int32)
        b2 = Bisectors(L, 0, _ptr(slot), _ptr(ids), _ptr(tw), _ptr(nx), _ptr(pv), None, None)
        verts = None
        if vertices:
            verts = np.zeros((L, 9), np.float32)
            b2.vertices = _ptr(verts)
        self._check(self.lib.cbt_query(self.h, C.byref(b2)))
        out.update(slot=slot, heap_id=ids, twin=tw, next=nx, prev=pv)
        if vertices:
            out["vertices"] = verts
        if tree:
            out["tree"] = heap
        return out

    def pool(self):
        """Per-slot arrays (heap ID 0 = free block), like a snapshot."""
        ids = np.zeros(self.cap, np.uint64)
        tw = np.zeros(self.cap, np.int32)
        nx = np.zeros(self.cap, np.int32)
        pv = np.zeros(self.cap, np.int32)
        self._check(self.lib.cbt_snapshot(self.h, _ptr(ids), _ptr(tw), _ptr(nx), _ptr(pv)))
        return ids, tw, nx, pv

    snapshot = pool

    def restore(self, ids, tw, nx, pv):
        ids = np.ascontiguousarray(ids, np.uint64)
        tw, nx, pv = (np.ascontiguousarray(a, np.int32) for a in (tw, nx, pv))
        self._check(self.lib.cbt_restore(self.h, _ptr(ids), _ptr(tw), _ptr(nx), _ptr(pv)))

    def decisions(self) -> np.ndarray:
        out = np.zeros(self.cap, np.uint8)
        self._check(self.lib.cbt_query_decisions(self.h, _ptr(out)))
        return out

    def frame_constants(self, camera) -> np.ndarray:
        cam = make_camera(camera)
        lp = self._lodp if self.lod is not None else LodParams(0, 1.0, 1.0, None, 0, 0.0)
        out = np.zeros(18, np.float32)
        self._check(self.lib.cbt_frame_constants(self.h, C.byref(cam), C.byref(lp), _ptr(out)))
        return out

    def time_stage(self, stage):
        """Record HIP events around one stage ('classify', ... or 'frame') in
        later updates; None stops."""
        self._check(self.lib.cbt_time_stage(self.h, 0 if stage is None else STAGES[stage]))

    def stage_time(self):
        """(timed launches, total milliseconds) since time_stage()."""
        n = C.c_int64()
        ms = C.c_double()
        self._check(self.lib.cbt_stage_time(self.h, C.byref(n), C.byref(ms)))
        return int(n.value), float(ms.value)

    def canonical(self):
        return canonical(self.query()["heap_id"], self.k)
