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
            "cbt_destroy", "cbt_status_string", "cbt_last_error", "cbt_time_stage", "cbt_stage_time",
            "cbt_set_schedule", "cbt_get_schedule", "cbt_stage_times", "cbt_batch_workspace_bytes", "cbt_batch_create",
            "cbt_batch_update", "cbt_batch_update_with_decisions", "cbt_batch_destroy", "cbt_update_converge",
            "cbt_export_triangles", "cbt_workspace_bytes_ex", "cbt_init_ex", "cbt_export_live", "cbt_import_live",
            "cbt_update_noalloc", "cbt_noalloc_scratch_bytes", "cbt_batch_fail_stage"]

INIT_FP64 = 1

STAGES = {"enumerate": 1, "classify": 2, "vote": 3, "budget": 4, "chain": 5, "owners": 6, "offsets": 7,
          "freelist": 8, "fill": 9, "resolve": 10, "reduce": 11, "frame": 12, "export": 13}


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
                ("table_res", C.c_int32), ("amplitude", C.c_float), ("criterion", C.c_int32)]


class FrameStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "live_before", "free_before", "split_requests", "split_accepted", "merge_requests", "merge_configs",
        "merge_accepted", "merges_executed", "split_consumed", "allocations", "frees", "live_after", "max_depth",
        "merge_candidates")]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class Bisectors(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("count", C.c_int64), ("slot", C.c_void_p), ("heap_id", C.c_void_p),
                ("twin", C.c_void_p), ("next", C.c_void_p), ("prev", C.c_void_p), ("vertices", C.c_void_p),
                ("tree", C.c_void_p), ("vertices64", C.c_void_p), ("root_h", C.c_void_p),
                ("subdiv_id", C.c_void_p)]


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
    lib.cbt_workspace_bytes_ex.argtypes = [C.c_int32, C.c_int32, C.c_uint32]
    lib.cbt_workspace_bytes_ex.restype = C.c_size_t
    lib.cbt_init_ex.argtypes = [C.POINTER(Mesh), C.c_int32, C.c_uint32, vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.cbt_update.argtypes = [vp, C.POINTER(Camera), C.POINTER(LodParams), C.POINTER(FrameStats)]
    lib.cbt_update_with_decisions.argtypes = [vp, vp, C.POINTER(FrameStats)]
    lib.cbt_update_noalloc.argtypes = [vp, C.POINTER(Camera), C.POINTER(LodParams), C.POINTER(FrameStats)]
    lib.cbt_noalloc_scratch_bytes.argtypes = []
    lib.cbt_noalloc_scratch_bytes.restype = C.c_size_t
    lib.cbt_query.argtypes = [vp, C.POINTER(Bisectors)]
    lib.cbt_query_decisions.argtypes = [vp, vp]
    lib.cbt_snapshot.argtypes = [vp, vp, vp, vp, vp]
    lib.cbt_restore.argtypes = [vp, vp, vp, vp, vp]
    lib.cbt_frame_constants.argtypes = [vp, C.POINTER(Camera), C.POINTER(LodParams), vp]
    lib.cbt_live_count.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.cbt_destroy.argtypes = [vp]
    lib.cbt_time_stage.argtypes = [vp, C.c_int32]
    lib.cbt_stage_time.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    lib.cbt_stage_times.argtypes = [vp, vp, C.c_int64, C.POINTER(C.c_int64)]
    lib.cbt_update_converge.argtypes = [vp, C.POINTER(Camera), C.POINTER(LodParams), C.c_int32,
                                        C.POINTER(C.c_int32), C.POINTER(FrameStats)]
    lib.cbt_export_triangles.argtypes = [vp, vp, C.c_int64, C.POINTER(C.c_int64)]
    lib.cbt_export_live.argtypes = [vp, vp, C.c_int64, C.POINTER(C.c_int64)]
    lib.cbt_import_live.argtypes = [vp, vp, C.c_int64, C.c_int32]
    lib.cbt_set_schedule.argtypes = [vp, C.c_int32, C.c_int32]
    lib.cbt_get_schedule.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.cbt_batch_workspace_bytes.argtypes = [vp, C.c_int32]
    lib.cbt_batch_workspace_bytes.restype = C.c_size_t
    lib.cbt_batch_create.argtypes = [vp, C.c_int32, vp, C.c_size_t, vp, C.c_int32, C.POINTER(vp)]
    lib.cbt_batch_update.argtypes = [vp, vp, vp, vp]
    lib.cbt_batch_update_with_decisions.argtypes = [vp, vp, vp]
    lib.cbt_batch_destroy.argtypes = [vp]
    lib.cbt_batch_fail_stage.argtypes = [vp, C.c_int32]
    lib.cbt_batch_fail_stage.restype = C.c_int32
    lib.cbt_status_string.argtypes = [C.c_int32]
    lib.cbt_status_string.restype = C.c_char_p
    lib.cbt_last_error.argtypes = [vp]
    lib.cbt_last_error.restype = C.c_char_p
    for f in ("cbt_init", "cbt_update", "cbt_update_with_decisions", "cbt_query", "cbt_query_decisions",
              "cbt_snapshot", "cbt_restore", "cbt_frame_constants", "cbt_live_count", "cbt_destroy",
              "cbt_time_stage", "cbt_stage_time", "cbt_stage_times", "cbt_set_schedule", "cbt_get_schedule", "cbt_batch_create",
              "cbt_batch_update", "cbt_batch_update_with_decisions", "cbt_batch_destroy", "cbt_update_converge",
              "cbt_export_triangles", "cbt_init_ex", "cbt_export_live", "cbt_import_live", "cbt_update_noalloc"):
        getattr(lib, f).restype = C.c_int32
    _LIB = lib
    return lib


def workspace_bytes(H: int, D: int, precision: int = 32) -> int:
    flags = INIT_FP64 if precision == 64 else 0
    return int(load_library().cbt_workspace_bytes_ex(H, D, flags))


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


class Instance:
    """One bisection-update instance resident on the GPU."""

    def __init__(self, mesh, depth: int, lod=None, device: str = "cuda", stream=None, tuned: bool = False,
                 precision: int = 32):
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
        if precision not in (32, 64):
            raise CbtError(-1, f"precision must be 32 or 64 bits, got {precision}")
        self.precision = int(precision)
        nbytes = workspace_bytes(self.H, self.D, self.precision)
        if nbytes == 0:
            raise CbtError(-3, f"invalid H={self.H} / D={self.D}")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._arrays = [np.ascontiguousarray(a, np.int32) for a in (mesh.twin, mesh.next, mesh.prev, mesh.vert)]
        pos = np.ascontiguousarray(mesh.pos, np.float32)
        m = Mesh(self.H, *(_ptr(a) for a in self._arrays), int(pos.shape[0]), _ptr(pos))
        h = C.c_void_p()
        flags = INIT_FP64 if self.precision == 64 else 0
        st = self.lib.cbt_init_ex(C.byref(m), self.D, flags, C.c_void_p(self.workspace.data_ptr()), nbytes,
                                  C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != CBT_OK:
            raise CbtError(st, self.lib.cbt_last_error(None).decode())
        self.h = h
        self.lod = None
        self._table = None
        if lod is not None:
            self.set_lod(lod)
        if tuned:
            self.apply_tuned(live=None)

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
                               int(lod.table_res), float(lod.amplitude), int(getattr(lod, "criterion", 0)))

    # -- frames -------------------------------------------------------------
    def update(self, camera, stats: bool = False):
        if self.lod is None:
            raise CbtError(-1, "no LOD parameters")
        cam = make_camera(camera)
        st = FrameStats() if stats else None
        self._check(self.lib.cbt_update(self.h, C.byref(cam), C.byref(self._lodp), C.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def update_noalloc(self, camera, stats: bool = False):
        """cbt_update_noalloc: the same frame with the scratch arrays in the
        library's static device array (pools of depth 20 at most)."""
        if self.lod is None:
            raise CbtError(-1, "no LOD parameters")
        cam = make_camera(camera)
        st = FrameStats() if stats else None
        self._check(self.lib.cbt_update_noalloc(self.h, C.byref(cam), C.byref(self._lodp),
                                                C.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def update_converge(self, camera, max_passes: int = 64):
        """Repeats the update with one camera until a pass changes nothing;
        returns (passes, counters of the last pass)."""
        if self.lod is None:
            raise CbtError(-1, "no LOD parameters")
        cam = make_camera(camera)
        n = C.c_int32()
        st = FrameStats()
        self._check(self.lib.cbt_update_converge(self.h, C.byref(cam), C.byref(self._lodp), int(max_passes),
                                                 C.byref(n), C.byref(st)))
        return int(n.value), st.as_dict()

    def export_triangles(self, out=None):
        """World positions of every live bisector's vertices, in block order,
        as a device tensor of shape (L, 3, 3)."""
        torch = self._torch
        n = C.c_int64()
        if out is None:
            st = self.lib.cbt_export_triangles(self.h, None, 0, C.byref(n))
            if st not in (CBT_OK, -4):
                self._check(st)
            out = torch.empty((max(1, int(n.value)), 3, 3), dtype=torch.float32, device=self.device)
        self._check(self.lib.cbt_export_triangles(self.h, C.c_void_p(out.data_ptr()), out.shape[0], C.byref(n)))
        return out[:int(n.value)]

    def export_live(self):
        """The live bisectors' records (block, id low, id high, twin, next,
        prev) in rank order, as a device int32 tensor of shape (L, 6)."""
        torch = self._torch
        n = C.c_int64()
        st = self.lib.cbt_export_live(self.h, None, 0, C.byref(n))
        if st not in (CBT_OK, -4):
            self._check(st)
        out = torch.empty((max(1, int(n.value)), 6), dtype=torch.int32, device=self.device)
        self._check(self.lib.cbt_export_live(self.h, C.c_void_p(out.data_ptr()), out.shape[0], C.byref(n)))
        return out[:int(n.value)]

    def import_live(self, records):
        """Replaces the state by records from export_live (a device tensor,
        or a host numpy array of shape (n, 6))."""
        if isinstance(records, np.ndarray):
            r = np.ascontiguousarray(records).view(np.uint32)
            self._check(self.lib.cbt_import_live(self.h, _ptr(r), int(r.shape[0]), 1))
        else:
            r = records.contiguous()
            self._check(self.lib.cbt_import_live(self.h, C.c_void_p(r.data_ptr()), int(r.shape[0]), 0))

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

    def query(self, vertices: bool = False, tree: bool = False, vertices64: bool = False):
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
        rh = np.zeros(L, np.int32)
        code = np.zeros(L, np.uint64)
        b2 = Bisectors(L, 0, _ptr(slot), _ptr(ids), _ptr(tw), _ptr(nx), _ptr(pv), None, None, None, _ptr(rh),
                       _ptr(code))
        verts = verts64 = None
        if vertices:
            verts = np.zeros((L, 9), np.float32)
            b2.vertices = _ptr(verts)
        if vertices64:
            verts64 = np.zeros((L, 9), np.float64)
            b2.vertices64 = _ptr(verts64)
        self._check(self.lib.cbt_query(self.h, C.byref(b2)))
        out.update(slot=slot, heap_id=ids, twin=tw, next=nx, prev=pv, root_h=rh, subdiv_id=code)
        if vertices:
            out["vertices"] = verts
        if vertices64:
            out["vertices64"] = verts64
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

    def stage_times(self) -> np.ndarray:
        """Milliseconds of each timed launch since time_stage(), in order."""
        n = C.c_int64()
        n_total, _ = self.stage_time()
        out = np.zeros(max(1, n_total), np.float64)
        self._check(self.lib.cbt_stage_times(self.h, _ptr(out), out.size, C.byref(n)))
        return out[:int(n.value)]

    def set_schedule(self, rank_groups: int, reduce_levels: int = 10):
        """Launch schedule of the per-bisector kernels (results do not depend
        on it)."""
        self._check(self.lib.cbt_set_schedule(self.h, int(rank_groups), int(reduce_levels)))

    def schedule(self):
        g = C.c_int32()
        r = C.c_int32()
        self._check(self.lib.cbt_get_schedule(self.h, C.byref(g), C.byref(r)))
        return int(g.value), int(r.value)

    def apply_tuned(self, live: int | None = -1):
        """Applies the tuned schedule of this depth for a live count: the
        instance's current one by default, the depth's busiest tuned state
        with live=None.  Returns the schedule, or None without a table."""
        from . import tune
        if live is not None and live < 0:
            live = self.live_count()
        entry = tune.lookup(self.D, tune.load_table(), live)
        if entry is not None:
            self.set_schedule(*entry)
        return entry

    def canonical(self):
        """The triangulation as the sorted (root halfedge, subdivision code)
        pairs the library reports (cbt_query's root_h / subdiv_id)."""
        q = self.query()
        return sorted(zip(q["root_h"].tolist(), q["subdiv_id"].tolist()))


BATCH_GRAPH = 1
BATCH_PERSISTENT = 2


class Batch:
    """Instances advanced together: one launch per pipeline stage for all of
    them, or one persistent launch per frame (persistent=True), optionally
    replayed from a captured HIP graph (cbt_batch_*)."""

    def __init__(self, instances, graph: bool = True, stream=None, persistent: bool = False):
        import torch
        self._torch = torch
        self.lib = load_library()
        self.members = list(instances)
        n = len(self.members)
        self._handles = (C.c_void_p * n)(*[m.h for m in self.members])
        nbytes = int(self.lib.cbt_batch_workspace_bytes(self._handles, n))
        if nbytes == 0:
            raise CbtError(-1, self.lib.cbt_last_error(None).decode())
        dev = self.members[0].device
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.Stream(dev)
        h = C.c_void_p()
        st = self.lib.cbt_batch_create(self._handles, n, C.c_void_p(self.workspace.data_ptr()), nbytes,
                                       C.c_void_p(self.stream.cuda_stream),
                                       (BATCH_GRAPH if graph else 0) | (BATCH_PERSISTENT if persistent else 0),
                                       C.byref(h))
        if st != CBT_OK:
            raise CbtError(st, self.lib.cbt_last_error(None).decode())
        self.h = h
        self.n = n

    def close(self):
        if getattr(self, "h", None):
            self.lib.cbt_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != CBT_OK:
            raise CbtError(st, self.lib.cbt_last_error(None).decode())

    def update(self, cameras, stats: bool = False):
        """One frame for every member; cameras[i] for member i (each member's
        LOD parameters are the ones set on its Instance)."""
        assert len(cameras) == self.n
        cams = (Camera * self.n)(*[make_camera(c) for c in cameras])
        lods = (LodParams * self.n)(*[m._lodp for m in self.members])
        st = (FrameStats * self.n)() if stats else None
        self._check(self.lib.cbt_batch_update(self.h, cams, lods, st))
        return [s.as_dict() for s in st] if stats else None

    def fail_stage(self, stage: int):
        """Test hook (persistent batches): the given stage's waits give up
        at once; -1 restores them."""
        self._check(self.lib.cbt_batch_fail_stage(self.h, int(stage)))

    def update_with_decisions(self, decisions, stats: bool = False):
        torch = self._torch
        devs = []
        for m, d in zip(self.members, decisions):
            if isinstance(d, np.ndarray):
                t = torch.from_numpy(np.ascontiguousarray(d, np.uint8)).to(m.device)
            else:
                t = d.to(m.device, torch.uint8).contiguous()
            assert t.numel() == m.cap
            devs.append(t)
        self._dec_keep = devs
        ptrs = (C.c_void_p * self.n)(*[t.data_ptr() for t in devs])
        st = (FrameStats * self.n)() if stats else None
        self._check(self.lib.cbt_batch_update_with_decisions(self.h, ptrs, st))
        return [s.as_dict() for s in st] if stats else None

    def synchronize(self):
        self.stream.synchronize()


class ServerConfig(C.Structure):
    _fields_ = [("memory_budget", C.c_int64), ("max_batch", C.c_int32), ("slots", C.c_int32),
                ("map_capacity", C.c_int64)]


class Completion(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("instance", C.c_int64), ("status", C.c_int32), ("batch_size", C.c_int32),
                ("latency_ms", C.c_double), ("queue_ms", C.c_double), ("live_before", C.c_int64),
                ("live_after", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "instances", "resident", "queued", "in_flight", "requests", "admissions", "evictions", "batches", "frames",
        "bisector_updates", "bytes_resident", "bytes_budget", "host_snapshots")] + [
        (n, C.c_double) for n in ("admit_ms", "admit_ms_max", "evict_ms", "evict_ms_max")]

    def as_dict(self):
        return {f: (float(getattr(self, f)) if t is C.c_double else int(getattr(self, f))) for f, t in self._fields_}


SERVER_EXPORTS = ["cbt_server_overhead_bytes", "cbt_server_create", "cbt_server_open", "cbt_server_set_schedule",
                  "cbt_server_set_schedule_table", "cbt_server_submit", "cbt_server_poll", "cbt_server_drain", "cbt_server_query",
                  "cbt_server_close", "cbt_server_get_stats", "cbt_server_destroy"]
EXPORTED += SERVER_EXPORTS


def _server_signatures(lib):
    vp = C.c_void_p
    lib.cbt_server_overhead_bytes.argtypes = [C.POINTER(ServerConfig)]
    lib.cbt_server_overhead_bytes.restype = C.c_size_t
    lib.cbt_server_create.argtypes = [C.POINTER(ServerConfig), vp, C.c_size_t, C.POINTER(vp)]
    lib.cbt_server_open.argtypes = [vp, C.POINTER(Mesh), C.c_int32, C.POINTER(LodParams), C.POINTER(C.c_int64)]
    lib.cbt_server_set_schedule.argtypes = [vp, C.c_int64, C.c_int32, C.c_int32]
    lib.cbt_server_set_schedule_table.argtypes = [vp, C.c_int32, vp, vp, vp, vp]
    lib.cbt_server_submit.argtypes = [vp, C.c_int64, C.POINTER(Camera), C.c_uint64]
    lib.cbt_server_poll.argtypes = [vp, C.c_int32, vp, C.c_int32, C.POINTER(C.c_int32)]
    lib.cbt_server_drain.argtypes = [vp]
    lib.cbt_server_query.argtypes = [vp, C.c_int64, C.POINTER(Bisectors)]
    lib.cbt_server_close.argtypes = [vp, C.c_int64]
    lib.cbt_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
    lib.cbt_server_destroy.argtypes = [vp]
    for f in SERVER_EXPORTS[1:]:
        getattr(lib, f).restype = C.c_int32


class Server:
    """Serving loop over resident instances (cbt_server_*): requests are
    submitted as they arrive and batched continuously on the device."""

    def __init__(self, arena_bytes: int, memory_budget: int = 0, max_batch: int = 128, slots: int = 2,
                 map_capacity: int = 1 << 22, device: str = "cuda", tuned: bool = False):
        import torch
        self._torch = torch
        self.lib = load_library()
        _server_signatures(self.lib)
        self.device = torch.device(device)
        self.cfg = ServerConfig(int(memory_budget), int(max_batch), int(slots), int(map_capacity))
        over = int(self.lib.cbt_server_overhead_bytes(C.byref(self.cfg)))
        if over == 0:
            raise CbtError(-1, "invalid server configuration")
        self.arena = torch.empty(int(arena_bytes) + over, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        st = self.lib.cbt_server_create(C.byref(self.cfg), C.c_void_p(self.arena.data_ptr()), self.arena.numel(),
                                        C.byref(h))
        if st != CBT_OK:
            raise CbtError(st, self.lib.cbt_last_error(None).decode())
        self.h = h
        self._tables = {}
        self._meta = {}
        self._buf = (Completion * 4096)()
        if tuned:
            from . import tune
            self.set_schedule_table([(d, live, g, lv) for d, rows in tune.load_table().items()
                                     for live, g, lv in rows])

    def set_schedule_table(self, entries):
        """(depth, live count, rank_groups, reduce_levels) entries the server
        picks from for instances without a schedule of their own."""
        n = len(entries)
        arr = [np.ascontiguousarray([e[i] for e in entries], dt) for i, dt in
               enumerate((np.int32, np.int64, np.int32, np.int32))]
        self._check(self.lib.cbt_server_set_schedule_table(self.h, n, *(_ptr(a) for a in arr)))

    def _check(self, st):
        if st != CBT_OK:
            raise CbtError(st, self.lib.cbt_last_error(None).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.cbt_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def open(self, mesh, depth: int, lod) -> int:
        torch = self._torch
        table = None
        if lod.table is not None:
            key = id(lod.table)
            if key not in self._tables:
                self._tables[key] = (lod.table, torch.from_numpy(np.ascontiguousarray(lod.table, np.float32)).to(self.device))
            table = self._tables[key][1]
        lp = LodParams(int(lod.mode), float(lod.split_px), float(lod.merge_px),
                       C.c_void_p(table.data_ptr()) if table is not None else None, int(lod.table_res),
                       float(lod.amplitude), int(getattr(lod, "criterion", 0)))
        arrays = [np.ascontiguousarray(a, np.int32) for a in (mesh.twin, mesh.next, mesh.prev, mesh.vert)]
        pos = np.ascontiguousarray(mesh.pos, np.float32)
        m = Mesh(int(mesh.H), *(_ptr(a) for a in arrays), int(pos.shape[0]), _ptr(pos))
        iid = C.c_int64()
        self._check(self.lib.cbt_server_open(self.h, C.byref(m), int(depth), C.byref(lp), C.byref(iid)))
        self._meta[int(iid.value)] = (int(mesh.H), int(depth))
        return int(iid.value)

    def set_schedule(self, iid: int, rank_groups: int, reduce_levels: int = 10):
        self._check(self.lib.cbt_server_set_schedule(self.h, int(iid), int(rank_groups), int(reduce_levels)))

    def submit(self, iid: int, camera, tag: int = 0):
        cam = make_camera(camera)
        self._check(self.lib.cbt_server_submit(self.h, int(iid), C.byref(cam), int(tag)))

    def poll(self, wait: bool = False):
        n = C.c_int32()
        out = []
        while True:
            self._check(self.lib.cbt_server_poll(self.h, 1 if wait else 0, self._buf, len(self._buf), C.byref(n)))
            out += [self._buf[i].as_dict() for i in range(n.value)]
            if n.value < len(self._buf):
                return out
            wait = False

    def drain(self):
        self._check(self.lib.cbt_server_drain(self.h))
        return self.poll()

    def query(self, iid: int, tree: bool = False):
        H, D = self._meta[int(iid)]
        b = Bisectors()
        b.capacity = 0
        self._check(self.lib.cbt_server_query(self.h, int(iid), C.byref(b)))
        L = int(b.count)
        slot = np.zeros(L, np.int32)
        ids = np.zeros(L, np.uint64)
        tw = np.zeros(L, np.int32)
        nx = np.zeros(L, np.int32)
        pv = np.zeros(L, np.int32)
        rh = np.zeros(L, np.int32)
        code = np.zeros(L, np.uint64)
        b2 = Bisectors(L, 0, _ptr(slot), _ptr(ids), _ptr(tw), _ptr(nx), _ptr(pv), None, None, None, _ptr(rh),
                       _ptr(code))
        heap = None
        if tree:
            heap = np.zeros(2 << D, np.uint32)
            b2.tree = _ptr(heap)
        self._check(self.lib.cbt_server_query(self.h, int(iid), C.byref(b2)))
        out = {"count": L, "slot": slot, "heap_id": ids, "twin": tw, "next": nx, "prev": pv, "root_h": rh,
               "subdiv_id": code}
        if tree:
            out["tree"] = heap
        return out

    def stats(self):
        s = ServerStats()
        self._check(self.lib.cbt_server_get_stats(self.h, C.byref(s)))
        return s.as_dict()

    def close_instance(self, iid: int):
        self._check(self.lib.cbt_server_close(self.h, int(iid)))
        self._meta.pop(int(iid), None)
