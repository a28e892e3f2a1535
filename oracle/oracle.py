"""ctypes binding of the CPU reference (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class OracleError(RuntimeError):
    pass


class _Stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "live_before", "free_before", "split_requests", "split_accepted", "merge_requests",
        "merge_configs", "merge_accepted", "merges_executed", "split_consumed", "allocations",
        "frees", "live_after", "max_depth")]


@dataclasses.dataclass
class Stats:
    live_before: int
    free_before: int
    split_requests: int
    split_accepted: int
    merge_requests: int
    merge_configs: int
    merge_accepted: int
    merges_executed: int
    split_consumed: int
    allocations: int
    frees: int
    live_after: int
    max_depth: int


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def load():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(_HERE, "libcbt_oracle.so")
    if not os.path.exists(path):
        from .build import build
        build()
    lib = C.CDLL(path)
    i32p, u32p, u64p, f32p, u8p = (C.POINTER(C.c_int32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
                                    C.POINTER(C.c_float), C.POINTER(C.c_uint8))
    lib.orc_cbt_reduce.argtypes = [u32p, C.c_int32]
    lib.orc_one_to_bit.argtypes = [u32p, C.c_int32, C.c_int64]
    lib.orc_one_to_bit.restype = C.c_int64
    lib.orc_zero_to_bit.argtypes = [u32p, C.c_int32, C.c_int64]
    lib.orc_zero_to_bit.restype = C.c_int64
    lib.orc_create.argtypes = [C.c_int32, i32p, i32p, i32p, i32p, C.c_int32, f32p, C.c_int32]
    lib.orc_create.restype = C.c_void_p
    lib.orc_destroy.argtypes = [C.c_void_p]
    lib.orc_set_lod.argtypes = [C.c_void_p, C.c_int32, C.c_float, C.c_float, f32p, C.c_int32, C.c_float]
    lib.orc_set_lod.restype = C.c_int32
    lib.orc_set_criterion.argtypes = [C.c_void_p, C.c_int32]
    lib.orc_set_criterion.restype = C.c_int32
    f64p = C.POINTER(C.c_double)
    lib.orc_set_precision.argtypes = [C.c_void_p, C.c_int32]
    lib.orc_set_precision.restype = C.c_int32
    lib.orc_world_position64.argtypes = [C.c_void_p, f64p, f64p]
    lib.orc_get_vertices64.argtypes = [C.c_void_p, f64p]
    lib.orc_get_vertices64.restype = C.c_int32
    lib.orc_decode64.argtypes = [C.c_void_p, C.c_uint64, f64p]
    lib.orc_decode64.restype = C.c_int32
    lib.orc_frame.argtypes = [C.c_void_p, f32p, u8p, C.POINTER(_Stats)]
    lib.orc_frame.restype = C.c_int32
    lib.orc_depth.argtypes = [C.c_void_p]
    lib.orc_depth.restype = C.c_int32
    lib.orc_root_bits.argtypes = [C.c_void_p]
    lib.orc_root_bits.restype = C.c_int32
    lib.orc_live_count.argtypes = [C.c_void_p]
    lib.orc_live_count.restype = C.c_int64
    lib.orc_get_pool.argtypes = [C.c_void_p, u64p, i32p, i32p, i32p]
    lib.orc_get_heap.argtypes = [C.c_void_p, u32p]
    lib.orc_get_vertices.argtypes = [C.c_void_p, f32p]
    lib.orc_get_decisions.argtypes = [C.c_void_p, u8p, f32p, f32p, f32p]
    lib.orc_frame_constants.argtypes = [C.c_void_p, f32p, f32p]
    lib.orc_frame_constants.restype = C.c_int32
    lib.orc_world_position.argtypes = [C.c_void_p, f32p, f32p]
    lib.orc_decode.argtypes = [C.c_void_p, C.c_uint64, f32p]
    lib.orc_decode.restype = C.c_int32
    lib.orc_root_triangle.argtypes = [C.c_void_p, C.c_int32, f32p]
    lib.orc_set_pool.argtypes = [C.c_void_p, u64p, i32p, i32p, i32p]
    lib.orc_set_pool.restype = C.c_int32
    lib.orc_check.argtypes = [C.c_void_p]
    lib.orc_check.restype = C.c_int32
    lib.orc_set_initiator_shuffle.argtypes = [C.c_void_p, C.c_uint64]
    lib.orc_last_error.restype = C.c_char_p
    _LIB = lib
    return lib


def _err(lib):
    return OracleError(lib.orc_last_error().decode())


# ---- CBT primitives on a full heap of 2^(D+1) counters ----

def cbt_reduce(heap: np.ndarray, D: int) -> np.ndarray:
    lib = load()
    h = np.ascontiguousarray(heap, dtype=np.uint32).copy()
    assert h.shape[0] == 2 << D
    lib.orc_cbt_reduce(_p(h, C.c_uint32), D)
    return h


def one_to_bit(heap: np.ndarray, D: int, i: int) -> int:
    h = np.ascontiguousarray(heap, dtype=np.uint32)
    return int(load().orc_one_to_bit(_p(h, C.c_uint32), D, i))


def zero_to_bit(heap: np.ndarray, D: int, i: int) -> int:
    h = np.ascontiguousarray(heap, dtype=np.uint32)
    return int(load().orc_zero_to_bit(_p(h, C.c_uint32), D, i))


class Oracle:
    """One bisection-update instance on the CPU."""

    def __init__(self, mesh, depth: int, lod=None, precision: int = 32):
        lib = load()
        self._lib = lib
        self._keep = []
        tw, nx, pv, vt = (np.ascontiguousarray(a, np.int32) for a in (mesh.twin, mesh.next, mesh.prev, mesh.vert))
        pos = np.ascontiguousarray(mesh.pos, np.float32)
        h = lib.orc_create(int(tw.shape[0]), _p(tw, C.c_int32), _p(nx, C.c_int32), _p(pv, C.c_int32),
                           _p(vt, C.c_int32), int(pos.shape[0]), _p(pos, C.c_float), int(depth))
        if not h:
            raise _err(lib)
        self._h = h
        self.D = int(depth)
        self.cap = 1 << self.D
        self.k = int(lib.orc_root_bits(h))
        self.precision = int(precision)
        if lib.orc_set_precision(h, self.precision):
            raise _err(lib)
        if lod is not None:
            self.set_lod(lod)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def set_lod(self, lod):
        t = None if lod.table is None else np.ascontiguousarray(lod.table, np.float32)
        rc = self._lib.orc_set_lod(self._h, int(lod.mode), float(lod.split_px), float(lod.merge_px),
                                   None if t is None else _p(t, C.c_float), lod.table_res, float(lod.amplitude))
        if rc:
            raise _err(self._lib)
        if self._lib.orc_set_criterion(self._h, int(getattr(lod, "criterion", 0))):
            raise _err(self._lib)

    def frame(self, camera=None, decisions=None) -> Stats:
        cam = None if camera is None else np.ascontiguousarray(camera.as_array(), np.float32)
        dec = None
        if decisions is not None:
            dec = np.ascontiguousarray(decisions, np.uint8)
            assert dec.shape[0] == self.cap
        st = _Stats()
        rc = self._lib.orc_frame(self._h, None if cam is None else _p(cam, C.c_float),
                                 None if dec is None else _p(dec, C.c_uint8), C.byref(st))
        if rc:
            raise _err(self._lib)
        return Stats(**{f: getattr(st, f) for f, _ in _Stats._fields_})

    # ---- inspection ----
    @property
    def live_count(self) -> int:
        return int(self._lib.orc_live_count(self._h))

    def pool(self):
        cap = self.cap
        ids = np.zeros(cap, np.uint64)
        tw = np.zeros(cap, np.int32)
        nx = np.zeros(cap, np.int32)
        pv = np.zeros(cap, np.int32)
        self._lib.orc_get_pool(self._h, _p(ids, C.c_uint64), _p(tw, C.c_int32), _p(nx, C.c_int32), _p(pv, C.c_int32))
        return ids, tw, nx, pv

    def heap(self) -> np.ndarray:
        h = np.zeros(2 * self.cap, np.uint32)
        self._lib.orc_get_heap(self._h, _p(h, C.c_uint32))
        return h

    def vertices(self) -> np.ndarray:
        v = np.zeros((self.cap, 9), np.float32)
        self._lib.orc_get_vertices(self._h, _p(v, C.c_float))
        return v

    def decisions(self):
        cap = self.cap
        dec = np.zeros(cap, np.uint8)
        A = np.zeros(cap, np.float32)
        Bs = np.zeros(cap, np.float32)
        Bm = np.zeros(cap, np.float32)
        self._lib.orc_get_decisions(self._h, _p(dec, C.c_uint8), _p(A, C.c_float), _p(Bs, C.c_float), _p(Bm, C.c_float))
        return dec, A, Bs, Bm

    def frame_constants(self, camera) -> np.ndarray:
        cam = np.ascontiguousarray(camera.as_array(), np.float32)
        out = np.zeros(18, np.float32)
        self._lib.orc_frame_constants(self._h, _p(cam, C.c_float), _p(out, C.c_float))
        return out

    def vertices64(self) -> np.ndarray:
        v = np.zeros((self.cap, 9), np.float64)
        if self._lib.orc_get_vertices64(self._h, _p(v, C.c_double)):
            raise _err(self._lib)
        return v

    def decode64(self, hid: int) -> np.ndarray:
        out = np.zeros(9, np.float64)
        if self._lib.orc_decode64(self._h, C.c_uint64(hid), _p(out, C.c_double)):
            raise _err(self._lib)
        return out.reshape(3, 3)

    def world_position64(self, v) -> np.ndarray:
        v = np.ascontiguousarray(v, np.float64)
        p = np.zeros(3, np.float64)
        self._lib.orc_world_position64(self._h, _p(v, C.c_double), _p(p, C.c_double))
        return p

    def world_position(self, v) -> np.ndarray:
        v = np.ascontiguousarray(v, np.float32)
        p = np.zeros(3, np.float32)
        self._lib.orc_world_position(self._h, _p(v, C.c_float), _p(p, C.c_float))
        return p

    def decode(self, hid: int) -> np.ndarray:
        out = np.zeros(9, np.float32)
        if self._lib.orc_decode(self._h, C.c_uint64(hid), _p(out, C.c_float)):
            raise _err(self._lib)
        return out.reshape(3, 3)

    def root_triangle(self, h: int) -> np.ndarray:
        out = np.zeros(9, np.float32)
        self._lib.orc_root_triangle(self._h, int(h), _p(out, C.c_float))
        return out.reshape(3, 3)

    def set_pool(self, ids, tw, nx, pv):
        ids = np.ascontiguousarray(ids, np.uint64)
        tw, nx, pv = (np.ascontiguousarray(a, np.int32) for a in (tw, nx, pv))
        rc = self._lib.orc_set_pool(self._h, _p(ids, C.c_uint64), _p(tw, C.c_int32), _p(nx, C.c_int32), _p(pv, C.c_int32))
        if rc:
            raise _err(self._lib)

    def check(self):
        if self._lib.orc_check(self._h):
            raise _err(self._lib)

    def set_initiator_shuffle(self, seed: int):
        self._lib.orc_set_initiator_shuffle(self._h, C.c_uint64(seed))

    def canonical(self):
        """Sorted (root halfedge, subdivision code) pairs of the live
        bisectors; the code is 1 followed by the d path bits."""
        ids = self.pool()[0]
        live = ids[ids != 0]
        out = []
        for x in live.tolist():
            d = x.bit_length() - 1 - self.k
            h = (x >> d) - (1 << self.k)
            out.append((h, (1 << d) | (x & ((1 << d) - 1))))
        return sorted(out)
