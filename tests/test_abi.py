"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every function declared in include/cbt.h, argument and mesh
validation happen before any device access, and the workspace size follows
the paper's memory model (Table 2, Section 4.2)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2407_02215_amd import build as hip_build
from paper_2407_02215_amd import cbt
from paper_2407_02215_amd import inputs as I
from tests.helpers import read_golden, we1_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(cbt.LIB_PATH):
        hip_build.build()
    return cbt.load_library()


def test_exports_every_declared_function():
    header = open(os.path.join(ROOT, "include", "cbt.h")).read()
    declared = set(re.findall(r"\b(cbt_[a-z_]+)\s*\(", header))
    lib = _lib()
    missing = [f for f in sorted(declared) if not hasattr(lib, f)]
    assert not missing, missing
    assert declared >= set(cbt.EXPORTED)


def _init(mesh, D, ws_bytes, ptr=0x100000):
    lib = _lib()
    arrs = [np.ascontiguousarray(a, np.int32) for a in (mesh.twin, mesh.next, mesh.prev, mesh.vert)]
    pos = np.ascontiguousarray(mesh.pos, np.float32)
    m = cbt.Mesh(mesh.H, *(a.ctypes.data_as(C.c_void_p) for a in arrs), pos.shape[0], pos.ctypes.data_as(C.c_void_p))
    h = C.c_void_p()
    st = lib.cbt_init(C.byref(m), D, C.c_void_p(ptr), ws_bytes, None, C.byref(h))
    return st, lib.cbt_last_error(None).decode()


@pytest.mark.parametrize("bad", ["twin", "nextprev", "vert", "corner"])
def test_invalid_mesh_rejected_before_device_access(bad):
    m = I.mesh_cube()
    tw, nx, pv, vt = m.twin.copy(), m.next.copy(), m.prev.copy(), m.vert.copy()
    if bad == "twin":
        tw[0], tw[1] = tw[1], tw[0]
    elif bad == "nextprev":
        pv[0] = 5
    elif bad == "vert":
        vt[3] = 99
    elif bad == "corner":
        two = I.mesh_two_triangles(False)
        tw, nx, pv, vt = two.twin.copy(), two.next.copy(), two.prev.copy(), two.vert.copy()
        tw[0] = 1   # twin inside its own corner, and not an involution
        m = two
    bm = I.HalfedgeMesh(tw, nx, pv, vt, m.edge, m.face, m.pos)
    st, msg = _init(bm, 10, 1 << 40)
    assert st == -2, msg


def test_depth_and_workspace_checks():
    mesh = we1_mesh()
    st, msg = _init(mesh, 3, 1 << 40)
    assert st == -3, msg                                  # D < ceil(log2 12)
    st, msg = _init(mesh, 31, 1 << 40)
    assert st == -3, msg
    need = cbt.workspace_bytes(mesh.H, 8)
    assert need > 0
    st, msg = _init(mesh, 8, need - 1)
    assert st == -6, msg                                  # workspace too small
    st, msg = _init(mesh, 8, need, ptr=0x100010)
    assert st == -1, msg                                  # misaligned workspace
    assert cbt.workspace_bytes(2, 8) == 0 and cbt.workspace_bytes(12, 3) == 0


def test_workspace_follows_paper_memory_model():
    """Per pool block the paper keeps three 32-bit pointers, a 64-bit index,
    a 32-bit command and four 32-bit allocation slots (40 bytes), plus two
    32-bit cached decode results; at D = 17 that, with a 2^18-entry CBT, is
    7 MiB.  This library keeps the same index (8), pointers (12, padded to
    16 with the bisector's fate this frame), command (4) and four slots
    (16), the same 8 bytes of rank and free lists, a 12-byte work list and a
    48-byte cache of the vertices' world positions, and stores the bitfield
    plus a tree that stops at the word level instead of the 2^(D+1) heap."""
    g = read_golden("we4_memory.txt")
    D = int(g["D"])
    paper = (1 << D) * (3 * 4 + 8 + 4 + 4 * 4) + (1 << D) * 8 + (1 << (D + 1)) * 4
    assert paper == int(g["total_mib"]) << 20
    ours = cbt.workspace_bytes(60, D)
    per_block = (8 + 16 + 4 + 16) + 8 + 12 + 48
    cbt_bytes = (1 << D) // 8 + (1 << (D - 4)) * 4
    assert ours >= (1 << D) * per_block + cbt_bytes
    assert ours <= (1 << D) * per_block + cbt_bytes + 64 * 1024
    assert cbt_bytes < (1 << (D + 1)) * 4
    # binary64 instances: the vertex record doubles to 96 bytes and the root
    # triangles to 72 bytes per halfedge
    ours64 = cbt.workspace_bytes(60, D, precision=64)
    assert (1 << D) * 48 + 60 * 36 - 256 <= ours64 - ours <= (1 << D) * 48 + 60 * 36 + 256


def test_init_flags_checked():
    lib = _lib()
    assert lib.cbt_workspace_bytes_ex(12, 8, 0) == lib.cbt_workspace_bytes(12, 8)
    assert lib.cbt_workspace_bytes_ex(12, 8, 2) == 0          # unknown flag
    mesh = we1_mesh()
    arrays = [np.ascontiguousarray(a, np.int32) for a in (mesh.twin, mesh.next, mesh.prev, mesh.vert)]
    pos = np.ascontiguousarray(mesh.pos, np.float32)
    m = cbt.Mesh(mesh.H, *(cbt._ptr(a) for a in arrays), int(pos.shape[0]), cbt._ptr(pos))
    h = C.c_void_p()
    st = lib.cbt_init_ex(C.byref(m), 8, 6, C.c_void_p(0x100000), 1 << 40, None, C.byref(h))
    assert st == -1 and b"flags" in lib.cbt_last_error(None)


def test_status_strings():
    lib = _lib()
    for code in range(-7, 1):
        assert lib.cbt_status_string(code)


def _header_structs():
    """Field names, in order, of every typedef'd struct of include/cbt.h."""
    header = open(os.path.join(ROOT, "include", "cbt.h")).read()
    header = re.sub(r"/\*.*?\*/", "", header, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct\s*\{(.*?)\}\s*(\w+)\s*;", header, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            names = decl.split(",")
            first = re.sub(r"\[.*?\]", "", names[0]).replace("*", " ").split()[-1]
            fields.append(first)
            fields += [re.sub(r"\[.*?\]", "", n).replace("*", " ").strip() for n in names[1:]]
        out[name] = fields
    return out


@pytest.mark.parametrize("cname,pyname", [("cbt_mesh", "Mesh"), ("cbt_camera", "Camera"),
                                          ("cbt_lod_params", "LodParams"), ("cbt_frame_stats", "FrameStats"),
                                          ("cbt_bisectors", "Bisectors"), ("cbt_server_config", "ServerConfig"),
                                          ("cbt_completion", "Completion"), ("cbt_server_stats", "ServerStats")])
def test_binding_structs_follow_the_header(cname, pyname):
    """The binding's ctypes structures have the header's fields in the
    header's order (including cbt_bisectors' canonical root_h / subdiv_id
    outputs)."""
    fields = _header_structs()[cname]
    assert [f for f, _ in getattr(cbt, pyname)._fields_] == fields
    if cname == "cbt_bisectors":
        assert fields[-2:] == ["root_h", "subdiv_id"]


def test_small_depths_accepted():
    """Section 3.3: any D >= ceil(log2 H) holds the roots; pools of fewer
    than 32 blocks keep one partial bitfield word."""
    _lib()
    assert cbt.workspace_bytes(12, 4) > 0          # the halfedge-table mesh at D = ceil(log2 12)
    assert cbt.workspace_bytes(6, 3) > 0           # two triangles at D = 3
    assert cbt.workspace_bytes(12, 3) == 0
    st, msg = _init(we1_mesh(), 4, cbt.workspace_bytes(12, 4) - 1)
    assert st == -6, msg                           # validated up to the workspace size, no device access
