"""cbt_update_noalloc (the frame with its scratch arrays in the library's
static device array) against cbt_update, through the C ABI: two instances
advanced frame by frame with the two entry points must hold identical pools,
trees and frame counters.  Two calls run back to back on different
instances, the second on a smaller pool, so the second finds the static
array as the first left it; then a pool too deep for the array is refused."""
import ctypes as C

import numpy as np
import pytest
import torch  # noqa: F401

from paper_2407_02215_amd import cbt
from paper_2407_02215_amd import inputs as I
from tests.gpu_checks import log

pytestmark = pytest.mark.gpu


def _state(inst):
    q = inst.query(tree=True)
    return [q[k] for k in ("slot", "heap_id", "twin", "next", "prev", "tree")]


def _same(a, b, label):
    for name, x, y in zip(("slot", "heap_id", "twin", "next", "prev", "tree"), _state(a), _state(b)):
        assert np.array_equal(x, y), f"{label}: {name} differs"


def test_noalloc_matches_update():
    # first: the planet (depth 20, the largest pool the array serves), then
    # the cube (depth 16), alternating frame by frame
    big = I.workload("planet", frames=24, table_res=128)
    small = I.workload("cube", frames=8)
    pairs = []
    for w in (big, small):
        pairs.append((w, cbt.Instance(w.mesh, w.depth, w.lod), cbt.Instance(w.mesh, w.depth, w.lod)))
    try:
        lib = cbt.load_library()
        log(f"[noalloc] scratch {int(lib.cbt_noalloc_scratch_bytes())} bytes")
        for f in range(24):
            for w, ref, got in pairs:
                if f >= len(w.cameras):
                    continue
                log(f"[noalloc] {w.name} D={w.depth} frame {f}")
                a = ref.update(w.cameras[f], stats=True)
                b = got.update_noalloc(w.cameras[f], stats=True)
                assert a == b, f"{w.name} frame {f}: counters {a} != {b}"
                _same(ref, got, f"{w.name} frame {f}")
        assert pairs[0][1].live_count() > 10000
    finally:
        for _, a, b in pairs:
            a.close()
            b.close()


def test_noalloc_refuses_deep_pool():
    w = I.workload("cube")
    inst = cbt.Instance(w.mesh, 21, w.lod)
    try:
        with pytest.raises(cbt.CbtError) as e:
            inst.update_noalloc(w.cameras[0])
        assert e.value.status == -4
        assert "static scratch" in str(e.value)
        # the handle stays usable through the ordinary entry point
        inst.update(w.cameras[0])
    finally:
        inst.close()
