"""Step parity on the benchmark's own workloads and frames.

The HIP path advances the workload exactly as the benchmark does (the
depth-24 terrain with its 2049^2 height table and the tuned launch schedule;
the depth-20 planet with its 6 x 512^2 cube map); at each listed frame its
pool is snapshotted into the CPU reference (set_pool), both run that frame,
and the decisions of every live bisector, the frame counters, every pool
slot and the full CBT heap must be identical.  This covers the frames the
benchmark times (its warm-up window and the steady state after it), which
the reference is too slow to reach in lock-step."""
import numpy as np
import pytest
import torch  # noqa: F401

from oracle import Oracle
from paper_2407_02215_amd import cbt
from paper_2407_02215_amd import inputs as I
from tests.gpu_checks import assert_same_state, assert_same_tree, log

pytestmark = pytest.mark.gpu

TERRAIN_FRAMES = [5, 12, 24, 40, 64, 128, 239]
PLANET_FRAMES = [64, 128, 200, 255]
KEYS = ("live_before", "split_requests", "split_accepted", "merge_requests", "merge_configs", "merge_accepted",
        "merges_executed", "split_consumed", "allocations", "frees", "live_after")


class _Run:
    def __init__(self, w, tuned):
        self.w = w
        self.inst = cbt.Instance(w.mesh, w.depth, w.lod, tuned=tuned)
        self.orc = Oracle(w.mesh, w.depth, w.lod)
        self.frame = 0

    def advance_to(self, f):
        while self.frame < f:
            self.inst.update(self.w.cameras[self.frame])
            self.frame += 1


@pytest.fixture(scope="module")
def terrain():
    r = _Run(I.workload("terrain", frames=max(TERRAIN_FRAMES) + 1), tuned=True)
    yield r
    r.inst.close()


@pytest.fixture(scope="module")
def planet():
    r = _Run(I.workload("planet", frames=256), tuned=True)
    yield r
    r.inst.close()


def _step(r, f, label):
    r.advance_to(f)
    log(f"[step] {label} frame {f}: snapshot")
    r.orc.set_pool(*r.inst.snapshot())
    cam = r.w.cameras[f]
    gst = r.inst.update(cam, stats=True)
    r.frame += 1
    log(f"[step] {label} frame {f}: reference frame, L={gst['live_before']}")
    ost = r.orc.frame(camera=cam)
    for key in KEYS:
        assert gst[key] == getattr(ost, key), f"{label} frame {f}: {key} gpu={gst[key]} ref={getattr(ost, key)}"
    gdec = r.inst.decisions()
    odec = r.orc.decisions()[0]
    was_live = gdec != 255
    assert was_live.sum() == ost.live_before
    bad = np.nonzero(gdec[was_live] != odec[was_live])[0]
    assert bad.size == 0, f"{label} frame {f}: {bad.size} decisions differ"
    assert_same_state(r.inst, r.orc, f"{label} frame {f}")
    assert_same_tree(r.inst, r.orc, f"{label} frame {f}")
    return gst


@pytest.mark.parametrize("frame", TERRAIN_FRAMES)
def test_terrain_step_parity(terrain, frame):
    st = _step(terrain, frame, "terrain")
    if frame >= 40:
        assert st["live_before"] > 500_000 and st["merges_executed"] > 0 and st["split_consumed"] > 0


@pytest.mark.parametrize("frame", PLANET_FRAMES)
def test_planet_step_parity(planet, frame):
    st = _step(planet, frame, "planet")
    assert st["live_before"] > 100_000
