"""The autotuner (fdtd_autotune): it times the candidate kernels of a grid,
keeps the fastest, restores the state it found, and caches its choice in the
JSON file named by GEMFDTD_TUNE_CACHE."""
import json
import os

import numpy as np
import pytest

from paper_2405_00814_amd import workloads as W

from helpers import assert_parity, rel_l2, run_oracle

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.mark.parametrize("dim", [2, 3])
def test_autotune_restores_state_and_caches(dim, tmp_path, monkeypatch):
    from paper_2405_00814_amd.sim import Sim
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("GEMFDTD_TUNE_CACHE", str(cache))
    if dim == 2:
        pb = W.dielectric2d(160, ny=192, steps=60, seed=3, nrect=6, side=(6, 30), npml=8, nprobes=3)
    else:
        pb = W.yee3d(shape=(24, 28, 64), steps=60, seed=3, nbox=4, side=(3, 8), npml=4, nprobes=3,
                     tau_steps=6.0)
    ref, rrec = run_oracle(pb, pb.steps)
    s = Sim.from_problem(pb)
    s.step(25)
    k = s.autotune(6)
    assert k["variant"] in (1, 2, 3)
    assert s.get_kernel() == k
    assert s.steps_done() == 25
    s.step(pb.steps - 25)
    got = {c: s.get_field(c) for c in ref}
    assert_parity(got, ref, TOL, "after autotune %s" % (k,))
    assert rel_l2(s.probe(), rrec) <= TOL
    s.close()
    d = json.loads(cache.read_text())
    assert len(d) == 1
    entry = list(d.values())[0]
    assert entry[0] == k["variant"] and tuple(entry[1:5]) == tuple(k["tile"])
    # a second handle on the same grid takes the cached choice
    s = Sim.from_problem(pb)
    assert s.autotune(6) == k
    s.close()
