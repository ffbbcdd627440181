"""fdtd_probe_noalloc (the probe read-out that allocates no device memory)
against fdtd_probe, called through the C ABI: two calls in a row, the second
with a smaller input, bit for bit (both are copies of the same records), and
the size limit.  It is a plain copy of the device records, so the bar is
equality."""
import ctypes as C

import numpy as np
import pytest

from paper_2405_00814_amd import _lib as L
from paper_2405_00814_amd import workloads as W
from paper_2405_00814_amd.sim import Sim

from helpers import log

pytestmark = pytest.mark.gpu

LIMIT = 4 << 20  # floats of the fixed device array


def _read(lib, fn, h, nprobes, cap):
    n = C.c_int64(-1)
    out = np.full((nprobes, max(cap, 1)), np.nan, np.float32)
    rc = getattr(lib, fn)(h, out.ctypes.data_as(C.POINTER(C.c_float)), cap, C.byref(n))
    return rc, out[:, :cap], n.value


def _case(pb, steps, caps):
    lib = L.load()
    s = Sim.from_problem(pb)
    try:
        s.step(steps)
        for cap in caps:
            log("no-alloc probe", pb.shape, "probes", s.nprobes, "steps", steps, "cap", cap)
            rc0, ref, n0 = _read(lib, "fdtd_probe", s.h, s.nprobes, cap)
            rc1, got, n1 = _read(lib, "fdtd_probe_noalloc", s.h, s.nprobes, cap)
            assert rc0 == 0 and rc1 == 0, lib.fdtd_last_error()
            assert n0 == n1 == steps
            m = min(cap, steps)
            assert np.array_equal(got[:, :m], ref[:, :m])
            assert np.all(np.isnan(got[:, m:]))  # nothing written past the recorded samples
            assert np.any(got[:, :m] != 0)
    finally:
        s.close()


def test_noalloc_probe_matches_fdtd_probe_two_calls():
    # first call: 2D grid with CPML, 6 probes, full record (cap == recorded)
    pb = W.dielectric2d(160, ny=144, steps=700, seed=3, nrect=6, side=(8, 32), npml=12, nprobes=6)
    _case(pb, 700, [700])
    # second call, smaller input: fewer probes and samples, and a cap below
    # the record (row stride != samples copied)
    pb2 = W.dielectric2d(96, ny=80, steps=250, seed=4, nrect=3, side=(6, 20), npml=8, nprobes=3)
    _case(pb2, 250, [250, 97])


def test_noalloc_probe_3d_and_graph():
    pb = W.yee3d(shape=(24, 22, 20), steps=60, seed=2, nbox=3, side=(3, 8), npml=4, nprobes=4, tau_steps=6.0)
    _case(pb, 60, [60, 17])
    pbg = W.dielectric2d(64, ny=56, steps=90, seed=5, nrect=3, side=(4, 16), npml=6, nprobes=2)
    lib = L.load()
    s = Sim.from_problem(pbg, graph=True)
    try:
        s.step(90)
        rc0, ref, _ = _read(lib, "fdtd_probe", s.h, s.nprobes, 90)
        rc1, got, _ = _read(lib, "fdtd_probe_noalloc", s.h, s.nprobes, 90)
        assert rc0 == 0 and rc1 == 0
        assert np.array_equal(got, ref)
    finally:
        s.close()


def test_noalloc_probe_limit():
    """A record block above the fixed array's size is refused (FDTD_EINVAL,
    nothing written); a read of fewer samples of the same record passes."""
    pb = W.cavity2d(64, steps=1030, seed=1)
    s = Sim.from_problem(pb)
    try:
        rng = np.random.default_rng(0)
        cells = np.stack([rng.integers(1, 63, 4096), rng.integers(1, 63, 4096)], 1)
        s.set_probes("ez", cells)
        s.step(1030)
        lib = L.load()
        assert 4096 * 1030 > LIMIT
        out = np.zeros((4096, 1030), np.float32)
        n = C.c_int64()
        rc = lib.fdtd_probe_noalloc(s.h, out.ctypes.data_as(C.POINTER(C.c_float)), 1030, C.byref(n))
        assert rc == L.FDTD_EINVAL and n.value == 1030
        assert b"no-allocation limit" in lib.fdtd_last_error()
        assert not out.any()
        rc0, ref, _ = _read(lib, "fdtd_probe", s.h, 4096, 1024)
        rc1, got, _ = _read(lib, "fdtd_probe_noalloc", s.h, 4096, 1024)
        assert rc0 == 0 and rc1 == 0
        assert np.array_equal(got, ref)
    finally:
        s.close()
