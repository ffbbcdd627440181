"""GPU parity: the HIP stepper (through the C ABI) against the FP64 oracle on
the same seeded inputs.  Bar: every field component and the probe series
within relative L2 1e-4 of the oracle."""
import math

import numpy as np
import pytest

from paper_2405_00814_amd import workloads as W

from helpers import assert_parity, assert_parity_energy, fields_of, log, rel_l2, run_gpu, run_oracle

pytestmark = pytest.mark.gpu
TOL = 1e-4


# ---------------------------------------------------------------------------
# 2D TMz
# ---------------------------------------------------------------------------

def test_cavity128_full_config():
    """128x128 PEC cavity, 1000 steps, Gaussian source, 4 probes."""
    pb = W.cavity2d(128, steps=1000, seed=0)
    ref, rrec = run_oracle(pb, pb.steps)
    for kernel in (None, (1,), (2, (1, 16)), (2, (2, 7)), (2, (4, 64))):
        log("cavity128 kernel", kernel)
        got, rec, cfg = run_gpu(pb, pb.steps, kernel)
        assert_parity(got, ref, TOL, "cavity128 %s" % (cfg,))
        assert rec.shape == rrec.shape
        assert rel_l2(rec, rrec) <= TOL


@pytest.mark.parametrize("shape,V,TX", [
    ((192, 160), 4, 16), ((203, 146), 2, 9), ((131, 97), 1, 32), ((70, 256), 4, 70),
    ((256, 64), 1, 1),
])
def test_dielectric2d_cpml_lossy(shape, V, TX):
    """Random rectangles (eps_r, sigma), 16-cell CPML, Ricker source; ragged
    tiles in x and y."""
    pb = W.dielectric2d(shape[0], ny=shape[1], steps=1500, seed=1, nrect=12, side=(8, 48),
                        npml=16, nprobes=6)
    log("dielectric2d", shape, V, TX)
    ref, rrec = run_oracle(pb, pb.steps)
    got, rec, cfg = run_gpu(pb, pb.steps, (2, (V, TX)))
    assert cfg["variant"] == 2 and cfg["tile"][:2] == (V, TX)
    assert_parity(got, ref, TOL, "dielectric2d %s" % (shape,))
    assert rel_l2(rec, rrec) <= TOL
    got1, rec1, _ = run_gpu(pb, pb.steps, (1,))
    assert_parity(got1, ref, TOL, "dielectric2d ref %s" % (shape,))


def test_cpml_kappa_alpha_and_mu_map():
    pb = W.dielectric2d(96, ny=88, steps=900, seed=2, nrect=8, side=(6, 30), npml=10, nprobes=3)
    pb.cpml = dict(m=3.0, sigma_max=0.0, kappa_max=4.0, alpha_max=0.1, m_alpha=1.0)
    pb.mu_r = np.random.default_rng(5).uniform(1.0, 2.5, pb.shape).astype(np.float32)
    ref, rrec = run_oracle(pb, pb.steps)
    for kernel in ((1,), (2, (4, 16)), (2, (2, 5))):
        got, rec, _ = run_gpu(pb, pb.steps, kernel)
        assert_parity(got, ref, TOL, "kappa/alpha/mu %s" % (kernel,))
        assert rel_l2(rec, rrec) <= TOL


def test_asymmetric_cpml_faces():
    pb = W.dielectric2d(80, ny=100, steps=700, seed=3, nrect=5, side=(6, 20), npml=8, nprobes=2)
    pb.npml = (4, 12, 0, 9)
    ref, _ = run_oracle(pb, pb.steps)
    for kernel in ((1,), (2, (4, 16)), (2, (1, 3))):
        got, _, _ = run_gpu(pb, pb.steps, kernel)
        assert_parity(got, ref, TOL, "asym cpml %s" % (kernel,))


def test_cavity_recurrence_on_gpu():
    """Discrete eigenmode: E^{n+1} + E^{n-1} = 2 cos(w dt) E^n holds on the
    GPU within FP32 rounding."""
    from paper_2405_00814_amd.sim import Sim
    nx, ny = 128, 128
    h = 1e-3
    dt = 0.99 / math.sqrt(2) * h / 299792458.0
    s = Sim((nx, ny), (h, h), dt)
    i = np.arange(nx)[:, None]
    j = np.arange(ny)[None, :]
    m, n = 8, 3
    s.set_field("ez", np.sin(m * math.pi * i / nx) * np.sin(n * math.pi * j / ny))
    s.set_probes("ez", [(37, 91), (64, 64), (100, 30)])
    s.step(300)
    rec = s.probe().astype(np.float64)
    w = 2 * math.asin(299792458.0 * dt / h * math.sqrt(math.sin(m * math.pi / (2 * nx)) ** 2 +
                                                        math.sin(n * math.pi / (2 * ny)) ** 2))
    err = np.abs(rec[:, 2:] + rec[:, :-2] - 2 * math.cos(w) * rec[:, 1:-1]).max()
    assert err / np.abs(rec).max() < 2e-5
    s.close()


def test_chunked_stepping_and_determinism():
    pb = W.dielectric2d(144, ny=128, steps=600, seed=4, nrect=6, side=(6, 30), npml=12, nprobes=3)
    a, ra, _ = run_gpu(pb, pb.steps)
    b, rb, _ = run_gpu(pb, pb.steps, chunks=7)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(ra, rb)


def test_resume_from_fields_bitwise():
    """run(2N) == run(N) -> get_field -> new handle -> set_field -> run(N)
    (PEC cavity: the state is the three fields)."""
    from paper_2405_00814_amd.sim import Sim
    pb = W.cavity2d(128, steps=400, seed=7)
    pb.source = None
    rng = np.random.default_rng(0)
    init = rng.standard_normal(pb.shape).astype(np.float32)
    init[0, :] = 0
    init[:, 0] = 0

    def mk():
        s = Sim.from_problem(pb)
        return s

    s = mk()
    s.set_field("ez", init)
    s.step(400)
    full = {k: s.get_field(k) for k in ("ez", "hx", "hy")}
    s.close()
    s = mk()
    s.set_field("ez", init)
    s.step(200)
    mid = {k: s.get_field(k) for k in ("ez", "hx", "hy")}
    s.close()
    s = mk()
    for k, v in mid.items():
        s.set_field(k, v)
    s.step(200)
    for k in full:
        assert np.array_equal(s.get_field(k), full[k]), k
    s.close()


@pytest.mark.parametrize("case", ["2d_default", "2d_multi", "2d_split_ref", "2d_graph", "3d_default", "3d_two"])
def test_resume_from_saved_state_with_cpml_bitwise(case):
    """run(2N) == run(N) -> fdtd_save_state -> new handle -> fdtd_load_state
    -> run(N), bit for bit in every field and in the probe samples of the
    second half, with a CPML (its auxiliary values are part of the state), a
    source still active across the cut (the step count is part of it), and
    the split-field PML and the graph form."""
    from paper_2405_00814_amd.sim import Sim
    graph = case == "2d_graph"
    if case.startswith("3d"):
        pb = W.yee3d(shape=(40, 36, 48), steps=120, seed=3, nbox=5, side=(3, 10), npml=6, nprobes=3,
                     tau_steps=10.0)
        N = 60
    else:
        pb = W.dielectric2d(140, ny=128, steps=400, seed=6, nrect=5, side=(6, 30), npml=12, nprobes=3)
        if case == "2d_split_ref":
            pb.cpml = dict(split=1)
            pb.sigma = None
            pb.eps_r = np.ones(pb.shape, np.float32)
        N = 200
    kernel = {"2d_multi": (3, (1, 8, 4)), "2d_split_ref": (1,), "3d_two": (3, (4,))}.get(case)

    def mk():
        s = Sim.from_problem(pb, graph=graph)
        if kernel is not None:
            s.set_kernel(*kernel)
        return s

    fields = fields_of(pb)
    s = mk()
    s.step(2 * N)
    full = {k: s.get_field(k) for k in fields}
    rec_full = s.probe()
    s.close()
    s = mk()
    s.step(N)
    st = s.save_state()
    s.close()
    s = mk()
    s.load_state(st)
    assert s.steps_done() == N
    s.step(N)
    for k in fields:
        assert np.array_equal(s.get_field(k), full[k]), (case, k)
    assert np.array_equal(s.probe(), rec_full[:, N:]), case
    assert np.abs(full[fields[0]]).max() > 0
    s.close()
    # a state of another grid is refused and leaves the handle as it was
    other = W.dielectric2d(64, ny=64, steps=10, seed=1, nrect=2, side=(4, 8), npml=8)
    o = Sim.from_problem(other)
    with pytest.raises(Exception):
        o.load_state(np.zeros(o.save_state().size, np.uint8))
    if case == "2d_default":
        with pytest.raises(Exception):
            o.load_state(st[:o.save_state().size])
    o.close()


def test_source_table_and_probe_components():
    from paper_2405_00814_amd.sim import Sim
    from oracle import oracle as O
    pb = W.dielectric2d(64, ny=72, steps=300, seed=8, nrect=3, side=(4, 12), npml=8, nprobes=3)
    tab = np.sin(np.arange(250) * 0.05).astype(np.float32) * np.hanning(250).astype(np.float32)
    s = Sim(pb.shape, pb.dx, pb.dt, pb.eps_r, None, pb.sigma, pb.npml)
    s.set_source("ez", pb.source.cell, 2, table=tab)
    s.set_probes("hy", pb.probes)
    s.step(300)
    rec = s.probe()
    g = {k: s.get_field(k) for k in ("ez", "hx", "hy")}
    s.close()
    o = O.Oracle2D(pb.shape, pb.dx, pb.dt, pb.eps_r, pb.sigma, None, pb.npml)
    o.src = None
    src_i = pb.source.cell[0] * pb.shape[1] + pb.source.cell[1]
    hy_rec = np.zeros((len(pb.probes), 300))
    vals = np.concatenate([tab.astype(np.float64), np.zeros(50)])
    for n in range(300):
        o.run(1)
        o.ez.ravel()[src_i] += vals[n]
        hy_rec[:, n] = [o.hy[tuple(c)] for c in pb.probes]
    assert_parity(g, {"ez": o.ez, "hx": o.hx, "hy": o.hy}, TOL, "table source")
    assert rel_l2(rec, hy_rec) <= TOL


def test_errors_on_device_handle():
    from paper_2405_00814_amd.sim import Sim
    from paper_2405_00814_amd import _lib as L
    pb = W.cavity2d(32, steps=10, seed=0)
    s = Sim.from_problem(pb)
    with pytest.raises(L.FdtdError) as e:
        s.set_source("ez", (0, 5), 0, (1.0, 1e-11, 1e-11))   # on the PEC wall
    assert e.value.code == L.FDTD_EINVAL
    with pytest.raises(L.FdtdError):
        s.set_probes("ez", [(32, 3)])                          # outside
    with pytest.raises(L.FdtdError):
        s.set_source("hx", (5, 5), 0, (1.0, 1e-11, 1e-11))   # not an E component
    assert s.check_finite()
    bad = np.zeros(pb.shape, np.float32)
    bad[3, 4] = np.nan
    s.set_field("hx", bad)
    assert not s.check_finite()
    s.reset()
    assert s.check_finite() and s.steps_done() == 0
    s.close()


# ---------------------------------------------------------------------------
# 3D Yee
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape,V,TX,npml", [
    ((40, 36, 30), 2, 0, (6,) * 6), ((33, 29, 70), 2, 5, (5, 3, 0, 7, 4, 2)),
    ((30, 26, 20), 4, 0, (6,) * 6), ((24, 21, 64), 4, 3, (0, 0, 0, 0, 6, 6)),
    ((26, 23, 300), 4, 0, (6,) * 6), ((21, 19, 45), 1, 0, (6,) * 6),
    ((44, 70, 128), 4, 0, (3, 5, 4, 6, 0, 0)), ((36, 41, 132), 2, 8, (4, 4, 7, 2, 5, 3)),
    ((30, 37, 256), 1, 1, (5, 0, 0, 5, 8, 8)), ((28, 90, 96), 4, 64, (4, 4, 20, 20, 40, 40)),
    ((20, 24, 96), 4, 2, (2, 2, 2, 2, 14, 3)),
])
def test_yee3d_cpml_boxes(shape, V, TX, npml):
    """Zero-mean (Ricker) source: every component within 1e-4.  The slab
    widths (some asymmetric or zero) make both the slab and the interior
    workgroups of the fused kernel run."""
    pb = W.yee3d(shape=shape, steps=260, seed=1, nbox=10, side=(3, 12), npml=min(npml[:4]) + 2,
                 nprobes=5, tau_steps=8.0)
    pb.npml = tuple(npml)
    # source at the centre of the region clear of every slab
    pb.source.cell = tuple((npml[2 * a] + shape[a] - npml[2 * a + 1]) // 2 for a in range(3))
    pb.source.kind = W.SRC_RICKER
    pb.source.params = (1.0, 40 * pb.dt, 1.0 / (20 * pb.dt))
    log("yee3d", shape, V, TX, npml)
    ref, rrec = run_oracle(pb, pb.steps)
    got, rec, cfg = run_gpu(pb, pb.steps, (2, (V, 0, TX)))
    assert tuple(cfg["tile"]) == (V, 0, TX, 0)
    assert cfg["variant"] == 2
    assert_parity(got, ref, TOL, "yee3d fused %s" % (shape,))
    assert rel_l2(rec, rrec) <= TOL
    got1, rec1, _ = run_gpu(pb, pb.steps, (1,))
    assert_parity(got1, ref, TOL, "yee3d ref %s" % (shape,))
    assert rel_l2(rec1, rrec) <= TOL


def test_yee3d_kernel_config_rejected():
    from paper_2405_00814_amd._lib import FdtdError
    from paper_2405_00814_amd.sim import Sim
    pb = W.yee3d(shape=(16, 16, 30), steps=10, seed=0, nbox=2, side=(2, 4), npml=3, nprobes=1,
                 tau_steps=4.0)
    s = Sim.from_problem(pb)
    for bad in ((4,), (3,), (2, 16), (2, 4), (1, 0, 0, 5), (1, 0, -1), (1, 0, 5000)):
        with pytest.raises(FdtdError):
            s.set_kernel(2, bad)
    s.set_kernel(2, (2,))
    assert s.get_kernel()["tile"] == (2, 0, 0, 0)
    s.close()


def test_yee3d_gaussian_source_energy_norm():
    """The headline source (Gaussian, nonzero mean) leaves a static curl-free
    E; the state is compared in the energy norm, E per component."""
    pb = W.yee3d(shape=(48, 44, 40), steps=600, seed=3, nbox=12, side=(4, 14), npml=8, nprobes=6,
                 tau_steps=12.0)
    ref, rrec = run_oracle(pb, pb.steps)
    for kernel in ((1,), (2, (4,)), (2, (2,)), (2, (1,))):
        got, rec, _ = run_gpu(pb, pb.steps, kernel)
        e = assert_parity_energy(got, ref, pb, TOL, "yee3d gaussian %s" % (kernel,))
        log("gaussian", kernel, "energy rel-L2 %.2e" % e,
            {k: "%.1e" % rel_l2(got[k], ref[k]) for k in ref})
        assert rel_l2(rec, rrec) <= TOL


def test_yee3d_long_z_and_lossy_mu():
    """nz > 256 (two z values per thread), lossy media, mu_r map, x-directed
    source, Hz probes."""
    pb = W.yee3d(shape=(14, 12, 300), steps=120, seed=2, nbox=4, side=(2, 20), npml=4,
                 nprobes=4, tau_steps=6.0)
    rng = np.random.default_rng(3)
    pb.sigma = rng.uniform(0, 0.05, pb.shape).astype(np.float32)
    pb.mu_r = rng.uniform(1, 2, pb.shape).astype(np.float32)
    pb.source.component = "ex"
    pb.probe_component = "hz"
    ref, rrec = run_oracle(pb, pb.steps)
    for kernel in ((1,), (2, (2,)), (2, (4,))):
        got, rec, _ = run_gpu(pb, pb.steps, kernel)
        assert_parity(got, ref, TOL, "yee3d lossy %s" % (kernel,))
        assert rel_l2(rec, rrec) <= TOL


def test_yee3d_tm_mode_recurrence_on_gpu():
    from paper_2405_00814_amd.sim import Sim
    nx, ny, nz = 40, 32, 24
    h = 1e-3
    dt = 0.99 / math.sqrt(3) * h / 299792458.0
    s = Sim((nx, ny, nz), (h, h, h), dt)
    i = np.arange(nx)[:, None, None]
    j = np.arange(ny)[None, :, None]
    m, n = 3, 2
    s.set_field("ez", np.sin(m * math.pi * i / nx) * np.sin(n * math.pi * j / ny) * np.ones((1, 1, nz)))
    s.set_probes("ez", [(7, 5, 2), (20, 11, 13)])
    s.step(200)
    rec = s.probe().astype(np.float64)
    w = 2 * math.asin(299792458.0 * dt / h * math.sqrt(math.sin(m * math.pi / (2 * nx)) ** 2 +
                                                        math.sin(n * math.pi / (2 * ny)) ** 2))
    err = np.abs(rec[:, 2:] + rec[:, :-2] - 2 * math.cos(w) * rec[:, 1:-1]).max()
    assert err / np.abs(rec).max() < 2e-5
    s.close()


def test_step_profile_matches_step():
    """Per-launch profiling advances the state exactly like fdtd_step, and its
    launches cover every cell once."""
    from paper_2405_00814_amd.sim import Sim
    pb = W.yee3d(shape=(40, 44, 96), steps=30, seed=4, nbox=6, side=(3, 10), npml=6, nprobes=3,
                 tau_steps=6.0)
    a = Sim.from_problem(pb)
    b = Sim.from_problem(pb)
    a.step(7)
    a.step(23)
    b.step(7)
    prof = b.step_profile(23)
    assert sum(p["cells"] for p in prof) == pb.cells
    # interior launch (z-slab code) and x/y-slab launch; every psi value once
    assert [p["cpml"] for p in prof] == [1, 2]
    sx, sy, sz = 12, 12, 12
    nx, ny, nz = pb.shape
    assert sum(p["psi"] for p in prof) == 4 * (sx * ny * nz + nx * sy * nz + nx * ny * sz)
    assert all(p["ms"] > 0 and p["launches"] == 1 for p in prof)
    assert b.steps_done() == 30
    for f in ("ex", "ey", "ez", "hx", "hy", "hz"):
        assert np.array_equal(a.get_field(f), b.get_field(f)), f
    assert np.array_equal(a.probe(), b.probe())
    a.set_kernel(1)
    prof = a.step_profile(2)
    assert len(prof) == 1 and prof[0]["cpml"] == -1 and prof[0]["cells"] == pb.cells
    assert prof[0]["psi"] == 4 * (sx * ny * nz + nx * sy * nz + nx * ny * sz)
    a.close()
    b.close()


@pytest.mark.parametrize("kind", ["sine", "modgauss"])
def test_sine_and_modulated_gaussian_sources(kind):
    """The sinusoidal (with its turn-on) and modulated-Gaussian sources in
    2D and 3D, through the single-step and the multi-step kernels."""
    pb = W.dielectric2d(120, ny=104, steps=420, seed=6, nrect=6, side=(8, 30), npml=10, nprobes=4)
    if kind == "sine":
        pb.source.kind, pb.source.params = W.SRC_SINE, (1.0, 1.2e9, 0.8e-9)
    else:
        pb.source.kind, pb.source.params = W.SRC_MODGAUSS, (1.0, 1.0e-9, 0.3e-9, 1.5e9)
    ref, rrec = run_oracle(pb, pb.steps)
    for kernel in ((2, (1, 4)), (3, (1, 4, 4)), (3, (2, 8, 2))):
        got, rec, _ = run_gpu(pb, pb.steps, kernel)
        assert_parity(got, ref, TOL, "2d %s %s" % (kind, kernel))
        assert rel_l2(rec, rrec) <= TOL
    pb3 = W.yee3d(shape=(36, 34, 48), steps=200, seed=4, nbox=8, side=(3, 10), npml=6, nprobes=4,
                  tau_steps=8.0)
    if kind == "sine":
        pb3.source.kind, pb3.source.params = W.SRC_SINE, (1.0, 30e9, 0.1e-9)
        pb3.source.component = "ey"
    else:
        pb3.source.kind, pb3.source.params = W.SRC_MODGAUSS, (1.0, 0.15e-9, 0.05e-9, 30e9)
    ref, rrec = run_oracle(pb3, pb3.steps)
    for kernel in ((2, (4,)), (3, (4,))):
        got, rec, _ = run_gpu(pb3, pb3.steps, kernel)
        assert_parity(got, ref, TOL, "3d %s %s" % (kind, kernel))
        assert rel_l2(rec, rrec) <= TOL


def test_line_and_box_sources():
    """Line sources (the box [cell, hi) driven with one waveform) along y and
    x in 2D, through the reference, fused, multi-step and graph forms; in 3D
    along z across the seam between a row's two wavefronts (nz > 256), along
    x across x chunks, and a plane, through the single- and two-step
    kernels."""
    import dataclasses
    base = W.dielectric2d(120, ny=104, steps=300, seed=6, nrect=6, side=(8, 30), npml=10, nprobes=4)
    for lo, hi in (((50, 20), (51, 80)), ((15, 60), (100, 61))):
        pb = dataclasses.replace(base, source=dataclasses.replace(base.source, cell=lo, hi=hi))
        ref, rrec = run_oracle(pb, pb.steps)
        for kernel in ((1,), (2, (1, 4)), (3, (1, 4, 4)), (3, (2, 8, 2))):
            got, rec, _ = run_gpu(pb, pb.steps, kernel)
            assert_parity(got, ref, TOL, "2d line %s %s" % (lo, kernel))
            assert rel_l2(rec, rrec) <= TOL
        got, rec, _ = run_gpu(pb, pb.steps, graph=True)
        assert_parity(got, ref, TOL, "2d line %s graph" % (lo,))
        assert rel_l2(rec, rrec) <= TOL
    base3 = W.yee3d(shape=(30, 28, 300), steps=120, seed=4, nbox=6, side=(3, 10), npml=5, nprobes=4,
                    tau_steps=8.0)
    base3.source.kind, base3.source.params = W.SRC_RICKER, (1.0, 40 * base3.dt, 1.0 / (20 * base3.dt))
    for comp, lo, hi in (("ez", (14, 12, 200), (15, 13, 290)), ("ex", (6, 14, 150), (24, 15, 151)),
                         ("ey", (10, 8, 140), (20, 18, 141))):
        src = dataclasses.replace(base3.source, cell=lo, hi=hi, component=comp)
        pb3 = dataclasses.replace(base3, source=src)
        ref, rrec = run_oracle(pb3, pb3.steps)
        for kernel in ((1,), (2, (4,)), (3, (4, 0, 5)), (3, (4, 1, 5))):
            got, rec, _ = run_gpu(pb3, pb3.steps, kernel)
            # a line or plane of dipoles leaves the H component along it
            # nearly zero by symmetry (rounding-sized): the state is gated in
            # the energy norm, E per component
            e = assert_parity_energy(got, ref, pb3, TOL, "3d box %s %s %s" % (comp, lo, kernel))
            log("box", comp, kernel, "energy %.1e" % e, {k: "%.1e" % rel_l2(got[k], ref[k]) for k in ref})
            assert rel_l2(rec, rrec) <= TOL


def test_dft_monitor():
    """Frequency-domain monitor (running DFT) of an E and an H component in
    2D (the multi-step default, which drops to single steps, and the graph
    form) and 3D, against the oracle's FP64 sums."""
    from paper_2405_00814_amd.sim import Sim
    from oracle import oracle as O
    pb = W.dielectric2d(120, ny=104, steps=360, seed=6, nrect=6, side=(8, 30), npml=10, nprobes=4)
    freqs = [0.5e9, 1.0e9, 1.7e9]
    for comp, lo, hi in (("ez", (20, 15), (90, 70)), ("hy", (0, 0), (120, 104))):
        o = O.for_problem(pb)
        o.set_dft(comp, lo, hi, freqs)
        o.run(pb.steps)
        ref = o.dft["X"]
        for kernel, graph in (((3, (1, 4, 4)), False), (None, True), ((2, (1, 4)), False)):
            s = Sim.from_problem(pb, graph=graph)
            if kernel is not None:
                s.set_kernel(*kernel)
            s.set_dft(comp, lo, hi, freqs)
            s.step(100)
            s.step(pb.steps - 100)
            X, n = s.get_dft()
            assert n == pb.steps
            e = float(np.linalg.norm(X - ref) / np.linalg.norm(ref))
            log("dft 2d", comp, kernel, graph, "%.2e" % e)
            assert e <= TOL, (comp, kernel, graph, e)
            s.close()
    pb3 = W.yee3d(shape=(36, 34, 48), steps=160, seed=4, nbox=8, side=(3, 10), npml=6, nprobes=4,
                  tau_steps=8.0)
    pb3.source.kind, pb3.source.params = W.SRC_RICKER, (1.0, 40 * pb3.dt, 1.0 / (20 * pb3.dt))
    f3 = [1.0 / (20 * pb3.dt), 1.0 / (40 * pb3.dt)]
    for comp, lo, hi in (("ey", (4, 5, 6), (30, 29, 40)), ("hz", (10, 10, 0), (26, 24, 48))):
        o = O.for_problem(pb3)
        o.set_dft(comp, lo, hi, f3)
        o.run(pb3.steps)
        s = Sim.from_problem(pb3)
        s.set_kernel(3, (4,))
        s.set_dft(comp, lo, hi, f3)
        s.step(pb3.steps)
        X, n = s.get_dft()
        e = float(np.linalg.norm(X - o.dft["X"]) / np.linalg.norm(o.dft["X"]))
        log("dft 3d", comp, "%.2e" % e)
        assert n == pb3.steps and e <= TOL
        s.close()


def test_dft_monitor_rules():
    from paper_2405_00814_amd._lib import FdtdError
    from paper_2405_00814_amd.sim import Sim
    pb = W.dielectric2d(64, ny=48, steps=20, seed=1, nrect=2, side=(4, 10), npml=6, nprobes=1)
    s = Sim.from_problem(pb)
    with pytest.raises(FdtdError):
        s.get_dft()                                    # none set
    for lo, hi, fr in (((0, 0), (65, 10), [1e9]), ((5, 5), (5, 9), [1e9]), ((0, 0), (4, 4), [-1.0]),
                       ((0, 0), (4, 4), [1e9] * 17)):
        with pytest.raises(FdtdError):
            s.set_dft("ez", lo, hi, fr)
    s.set_field("ez", np.random.default_rng(0).standard_normal(pb.shape).astype(np.float32))
    s.set_dft("ez", (2, 2), (30, 20), [1e9, 2e9])
    s.step(10)
    X, n = s.get_dft()
    assert n == 10 and X.shape == (2, 28, 18) and np.abs(X).max() > 0
    with pytest.raises(FdtdError):
        s.step_profile(4)
    with pytest.raises(FdtdError):
        s.autotune(4)
    s.reset()
    X, n = s.get_dft()
    assert n == 0 and np.abs(X).max() == 0
    s.set_dft("ez", (2, 2), (30, 20), [])              # removed
    with pytest.raises(FdtdError):
        s.get_dft()
    s.step_profile(4)
    s.close()
    # samples are summed in batches of steps: reading the sums between
    # uneven chunks (partial batches) gives the sums of one run
    st0 = np.random.default_rng(1).standard_normal(pb.shape).astype(np.float32)
    out = []
    for chunks in ((37,), (5, 13, 19), (1, 7, 8, 21)):
        s = Sim.from_problem(pb)
        s.set_field("ez", st0)
        s.set_dft("hy", (1, 3), (40, 44), [0.7e9, 3e9, 0.0])
        for c in chunks:
            s.step(c)
            X, n = s.get_dft()
        assert n == 37
        out.append(X)
        s.close()
    for X in out[1:]:
        assert np.abs(X - out[0]).max() <= 1e-12 * np.abs(out[0]).max()


def test_sar_layered():
    """Absorption rate in the layered lossy case (the paper's tissue setup,
    Sec. V-B, with synthetic layer properties) from the GPU monitor against
    the oracle's, sigma |X|^2 / (2 rho norm^2) per frequency, without and
    with a source-spectrum norm; zero in the lossless air rows; the rules."""
    from paper_2405_00814_amd._lib import FdtdError
    from paper_2405_00814_amd.sim import Sim
    from oracle import oracle as O
    pb = W.layered2d(160, ny=120, steps=600, seed=2)
    f0 = pb.source.params[3]
    freqs = [0.6 * f0, f0, 1.4 * f0]
    lo, hi = (30, 20), (140, 100)
    box = (slice(lo[0], hi[0]), slice(lo[1], hi[1]))
    o = O.for_problem(pb)
    o.set_dft("ez", lo, hi, freqs)
    o.run(pb.steps)
    air = pb.sigma[box] == 0
    assert air.any() and (~air).any()
    for kernel in (None, (2, (1, 4)), (1,)):
        s = Sim.from_problem(pb)
        if kernel is not None:
            s.set_kernel(*kernel)
        s.set_dft("ez", lo, hi, freqs)
        s.step(pb.steps)
        for nm in (None, [2.0, 0.5, 3.0]):
            got = s.dft_sar(pb.rho[box], nm)
            ref = O.sar(o.dft["X"], pb.sigma[box], pb.rho[box], nm)
            e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            log("sar", kernel, nm, "rel-L2 %.2e" % e, "max %.3e" % ref.max())
            assert e <= TOL, (kernel, nm, e)
            assert np.all(got[:, air] == 0) and got.max() > 0
        with pytest.raises(FdtdError):
            s.dft_sar(np.zeros_like(pb.rho[box]))            # rho must be > 0
        with pytest.raises(FdtdError):
            s.dft_sar(pb.rho[box], [1.0, -1.0, 1.0])         # norm must be > 0
        s.set_dft("hx", lo, hi, freqs)
        with pytest.raises(FdtdError):
            s.dft_sar(pb.rho[box])                            # an H monitor
        s.set_dft("ez", lo, hi, [])
        with pytest.raises(FdtdError):
            s.dft_sar(np.zeros(0, np.float32))                # no monitor
        s.close()


def test_split_field_pml():
    """The paper's split-field PML (Sec. III-C): the reference kernels and the
    4-nodes-per-cell explicit graph against the split-field oracle; the
    rules that keep it to those forms and to a vacuum layer."""
    from paper_2405_00814_amd._lib import FdtdError
    from paper_2405_00814_amd.sim import Batch, Sim
    pb = W.dielectric2d(120, ny=104, steps=400, seed=6, nrect=6, side=(8, 30), npml=12, nprobes=4)
    pb.cpml = dict(pb.cpml, split=1)
    pb.npml = (12, 9, 10, 12)
    ref, rrec = run_oracle(pb, pb.steps)
    got, rec, cfg = run_gpu(pb, pb.steps)
    assert cfg["variant"] == 1
    assert_parity(got, ref, TOL, "split pml implicit")
    assert rel_l2(rec, rrec) <= TOL
    got, rec, _ = run_gpu(pb, pb.steps, graph=True)
    assert_parity(got, ref, TOL, "split pml graph")
    assert rel_l2(rec, rrec) <= TOL
    # a line source through the layer edge and a seeded initial Ez
    s = Sim.from_problem(pb)
    for bad in ((2, (1, 4)), (3, (1, 4, 4))):
        with pytest.raises(FdtdError):
            s.set_kernel(*bad)
    with pytest.raises(FdtdError):   # material in the layer
        s.set_material((0, 0), (4, 4), np.full((4, 4), 2.0, np.float32))
    s.close()
    g = Sim.from_problem(pb, graph=True)
    with pytest.raises(FdtdError):
        g.set_dft("ez", (20, 20), (30, 30), [1e9])
    g.close()
    with pytest.raises(FdtdError):
        Batch([pb])
    pb3 = W.yee3d(shape=(16, 16, 16), steps=4, seed=0, nbox=1, side=(2, 4), npml=3, nprobes=1)
    pb3.cpml = dict(pb3.cpml, split=1)
    with pytest.raises(FdtdError):
        Sim.from_problem(pb3)


def test_gaussian_h_error_is_the_fp32_floor():
    """The headline scene's 3D Gaussian source at 192^3 for 600 steps: the
    GPU kernels (two-step default, fused single step, two-pass reference)
    and the FP32 build of the oracle (the oracle's own code in single
    precision) miss the relative 1e-4 bar on H alike, against the FP64
    oracle; the GPU's H error is within 2x of the CPU FP32 build's and every
    component's error is far inside 1e-4 of the peak energy norm."""
    from oracle import oracle as O
    from paper_2405_00814_amd.sim import Sim
    from helpers import energy_weights, run_errors, run_oracle_tracked
    pb = W.yee3d(shape=(192, 192, 192), steps=600, seed=0, nbox=24, side=(3, 36), npml=12)
    w = energy_weights(pb)
    o = O.for_problem(pb)
    f32, _ = O.run_fp32(o, 600)
    rec, peak, _ = run_oracle_tracked(o, 600, 50, w)
    ref = {f: getattr(o, f) for f in O.F3}
    cpu = run_errors({f: f32[f] for f in O.F3}, ref, peak, w)
    log("cpu fp32", {f: "%.1e/%.1e" % v[:2] for f, v in cpu.items()})
    assert max(cpu[f][0] for f in ("hx", "hy", "hz")) > TOL  # the relative bar is out of FP32 reach on H
    for kernel in (None, (2, (4,)), (1,)):
        got, grec, cfg = run_gpu(pb, 600, kernel)
        e = run_errors(got, ref, peak, w)
        log("gpu", cfg["variant"], {f: "%.1e/%.1e" % v[:2] for f, v in e.items()})
        for f in O.F3:
            assert e[f][1] <= 1e-5, (cfg, f, e[f])
            assert e[f][1] <= 2 * cpu[f][1] + 1e-8, (cfg, f, e[f], cpu[f])
        for f in ("ex", "ey", "ez"):
            assert e[f][0] <= TOL, (cfg, f)
        assert rel_l2(grec, rec) <= TOL


def test_stream_copy_kernel():
    """The library's copy kernel (the bandwidth reference of the bench):
    every byte copied for sizes that leave a partial last block, on a torch
    stream, and nothing written past the end."""
    import ctypes as C
    import torch
    from paper_2405_00814_amd import _lib
    L = _lib.load()
    st = torch.cuda.Stream()
    for n in (4, 256 * 4 + 4, 3 * 1024 * 1024 + 12):  # floats; bytes a multiple of 16
        a = torch.randn(n, device="cuda")
        b = torch.full((n + 64,), -7.0, device="cuda")
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            rc = L.fdtd_stream_copy(C.c_void_p(b.data_ptr()), C.c_void_p(a.data_ptr()), n * 4,
                                    C.c_void_p(st.cuda_stream))
        assert rc == 0
        st.synchronize()
        assert torch.equal(b[:n], a)
        assert torch.all(b[n:] == -7.0)

