"""GPU parity of the 2D multi-step stepper (kernel variant 3: TB = 2 or 4
leapfrog steps per pass, one wavefront per tile, halo columns and rows
recomputed).  Bar: every field and the probe series within relative L2 1e-4
of the FP64 oracle, and the single-step fused stepper's result within 1e-5
(the same formulas; the compiler may contract a product and a sum into one
fused multiply-add differently in the two kernels, so last bits differ)."""
import numpy as np
import pytest

from paper_2405_00814_amd import workloads as W

from helpers import assert_parity, log, rel_l2, run_gpu, run_oracle

pytestmark = pytest.mark.gpu
TOL = 1e-4


# ragged shapes; tiles of 1 .. 64 rows; slabs of both kinds in the cones;
# odd row lengths (one column per lane)
CASES = [
    ((192, 160), 4, 2, 16, 601), ((203, 146), 2, 2, 9, 600), ((131, 96), 2, 4, 32, 603),
    ((70, 256), 4, 4, 70, 602), ((256, 64), 2, 4, 1, 301), ((300, 520), 4, 2, 3, 400),
    ((203, 147), 1, 4, 9, 600), ((97, 251), 1, 2, 33, 401), ((130, 129), 1, 4, 16, 500),
]


@pytest.mark.parametrize("shape,V,TB,TX,steps", CASES)
def test_tb2d_dielectric_cpml_lossy(shape, V, TB, TX, steps):
    pb = W.dielectric2d(shape[0], ny=shape[1], steps=steps, seed=1, nrect=12, side=(8, 48),
                        npml=16, nprobes=6)
    log("tb2d", shape, V, TB, TX, steps)
    ref, rrec = run_oracle(pb, steps)
    got, rec, cfg = run_gpu(pb, steps, (3, (V, TX, TB)))
    assert cfg["variant"] == 3 and cfg["tile"][:3] == (V, TX, TB)
    assert_parity(got, ref, TOL, "tb2d %s" % (shape,))
    assert rel_l2(rec, rrec) <= TOL
    one, rec1, _ = run_gpu(pb, steps, (2, (2 if shape[1] % 2 == 0 else 1, 4)))
    same = all(np.array_equal(got[k], one[k]) for k in got)
    log("  bitwise equal to the single-step stepper:", same,
        {k: "%.1e" % rel_l2(got[k], one[k]) for k in got})
    for k in got:
        assert rel_l2(got[k], one[k]) <= 1e-5, k
    assert rel_l2(rec, rec1) <= 1e-5


def test_tb2d_mu_map_kappa_alpha_asymmetric():
    pb = W.dielectric2d(96, ny=88, steps=501, seed=2, nrect=8, side=(6, 30), npml=10, nprobes=3)
    pb.cpml = dict(m=3.0, sigma_max=0.0, kappa_max=4.0, alpha_max=0.1, m_alpha=1.0)
    pb.mu_r = np.random.default_rng(5).uniform(1.0, 2.5, pb.shape).astype(np.float32)
    pb.npml = (4, 12, 0, 9)
    ref, rrec = run_oracle(pb, pb.steps)
    for kernel in ((3, (2, 8, 2)), (3, (4, 5, 4)), (3, (2, 64, 4, 3))):
        got, rec, _ = run_gpu(pb, pb.steps, kernel)
        assert_parity(got, ref, TOL, "tb2d mu %s" % (kernel,))
        assert rel_l2(rec, rrec) <= TOL


def test_tb2d_chunks_sources_probes_at_edges():
    """Source and probes on tile seams, next to slabs and near the walls;
    steps in uneven chunks (remainders run single steps)."""
    pb = W.dielectric2d(130, ny=400, steps=203, seed=4, nrect=6, side=(6, 30), npml=8, nprobes=2)
    ow = 248  # own columns of a V=4, TB=4 strip
    pb.source.cell = (33, ow)
    pb.probes = np.array([(32, ow - 1), (33, ow), (31, 1), (1, 120), (128, 398), (9, 9),
                          (64, 8), (120, 391), (96, ow + 1), (95, ow - 2)], dtype=np.int32)
    ref, rrec = run_oracle(pb, pb.steps)
    for chunks in (1, 5, 13):
        got, rec, _ = run_gpu(pb, pb.steps, (3, (4, 32, 4)), chunks=chunks)
        log("chunks", chunks, {k: "%.1e" % rel_l2(got[k], ref[k]) for k in ref})
        assert_parity(got, ref, TOL, "tb2d chunks %d" % chunks)
        assert rel_l2(rec, rrec) <= TOL


def test_tb2d_cpml_tiles_on_second_stream():
    """The CPML tiles (quarter chunks) run beside the interior tiles on a
    second stream: parity, and the same bits on a second run."""
    pb = W.dielectric2d(700, ny=600, steps=301, seed=7, nrect=10, side=(8, 48), npml=16, nprobes=5)
    ref, rrec = run_oracle(pb, pb.steps)
    for kernel in ((3, (2, 32, 4, 8)), (3, (1, 16, 4, 4))):
        runs = [run_gpu(pb, pb.steps, kernel) for _ in range(2)]
        got, rec, cfg = runs[0]
        assert cfg["tile"] == kernel[1]
        log("tb2d second stream", kernel, {k: "%.1e" % rel_l2(got[k], ref[k]) for k in ref})
        assert_parity(got, ref, TOL, "tb2d second stream %s" % (kernel,))
        assert rel_l2(rec, rrec) <= TOL
        for k in got:
            assert np.array_equal(got[k], runs[1][0][k]), k
        assert np.array_equal(rec, runs[1][1])


def test_tb2d_forked_pass_on_a_torch_stream():
    """The second stream forks from and joins to the simulation's stream,
    whichever it is: on a non-default torch stream the forked passes, in
    uneven chunks, give the bits of the default stream."""
    import torch
    from paper_2405_00814_amd.sim import Sim
    pb = W.dielectric2d(700, ny=600, steps=201, seed=8, nrect=10, side=(8, 48), npml=16, nprobes=5)
    kernel = (3, (2, 32, 4, 8))
    got, rec, _ = run_gpu(pb, pb.steps, kernel)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s = Sim.from_problem(pb)
        s.set_kernel(*kernel)
        for c in (60, 141):
            s.step(c)
        f = {k: s.get_field(k) for k in got}
        r = s.probe()
        s.close()
    for k in got:
        assert np.array_equal(f[k], got[k]), k
    assert np.array_equal(r, rec)


def test_tb2d_cavity_full_config():
    pb = W.cavity2d(128, steps=1000, seed=0)
    ref, rrec = run_oracle(pb, pb.steps)
    for kernel in ((3, (4, 16, 4)), (3, (2, 32, 2))):
        got, rec, _ = run_gpu(pb, pb.steps, kernel)
        assert_parity(got, ref, TOL, "cavity tb2d %s" % (kernel,))
        assert rel_l2(rec, rrec) <= TOL


def test_tb2d_profile_and_rules():
    from paper_2405_00814_amd._lib import FdtdError
    from paper_2405_00814_amd.sim import Sim
    pb = W.dielectric2d(200, ny=300, steps=40, seed=6, nrect=6, side=(6, 30), npml=10, nprobes=3)
    a = Sim.from_problem(pb)
    b = Sim.from_problem(pb)
    for s in (a, b):
        s.set_kernel(3, (4, 16, 4))
    a.step(3)
    a.step(37)
    b.step(3)
    prof = b.step_profile(37)
    assert len(prof) == 1 and prof[0]["steps"] == 4 and prof[0]["cells"] == pb.cells
    assert b.steps_done() == 40
    for f in ("ez", "hx", "hy"):
        assert np.array_equal(a.get_field(f), b.get_field(f)), f
    assert np.array_equal(a.probe(), b.probe())
    for bad in ((3, (4, 16, 3)), (3, (8, 16, 2)), (3, (3, 16, 2)), (3, (4, 16, 2, -1))):
        with pytest.raises(FdtdError):
            a.set_kernel(*bad)
    a.close()
    b.close()
    pb = W.dielectric2d(64, ny=66, steps=10, seed=0, nrect=2, side=(4, 8), npml=4, nprobes=1)
    s = Sim.from_problem(pb)
    with pytest.raises(FdtdError):  # ny % 4 != 0
        s.set_kernel(3, (4, 16, 2))
    s.set_kernel(3, (2, 16, 2))
    s.step(5)
    assert s.check_finite()
    s.close()
    pb = W.dielectric2d(64, ny=67, steps=10, seed=0, nrect=2, side=(4, 8), npml=4, nprobes=1)
    s = Sim.from_problem(pb)
    with pytest.raises(FdtdError):  # ny % 2 != 0
        s.set_kernel(3, (2, 16, 2))
    s.set_kernel(3, (1, 16, 2))
    s.step(10)
    assert s.check_finite() and s.get_kernel()["tile"][0] == 1
    s.close()


@pytest.mark.parametrize("shape,V,TX,TB,G", [((128, 128), 1, 8, 4, 32), ((203, 146), 2, 5, 2, 8),
                                             ((160, 96), 1, 16, 4, 64)])
def test_graph_replay_matches_eager_passes(shape, V, TX, TB, G):
    """Multi-step passes replayed from a captured graph (kernel config tb =
    G steps per replay): the same fields and probe records as the passes
    launched one by one, over calls that start on either buffer set and
    leave remainders, and the oracle's within 1e-4."""
    from paper_2405_00814_amd.sim import Sim
    pb = W.dielectric2d(shape[0], ny=shape[1], steps=0, seed=4, nrect=5, side=(6, 30), npml=12, nprobes=5)
    chunks = (TB, 3 * G + TB, G, 2 * G + 3, 5)
    n = sum(chunks)
    out = []
    for g in (1, G):
        s = Sim.from_problem(pb)
        s.set_kernel(3, (V, TX, TB), tb=g)
        for c in chunks:
            s.step(c)
        assert s.get_kernel()["tb"] == g
        out.append(({k: s.get_field(k) for k in ("ez", "hx", "hy")}, s.probe()))
        ms, launches = s.last_step_time()
        s.close()
    (a, ra), (b, rb) = out
    for k in a:
        assert rel_l2(b[k], a[k]) <= 1e-6, k
    assert rel_l2(rb, ra) <= 1e-6
    ref, rrec = run_oracle(pb, n)
    assert_parity(b, ref, 1e-4, "graph %s" % (shape,))
    assert rel_l2(rb, rrec) <= 1e-4
