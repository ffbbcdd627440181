"""Parity at the full sizes and step counts of the measured workloads, in
the launch configuration bench.py times (the grid's default kernel, the
batch's default configuration), against the FP64 oracle run to the same
step.

  * 512^3 and 4096^2 also from a seeded random state (every component
    nonzero in every cell, so the CPML slabs, the boundaries and every tile
    take part from the first step) for a few steps, element by element;
  * the whole runs (512^3 x 2000, 4096^2 x 10000, 16 problems of the
    256-problem batch x 4000, the 1024^2 adjoint at T = 4000) element by
    element at checkpoints and at the final step, with the probe records
    over the whole run.  The bar at a checkpoint (helpers.assert_run_parity):
    every component's error in the energy norm within 1e-4 of the peak
    energy norm the state reached over the run, and within 1e-4 of its own
    norm while it holds at least 0.1 of that peak; the FP32 build of the
    oracle shows that no FP32 evaluation of the update meets the relative
    bar on a component far below the peak (tests/test_oracle_fp32.py), and
    on 512^3 that the GPU kernels and the CPU FP32 build have the same H
    error;
  * the adjoint's gradient over the whole 256^2 design box against the
    oracle's discrete adjoint, and on 8 seeded cells against FP64 central
    differences of the oracle.
"""
import os

import numpy as np
import pytest

from paper_2405_00814_amd import workloads as W

from helpers import (assert_parity, assert_run_parity, energy_rel_l2, energy_weights, fields_of, log, progress,
                     rel_l2, run_oracle_tracked)

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _random_state(pb, seed):
    rng = np.random.default_rng(seed)
    return {f: rng.standard_normal(pb.shape).astype(np.float32) for f in fields_of(pb)}


def _gpu_from_state(pb, st, steps, kernel=None):
    from paper_2405_00814_amd.sim import Sim
    s = Sim.from_problem(pb)
    if kernel is not None:
        s.set_kernel(*kernel)
    cfg = s.get_kernel()
    for f, a in st.items():
        s.set_field(f, a)
    s.step(steps)
    got = {f: s.get_field(f) for f in st}
    rec = s.probe()
    s.close()
    return got, rec, cfg


def _oracle_from_state(pb, st, steps):
    from oracle import oracle as O
    o = O.for_problem(pb)
    o.set_state({f: a.astype(np.float64) for f, a in st.items()})
    rec = o.run(steps)
    ref = {f: getattr(o, f) for f in st}
    return ref, rec


def test_full_yee3d_512_short_run_vs_oracle():
    pb = W.yee3d(512, steps=6, seed=0)
    st = _random_state(pb, 11)
    log("yee3d 512^3: bench kernel, random state, 6 steps")
    got, rec, cfg = _gpu_from_state(pb, st, 6)
    log("kernel", cfg)
    assert cfg["variant"] == 3 and cfg["tile"][1] == 0  # two steps per pass, slab tiles included
    ref, rrec = _oracle_from_state(pb, st, 6)
    errs = {f: rel_l2(got[f], ref[f]) for f in got}
    log("rel-L2", {f: "%.2e" % e for f, e in errs.items()}, "probes %.2e" % rel_l2(rec, rrec))
    assert_parity(got, ref, TOL, "yee3d 512^3")
    assert rel_l2(rec, rrec) <= TOL
    # every plane, including the CPML slabs and the x/y/z ends
    for f in ("ex", "hz"):
        d = np.abs(got[f].astype(np.float64) - ref[f])
        plane = d.max(axis=(1, 2)) / np.abs(ref[f]).max()
        assert plane.max() <= 1e-4, (f, int(plane.argmax()))


def _log_errs(tag, errs):
    progress(tag, " ".join("%s rel %.2e (energy/peak %.2e, share %.2g)" % (f, *v) for f, v in errs.items()))


def test_full_yee3d_512_2000_steps_vs_oracle():
    """The headline workload, 512^3 x 2000 steps with its Gaussian source,
    against the oracle at steps 500, 1000 and 2000."""
    from oracle import oracle as O
    from paper_2405_00814_amd.sim import Sim
    pb = W.yee3d(512, steps=2000, seed=0)
    checks = (500, 1000, 2000)
    s = Sim.from_problem(pb)
    o = O.for_problem(pb)
    w = energy_weights(pb)
    done, recs, peak = 0, [], 0.0
    for c in checks:
        progress("yee3d 512^3: GPU to step", c)
        s.step(c - done)
        got = {f: s.get_field(f) for f in fields_of(pb)}

        rec, pk, _ = run_oracle_tracked(o, c - done, 100, w, tag="yee3d 512^3 from step %d" % done)
        recs.append(rec)
        peak = max(peak, pk)
        done = c
        ref = {f: getattr(o, f) for f in fields_of(pb)}
        errs = assert_run_parity(got, ref, peak, w, TOL, "yee3d 512^3 step %d" % c)
        _log_errs("step %d" % c, errs)
        progress("step %d energy-norm rel-L2 %.2e" % (c, energy_rel_l2(got, ref, pb)))
        for f in ("ex", "ey", "ez"):  # the static E of the Gaussian holds the energy
            assert errs[f][2] >= 0.1, f
        del got, ref
    assert s.get_kernel()["variant"] == 3 and s.check_finite()
    rec, rrec = s.probe(), np.concatenate(recs, axis=1)
    s.close()
    progress("probes rel-L2 %.2e" % rel_l2(rec, rrec))
    assert rec.shape == rrec.shape
    # the probes lie in the far field (signals 1e-6..3e-5 V/m) of a source
    # whose static near field is of order 1: their records carry the FP32
    # rounding of the run; the FP32 build of the oracle on this workload
    # misses the FP64 record by 7.8e-4 (per probe 2e-5..9e-4), the GPU by
    # 8.4e-4 (test_full_yee3d_probe_floor_fp32_build)
    assert rel_l2(rec, rrec) <= 2e-3


@pytest.mark.skipif(os.environ.get("GEMFDTD_FULL_FP32") != "1",
                    reason="about 7 min of host time (the FP64 and FP32 oracles at 512^3 x 2000); "
                           "set GEMFDTD_FULL_FP32=1")
def test_full_yee3d_probe_floor_fp32_build():
    """The probe records of the headline workload against the FP64 oracle,
    for the GPU and for the FP32 build of the oracle (the oracle's own code
    in single precision, run in chunks): the GPU's error per probe is within
    1.5x of the FP32 build's (measured: all probes 8.4e-4 GPU, 7.8e-4 FP32
    build)."""
    from oracle import oracle as O
    from paper_2405_00814_amd.sim import Sim
    pb = W.yee3d(512, steps=2000, seed=0)
    s = Sim.from_problem(pb)
    s.step(2000)
    g = s.probe().astype(np.float64)
    s.close()
    o32 = O.for_problem(pb)
    recs32 = []
    for k in range(0, 2000, 100):
        f32, r = O.run_fp32(o32, 100)
        o32.set_state({n: v.astype(np.float64) for n, v in f32.items()})
        o32.n += 100
        recs32.append(r)
        progress("  fp32 build: step", k + 100)
    del o32, f32
    r32 = np.concatenate(recs32, axis=1).astype(np.float64)
    o = O.for_problem(pb)
    ref, _, _ = run_oracle_tracked(o, 2000, 100, energy_weights(pb), tag="fp64")
    for p in range(len(ref)):
        eg = rel_l2(g[p], ref[p])
        ec = rel_l2(r32[p], ref[p])
        log("probe %d: gpu %.2e fp32 build %.2e" % (p, eg, ec))
        assert eg <= 1.5 * ec + 1e-5, p


def test_full_dielectric2d_4096():
    pb = W.dielectric2d(4096, steps=8, seed=0)
    st = _random_state(pb, 12)
    log("dielectric2d 4096^2: bench kernel, random state, 8 steps")
    got, rec, cfg = _gpu_from_state(pb, st, 8)
    log("kernel", cfg)
    assert cfg["variant"] == 3
    ref, rrec = _oracle_from_state(pb, st, 8)
    assert_parity(got, ref, TOL, "dielectric2d 4096^2")
    assert rel_l2(rec, rrec) <= TOL
    # the whole 10000 steps against the oracle at steps 2500, 5000, 10000
    from oracle import oracle as O
    from paper_2405_00814_amd.sim import Sim
    pb = W.dielectric2d(4096, steps=10000, seed=0)
    s = Sim.from_problem(pb)
    o = O.for_problem(pb)
    w = energy_weights(pb)
    done, recs, peak = 0, [], 0.0
    for c in (2500, 5000, 10000):
        progress("dielectric2d 4096^2: GPU and oracle to step", c)
        s.step(c - done)
        got = {f: s.get_field(f) for f in fields_of(pb)}
        rec, pk, _ = run_oracle_tracked(o, c - done, 250, w, tag="dielectric2d 4096^2 from step %d" % done)
        recs.append(rec)
        peak = max(peak, pk)
        done = c
        errs = assert_run_parity(got, {f: getattr(o, f) for f in got}, peak, w, TOL,
                                 "dielectric2d 4096^2 step %d" % c)
        _log_errs("step %d" % c, errs)
    assert s.get_kernel()["variant"] == 3 and s.check_finite()
    rec, rrec = s.probe(), np.concatenate(recs, axis=1)
    s.close()
    progress("probes rel-L2 %.2e" % rel_l2(rec, rrec))
    assert rel_l2(rec, rrec) <= TOL


def test_full_batch_256_4000_steps_sampled():
    """The 256-problem batch in its default configuration for 4000 steps;
    its 4 smallest, 4 largest and 8 seeded other problems against the oracle
    at steps 1000 and 4000, with their probe records."""
    from oracle import oracle as O
    from paper_2405_00814_amd.sim import Batch
    probs = W.batch2d(count=256, steps=4000, seed=0)
    order = sorted(range(len(probs)), key=lambda q: probs[q].cells)
    rest = order[4:-4]
    rng = np.random.default_rng(3)
    sample = order[:4] + order[-4:] + [rest[int(k)] for k in rng.choice(len(rest), 8, replace=False)]
    b = Batch(probs)
    log("batch: 256 problems, to step 1000")
    b.step(1000)
    mid = {q: {f: b.get_field(q, f) for f in ("ez", "hx", "hy")} for q in sample}
    log("batch: to step 4000")
    b.step(3000)
    for q in sample:
        pb = probs[q]
        log("batch problem", q, pb.shape)
        o = O.for_problem(pb)
        w = energy_weights(pb)
        r1, peak, _ = run_oracle_tracked(o, 1000, 200, w)
        errs = assert_run_parity(mid[q], {f: getattr(o, f) for f in mid[q]}, peak, w, TOL,
                                 "batch[%d] step 1000" % q)
        _log_errs("  step 1000", errs)
        r2, pk, _ = run_oracle_tracked(o, 3000, 200, w)
        progress("  batch[%d] %s: oracle done" % (q, pb.shape))
        peak = max(peak, pk)
        rrec = np.concatenate([r1, r2], axis=1)
        got = {f: b.get_field(q, f) for f in ("ez", "hx", "hy")}
        errs = assert_run_parity(got, {f: getattr(o, f) for f in got}, peak, w, TOL, "batch[%d] step 4000" % q)
        _log_errs("  step 4000", errs)
        rec = b.probe(q)
        progress("  probes rel-L2 %.2e" % rel_l2(rec, rrec))
        assert rec.shape == rrec.shape
        assert rel_l2(rec, rrec) <= TOL
    b.close()


def test_full_adjoint_1024_T4000():
    from oracle import oracle as O
    from paper_2405_00814_amd.sim import Sim
    pb = W.adjoint2d(1024, steps=4000, seed=0)
    i0, i1, j0, j1 = pb.design
    s = Sim.from_problem(pb)
    loss, grad = s.adjoint_eps(pb.steps, pb.window, pb.design)
    g = grad.cpu().numpy().reshape(i1 - i0, j1 - j0)
    s.close()
    assert np.isfinite(g).all()

    def oracle_loss(eps):
        o = O.Oracle2D(pb.shape, pb.dx, pb.dt, eps, pb.sigma, pb.mu_r, pb.npml, pb.cpml)
        o.set_source(pb.source.cell, pb.source.kind, pb.source.params)
        o.set_probes(pb.probes)
        r = o.run(pb.steps)
        return float(np.sum(r[:, pb.window[0]:pb.window[1]] ** 2))

    # the whole design box against the oracle's discrete adjoint
    progress("adjoint 1024^2 T=4000: oracle adjoint over the 256^2 design box")
    o = O.for_problem(pb)
    lref, gref, gmref = o.loss_and_grad(pb.steps, pb.window, pb.design, mu=True)
    eg = rel_l2(g, gref)
    progress("loss gpu %.6e oracle adjoint %.6e; gradient rel-L2 over %d cells %.2e, max |diff| / max |g| %.2e"
        % (loss, lref, gref.size, eg, np.abs(g - gref).max() / np.abs(gref).max()))
    assert abs(loss - lref) <= TOL * abs(lref)
    assert eg <= 1e-3
    del o
    # dL/d mu_r (the H layer's weight) over the same box from one more run
    s = Sim.from_problem(pb)
    lm, ge2, _, gm = s.adjoint_grads(pb.steps, pb.window, pb.design, 0, mu=True)
    gm = gm.cpu().numpy().reshape(gmref.shape)
    s.close()
    progress("mu_r gradient rel-L2 over the box %.2e" % rel_l2(gm, gmref))
    assert lm == loss and np.array_equal(ge2.cpu().numpy().reshape(g.shape), g)
    assert rel_l2(gm, gmref) <= 1e-3
    e0 = pb.eps_r.astype(np.float64)
    l0 = oracle_loss(e0)
    log("loss gpu %.6e oracle %.6e" % (loss, l0))
    assert abs(loss - l0) <= TOL * abs(l0)
    assert abs(l0 - lref) <= 1e-12 * abs(l0)
    rng = np.random.default_rng(8)
    fd, gg = [], []
    for _ in range(8):
        c = (int(rng.integers(i0, i1)), int(rng.integers(j0, j1)))
        vals = []
        for sgn in (+1, -1):
            e = e0.copy()
            e[c] += sgn * 1e-4 * e[c]
            vals.append(oracle_loss(e))
        fd.append((vals[0] - vals[1]) / (2e-4 * e0[c]))
        gg.append(g[c[0] - i0, c[1] - j0])
        progress("  cell", c, "fd %.6e gpu %.6e" % (fd[-1], gg[-1]))
    fd, gg = np.array(fd), np.array(gg)
    assert np.linalg.norm(gg - fd) <= 1e-3 * np.linalg.norm(fd)
