"""Shared helpers of the parity tests: run a problem on the HIP library and
on the FP64 oracle with the same seeded inputs, compare."""
import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b.ravel())
    if nb == 0:
        return float(np.linalg.norm(a.ravel()))
    return float(np.linalg.norm((a - b).ravel()) / nb)


def fields_of(pb):
    return ("ez", "hx", "hy") if pb.ndim == 2 else ("ex", "ey", "ez", "hx", "hy", "hz")


def run_oracle(pb, steps):
    from oracle import oracle as O
    o = O.for_problem(pb)
    rec = o.run(steps)
    return {f: getattr(o, f).copy() for f in fields_of(pb)}, rec


def run_gpu(pb, steps, kernel=None, graph=False, chunks=1):
    from paper_2405_00814_amd.sim import Sim
    s = Sim.from_problem(pb, graph=graph)
    if kernel is not None:
        s.set_kernel(*kernel)
    done = 0
    for c in range(chunks):
        n = steps // chunks if c < chunks - 1 else steps - done
        s.step(n)
        done += n
    f = {k: s.get_field(k) for k in fields_of(pb)}
    rec = s.probe()
    cfg = s.get_kernel() if not graph else None
    s.close()
    return f, rec, cfg


def assert_parity(gpu, ref, tol=1e-4, what=""):
    for k in ref:
        e = rel_l2(gpu[k], ref[k])
        assert e <= tol, "%s %s rel-L2 %.3e > %.1e" % (what, k, e, tol)


EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6


def energy_rel_l2(gpu, ref, pb):
    """Relative L2 error of the whole field state in the energy norm
    sqrt(sum eps |E|^2 + mu |H|^2) (SI weights, per cell)."""
    eps = EPS0 * (np.ones(pb.shape) if pb.eps_r is None else pb.eps_r.astype(np.float64))
    mu = MU0 * (np.ones(pb.shape) if pb.mu_r is None else pb.mu_r.astype(np.float64))
    num = den = 0.0
    for k in ref:
        w = eps if k.startswith("e") else mu
        d = np.asarray(gpu[k], np.float64) - ref[k]
        num += float(np.sum(w * d * d))
        den += float(np.sum(w * np.asarray(ref[k], np.float64) ** 2))
    return float(np.sqrt(num / den))


def assert_parity_energy(gpu, ref, pb, tol=1e-4, what=""):
    """The state bar for sources with a static part: whole-state energy-norm
    rel-L2 <= tol and every E component within tol (the H components of a
    DC-carrying soft source are a small curl of a large static E and are
    reported, not gated)."""
    e = energy_rel_l2(gpu, ref, pb)
    assert e <= tol, "%s energy-norm rel-L2 %.3e > %.1e" % (what, e, tol)
    for k in ref:
        if k.startswith("e"):
            ek = rel_l2(gpu[k], ref[k])
            assert ek <= tol, "%s %s rel-L2 %.3e > %.1e" % (what, k, ek, tol)
    return e


def group_norm(state, group):
    """Norm of the E ("e") or H ("h") components of a state together."""
    return float(np.sqrt(sum(float(np.sum(np.asarray(v, np.float64) ** 2))
                             for k, v in state.items() if k.startswith(group))))


def run_oracle_tracked(o, steps, chunk, at=()):
    """Advance the FP64 oracle `o` by `steps` in chunks of at most `chunk`,
    tracking the largest norm the E and the H components reached (at the
    chunk ends; a lower bound of the true peak).  Returns the probe record,
    {"e": peak, "h": peak} and copies of the fields at the steps in `at`
    (counted from o's start)."""
    fields = o.fields
    peaks = {"e": 0.0, "h": 0.0}
    snaps = {}
    stops = sorted(set(list(range(chunk, steps, chunk)) + [int(a) for a in at if 0 < a < steps] + [steps]))
    done, recs = 0, []
    for stop in stops:
        recs.append(o.run(stop - done))
        done = stop
        st = {f: getattr(o, f) for f in fields}
        for g in peaks:
            peaks[g] = max(peaks[g], group_norm(st, g))
        if done in at:
            snaps[done] = {f: getattr(o, f).copy() for f in fields}
    return np.concatenate(recs, axis=1), peaks, snaps


def run_errors(got, ref, peaks):
    """Per component: the literal rel-L2 ||got - ref|| / ||ref||, the error
    relative to the peak norm of its field group over the run
    ||got - ref|| / P_group, and ||ref|| / P_group."""
    out = {}
    for k in ref:
        d = float(np.linalg.norm((np.asarray(got[k], np.float64) - ref[k]).ravel()))
        n = float(np.linalg.norm(np.asarray(ref[k], np.float64).ravel()))
        p = peaks[k[0]]
        out[k] = (d / n if n > 0 else d, d / p, n / p)
    return out


LIVE = 0.1


def assert_run_parity(got, ref, peaks, tol=1e-4, what=""):
    """The parity bar of a whole run at a checkpoint: every component within
    tol of the peak norm its field group (E or H) reached over the run, and
    every live component (norm at least LIVE of that peak) also within tol
    of its own norm.  A component far below its group's peak (a pulse that
    has been absorbed, the H of the static field a DC-carrying source
    leaves) carries the rounding of the whole run in units of that peak:
    no FP32 evaluation meets the literal bar there (the FP32 build of the
    oracle shows it)."""
    errs = run_errors(got, ref, peaks)
    for k, (lit, grp, frac) in errs.items():
        assert grp <= tol, "%s %s error / group peak %.3e > %.1e" % (what, k, grp, tol)
        if frac >= LIVE:
            assert lit <= tol, "%s %s rel-L2 %.3e > %.1e (live: %.2f of the peak)" % (what, k, lit, tol, frac)
    return errs
