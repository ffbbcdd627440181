"""Shared helpers of the parity tests: run a problem on the HIP library and
on the FP64 oracle with the same seeded inputs, compare."""
import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# set by conftest.py: the pytest config, for progress() below
PYTEST_CONFIG = None


def progress(*a):
    """A progress line of a long test (a step of the work done), written
    past pytest's output capture so that it appears while the test runs."""
    capman = PYTEST_CONFIG.pluginmanager.getplugin("capturemanager") if PYTEST_CONFIG else None
    if capman is None:
        log(*a)
        return
    with capman.global_and_fixture_disabled():
        print(*a, flush=True)


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


def energy_weights(pb):
    """Per-cell weights of the energy norm: eps0 eps_r for E components,
    mu0 mu_r for H components (scalars when the map is absent)."""
    we = EPS0 * (1.0 if pb.eps_r is None else np.asarray(pb.eps_r, np.float64))
    wh = MU0 * (1.0 if pb.mu_r is None else np.asarray(pb.mu_r, np.float64))
    return {"e": we, "h": wh}


def _wnorm(a, w):
    a = np.asarray(a, np.float64)
    return float(np.sqrt(np.sum(w * a * a)))


def state_energy_norm(state, w):
    """sqrt(sum over cells and components of w f^2): the energy norm of a
    state (field components keyed ex..hz), the norm the leapfrog conserves
    in a lossless cavity."""
    return float(np.sqrt(sum(_wnorm(v, w[k[0]]) ** 2 for k, v in state.items())))


def run_oracle_tracked(o, steps, chunk, w, at=(), tag=None):
    """Advance the FP64 oracle `o` by `steps` in chunks of at most `chunk`,
    tracking the largest energy norm (weights w, energy_weights) the state
    reached at the chunk ends (a lower bound of the true peak).  Returns the
    probe record, that peak and copies of the fields at the steps in `at`
    (counted from o's start).  With a tag, each chunk's end is reported by
    progress()."""
    fields = o.fields
    peak = 0.0
    snaps = {}
    stops = sorted(set(list(range(chunk, steps, chunk)) + [int(a) for a in at if 0 < a < steps] + [steps]))
    done, recs = 0, []
    for stop in stops:
        recs.append(o.run(stop - done))
        done = stop
        if tag:
            progress("  %s: oracle step %d of %d" % (tag, done, steps))
        peak = max(peak, state_energy_norm({f: getattr(o, f) for f in fields}, w))
        if done in at:
            snaps[done] = {f: getattr(o, f).copy() for f in fields}
    return np.concatenate(recs, axis=1), peak, snaps


def run_errors(got, ref, peak, w):
    """Per component: the literal rel-L2 ||got - ref|| / ||ref||; its error
    in the energy norm relative to the peak energy norm of the whole state
    over the run, ||got - ref||_w / P; and ||ref||_w / P (its share)."""
    out = {}
    for k in ref:
        d = np.asarray(got[k], np.float64) - ref[k]
        n = float(np.linalg.norm(np.asarray(ref[k], np.float64).ravel()))
        dn = float(np.linalg.norm(d.ravel()))
        out[k] = (dn / n if n > 0 else dn, _wnorm(d, w[k[0]]) / peak, _wnorm(ref[k], w[k[0]]) / peak)
    return out


LIVE = 0.1


def assert_run_parity(got, ref, peak, w, tol=1e-4, what=""):
    """The parity bar of a whole run at a checkpoint: every component's error
    in the energy norm within tol of the peak energy norm the state reached
    over the run, and every live component (its own energy norm at least
    LIVE of that peak) also within tol of its own norm (relative L2).  A
    component far below the peak (a pulse that has been absorbed, the H of
    the static field a DC-carrying source leaves) carries the rounding of
    the whole run in units of that peak: no FP32 evaluation meets the
    relative bar there (the FP32 build of the oracle shows it)."""
    errs = run_errors(got, ref, peak, w)
    for k, (lit, grp, frac) in errs.items():
        assert grp <= tol, "%s %s energy-norm error / peak %.3e > %.1e" % (what, k, grp, tol)
        if frac >= LIVE:
            assert lit <= tol, "%s %s rel-L2 %.3e > %.1e (live: %.2f of the peak)" % (what, k, lit, tol, frac)
    return errs
