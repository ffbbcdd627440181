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
