"""Regression fixtures of the oracle (written by tests/golden/make_golden.py)."""
import os

import numpy as np

from paper_2405_00814_amd import workloads as W

G = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    return np.loadtxt(os.path.join(G, name), comments="#", ndmin=2)


def test_golden_cavity128(orc):
    ref = _load("cavity2d_128_seed0_probes.txt")
    pb = W.cavity2d(128, steps=1000, seed=0)
    rec = orc.for_problem(pb).run(pb.steps)
    got = rec[:, 49::50].T
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_golden_adjoint_small(orc):
    with open(os.path.join(G, "adjoint2d_48_seed1_grad.txt")) as f:
        rows = [l for l in f if not l.startswith("#")]
    loss_ref = float(rows[0])
    grad_ref = np.array([[float(v) for v in r.split()] for r in rows[1:]])
    pb = W.adjoint2d(n=48, steps=300, seed=1, design=(18, 30, 18, 30), npml=8, nprobes=4)
    loss, grad = orc.for_problem(pb).loss_and_grad(pb.steps, pb.window, pb.design)
    assert abs(loss - loss_ref) <= 1e-12 * abs(loss_ref)
    assert np.abs(grad - grad_ref).max() <= 1e-11 * np.abs(grad_ref).max()
