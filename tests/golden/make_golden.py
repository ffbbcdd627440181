"""Writes the stored expected values under tests/golden/ (calls only oracle/).

The paper prints no worked numeric example (its figures carry no data), so
the fixtures here are FP64 oracle outputs on the seeded workloads, kept to
detect unintended changes of the oracle's arithmetic.  Each file names the
workload, seed and command that produced it.

    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2405_00814_amd import workloads as W  # noqa: E402


def cavity128():
    pb = W.cavity2d(128, steps=1000, seed=0)
    o = O.for_problem(pb)
    rec = o.run(pb.steps)
    path = os.path.join(HERE, "cavity2d_128_seed0_probes.txt")
    with open(path, "w") as f:
        f.write("# FP64 oracle, 2D TMz PEC cavity 128x128, dx=1mm, S=0.99/sqrt(2), Gaussian\n")
        f.write("# tau=20dt t0=100dt, seed 0; rows = steps 1..1000 (every 50th), cols = 4 probes\n")
        f.write("# source cell %s probes %s\n" % (pb.source.cell, pb.probes.tolist()))
        f.write("# made by: python tests/golden/make_golden.py\n")
        for k in range(49, pb.steps, 50):
            f.write(" ".join("%.17e" % v for v in rec[:, k]) + "\n")


def adjoint_small():
    pb = W.adjoint2d(n=48, steps=300, seed=1, design=(18, 30, 18, 30), npml=8, nprobes=4)
    o = O.for_problem(pb)
    loss, grad = o.loss_and_grad(pb.steps, pb.window, pb.design)
    path = os.path.join(HERE, "adjoint2d_48_seed1_grad.txt")
    with open(path, "w") as f:
        f.write("# FP64 oracle, 2D TMz 48x48, 8-cell CPML, design [18,30)^2, 300 steps,\n")
        f.write("# window (150,300], seed 1; first line = loss, then dL/deps_r rows of the design box\n")
        f.write("# made by: python tests/golden/make_golden.py\n")
        f.write("%.17e\n" % loss)
        for row in grad:
            f.write(" ".join("%.17e" % v for v in row) + "\n")


if __name__ == "__main__":
    cavity128()
    adjoint_small()
