"""Seeded synthetic workloads (inputs only).

This module builds the inputs that both the FP32 HIP path and the FP64 oracle
consume: grid sizes, spatial and time steps, per-cell material maps, CPML
thickness, source description, probe cells and the design box of the
sensitivity study.  It holds none of the update arithmetic: no coefficient
folding, no CPML profile, no source waveform.  Each consumer turns the
description below into its own numbers.

Scenes follow the paper's proof-of-concept experiments (Sec. V-A): randomly
placed axis-aligned objects with random permittivity and conductivity on a
vacuum background, a point source at a random position, waveforms sampled at
random cells.  Objects are painted in draw order (later wins) and are kept
out of the absorbing layer.  All randomness is numpy PCG64 with an explicit
seed.

The time step comes from a Courant number S: dt = S * min(dx) / c0.  The
spatial step of the dielectric scenes follows the paper's sampling rule of
twenty cells per shortest wavelength (Sec. V-B), with that wavelength taken at
three times the Ricker peak frequency in the densest medium.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

C0 = 299792458.0  # speed of light in vacuum, m/s (exact, SI)

SRC_GAUSSIAN = 0
SRC_RICKER = 1
SRC_SINE = 3
SRC_MODGAUSS = 4


@dataclasses.dataclass
class Source:
    """A soft source: E[cell] += amp * g((n+1) dt) after each E update; with
    hi set, on every cell of the box [cell, hi) (a line source when one
    extent exceeds 1).

    kind: SRC_GAUSSIAN with params (amp, t0, tau), g = exp(-((t - t0)/tau)^2)
          SRC_RICKER   with params (amp, t0, f),   g = (1 - 2 pi^2 f^2 s^2) exp(-pi^2 f^2 s^2), s = t - t0
          SRC_SINE     with params (amp, f, T),    g = w(t) sin(2 pi f t), turn-on w = sin^2(pi t / 2T) for t < T
          SRC_MODGAUSS with params (amp, t0, tau, f), g = exp(-((t - t0)/tau)^2) sin(2 pi f (t - t0))
    """
    cell: Tuple[int, ...]
    kind: int
    params: Tuple[float, ...]
    component: str = "ez"
    hi: Optional[Tuple[int, ...]] = None


@dataclasses.dataclass
class Problem:
    """One FDTD problem.  Arrays are float32, C order, last axis contiguous."""
    name: str
    ndim: int
    shape: Tuple[int, ...]          # (nx, ny) or (nx, ny, nz), cells incl. CPML
    dx: Tuple[float, ...]           # per-axis spatial step (m)
    dt: float                       # time step (s)
    steps: int                      # number of leapfrog steps of the workload
    npml: Tuple[int, ...]           # cells per face: -x,+x,-y,+y(,-z,+z)
    eps_r: Optional[np.ndarray]     # None => vacuum
    sigma: Optional[np.ndarray]     # None => lossless (S/m)
    mu_r: Optional[np.ndarray]      # None => 1
    source: Optional[Source]
    probes: np.ndarray              # int32 [P, ndim]
    probe_component: str = "ez"
    design: Optional[Tuple[int, int, int, int]] = None   # [i0, i1) x [j0, j1)
    window: Optional[Tuple[int, int]] = None              # loss window (n0, n1]
    cpml: dict = dataclasses.field(default_factory=lambda: dict(
        m=3.0, sigma_max=0.0, kappa_max=1.0, alpha_max=0.0, m_alpha=1.0))
    rho: Optional[np.ndarray] = None  # mass density (kg/m^3), for absorption rates

    @property
    def cells(self) -> int:
        return int(np.prod(self.shape))


def _interior_cell(rng, shape, margin, avoid=None):
    for _ in range(100000):
        c = tuple(int(rng.integers(min(margin, (n - 1) // 2), n - min(margin, (n - 1) // 2)))
                  for n in shape)
        if avoid is None or not avoid(c):
            return c
    raise ValueError("no admissible cell in grid %s" % (shape,))


def _paint_boxes(rng, shape, npml, count, side_lo, side_hi, eps_lo, eps_hi,
                 sig_hi, eps, sigma):
    """Axis-aligned boxes with integer sides U{side_lo..side_hi}, corners
    uniform inside the non-CPML interior, painted in draw order."""
    nd = len(shape)
    for _ in range(count):
        lo, hi = [], []
        for a in range(nd):
            inner = shape[a] - npml[2 * a] - npml[2 * a + 1]
            w = int(rng.integers(side_lo, side_hi + 1))
            w = min(w, inner)
            c0 = int(rng.integers(npml[2 * a], npml[2 * a] + inner - w + 1))
            lo.append(c0)
            hi.append(c0 + w)
        er = float(rng.uniform(eps_lo, eps_hi))
        sl = tuple(slice(l, h) for l, h in zip(lo, hi))
        eps[sl] = er
        if sigma is not None:
            sigma[sl] = float(rng.uniform(0.0, sig_hi))


def courant_dt(S: float, dx: Sequence[float]) -> float:
    return S * min(dx) / C0


def dx_for_ricker(f_peak: float, eps_max: float, ppw: int = 20) -> float:
    """Spatial step giving ppw cells per shortest wavelength, shortest
    wavelength at 3 * f_peak in the densest medium."""
    return C0 / (3.0 * f_peak * math.sqrt(eps_max) * ppw)


# ---------------------------------------------------------------------------
# The five workloads (and scaled-down versions of them for parity tests)
# ---------------------------------------------------------------------------

def cavity2d(n: int = 128, steps: int = 1000, seed: int = 0, nprobes: int = 4,
             ny: Optional[int] = None) -> Problem:
    """2D TMz PEC cavity, vacuum, dx = 1 mm, S = 0.99/sqrt(2), Gaussian pulse
    (tau = 20 dt, t0 = 100 dt) at a seeded interior cell, seeded probes."""
    rng = np.random.default_rng(seed)
    ny = n if ny is None else ny
    shape = (n, ny)
    dx = (1e-3, 1e-3)
    dt = courant_dt(0.99 / math.sqrt(2.0), dx)
    margin = min(8, min(shape) // 4)
    src = Source(_interior_cell(rng, shape, margin), SRC_GAUSSIAN,
                 (1.0, 100.0 * dt, 20.0 * dt))
    probes = np.array([_interior_cell(rng, shape, margin) for _ in range(nprobes)],
                      dtype=np.int32)
    return Problem("cavity2d_%dx%d" % shape, 2, shape, dx, dt, steps,
                   (0, 0, 0, 0), None, None, None, src, probes)


def dielectric2d(n: int = 4096, steps: int = 10000, seed: int = 0,
                 nrect: int = 200, side: Tuple[int, int] = (16, 512),
                 npml: int = 16, nprobes: int = 8, ny: Optional[int] = None,
                 lossy: bool = True, f_peak: float = 1e9) -> Problem:
    """2D TMz with CPML and a random-rectangle scene: eps_r ~ U[1,6],
    sigma ~ U[0, 0.01] S/m, Ricker source at f_peak, t0 = 1.5/f_peak,
    dx = lambda_min/20, S = 0.99/sqrt(2)."""
    rng = np.random.default_rng(seed)
    ny = n if ny is None else ny
    shape = (n, ny)
    pml = (npml,) * 4
    eps = np.ones(shape, np.float32)
    sig = np.zeros(shape, np.float32) if lossy else None
    _paint_boxes(rng, shape, pml, nrect, side[0], side[1], 1.0, 6.0, 0.01, eps, sig)
    h = dx_for_ricker(f_peak, 6.0)
    dx = (h, h)
    dt = courant_dt(0.99 / math.sqrt(2.0), dx)
    margin = npml + min(8, (min(shape) - 2 * npml) // 4)
    src = Source(_interior_cell(rng, shape, margin), SRC_RICKER, (1.0, 1.5 / f_peak, f_peak))
    probes = np.array([_interior_cell(rng, shape, margin) for _ in range(nprobes)],
                      dtype=np.int32)
    return Problem("dielectric2d_%dx%d" % shape, 2, shape, dx, dt, steps, pml,
                   eps, sig, None, src, probes)


def yee3d(n: int = 512, steps: int = 2000, seed: int = 0, nbox: int = 500,
          side: Tuple[int, int] = (8, 96), npml: int = 12, nprobes: int = 8,
          shape: Optional[Tuple[int, int, int]] = None,
          tau_steps: float = 68.0) -> Problem:
    """3D Yee, CPML, random dielectric boxes eps_r ~ U[1,8], sigma = 0,
    mu_r = 1, z-directed soft Ez source with a Gaussian pulse
    (tau = tau_steps * dt, t0 = 5 tau), dx = 1 mm, S = 0.99/sqrt(3)."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n) if shape is None else tuple(shape)
    pml = (npml,) * 6
    eps = np.ones(shape, np.float32)
    _paint_boxes(rng, shape, pml, nbox, side[0], side[1], 1.0, 8.0, 0.0, eps, None)
    dx = (1e-3, 1e-3, 1e-3)
    dt = courant_dt(0.99 / math.sqrt(3.0), dx)
    margin = npml + min(8, (min(shape) - 2 * npml) // 4)
    tau = tau_steps * dt
    src = Source(_interior_cell(rng, shape, margin), SRC_GAUSSIAN, (1.0, 5.0 * tau, tau))
    probes = np.array([_interior_cell(rng, shape, margin) for _ in range(nprobes)],
                      dtype=np.int32)
    return Problem("yee3d_%dx%dx%d" % shape, 3, shape, dx, dt, steps, pml,
                   eps, None, None, src, probes)


def batch2d(count: int = 256, steps: int = 4000, seed: int = 0,
            side: Tuple[int, int] = (256, 2048), npml: int = 16,
            nprobes: int = 4, rect_side: Tuple[int, int] = (16, 256),
            rect_density: float = 200.0 / 4096 ** 2) -> List[Problem]:
    """Independent 2D TMz problems with sides drawn independently and
    uniformly from {side[0]..side[1]} (ny redrawn while equal to nx), each with
    its own random-rectangle scene (eps_r ~ U[1,6], sigma = 0), Ricker 1 GHz
    at its own cell, 16-cell CPML, dx = 2.0398 mm, S = 0.99/sqrt(2)."""
    rng = np.random.default_rng(seed)
    out = []
    h = dx_for_ricker(1e9, 6.0)
    dx = (h, h)
    dt = courant_dt(0.99 / math.sqrt(2.0), dx)
    for p in range(count):
        nx = int(rng.integers(side[0], side[1] + 1))
        ny = int(rng.integers(side[0], side[1] + 1))
        while ny == nx:
            ny = int(rng.integers(side[0], side[1] + 1))
        shape = (nx, ny)
        pml = (npml,) * 4
        eps = np.ones(shape, np.float32)
        nrect = max(1, int(round(rect_density * nx * ny)))
        _paint_boxes(rng, shape, pml, nrect, rect_side[0], rect_side[1], 1.0, 6.0,
                     0.0, eps, None)
        margin = npml + min(8, (min(shape) - 2 * npml) // 4)
        src = Source(_interior_cell(rng, shape, margin), SRC_RICKER, (1.0, 1.5e-9, 1e9))
        probes = np.array([_interior_cell(rng, shape, margin) for _ in range(nprobes)],
                          dtype=np.int32)
        out.append(Problem("batch2d[%d]_%dx%d" % (p, nx, ny), 2, shape, dx, dt, steps,
                           pml, eps, None, None, src, probes))
    return out


def adjoint2d(n: int = 1024, steps: int = 4000, seed: int = 0,
              design: Optional[Tuple[int, int, int, int]] = None,
              npml: int = 16, nprobes: int = 16) -> Problem:
    """2D TMz sensitivity study: vacuum with a design box whose eps_r is
    i.i.d. U[1,4] per cell, Ricker 1 GHz outside the box, probes outside the
    box and the CPML, loss window (T/2, T]."""
    rng = np.random.default_rng(seed)
    shape = (n, n)
    pml = (npml,) * 4
    if design is None:
        a, b = (3 * n) // 8, (5 * n) // 8
        design = (a, b, a, b)
    i0, i1, j0, j1 = design
    eps = np.ones(shape, np.float32)
    eps[i0:i1, j0:j1] = rng.uniform(1.0, 4.0, size=(i1 - i0, j1 - j0)).astype(np.float32)
    h = dx_for_ricker(1e9, 4.0)
    dx = (h, h)
    dt = courant_dt(0.99 / math.sqrt(2.0), dx)
    margin = npml + min(8, (n - 2 * npml) // 8)

    def in_design(c):
        return i0 - 2 <= c[0] < i1 + 2 and j0 - 2 <= c[1] < j1 + 2

    src = Source(_interior_cell(rng, shape, margin, in_design), SRC_RICKER, (1.0, 1.5e-9, 1e9))
    probes = np.array([_interior_cell(rng, shape, margin, in_design) for _ in range(nprobes)],
                      dtype=np.int32)
    return Problem("adjoint2d_%dx%d" % shape, 2, shape, dx, dt, steps, pml, eps,
                   None, None, src, probes, design=design, window=(steps // 2, steps))


def layered2d(n: int = 400, steps: int = 4000, seed: int = 0, ny: Optional[int] = None,
              npml: int = 12, f0: float = 6.8e9, nprobes: int = 4) -> Problem:
    """2D TMz layered lossy medium of the shape of the paper's tissue case
    (Sec. V-B: air over a thin, a thick and a semi-infinite layer, a pulsed
    point source above the first layer, 20 cells per shortest wavelength,
    Courant number 0.95).  The layer properties are synthetic draws from
    broad tissue-like ranges, not measured data: thin layer eps_r U[25, 45],
    sigma U[1, 5] S/m; thick layer eps_r U[3, 8], sigma U[0.05, 0.5];
    last layer eps_r U[35, 55], sigma U[2, 8]; density U[900, 1150] kg/m^3
    per layer (air: 1.2).  Layers run along x (rows): air to 30 % of the
    rows, the thin layer 4 %, the thick one 30 %, the last to the end.
    Source: modulated Gaussian at f0 (tau = 1/f0, t0 = 4 tau), 8 % of the
    rows above the first layer, mid column; probes on that column."""
    rng = np.random.default_rng(seed)
    ny = n if ny is None else ny
    shape = (n, ny)
    pml = (npml,) * 4
    props = [(1.0, 0.0, 1.2),
             (float(rng.uniform(25, 45)), float(rng.uniform(1, 5)), float(rng.uniform(900, 1150))),
             (float(rng.uniform(3, 8)), float(rng.uniform(0.05, 0.5)), float(rng.uniform(900, 1150))),
             (float(rng.uniform(35, 55)), float(rng.uniform(2, 8)), float(rng.uniform(900, 1150)))]
    edges = [0, int(0.30 * n), int(0.34 * n), int(0.64 * n), n]
    eps = np.ones(shape, np.float32)
    sig = np.zeros(shape, np.float32)
    rho = np.ones(shape, np.float32)
    for (er, sg, rh), a, b in zip(props, edges[:-1], edges[1:]):
        eps[a:b] = er
        sig[a:b] = sg
        rho[a:b] = rh
    h = C0 / (f0 * math.sqrt(max(p[0] for p in props)) * 20)
    dx = (h, h)
    dt = courant_dt(0.95 / math.sqrt(2.0), dx)
    tau = 1.0 / f0
    src = Source((max(npml + 1, edges[1] - int(0.08 * n)), ny // 2), SRC_MODGAUSS, (1.0, 4 * tau, tau, f0))
    rows = np.linspace(edges[1] + 1, n - npml - 2, nprobes).astype(np.int32)
    probes = np.array([(int(r), ny // 2) for r in rows], dtype=np.int32)
    pb = Problem("layered2d_%dx%d" % shape, 2, shape, dx, dt, steps, pml, eps, sig, None, src, probes)
    pb.rho = rho
    pb.cpml = dict(m=3.0, sigma_max=0.0, kappa_max=1.0, alpha_max=0.0, m_alpha=1.0)
    return pb


def freespace2d(n: int, steps: int = 1024, npml: int = 16) -> Problem:
    """Paper-shape sweep (Sec. V-C): free space square grid, absorbing layer,
    Gaussian source at the centre."""
    shape = (n, n)
    h = dx_for_ricker(1e9, 1.0)
    dx = (h, h)
    dt = courant_dt(0.99 / math.sqrt(2.0), dx)
    tau = 20.0 * dt
    src = Source((n // 2, n // 2), SRC_GAUSSIAN, (1.0, 5.0 * tau, tau))
    probes = np.array([(n // 2 + 3, n // 2 - 5)], dtype=np.int32)
    return Problem("freespace2d_%dx%d" % shape, 2, shape, dx, dt, steps,
                   (npml,) * 4, None, None, None, src, probes)


def random_state(rng: np.random.Generator, shape, ncomp: int, dtype=np.float64):
    """Random field components (for linearity / adjoint / resume tests)."""
    return [rng.standard_normal(shape).astype(dtype) for _ in range(ncomp)]
