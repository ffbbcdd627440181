"""FP64 CPU oracle of the split-field PML (test infrastructure only).

The paper terminates its grid with a perfectly matched layer in which the
electric field is split in two parts, one per transverse axis, each damped
by the conductivity along its own axis, while the magnetic field is damped
by a magnetic conductivity along the axis of its curl term; the magnetic
conductivity is matched to the electric one (ratio mu/eps) so the layer's
impedance equals the grid's (Sec. III-C, Eq. 10-13).  In the TMz form used
here (the paper's TE equations relabelled Ey -> Ez, Hz -> Hy, z -> y):

    eps dEzx/dt + (sigma + sx) Ezx =  dHy/dx
    eps dEzy/dt + (sigma + sy) Ezy = -dHx/dy        Ez = Ezx + Ezy
    mu  dHx/dt  + sy* Hx           = -dEz/dy
    mu  dHy/dt  + sx* Hy           =  dEz/dx        s*/mu0 = s/eps0

(sigma: the cell's own conductivity; sx, sy: the layer's, zero outside it;
the printed magnetic subscripts are read as the axis of each curl term).
Each equation is discretised like Eq. 7-9: central differences on the Yee
grid, the loss term averaged over the time step, giving
    F <- (1 - a)/(1 + a) F + (dt/m)/(1 + a) D,   a = s dt / (2 m)
with m = eps or mu.  The field is split in every cell, so outside the
layer the two parts simply add up to the unsplit update.  The layer's
conductivity is graded as s = s_max rho^m (rho: normalised depth at x = i
for E and i + 1/2 for H, s_max = 0.8 (m + 1) / (eta0 d) unless given).

Nothing here is shared with the library under test.
"""
from __future__ import annotations

import math

import numpy as np

from .oracle import source_samples

EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6


def layer_sigma(n, lo, hi, delta, m, sigma_max, half):
    """Graded layer conductivity along one axis at x = i (+ 1/2 if half)."""
    x = np.arange(n, dtype=np.float64) + (0.5 if half else 0.0)
    rho = np.zeros(n)
    if lo > 0:
        rho = np.where(x < lo, (lo - x) / lo, rho)
    if hi > 0:
        rho = np.maximum(rho, np.where(x > n - hi, (x - (n - hi)) / hi, 0.0))
    smax = sigma_max if sigma_max > 0 else 0.8 * (m + 1.0) / (math.sqrt(MU0 / EPS0) * delta)
    return smax * rho ** m


class Oracle2DSplit:
    """FP64 2D TMz stepper with the split-field PML."""

    fields = ("ez", "hx", "hy")

    def __init__(self, shape, dx, dt, eps_r=None, sigma=None, mu_r=None, npml=(0, 0, 0, 0), cpml=None):
        nx, ny = shape
        self.shape = (nx, ny)
        self.dx = tuple(dx)
        self.dt = float(dt)
        cp = dict(m=3.0, sigma_max=0.0)
        cp.update(cpml or {})
        eps = EPS0 * (np.ones(shape) if eps_r is None else np.asarray(eps_r, np.float64).reshape(shape))
        mu = MU0 * (np.ones(shape) if mu_r is None else np.asarray(mu_r, np.float64).reshape(shape))
        sg = np.zeros(shape) if sigma is None else np.asarray(sigma, np.float64).reshape(shape)
        sxE = layer_sigma(nx, npml[0], npml[1], dx[0], cp["m"], cp["sigma_max"], False)[:, None]
        syE = layer_sigma(ny, npml[2], npml[3], dx[1], cp["m"], cp["sigma_max"], False)[None, :]
        sxH = layer_sigma(nx, npml[0], npml[1], dx[0], cp["m"], cp["sigma_max"], True)[:, None]
        syH = layer_sigma(ny, npml[2], npml[3], dx[1], cp["m"], cp["sigma_max"], True)[None, :]

        def coef(s, m):
            a = s * self.dt / (2.0 * m)
            return (1.0 - a) / (1.0 + a), (self.dt / m) / (1.0 + a)

        self.ax, self.bx = coef(sg + sxE, eps)         # Ezx
        self.ay, self.by = coef(sg + syE, eps)         # Ezy
        self.hxa, self.hxb = coef(syH * MU0 / EPS0, mu)  # Hx: curl along y
        self.hya, self.hyb = coef(sxH * MU0 / EPS0, mu)  # Hy: curl along x
        self.ezx = np.zeros(shape)
        self.ezy = np.zeros(shape)
        self.hx = np.zeros(shape)
        self.hy = np.zeros(shape)
        self.src = None
        self.probes = np.zeros((0, 2), np.int64)
        self.n = 0
        self.rec = []

    @classmethod
    def from_problem(cls, pb):
        o = cls(pb.shape, pb.dx, pb.dt, pb.eps_r, pb.sigma, pb.mu_r, pb.npml, pb.cpml)
        if pb.source is not None:
            o.set_source(pb.source.cell, pb.source.kind, pb.source.params, hi=getattr(pb.source, "hi", None))
        o.set_probes(pb.probes)
        return o

    @property
    def ez(self):
        return self.ezx + self.ezy

    def set_source(self, cell, kind, params, hi=None):
        """Soft source on Ez (its x part) at cell or on the box [cell, hi)."""
        hi = tuple(hi) if hi is not None else (cell[0] + 1, cell[1] + 1)
        self.src = ((slice(cell[0], hi[0]), slice(cell[1], hi[1])), int(kind), tuple(params))

    def set_probes(self, cells):
        self.probes = np.asarray(cells, np.int64).reshape(-1, 2)

    def step(self, gval):
        dx, dy = self.dx
        ez = self.ezx + self.ezy
        # H layer (ghost Ez beyond the last row and column is zero)
        dey = np.zeros_like(ez)
        dey[:, :-1] = ez[:, 1:] - ez[:, :-1]
        dey[:, -1] = -ez[:, -1]
        dex = np.zeros_like(ez)
        dex[:-1, :] = ez[1:, :] - ez[:-1, :]
        dex[-1, :] = -ez[-1, :]
        self.hx = self.hxa * self.hx - self.hxb * dey / dy
        self.hy = self.hya * self.hy + self.hyb * dex / dx
        # E layer on the cells off the PEC planes i = 0, j = 0
        dhy = (self.hy[1:, 1:] - self.hy[:-1, 1:]) / dx
        dhx = (self.hx[1:, 1:] - self.hx[1:, :-1]) / dy
        self.ezx[1:, 1:] = self.ax[1:, 1:] * self.ezx[1:, 1:] + self.bx[1:, 1:] * dhy
        self.ezy[1:, 1:] = self.ay[1:, 1:] * self.ezy[1:, 1:] - self.by[1:, 1:] * dhx
        if self.src is not None:
            self.ezx[self.src[0]] += gval

    def run(self, nsteps):
        g = np.zeros(nsteps)
        if self.src is not None:
            g = source_samples(self.src[1], self.src[2], self.dt, self.n, nsteps)
        rec = np.zeros((len(self.probes), nsteps))
        for k in range(nsteps):
            self.step(g[k])
            if len(self.probes):
                ez = self.ezx + self.ezy
                rec[:, k] = ez[self.probes[:, 0], self.probes[:, 1]]
        self.n += nsteps
        self.rec.append(rec)
        return rec

    def probe_series(self):
        return np.concatenate(self.rec, axis=1) if self.rec else np.zeros((len(self.probes), 0))
