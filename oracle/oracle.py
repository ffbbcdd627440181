"""FP64 CPU oracle: Python side (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It wraps the plain C stepper in ``fdtd_oracle.c``
(built with gcc into ``liborc.so`` next to this file) and keeps the state in
numpy float64 arrays.  The library under test is never imported here.

What each class computes is documented in ``fdtd_oracle.c``: the Yee
leapfrog of the paper's Eq. 7-9 (TMz form of its 2D TE equations, and the
3D extension), CPML boundary, soft source, probes, and the discrete adjoint
of a probe-energy loss with respect to eps_r.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fdtd_oracle.c")
LIB = os.path.join(HERE, "liborc.so")
# the same C source built in single precision (run_fp32 below)
LIB32 = os.path.join(HERE, "liborc32.so")

_lock = threading.Lock()
_lib = None

DP = C.POINTER(C.c_double)
LP = C.POINTER(C.c_long)
IP = C.POINTER(C.c_int)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no GPU code involved), and the same
    source in single precision (-DORC_FP32) for run_fp32."""
    for out, extra in ((LIB, []), (LIB32, ["-DORC_FP32"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
            tmp = out + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                                   "-Wall"] + extra + ["-o", tmp, SRC, "-lm"])
            os.replace(tmp, out)
    return LIB


class _O2(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("dx", C.c_double), ("dy", C.c_double),
                ("ez", DP), ("hx", DP), ("hy", DP), ("ca", DP), ("cb", DP), ("db", DP),
                ("psi_hx", DP), ("psi_hy", DP), ("psi_ezx", DP), ("psi_ezy", DP),
                ("prof_x", DP), ("prof_y", DP)]


class _A2(C.Structure):
    _fields_ = [(n, DP) for n in ("ez", "hx", "hy", "psi_hx", "psi_hy", "psi_ezx", "psi_ezy")]


F3 = ("ex", "ey", "ez", "hx", "hy", "hz")
PSI3 = ("psi_hxy", "psi_hxz", "psi_hyz", "psi_hyx", "psi_hzx", "psi_hzy",
        "psi_exy", "psi_exz", "psi_eyz", "psi_eyx", "psi_ezx", "psi_ezy")


class _O3(C.Structure):
    _fields_ = ([("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                 ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double)]
                + [(n, DP) for n in F3] + [("ca", DP), ("cb", DP), ("db", DP)]
                + [(n, DP) for n in PSI3]
                + [("prof_x", DP), ("prof_y", DP), ("prof_z", DP)])


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(LIB)
            L.orc_coeffs.argtypes = [C.c_long, C.c_double, DP, DP, DP, DP, DP, DP]
            L.orc_cpml_axis.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                        C.c_double, C.c_double, C.c_double, C.c_double,
                                        C.c_double, DP]
            L.orc_source.argtypes = [C.c_int, DP, C.c_double, C.c_long, C.c_long, DP]
            L.orc2d_h_layer.argtypes = [C.POINTER(_O2)]
            L.orc2d_e_layer.argtypes = [C.POINTER(_O2), DP]
            L.orc2d_run.argtypes = [C.POINTER(_O2), C.c_long, C.c_long, LP, DP, C.c_int, LP, DP,
                                    C.c_long, IP, DP, DP]
            L.orc2d_adj_step.argtypes = [C.POINTER(_O2), C.POINTER(_A2)]
            L.orc2d_adjoint.argtypes = [C.POINTER(_O2), C.POINTER(_A2), C.c_long, C.c_int, LP,
                                        DP, C.c_long, C.c_long, IP, DP, DP, DP, DP,
                                        C.c_double, DP]
            L.orc2d_run_mu.argtypes = L.orc2d_run.argtypes + [DP, DP]
            L.orc2d_adjoint_mu.argtypes = L.orc2d_adjoint.argtypes + [DP, DP, DP, DP]
            L.orc3d_h_layer.argtypes = [C.POINTER(_O3)]
            L.orc3d_e_layer.argtypes = [C.POINTER(_O3)]
            L.orc3d_run.argtypes = [C.POINTER(_O3), C.c_long, DP, C.c_long, LP, DP, DP, C.c_int,
                                    LP, DP, C.c_long]
            _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(DP)


def _f64(a, shape=None):
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def cpml_axis(n, d_lo, d_hi, delta, dt, cp):
    prof = np.zeros(6 * n, np.float64)
    lib().orc_cpml_axis(n, d_lo, d_hi, delta, dt, cp.get("m", 3.0), cp.get("sigma_max", 0.0),
                        cp.get("kappa_max", 1.0), cp.get("alpha_max", 0.0),
                        cp.get("m_alpha", 1.0), _p(prof))
    return prof


def source_samples(kind, params, dt, n0, count):
    out = np.zeros(count, np.float64)
    par = np.asarray(params, np.float64)
    lib().orc_source(int(kind), _p(par), dt, int(n0), int(count), _p(out))
    return out


def coeffs(dt, eps_r, sigma, mu_r, ncell):
    ca = np.zeros(ncell, np.float64)
    cb = np.zeros(ncell, np.float64)
    db = np.zeros(ncell, np.float64)
    e = _f64(eps_r.ravel()) if eps_r is not None else None
    s = _f64(sigma.ravel()) if sigma is not None else None
    m = _f64(mu_r.ravel()) if mu_r is not None else None
    lib().orc_coeffs(ncell, dt, _p(e), _p(s), _p(m), _p(ca), _p(cb), _p(db))
    return ca, cb, db


class Oracle2D:
    """FP64 2D TMz stepper.  Fields: ez, hx, hy (shape (nx, ny)); psi arrays
    psi_hx, psi_hy, psi_ezx, psi_ezy on the full grid."""

    fields = ("ez", "hx", "hy")
    psis = ("psi_hx", "psi_hy", "psi_ezx", "psi_ezy")

    def __init__(self, shape, dx, dt, eps_r=None, sigma=None, mu_r=None,
                 npml=(0, 0, 0, 0), cpml=None):
        nx, ny = shape
        self.shape = (nx, ny)
        self.dx = tuple(dx)
        self.dt = float(dt)
        cpml = cpml or {}
        self.eps_r = None if eps_r is None else _f64(eps_r).reshape(shape)
        self.sigma = None if sigma is None else _f64(sigma).reshape(shape)
        self.mu_r = None if mu_r is None else _f64(mu_r).reshape(shape)
        self.ca, self.cb, self.db = coeffs(dt, self.eps_r, self.sigma, self.mu_r, nx * ny)
        self.prof_x = cpml_axis(nx, npml[0], npml[1], dx[0], dt, cpml)
        self.prof_y = cpml_axis(ny, npml[2], npml[3], dx[1], dt, cpml)
        for n in self.fields + self.psis:
            setattr(self, n, np.zeros(shape, np.float64))
        self.src = None
        self.probes = np.zeros((0,), np.int64)
        self.n = 0
        self.rec = []
        self.dft = None

    @classmethod
    def from_problem(cls, pb):
        o = cls(pb.shape, pb.dx, pb.dt, pb.eps_r, pb.sigma, pb.mu_r, pb.npml, pb.cpml)
        if pb.source is not None:
            o.set_source(pb.source.cell, pb.source.kind, pb.source.params, hi=getattr(pb.source, "hi", None))
        o.set_probes(pb.probes)
        return o

    def _struct(self):
        s = _O2()
        s.nx, s.ny = self.shape
        s.dx, s.dy = self.dx
        for n in self.fields + self.psis:
            setattr(s, n, _p(getattr(self, n)))
        s.ca, s.cb, s.db = _p(self.ca), _p(self.cb), _p(self.db)
        s.prof_x, s.prof_y = _p(self.prof_x), _p(self.prof_y)
        self._keep = s
        return s

    def set_source(self, cell, kind, params, hi=None):
        """Soft Ez source at cell, or on every cell of the box [cell, hi)."""
        hi = tuple(hi) if hi is not None else (cell[0] + 1, cell[1] + 1)
        cells = [i * self.shape[1] + j for i in range(cell[0], hi[0]) for j in range(cell[1], hi[1])]
        self.src = (np.array(cells, np.int64), int(kind), tuple(params))

    def set_dft(self, comp, lo, hi, freqs):
        _set_dft(self, comp, lo, hi, freqs)

    def set_probes(self, cells):
        cells = np.asarray(cells, np.int64).reshape(-1, 2)
        self.probes = np.ascontiguousarray(cells[:, 0] * self.shape[1] + cells[:, 1])

    def run(self, nsteps, design=None, hbr=False):
        """Advance nsteps; returns probe samples [P, nsteps] and, with a
        design box, the per-step (Ez before E layer, bracket) trajectories,
        and with hbr also those of the H layer's brackets (Hx -= Db bx,
        Hy += Db by)."""
        if self.dft is not None and design is None and nsteps > 1:
            return np.concatenate([self.run(1) for _ in range(nsteps)], axis=1)
        s = self._struct()
        P = len(self.probes)
        rec = np.zeros((P, nsteps), np.float64)
        cells, vals = np.zeros(1, np.int64), None
        if self.src is not None:
            cells = self.src[0]
            vals = source_samples(self.src[1], self.src[2], self.dt, self.n, nsteps)
        nsrc = len(cells) if self.src is not None else 0
        dz = tz = tb = hx = hy = None
        if design is not None:
            dz = (C.c_int * 4)(*design)
            nd = (design[1] - design[0]) * (design[3] - design[2])
            tz = np.zeros((nsteps, nd), np.float64)
            tb = np.zeros((nsteps, nd), np.float64)
            if hbr:
                hx = np.zeros((nsteps, nd), np.float64)
                hy = np.zeros((nsteps, nd), np.float64)
        pr = self.probes if P else np.zeros(1, np.int64)
        lib().orc2d_run_mu(C.byref(s), nsteps, nsrc, cells.ctypes.data_as(LP), _p(vals), P,
                           pr.ctypes.data_as(LP), _p(rec), nsteps, dz, _p(tz), _p(tb), _p(hx), _p(hy))
        self.n += nsteps
        self.rec.append(rec)
        if self.dft is not None:
            _dft_sample(self, nsteps)
        if design is not None:
            return (rec, tz, tb, hx, hy) if hbr else (rec, tz, tb)
        return rec

    def h_layer(self):
        s = self._struct()
        lib().orc2d_h_layer(C.byref(s))

    def e_layer(self):
        s = self._struct()
        lib().orc2d_e_layer(C.byref(s), None)

    def probe_series(self):
        return np.concatenate(self.rec, axis=1) if self.rec else np.zeros((len(self.probes), 0))

    def state(self):
        return {n: getattr(self, n).copy() for n in self.fields + self.psis}

    def set_state(self, st):
        for n, v in st.items():
            getattr(self, n)[...] = v

    # ---- adjoint -----------------------------------------------------
    def adj_step(self, adj):
        """Apply the transpose of one step (without source) to adjoint arrays
        given as a dict with the keys of state()."""
        s = self._struct()
        a = _A2()
        for n in self.fields + self.psis:
            assert adj[n].dtype == np.float64 and adj[n].flags.c_contiguous
            setattr(a, n, _p(adj[n]))
        lib().orc2d_adj_step(C.byref(s), C.byref(a))

    def loss_and_grad(self, T, window, design, mu=False):
        """From the zero state: run T steps, L = sum over probes and
        m in (n0, n1] of Ez^m[p]^2, and dL/d eps_r on the design box (with
        mu: also dL/d mu_r, returned third)."""
        for n in self.fields + self.psis:
            getattr(self, n)[...] = 0.0
        self.n = 0
        self.rec = []
        if mu:
            rec, tz, tb, hx, hy = self.run(T, design=design, hbr=True)
        else:
            rec, tz, tb = self.run(T, design=design)
            hx = hy = None
        n0, n1 = window
        loss = float(np.sum(rec[:, n0:n1] ** 2))
        for n in self.fields + self.psis:
            getattr(self, n)[...] = 0.0
        adj = {n: np.zeros(self.shape, np.float64) for n in self.fields + self.psis}
        a = _A2()
        for n in adj:
            setattr(a, n, _p(adj[n]))
        s = self._struct()
        nd = (design[1] - design[0]) * (design[3] - design[2])
        grad = np.zeros(nd, np.float64)
        er = self.eps_r if self.eps_r is not None else np.ones(self.shape)
        er = np.ascontiguousarray(er, np.float64)
        sg = self.sigma
        gmu = np.zeros(nd, np.float64) if mu else None
        mr = None if self.mu_r is None else np.ascontiguousarray(self.mu_r, np.float64)
        lib().orc2d_adjoint_mu(C.byref(s), C.byref(a), T, len(self.probes),
                               self.probes.ctypes.data_as(LP), _p(np.ascontiguousarray(rec)),
                               n0, n1, (C.c_int * 4)(*design), _p(tz), _p(tb), _p(er), _p(sg),
                               self.dt, _p(grad), _p(hx), _p(hy), _p(mr), _p(gmu))
        shape = (design[1] - design[0], design[3] - design[2])
        if mu:
            return loss, grad.reshape(shape), gmu.reshape(shape)
        return loss, grad.reshape(shape)


class Oracle3D:
    """FP64 3D Yee stepper (six components, twelve psi arrays)."""

    fields = F3
    psis = PSI3

    def __init__(self, shape, dx, dt, eps_r=None, sigma=None, mu_r=None,
                 npml=(0,) * 6, cpml=None):
        nx, ny, nz = shape
        self.shape = (nx, ny, nz)
        self.dx = tuple(dx)
        self.dt = float(dt)
        cpml = cpml or {}
        ncell = nx * ny * nz
        er = None if eps_r is None else _f64(eps_r)
        sg = None if sigma is None else _f64(sigma)
        mr = None if mu_r is None else _f64(mu_r)
        self.ca, self.cb, self.db = coeffs(dt, er, sg, mr, ncell)
        del er, sg, mr
        self.prof_x = cpml_axis(nx, npml[0], npml[1], dx[0], dt, cpml)
        self.prof_y = cpml_axis(ny, npml[2], npml[3], dx[1], dt, cpml)
        self.prof_z = cpml_axis(nz, npml[4], npml[5], dx[2], dt, cpml)
        for n in self.fields + self.psis:
            setattr(self, n, np.zeros(shape, np.float64))
        self.src = None
        self.probes = np.zeros((0,), np.int64)
        self.probe_comp = "ez"
        self.n = 0
        self.rec = []
        self.dft = None

    @classmethod
    def from_problem(cls, pb):
        o = cls(pb.shape, pb.dx, pb.dt, pb.eps_r, pb.sigma, pb.mu_r, pb.npml, pb.cpml)
        if pb.source is not None:
            o.set_source(pb.source.cell, pb.source.kind, pb.source.params, pb.source.component,
                         hi=getattr(pb.source, "hi", None))
        o.set_probes(pb.probes, pb.probe_component)
        return o

    def _lin(self, cell):
        nx, ny, nz = self.shape
        return (int(cell[0]) * ny + int(cell[1])) * nz + int(cell[2])

    def _struct(self):
        s = _O3()
        s.nx, s.ny, s.nz = self.shape
        s.dx, s.dy, s.dz = self.dx
        for n in self.fields + self.psis:
            setattr(s, n, _p(getattr(self, n)))
        s.ca, s.cb, s.db = _p(self.ca), _p(self.cb), _p(self.db)
        s.prof_x, s.prof_y, s.prof_z = _p(self.prof_x), _p(self.prof_y), _p(self.prof_z)
        self._keep = s
        return s

    def set_source(self, cell, kind, params, component="ez", hi=None):
        """Soft source on `component` at cell, or on every cell of the box
        [cell, hi)."""
        hi = tuple(hi) if hi is not None else tuple(int(c) + 1 for c in cell)
        cells = [self._lin((i, j, k)) for i in range(cell[0], hi[0]) for j in range(cell[1], hi[1])
                 for k in range(cell[2], hi[2])]
        self.src = (np.array(cells, np.int64), int(kind), tuple(params), component)

    def set_dft(self, comp, lo, hi, freqs):
        _set_dft(self, comp, lo, hi, freqs)

    def set_probes(self, cells, component="ez"):
        cells = np.asarray(cells, np.int64).reshape(-1, 3)
        self.probes = np.ascontiguousarray(np.array([self._lin(c) for c in cells], np.int64))
        self.probe_comp = component

    def run(self, nsteps):
        if self.dft is not None and nsteps > 1:
            return np.concatenate([self.run(1) for _ in range(nsteps)], axis=1)
        s = self._struct()
        P = len(self.probes)
        rec = np.zeros((P, nsteps), np.float64)
        sf, cells, vals = None, np.zeros(1, np.int64), None
        if self.src is not None:
            cells = self.src[0]
            sf = _p(getattr(self, self.src[3]))
            vals = source_samples(self.src[1], self.src[2], self.dt, self.n, nsteps)
        nsrc = len(cells) if self.src is not None else 0
        pr = self.probes if P else np.zeros(1, np.int64)
        lib().orc3d_run(C.byref(s), nsteps, sf, nsrc, cells.ctypes.data_as(LP), _p(vals),
                        _p(getattr(self, self.probe_comp)), P, pr.ctypes.data_as(LP),
                        _p(rec), nsteps)
        self.n += nsteps
        self.rec.append(rec)
        if self.dft is not None:
            _dft_sample(self, nsteps)
        return rec

    def h_layer(self):
        s = self._struct()
        lib().orc3d_h_layer(C.byref(s))

    def e_layer(self):
        s = self._struct()
        lib().orc3d_e_layer(C.byref(s))

    def probe_series(self):
        return np.concatenate(self.rec, axis=1) if self.rec else np.zeros((len(self.probes), 0))

    def state(self):
        return {n: getattr(self, n).copy() for n in self.fields + self.psis}

    def set_state(self, st):
        for n, v in st.items():
            getattr(self, n)[...] = v


def _set_dft(o, comp, lo, hi, freqs):
    """Frequency-domain monitor (the paper motivates frequency-domain
    responses, Sec. I; no formulation given): the discrete Fourier sum
    X_q = sum_n F^{n+1}[box] exp(-2 pi i f_q t_n) dt over the steps run from
    now on, t_n = (n+1) dt for E and (n+1/2) dt for H (the sample's time on
    the leapfrog grid)."""
    box = tuple(slice(int(a), int(b)) for a, b in zip(lo, hi))
    o.dft = dict(comp=comp, box=box, f=np.asarray(freqs, np.float64),
                 X=np.zeros((len(freqs),) + tuple(b.stop - b.start for b in box), np.complex128), n=0)


def _dft_sample(o, nsteps):
    # called after exactly one step (run steps one by one while a monitor is set)
    assert nsteps == 1
    d = o.dft
    step = o.n - 1
    t = (step + (0.5 if d["comp"].startswith("h") else 1.0)) * o.dt
    v = getattr(o, d["comp"])[d["box"]]
    for q, f in enumerate(d["f"]):
        d["X"][q] += v * np.exp(-2j * np.pi * f * t) * o.dt
    d["n"] += 1


def sar(X, sigma, rho, norm=None):
    """Specific absorption rate (W/kg) of a time-harmonic field whose complex
    amplitude at frequency q is X[q] (the paper estimates SAR in layered
    tissue, Sec. V-B, without stating the formula): the time-averaged Joule
    power per unit mass, sigma |X|^2 / (2 rho), with X divided by norm[q]
    (the source spectrum, for a per-unit-source result; None: 1).  sigma and
    rho have the shape of one X[q]."""
    X = np.asarray(X, np.complex128)
    n = np.ones(X.shape[0]) if norm is None else np.asarray(norm, np.float64)
    n = n.reshape((-1,) + (1,) * (X.ndim - 1))
    a2 = X.real ** 2 + X.imag ** 2
    return np.asarray(sigma, np.float64)[None] * a2 / (2.0 * np.asarray(rho, np.float64)[None] * n ** 2)


def for_problem(pb):
    if pb.ndim == 2 and (pb.cpml or {}).get("split", 0):
        from .split import Oracle2DSplit
        return Oracle2DSplit.from_problem(pb)
    return (Oracle2D if pb.ndim == 2 else Oracle3D).from_problem(pb)


# ---------------------------------------------------------------------------
# FP32 evaluation of the same update (rounding studies; not the oracle)
# ---------------------------------------------------------------------------
FP = C.POINTER(C.c_float)


class _O2f(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("dx", C.c_float), ("dy", C.c_float)] + \
               [(n, FP) for n in ("ez", "hx", "hy", "ca", "cb", "db", "psi_hx", "psi_hy", "psi_ezx",
                                  "psi_ezy", "prof_x", "prof_y")]


class _O3f(C.Structure):
    _fields_ = ([("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                 ("dx", C.c_float), ("dy", C.c_float), ("dz", C.c_float)]
                + [(n, FP) for n in F3] + [("ca", FP), ("cb", FP), ("db", FP)]
                + [(n, FP) for n in PSI3]
                + [("prof_x", FP), ("prof_y", FP), ("prof_z", FP)])


_lib32 = None


def lib32():
    global _lib32
    with _lock:
        if _lib32 is None:
            build()
            L = C.CDLL(LIB32)
            L.orc2d_run.argtypes = [C.POINTER(_O2f), C.c_long, C.c_long, LP, FP, C.c_int, LP, FP,
                                    C.c_long, IP, FP, FP]
            L.orc3d_run.argtypes = [C.POINTER(_O3f), C.c_long, FP, C.c_long, LP, FP, FP, C.c_int,
                                    LP, FP, C.c_long]
            _lib32 = L
    return _lib32


def run_fp32(o, nsteps):
    """Advance the problem of the FP64 oracle `o` by nsteps from o's current
    state with the single-precision build of the same stepping code: the
    state, the coefficients, the CPML profiles and the source samples (all
    computed in FP64) rounded once to float32, every operation of the steps
    in float32.  `o` is not modified.  Returns ({name: float32 array} of the
    fields and psi arrays, float32 probe record [P, nsteps])."""
    f32 = {n: np.ascontiguousarray(getattr(o, n), np.float32) for n in o.fields + o.psis}
    tabs = {n: np.ascontiguousarray(getattr(o, n), np.float32)
            for n in ("ca", "cb", "db", "prof_x", "prof_y") + (("prof_z",) if len(o.shape) == 3 else ())}

    def fp(a):
        return a.ctypes.data_as(FP)

    P = len(o.probes)
    rec = np.zeros((P, nsteps), np.float32)
    pr = o.probes if P else np.zeros(1, np.int64)
    cells, vals, nsrc = np.zeros(1, np.int64), None, 0
    if o.src is not None:
        cells = o.src[0]
        nsrc = len(cells)
        vals = source_samples(o.src[1], o.src[2], o.dt, o.n, nsteps).astype(np.float32)
    if len(o.shape) == 2:
        s = _O2f()
        s.nx, s.ny = o.shape
        s.dx, s.dy = o.dx
        for n, a in list(f32.items()) + list(tabs.items()):
            setattr(s, n, fp(a))
        lib32().orc2d_run(C.byref(s), nsteps, nsrc, cells.ctypes.data_as(LP),
                          fp(vals) if vals is not None else None, P, pr.ctypes.data_as(LP), fp(rec),
                          nsteps, None, None, None)
    else:
        s = _O3f()
        s.nx, s.ny, s.nz = o.shape
        s.dx, s.dy, s.dz = o.dx
        for n, a in list(f32.items()) + list(tabs.items()):
            setattr(s, n, fp(a))
        sf = fp(f32[o.src[3]]) if o.src is not None else None
        lib32().orc3d_run(C.byref(s), nsteps, sf, nsrc, cells.ctypes.data_as(LP),
                          fp(vals) if vals is not None else None, fp(f32[o.probe_comp]), P,
                          pr.ctypes.data_as(LP), fp(rec), nsteps)
    return f32, rec
