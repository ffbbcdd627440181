"""Thin Python objects over the C ABI (marshalling only).

``Sim`` wraps one fdtd_sim handle, ``Batch`` one fdtd_batch handle.  Device
memory comes from torch's caching allocator and work is enqueued on torch's
current HIP stream; torch is used for nothing else.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _lib as L

COMP = {"ex": L.FDTD_EX, "ey": L.FDTD_EY, "ez": L.FDTD_EZ,
        "hx": L.FDTD_HX, "hy": L.FDTD_HY, "hz": L.FDTD_HZ}


def _comp(c):
    return COMP[c] if isinstance(c, str) else int(c)


# ---------------------------------------------------------------------------
# torch plumbing: stream and caching allocator
# ---------------------------------------------------------------------------
_torch_alloc_cb = None
_torch_free_cb = None
_torch_allocator = None


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible to torch")
    return torch


def torch_allocator():
    """fdtd_allocator backed by torch.cuda.caching_allocator_alloc/delete."""
    global _torch_alloc_cb, _torch_free_cb, _torch_allocator
    if _torch_allocator is None:
        torch = _torch()

        def _alloc(ctx, size, stream):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(size), stream=int(stream or 0)))
            except Exception:
                return None

        def _free(ctx, ptr, stream):
            try:
                torch.cuda.caching_allocator_delete(int(ptr))
            except Exception:
                pass

        _torch_alloc_cb = L.ALLOC_FN(_alloc)
        _torch_free_cb = L.FREE_FN(_free)
        _torch_allocator = L.fdtd_allocator(None, _torch_alloc_cb, _torch_free_cb)
    return _torch_allocator


def current_stream() -> int:
    torch = _torch()
    return int(torch.cuda.current_stream().cuda_stream)


def _f32(a, n):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(-1))
    assert a.size == n, (a.size, n)
    return a


def make_desc(shape, dx, dt, eps_r=None, mu_r=None, sigma=None, npml=None, cpml=None,
              stream: Optional[int] = None, allocator=True):
    """Build an fdtd_desc (and the host arrays it points to)."""
    nd = len(shape)
    nx, ny = int(shape[0]), int(shape[1])
    nz = int(shape[2]) if nd == 3 else 1
    n = nx * ny * nz
    keep = [_f32(eps_r, n), _f32(mu_r, n), _f32(sigma, n)]
    d = L.fdtd_desc()
    d.ndim = nd
    d.nx, d.ny, d.nz = nx, ny, nz
    d.dx, d.dy = float(dx[0]), float(dx[1])
    d.dz = float(dx[2]) if nd == 3 else 1.0
    d.dt = float(dt)
    fp = C.POINTER(C.c_float)
    d.eps_r = keep[0].ctypes.data_as(fp) if keep[0] is not None else fp()
    d.mu_r = keep[1].ctypes.data_as(fp) if keep[1] is not None else fp()
    d.sigma = keep[2].ctypes.data_as(fp) if keep[2] is not None else fp()
    np6 = list(npml or ()) + [0] * 6
    cp = dict(m=3.0, sigma_max=0.0, kappa_max=1.0, alpha_max=0.0, m_alpha=1.0, split=0)
    cp.update(cpml or {})
    d.cpml.npml = (C.c_int32 * 6)(*[int(v) for v in np6[:6]])
    d.cpml.m, d.cpml.sigma_max = cp["m"], cp["sigma_max"]
    d.cpml.kappa_max, d.cpml.alpha_max, d.cpml.m_alpha = cp["kappa_max"], cp["alpha_max"], cp["m_alpha"]
    d.cpml.split = int(cp["split"])
    d.stream = current_stream() if stream is None else stream
    if allocator:
        d.allocator = C.pointer(torch_allocator())
    return d, keep


class Sim:
    """One simulation (implicit Yee graph, or explicit CSR graph with graph=True)."""

    def __init__(self, shape, dx, dt, eps_r=None, mu_r=None, sigma=None, npml=None,
                 cpml=None, graph=False, stream=None, allocator=True):
        self.shape = tuple(int(v) for v in shape)
        self.ndim = len(self.shape)
        self._desc, self._keep = make_desc(shape, dx, dt, eps_r, mu_r, sigma, npml, cpml,
                                           stream, allocator)
        h = C.c_void_p()
        L.call("fdtd_create_graph" if graph else "fdtd_create", C.byref(self._desc), C.byref(h))
        self.h = h
        self.nprobes = 0

    @classmethod
    def from_problem(cls, pb, graph=False, **kw):
        s = cls(pb.shape, pb.dx, pb.dt, pb.eps_r, pb.mu_r, pb.sigma, pb.npml, pb.cpml,
                graph=graph, **kw)
        if pb.source is not None and pb.source.hi is not None:
            s.set_source_box(pb.source.component, pb.source.cell, pb.source.hi, pb.source.kind, pb.source.params)
        elif pb.source is not None:
            s.set_source(pb.source.component, pb.source.cell, pb.source.kind, pb.source.params)
        if len(pb.probes):
            s.set_probes(pb.probe_component, pb.probes)
        return s

    def close(self):
        if getattr(self, "h", None):
            L.load().fdtd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def cells(self):
        return int(np.prod(self.shape))

    def set_source(self, comp, cell, kind, params=(0.0, 0.0, 0.0), table=None):
        ijk = (C.c_int32 * 3)(*[int(v) for v in cell] + [0] * (3 - len(cell)))
        par = (C.c_double * 4)(*[float(v) for v in params])
        tp, nt = None, 0
        if table is not None:
            self._table = np.ascontiguousarray(np.asarray(table, np.float32))
            tp = self._table.ctypes.data_as(C.POINTER(C.c_float))
            nt = self._table.size
        L.call("fdtd_set_source", self.h, _comp(comp), ijk, int(kind), par, tp, nt)

    def set_source_box(self, comp, lo, hi, kind, params=(0.0, 0.0, 0.0), table=None):
        """Soft source on every cell of [lo, hi) (a line source when one
        extent exceeds 1)."""
        a = (C.c_int32 * 3)(*[int(v) for v in lo] + [0] * (3 - len(lo)))
        b = (C.c_int32 * 3)(*[int(v) for v in hi] + [1] * (3 - len(hi)))
        par = (C.c_double * 4)(*[float(v) for v in params])
        tp, nt = None, 0
        if table is not None:
            self._table = np.ascontiguousarray(np.asarray(table, np.float32))
            tp = self._table.ctypes.data_as(C.POINTER(C.c_float))
            nt = self._table.size
        L.call("fdtd_set_source_box", self.h, _comp(comp), a, b, int(kind), par, tp, nt)

    def set_dft(self, comp, lo, hi, freqs):
        """Frequency-domain monitor of `comp` on the box [lo, hi) at freqs
        (Hz); an empty freqs removes it."""
        a = (C.c_int32 * 3)(*[int(v) for v in lo] + [0] * (3 - len(lo)))
        b = (C.c_int32 * 3)(*[int(v) for v in hi] + [1] * (3 - len(hi)))
        fr = (C.c_double * max(1, len(freqs)))(*[float(v) for v in freqs])
        L.call("fdtd_set_dft", self.h, _comp(comp), a, b, len(freqs), fr)
        self._dft = (tuple(int(h) - int(l) for l, h in zip(lo, hi)), len(freqs))

    def get_dft(self):
        """(X, nsteps): X complex128 [nf, *box shape]."""
        shape, nf = getattr(self, "_dft", ((0,), 0))
        if nf == 0:  # no monitor: the library reports it
            L.call("fdtd_get_dft", self.h, None, None, None)
        n = int(np.prod(shape))
        re = np.zeros(nf * n, np.float64)
        im = np.zeros(nf * n, np.float64)
        ns = C.c_int64()
        L.call("fdtd_get_dft", self.h, re.ctypes.data_as(C.POINTER(C.c_double)),
               im.ctypes.data_as(C.POINTER(C.c_double)), C.byref(ns))
        return (re + 1j * im).reshape((nf,) + shape), ns.value

    def dft_sar(self, rho, norm=None):
        """Specific absorption rate (W/kg) from the monitor's sums, float32
        [nf, *box shape]: sigma |X|^2 / (2 rho norm^2); rho over the box
        (kg/m^3), norm per frequency (None: 1)."""
        shape, nf = getattr(self, "_dft", ((0,), 0))
        if nf == 0:  # no monitor: the library reports it
            one = np.ones(1, np.float32)
            L.call("fdtd_dft_sar", self.h, one.ctypes.data_as(C.POINTER(C.c_float)), None,
                   one.ctypes.data_as(C.POINTER(C.c_float)))
        n = int(np.prod(shape))
        r = np.ascontiguousarray(np.asarray(rho, np.float32).reshape(-1))
        if r.size != n:
            raise ValueError("rho must have one value per monitored cell")
        out = np.zeros(max(1, nf * n), np.float32)
        nm = None if norm is None else (C.c_double * nf)(*[float(v) for v in norm])
        L.call("fdtd_dft_sar", self.h, r.ctypes.data_as(C.POINTER(C.c_float)), nm,
               out.ctypes.data_as(C.POINTER(C.c_float)))
        return out[:nf * n].reshape((nf,) + shape)

    def clear_source(self):
        L.call("fdtd_set_source", self.h, L.FDTD_EZ, None, -1, None, None, 0)

    def set_probes(self, comp, cells):
        cells = np.ascontiguousarray(np.asarray(cells, np.int32).reshape(-1, self.ndim))
        L.call("fdtd_set_probes", self.h, _comp(comp),
               cells.ctypes.data_as(C.POINTER(C.c_int32)), int(cells.shape[0]))
        self.nprobes = int(cells.shape[0])

    def step(self, n: int):
        L.call("fdtd_step", self.h, int(n))

    def probe(self) -> np.ndarray:
        n = C.c_int64()
        L.call("fdtd_probe", self.h, None, 0, C.byref(n))
        out = np.zeros((self.nprobes, max(n.value, 0)), np.float32)
        if self.nprobes and n.value:
            L.call("fdtd_probe", self.h, out.ctypes.data_as(C.POINTER(C.c_float)), n.value,
                   C.byref(n))
        return out

    def get_field(self, comp) -> np.ndarray:
        out = np.zeros(self.shape, np.float32)
        L.call("fdtd_get_field", self.h, _comp(comp), out.ctypes.data_as(C.c_void_p), 0)
        return out

    def get_field_device(self, comp, tensor):
        """Copy into a torch float32 CUDA tensor of self.cells elements (async)."""
        assert tensor.is_cuda and tensor.dtype.is_floating_point and tensor.numel() == self.cells
        L.call("fdtd_get_field", self.h, _comp(comp), C.c_void_p(tensor.data_ptr()), 1)

    def set_field(self, comp, arr):
        a = np.ascontiguousarray(np.asarray(arr, np.float32).reshape(self.shape))
        L.call("fdtd_set_field", self.h, _comp(comp), a.ctypes.data_as(C.c_void_p), 0)

    def save_state(self) -> np.ndarray:
        """The whole stepping state (fdtd_save_state) as a host byte array."""
        n = C.c_int64()
        L.call("fdtd_state_bytes", self.h, C.byref(n))
        buf = np.zeros(n.value, np.uint8)
        L.call("fdtd_save_state", self.h, buf.ctypes.data_as(C.c_void_p), 0)
        return buf

    def load_state(self, buf: np.ndarray):
        """Resume from a state saved by save_state (fdtd_load_state)."""
        n = C.c_int64()
        L.call("fdtd_state_bytes", self.h, C.byref(n))
        b = np.ascontiguousarray(buf, np.uint8)
        if b.size != n.value:
            raise ValueError("saved state has %d bytes, this handle's state %d" % (b.size, n.value))
        L.call("fdtd_load_state", self.h, b.ctypes.data_as(C.c_void_p), 0)

    def reset(self):
        L.call("fdtd_reset", self.h)

    def steps_done(self) -> int:
        n = C.c_int64()
        L.call("fdtd_steps_done", self.h, C.byref(n))
        return n.value

    def check_finite(self) -> bool:
        r = L.load().fdtd_check_finite(self.h)
        if r == L.FDTD_ENONFINITE:
            return False
        L.check(r, "fdtd_check_finite")
        return True

    def set_material(self, lo, hi, eps_r, sigma=None):
        nd = self.ndim
        lo_ = (C.c_int32 * 3)(*[int(v) for v in lo] + [0] * (3 - nd))
        hi_ = (C.c_int32 * 3)(*[int(v) for v in hi] + [1] * (3 - nd))
        e = np.ascontiguousarray(np.asarray(eps_r, np.float32).reshape(-1))
        s = None if sigma is None else np.ascontiguousarray(np.asarray(sigma, np.float32).reshape(-1))
        fp = C.POINTER(C.c_float)
        L.call("fdtd_set_material", self.h, lo_, hi_, e.ctypes.data_as(fp),
               s.ctypes.data_as(fp) if s is not None else None)

    def set_kernel(self, variant, tile=(0, 0, 0, 0), tb=1):
        k = L.fdtd_kernel_config()
        k.variant = int(variant)
        k.tile = (C.c_int32 * 4)(*[int(v) for v in list(tile) + [0] * (4 - len(tile))])
        k.tb = int(tb)
        L.call("fdtd_set_kernel", self.h, C.byref(k))

    def get_kernel(self):
        k = L.fdtd_kernel_config()
        L.call("fdtd_get_kernel", self.h, C.byref(k))
        return dict(variant=k.variant, tile=tuple(k.tile), tb=k.tb)

    def autotune(self, trial_steps=20):
        k = L.fdtd_kernel_config()
        L.call("fdtd_autotune", self.h, int(trial_steps), C.byref(k))
        return dict(variant=k.variant, tile=tuple(k.tile), tb=k.tb)

    def last_step_time(self):
        ms = C.c_float()
        n = C.c_int64()
        L.call("fdtd_last_step_time", self.h, C.byref(ms), C.byref(n))
        return ms.value, n.value

    def step_profile(self, steps=1):
        """Advance `steps` steps with per-launch HIP events; list of dicts
        (ms, cells, psi, cpml, launches, steps) with the mean duration of each
        launch per step (per step pair for the two-step pass)."""
        arr = (L.fdtd_launch_stat * 64)()
        n = C.c_int32()
        L.call("fdtd_step_profile", self.h, int(steps), arr, 64, C.byref(n))
        return [dict(ms=arr[q].ms, cells=arr[q].cells, psi=arr[q].psi, cpml=arr[q].cpml,
                     launches=arr[q].launches, steps=arr[q].steps)
                for q in range(min(n.value, 64))]

    def adjoint_eps(self, T, window, design, ckpt_interval=0, grad=None):
        """Loss and dL/d eps_r on the design box; grad is a torch float32
        CUDA tensor of the box size (allocated if None)."""
        torch = _torch()
        i0, i1, j0, j1 = design
        if grad is None:
            grad = torch.empty((i1 - i0) * (j1 - j0), dtype=torch.float32, device="cuda")
        d = (C.c_int32 * 4)(*[int(v) for v in design])
        loss = C.c_double()
        L.call("fdtd_adjoint_eps", self.h, int(T), int(window[0]), int(window[1]), d,
               int(ckpt_interval), C.byref(loss), C.cast(C.c_void_p(grad.data_ptr()), C.POINTER(C.c_float)))
        return loss.value, grad

    def adjoint_grads(self, T, window, design, ckpt_interval=0, mu=False):
        """Loss and its gradients with respect to eps_r and sigma (per S/m)
        on the design box, from one adjoint run: (loss, g_eps, g_sigma) with
        torch float32 CUDA tensors of the box size; with mu, also the
        gradient with respect to mu_r: (loss, g_eps, g_sigma, g_mu)."""
        torch = _torch()
        i0, i1, j0, j1 = design
        n = (i1 - i0) * (j1 - j0)
        ge = torch.empty(n, dtype=torch.float32, device="cuda")
        gs = torch.empty(n, dtype=torch.float32, device="cuda")
        gm = torch.empty(n, dtype=torch.float32, device="cuda") if mu else None
        d = (C.c_int32 * 4)(*[int(v) for v in design])
        loss = C.c_double()
        fp = C.POINTER(C.c_float)

        def ptr(t):
            return C.cast(C.c_void_p(t.data_ptr()), fp) if t is not None else None
        L.call("fdtd_adjoint_grads", self.h, int(T), int(window[0]), int(window[1]), d, int(ckpt_interval),
               C.byref(loss), ptr(ge), ptr(gs), ptr(gm))
        return (loss.value, ge, gs, gm) if mu else (loss.value, ge, gs)


class Batch:
    """Many independent 2D problems advanced together."""

    def __init__(self, problems, stream=None, allocator=True):
        self.problems = list(problems)
        n = len(self.problems)
        arr = (L.fdtd_desc * n)()
        self._keep = []
        for q, pb in enumerate(self.problems):
            d, keep = make_desc(pb.shape, pb.dx, pb.dt, pb.eps_r, pb.mu_r, pb.sigma, pb.npml,
                                pb.cpml, stream, allocator)
            arr[q] = d
            self._keep.append((d, keep))
        h = C.c_void_p()
        L.call("fdtd_batch_create", arr, n, C.byref(h))
        self.h = h
        self.nprobes = [0] * n
        for q, pb in enumerate(self.problems):
            if pb.source is not None:
                self.set_source(q, pb.source.cell, pb.source.kind, pb.source.params)
            if len(pb.probes):
                self.set_probes(q, pb.probes)

    def close(self):
        if getattr(self, "h", None):
            L.load().fdtd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_source(self, q, cell, kind, params):
        ijk = (C.c_int32 * 3)(*[int(v) for v in cell] + [0])
        par = (C.c_double * 4)(*[float(v) for v in params])
        L.call("fdtd_batch_set_source", self.h, int(q), ijk, int(kind), par, None, 0)

    def set_probes(self, q, cells):
        cells = np.ascontiguousarray(np.asarray(cells, np.int32).reshape(-1, 2))
        L.call("fdtd_batch_set_probes", self.h, int(q), cells.ctypes.data_as(C.POINTER(C.c_int32)),
               int(cells.shape[0]))
        self.nprobes[q] = int(cells.shape[0])

    def step(self, n):
        L.call("fdtd_batch_step", self.h, int(n))

    def set_kernel(self, tb=4, tx=16, vmax=2, txo=0):
        """Steps per pass (1, 2, 4), rows per tile, widest column vector,
        rows per tile near a CPML slab (0: tx)."""
        L.call("fdtd_batch_set_kernel", self.h, int(tb), int(tx), int(vmax), int(txo))

    def autotune(self, trial_steps=64):
        """Time the batch configurations and keep the fastest
        (fdtd_batch_autotune); returns (tb, tx, vmax, txo)."""
        out = (C.c_int32 * 4)()
        L.call("fdtd_batch_autotune", self.h, int(trial_steps), out)
        return tuple(int(v) for v in out)

    def probe(self, q):
        n = C.c_int64()
        L.call("fdtd_batch_probe", self.h, int(q), None, 0, C.byref(n))
        out = np.zeros((self.nprobes[q], n.value), np.float32)
        if self.nprobes[q] and n.value:
            L.call("fdtd_batch_probe", self.h, int(q), out.ctypes.data_as(C.POINTER(C.c_float)),
                   n.value, C.byref(n))
        return out

    def get_field(self, q, comp):
        out = np.zeros(self.problems[q].shape, np.float32)
        L.call("fdtd_batch_get_field", self.h, int(q), _comp(comp), out.ctypes.data_as(C.c_void_p), 0)
        return out

    def cells(self):
        n = C.c_int64()
        L.call("fdtd_batch_cells", self.h, C.byref(n))
        return n.value

    def last_step_time(self):
        ms = C.c_float()
        n = C.c_int64()
        L.call("fdtd_batch_last_step_time", self.h, C.byref(ms), C.byref(n))
        return ms.value, n.value
