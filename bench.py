"""Benchmark: Gcell-updates/s and fraction of the HBM roofline on MI355X.

One "step" is one leapfrog time step (H layer + E layer + CPML + source +
probes) of the whole 3D Yee grid of the headline workload: 512^3 cells with
a 12-cell CPML, 500 random dielectric boxes (eps_r ~ U[1,8]), a z-directed
Gaussian soft source and 8 probes (inputs already resident in HBM).  The
same JSON line also reports the other forms of the method on their
workloads: the 2D TMz 4096^2 CPML stepper, the explicit CSR graph form on
that grid, 256 batched 2D problems against the plain stepper over the same
problems, and the adjoint against the plain forward on the 1024^2
sensitivity workload.  `roofline` describes the dominant kernel of the
headline step; `cpu_baseline` is the FP64 oracle on the host cores, timed on
a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 2000] [--warmup 20]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12  # MI355X published HBM3E bandwidth, B/s
METRIC = "Gcell-updates/s and % of HBM roofline; batched and adjoint vs plain step"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes_implicit(sim_cells, psi_floats, nfields, ncoef):
    """Algorithmic HBM bytes of one step of the implicit stepper: every field
    read and written once, every per-cell coefficient map read once, every
    CPML auxiliary value read and written once (1D profiles ~0)."""
    return sim_cells * (8 * nfields + 4 * ncoef) + 8 * psi_floats


def psi_floats_of(pb):
    nd = pb.ndim
    n = pb.shape
    tot = 0
    if nd == 2:
        sx, sy = pb.npml[0] + pb.npml[1], pb.npml[2] + pb.npml[3]
        tot = 2 * n[0] * sy + 2 * sx * n[1]
    else:
        s = [pb.npml[0] + pb.npml[1], pb.npml[2] + pb.npml[3], pb.npml[4] + pb.npml[5]]
        X, Y, Z = s[0] * n[1] * n[2], n[0] * s[1] * n[2], n[0] * n[1] * s[2]
        tot = 4 * (X + Y + Z)
    return tot


def ncoef_of(pb):
    nc = 1  # Cb
    if pb.sigma is not None and np.any(pb.sigma > 0):
        nc += 1
    if pb.mu_r is not None and np.any(pb.mu_r != pb.mu_r.ravel()[0]):
        nc += 1
    return nc


def kernel_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_record(name, src):
    """Measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled
    by a copy kernel of known size) if they were taken on the current kernel
    source, else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))[name]
    except Exception:
        return None
    if d.get("kernel_sha") != kernel_hash(src):
        return None
    return d.get("bytes_per_launch")


def timed_steps(sim, steps, warmup):
    import torch
    if warmup:
        sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    ms_dev, launches = sim.last_step_time()   # HIP events on the launch stream
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ms_dev / 1e3, wall, launches


def bench_3d(args):
    from paper_2405_00814_amd import workloads as W
    from paper_2405_00814_amd.sim import Sim
    pb = W.yee3d(512, steps=args.steps, seed=0)
    log("3d: building %s" % (pb.shape,))
    sim = Sim.from_problem(pb)
    if args.tune:
        log("3d: autotune", sim.autotune(10))
    cfg = sim.get_kernel()
    t, wall, launches = timed_steps(sim, args.steps, args.warmup)
    cells = pb.cells
    rate = cells * args.steps / t
    ab = alg_bytes_implicit(cells, psi_floats_of(pb), 6, ncoef_of(pb))
    # the same number of steps again with HIP events around every launch
    prof = sim.step_profile(args.steps)
    ok = sim.check_finite()
    sim.close()
    dom = max(range(len(prof)), key=lambda q: prof[q]["ms"])
    d = prof[dom]
    # algorithmic bytes per cell-update of the dominant launch: its cells'
    # fields read and written once, the coefficient maps read once, its psi
    # values read and written once.  A launch that advances its cells by two
    # steps processes two cell-updates per cell; the bytes it must move at
    # least are those of one pass (state n in, state n+2 out).
    pass_bytes = alg_bytes_implicit(d["cells"], d["psi"], 6, ncoef_of(pb))
    k = d.get("steps", 1)
    return dict(pb=pb, cfg=cfg, t=t, wall=wall, launches=launches, rate=rate, bytes=ab,
                step_achieved=ab * args.steps / t, finite=ok, prof=prof, dom=dom,
                dom_steps=k, dom_pass_bytes=pass_bytes, dom_bytes=k * pass_bytes,
                dom_ms=d["ms"], dom_bpc=pass_bytes / d["cells"],
                dom_achieved=k * pass_bytes / (d["ms"] / 1e3))


def bench_2d(args, steps=10000):
    from paper_2405_00814_amd import workloads as W
    from paper_2405_00814_amd.sim import Sim
    pb = W.dielectric2d(4096, steps=steps, seed=0)
    sim = Sim.from_problem(pb)
    t, wall, launches = timed_steps(sim, steps, 20)
    ab = alg_bytes_implicit(pb.cells, psi_floats_of(pb), 3, ncoef_of(pb))
    k = sim.get_kernel()
    tb = k["tile"][2] if k["variant"] == 3 else 1
    # hbm_frac: a pass of tb steps must move one step's algorithmic bytes
    # (state in and out once); step_equiv_frac counts them per step
    out = dict(workload="dielectric2d_4096x4096_cpml16_200rects", steps=steps,
               kernel=k, steps_per_pass=tb, gcells_per_s=pb.cells * steps / t / 1e9,
               bytes_per_cell_pass=ab / pb.cells,
               achieved_GBps=ab * steps / tb / t / 1e9,
               hbm_frac=ab * steps / tb / t / PEAK_HBM,
               step_equiv_frac=ab * steps / t / PEAK_HBM)
    sim.close()
    # explicit graph form on the same grid
    g = Sim.from_problem(pb, graph=True)
    gs = 200
    tg, _, lg = timed_steps(g, gs, 5)
    gbytes = csr_alg_bytes(pb)
    out["graph_form"] = dict(steps=gs, gcells_per_s=pb.cells * gs / tg / 1e9,
                             bytes_per_cell_update=gbytes / pb.cells,
                             achieved_GBps=gbytes * gs / tg / 1e9,
                             hbm_frac=gbytes * gs / tg / PEAK_HBM, launches_per_step=lg / gs,
                             impl_bytes_per_cell_update=csr_impl_bytes(pb) / pb.cells)
    g.close()
    # frequency-domain monitor: Ez on the central 2048^2 box at 4 frequencies
    # (single steps while it is set), against single steps without it
    ms = 400
    m = Sim.from_problem(pb)
    m.set_kernel(2, (2, 4))
    tp, _, _ = timed_steps(m, ms, 5)
    m.set_dft("ez", (1024, 1024), (3072, 3072), [0.5e9, 1.0e9, 1.5e9, 2.0e9])
    tm, _, _ = timed_steps(m, ms, 5)
    m.close()
    out["dft_monitor"] = dict(steps=ms, box_cells=2048 * 2048, frequencies=4,
                              single_step_gcells_per_s=pb.cells * ms / tp / 1e9,
                              with_monitor_gcells_per_s=pb.cells * ms / tm / 1e9,
                              monitor_us_per_step=(tm - tp) / ms * 1e6)
    # the paper's split-field PML (two-pass reference kernels), against the
    # CPML through the same kernels, and its 4-node explicit graph
    import dataclasses
    ps = dataclasses.replace(pb, cpml=dict(pb.cpml, split=1))
    rates = {}
    for name, prob, graph in (("cpml_reference", pb, False), ("split_reference", ps, False),
                              ("split_graph", ps, True)):
        r = Sim.from_problem(prob, graph=graph)
        if not graph:
            r.set_kernel(1)
        tr, _, _ = timed_steps(r, 200, 5)
        rates[name + "_gcells_per_s"] = pb.cells * 200 / tr / 1e9
        r.close()
    out["split_pml"] = rates
    return out


def _csr_counts(pb):
    """(nonzeros, rows, nodes) of one step of the explicit graph of a 2D
    CPML problem: H rows (Hx, Hy: self, two E nodes, psi in a slab), psi_H
    rows (self, two E nodes), E rows (self, four H nodes, psi in a slab),
    psi_E rows (self, two H nodes)."""
    nx, ny = pb.shape
    N = nx * ny
    sx, sy = pb.npml[0] + pb.npml[1], pb.npml[2] + pb.npml[3]
    slab = nx * sy + sx * ny        # psi values of one layer's field (x and y slabs)
    nnz_h = 2 * 3 * N + slab + 3 * slab
    nnz_e = 5 * N + slab + 3 * slab
    rows = 3 * N + 2 * slab
    return nnz_h + nnz_e, rows, rows


def csr_alg_bytes(pb):
    """Algorithmic bytes of one step of the explicit graph (the method's
    matrices): every matrix entry (column index and weight, 8 B) and every
    row pointer (4 B) read once, every node value read once and written once
    (8 B).  124 B per interior cell."""
    nnz, rows, nodes = _csr_counts(pb)
    return 8 * nnz + 4 * rows + 8 * nodes


def csr_impl_bytes(pb):
    """Bytes the CSR kernels move at least: the algorithmic bytes plus a
    second read of every field node (the H layer gathers E and its own H,
    the E layer H and its own E).  Destinations come from a table of 8 B per
    64 rows (the per-row index only where a chunk straddles a grid row) and
    the psi rows run inside the field rows that read them."""
    nnz, rows, nodes = _csr_counts(pb)
    return 8 * nnz + 4 * rows + 8 * nodes + 4 * 3 * pb.cells


def bench_batch(args, steps=4000):
    from paper_2405_00814_amd import workloads as W
    from paper_2405_00814_amd.sim import Batch, Sim
    import torch
    probs = W.batch2d(count=256, steps=steps, seed=0)
    cells = sum(p.cells for p in probs)
    log("batch: %d problems, %.3e cells" % (len(probs), cells))
    b = Batch(probs)
    # the autotuner picks steps per pass, tile rows and vector width for this
    # size mix (state restored; cached when $GEMFDTD_TUNE_CACHE is set)
    t0 = time.perf_counter()
    tuned = b.autotune(64)
    tune_s = time.perf_counter() - t0
    b.step(64)
    torch.cuda.synchronize()
    b.step(steps)
    tb, lb = b.last_step_time()
    tb /= 1e3
    ok = all(np.isfinite(b.get_field(q, "ez")).all() for q in (0, 255))
    b.close()
    # the plain stepper over the same problems, one after the other
    tp = 0.0
    for pb in probs:
        s = Sim.from_problem(pb)
        s.step(8)
        torch.cuda.synchronize()
        s.step(steps)
        t, _ = s.last_step_time()
        tp += t / 1e3
        s.close()
    ab = sum(alg_bytes_implicit(p.cells, psi_floats_of(p), 3, ncoef_of(p)) for p in probs)
    return dict(workload="batch2d_256_problems_sides_256_2048_cpml16", problems=len(probs),
                cells=cells, steps=steps, tuned=dict(tb=tuned[0], tx=tuned[1], vmax=tuned[2], txo=tuned[3],
                                                     seconds=tune_s),
                steps_per_pass=tuned[0], gcells_per_s=cells * steps / tb / 1e9,
                hbm_frac=ab * steps / tuned[0] / tb / PEAK_HBM, step_equiv_frac=ab * steps / tb / PEAK_HBM,
                plain_sequential_gcells_per_s=cells * steps / tp / 1e9,
                speedup_vs_plain=tp / tb, launches=lb, finite=bool(ok))


def bench_cavity(args, steps=1000, runs=5):
    """The 128^2 PEC cavity (1000 steps, Gaussian source, 4 probes): a grid
    that fits one XCD's L2 many times over, so a step costs its launch; the
    median of `runs` timed runs of the default kernel."""
    from paper_2405_00814_amd import workloads as W
    from paper_2405_00814_amd.sim import Sim
    pb = W.cavity2d(128, steps=steps, seed=0)
    s = Sim.from_problem(pb)
    ts, launches = [], 0
    s.step(steps)
    for _ in range(runs):
        s.reset()
        t, _, launches = timed_steps(s, steps, 0)
        ts.append(t)
    cfg = s.get_kernel()
    s.close()
    t = float(np.median(ts))
    return dict(workload="cavity2d_128x128_pec_gaussian", steps=steps, runs=runs, kernel=cfg,
                gcells_per_s=pb.cells * steps / t / 1e9, us_per_step=t / steps * 1e6,
                launches_per_step=launches / steps)


def _ci95(v):
    """Median, and the 95 % confidence interval of the mean (Student t)."""
    v = np.asarray(v, np.float64)
    tq = {2: 12.706, 3: 4.303, 4: 3.182, 5: 2.776, 6: 2.571, 7: 2.447, 8: 2.365}.get(len(v), 2.0)
    h = tq * v.std(ddof=1) / math.sqrt(len(v)) if len(v) > 1 else 0.0
    return float(np.median(v)), float(v.mean() - h), float(v.mean() + h)


def bench_sweep(args, sides=(250, 1000, 2000, 3000, 4000, 5000, 6400), steps=1024, runs=5):
    """The paper's timing experiment in shape: free-space squares of the
    given sides with a 16-cell CPML and a Gaussian source at the centre,
    1024 steps, `runs` timed runs each: Gcell-updates/s median and 95 %
    confidence interval, default kernel."""
    from paper_2405_00814_amd import workloads as W
    from paper_2405_00814_amd.sim import Sim
    out = []
    for n in sides:
        pb = W.freespace2d(n, steps=steps)
        s = Sim.from_problem(pb)
        s.step(8)
        rates = []
        for _ in range(runs):
            s.reset()
            t, _, _ = timed_steps(s, steps, 0)
            rates.append(pb.cells * steps / t / 1e9)
        k = s.get_kernel()
        s.close()
        med, lo, hi = _ci95(rates)
        out.append(dict(side=n, cells=pb.cells, kernel_variant=k["variant"], gcells_per_s=med,
                        ci95=[lo, hi], seconds_per_sim=pb.cells * steps / (med * 1e9)))
    return dict(workload="freespace2d_sides_250_6400_cpml16_1024steps", steps=steps, runs=runs,
                points=out)


def bench_adjoint(args):
    from paper_2405_00814_amd import workloads as W
    from paper_2405_00814_amd.sim import Sim
    import torch
    pb = W.adjoint2d(1024, steps=4000, seed=0)
    s = Sim.from_problem(pb)
    s.step(50)
    s.reset()
    torch.cuda.synchronize()
    s.step(pb.steps)
    tf, _ = s.last_step_time()
    s.reset()
    loss, grad = s.adjoint_eps(pb.steps, pb.window, pb.design, 0)
    ta, _ = s.last_step_time()
    g = grad.cpu().numpy()
    # the same run holding the design values of all T steps (no recompute:
    # 8 B per design cell and step, 2.1 GB here)
    s.reset()
    loss_f, grad_f = s.adjoint_eps(pb.steps, pb.window, pb.design, pb.steps)
    tn, _ = s.last_step_time()
    same = bool(loss_f == loss and torch.equal(grad_f, grad))
    s.close()
    return dict(workload="adjoint2d_1024x1024_design_256x256_T4000", steps=pb.steps,
                forward_ms=tf, forward_gcells_per_s=pb.cells * pb.steps / (tf / 1e3) / 1e9,
                forward_us_per_step=tf / pb.steps * 1e3, adjoint_ms=ta, adjoint_over_forward=ta / tf,
                checkpoint_interval=int(math.ceil(math.sqrt(pb.steps))),
                no_recompute_ms=tn, no_recompute_over_forward=tn / tf, no_recompute_same_bits=same,
                loss=loss, grad_finite=bool(np.isfinite(g).all()))


def _oracle_rate(planes, target_s, threads=None):
    """Gcell-updates/s of the FP64 oracle on the first `planes` x planes of
    the 512^3 scene (CPML on the five faces it keeps), as many steps as fit
    in about target_s seconds; threads: OpenMP threads (None: all)."""
    import ctypes as C
    from oracle import oracle as O
    from paper_2405_00814_amd import workloads as W
    gomp = C.CDLL("libgomp.so.1")
    pb = W.yee3d(512, steps=1, seed=0)
    sub = (planes, 512, 512)
    o = O.Oracle3D(sub, pb.dx, pb.dt, pb.eps_r[:planes], None, None, (12, 0, 12, 12, 12, 12), pb.cpml)
    o.set_source((min(20, planes - 2), 256, 256), pb.source.kind, pb.source.params)
    o.set_probes([(planes - 2, 100, 100)])
    if threads:
        gomp.omp_set_num_threads(int(threads))
    try:
        o.run(2)  # warm-up (thread start, first touch)
        t0 = time.perf_counter()
        o.run(2)
        t1 = time.perf_counter() - t0
        n = max(2, int(target_s / max(t1 / 2, 1e-3)))
        t0 = time.perf_counter()
        o.run(n)
        t = time.perf_counter() - t0
    finally:
        if threads:
            gomp.omp_set_num_threads(len(os.sched_getaffinity(0)))
    return int(np.prod(sub)) * n / t / 1e9, n, t


def cpu_baseline(target_s=12.0):
    """FP64 oracle on the host cores, on a bounded sample of the headline
    workload: the first 48 x planes (incl. the low CPML slab) of the 512^3
    scene with all cores, the first 12 with one core."""
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    v, n, t = _oracle_rate(48, target_s)
    v1, n1, t1 = _oracle_rate(12, target_s / 3, threads=1)
    return dict(value=v, unit="Gcell-updates/s", cores=cores, kind="oracle",
                cpu_model=cpu_model(), single_thread_value=v1,
                sample="FP64 oracle, first 48 x-planes of the 512^3 scene (48x512x512 cells, "
                       "CPML on 5 faces), %d steps, %.1f s on %d threads; single thread: first 12 "
                       "x-planes, %d steps, %.1f s" % (n, t, cores, n1, t1))


def stream_copy(nbytes=1 << 30, reps=10):
    """The library's copy kernel (fdtd_stream_copy) on two nbytes device
    buffers: bytes read plus written per second, the practical HBM ceiling."""
    import ctypes as C
    import torch
    from paper_2405_00814_amd import _lib as L
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    lib = L.load()

    def go():
        L.check(lib.fdtd_stream_copy(C.c_void_p(b.data_ptr()), C.c_void_p(a.data_ptr()), nbytes,
                                     C.c_void_p(st.cuda_stream)), "fdtd_stream_copy")
    for _ in range(3):
        go()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(reps):
        go()
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(a[:1024], b[:1024]) and torch.equal(a[-1024:], b[-1024:]))
    del a, b
    return dict(bytes=nbytes, ms=ms, GBps=2 * nbytes / (ms / 1e3) / 1e9, correct=ok)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_calibration(nbytes=1 << 30, reps=5):
    """A plain device copy of known size (the library's copy kernel,
    k_stream_copy): the reference point that scales rocprofv3's FETCH_SIZE /
    WRITE_SIZE readings to bytes."""
    r = stream_copy(nbytes, reps)
    print(json.dumps(dict(copy_bytes_read=nbytes, copy_bytes_written=nbytes, reps=reps, ms=r["ms"],
                          GBps=r["GBps"])), flush=True)


def forms_brief():
    """A few steps of every form in its bench configuration: one kernel
    dispatch per step or pass of each, for rocprofv3 counter runs (which
    serialise dispatches)."""
    import torch
    from paper_2405_00814_amd import workloads as W
    from paper_2405_00814_amd.sim import Batch, Sim
    pb = W.dielectric2d(4096, steps=8, seed=0)
    s = Sim.from_problem(pb)
    s.step(8)
    s.close()
    g = Sim.from_problem(pb, graph=True)
    g.step(4)
    g.close()
    b = Batch(W.batch2d(count=256, steps=8, seed=0))
    b.step(8)
    b.close()
    pa = W.adjoint2d(1024, steps=64, seed=0)
    a = Sim.from_problem(pa)
    a.adjoint_eps(64, (32, 64), pa.design, 0)
    a.close()
    torch.cuda.synchronize()
    print(json.dumps(dict(forms_brief="done")), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--tune", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (for scaling HBM counters)")
    ap.add_argument("--forms-brief", action="store_true",
                    help="only a few steps of each form (2D 4096^2, its CSR graph, the 256-problem batch, "
                         "the 1024^2 adjoint), for hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only (the method's independent grids and batches run "
              "one per GPU); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.forms_brief:
        forms_brief()
        return

    r = bench_3d(args)
    pb = r["pb"]
    two = r["dom_steps"] == 2
    src3 = os.path.join(ROOT, "paper_2405_00814_amd", "csrc", "k3dt.hip" if two else "k3dw.hip")
    traffic = traffic_record("yee3d_512_two" if two else "yee3d_512_interior", src3)
    dcells = r["prof"][r["dom"]]["cells"]
    launch_s = r["dom_ms"] / 1e3
    copy = stream_copy()
    # achieved: the algorithmic bytes one launch must move (its cells' state
    # read once and written once, coefficient maps and CPML values once: one
    # pass, whatever the steps it advances) over its mean duration
    achieved = r["dom_pass_bytes"] / launch_s
    roof = dict(bound="hbm", achieved=achieved / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s",
                frac=achieved / PEAK_HBM,
                traffic=traffic,
                traffic_GBps=(traffic / launch_s / 1e9) if traffic else None,
                kernel=("k3d_two launch (interior tiles, two steps per pass, z-slab CPML)" if two
                        else "k3d_march interior launch (z-slab CPML only)"),
                bytes_per_launch=r["dom_pass_bytes"], bytes_per_cell_per_pass=r["dom_bpc"],
                cells_per_launch=dcells, steps_per_launch=r["dom_steps"],
                cell_updates_per_launch=r["dom_steps"] * dcells,
                psi_per_launch=r["prof"][r["dom"]]["psi"], avg_launch_ms=r["dom_ms"],
                stream_copy_GBps=copy["GBps"], frac_of_stream_copy=achieved / 1e9 / copy["GBps"],
                # the same launch counted per cell-update (bytes of one step
                # per step it advances): above 1 when steps share a pass
                step_equiv_achieved=r["dom_achieved"] / 1e9, step_equiv_frac=r["dom_achieved"] / PEAK_HBM,
                step=dict(launches_per_step=r["launches"] / args.steps,
                          bytes_per_step=r["bytes"], bytes_per_cell_update=r["bytes"] / pb.cells,
                          step_equiv_achieved=r["step_achieved"] / 1e9,
                          step_equiv_frac=r["step_achieved"] / PEAK_HBM,
                          launch_ms=[round(x["ms"], 4) for x in r["prof"]],
                          launch_cells=[x["cells"] for x in r["prof"]],
                          launch_steps=[x["steps"] for x in r["prof"]]))
    forms = {}
    if not args.no_forms:
        log("2d ...")
        forms["tmz2d"] = bench_2d(args)
        log("batch ...")
        forms["batched"] = bench_batch(args)
        log("adjoint ...")
        forms["adjoint"] = bench_adjoint(args)
        log("cavity ...")
        forms["cavity128"] = bench_cavity(args)
        log("sweep ...")
        forms["sweep"] = bench_sweep(args)
    cpu = None
    if not args.no_cpu:
        log("cpu baseline ...")
        cpu = cpu_baseline()
    out = {
        "metric": METRIC,
        "value": r["rate"] / 1e9,
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["t"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "yee3d_512x512x512_cpml12_500boxes_gaussian_ez",
                   "cells": pb.cells, "kernel": r["cfg"], "finite": r["finite"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": forms,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
