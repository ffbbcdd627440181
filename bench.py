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
    # hbm_frac: algorithmic bytes per cell-update x cell-updates/s; a pass of
    # tb steps moves one step's bytes, so pass_frac is the memory-side view
    out = dict(workload="dielectric2d_4096x4096_cpml16_200rects", steps=steps,
               kernel=k, steps_per_pass=tb, gcells_per_s=pb.cells * steps / t / 1e9,
               bytes_per_cell_update=ab / pb.cells,
               achieved_GBps=ab * steps / t / 1e9,
               hbm_frac=ab * steps / t / PEAK_HBM,
               pass_frac=ab * steps / tb / t / PEAK_HBM)
    sim.close()
    # explicit graph form on the same grid
    g = Sim.from_problem(pb, graph=True)
    gs = 200
    tg, _, lg = timed_steps(g, gs, 5)
    gbytes = csr_alg_bytes(pb)
    out["graph_form"] = dict(steps=gs, gcells_per_s=pb.cells * gs / tg / 1e9,
                             bytes_per_cell_update=gbytes / pb.cells,
                             achieved_GBps=gbytes * gs / tg / 1e9,
                             hbm_frac=gbytes * gs / tg / PEAK_HBM, launches_per_step=lg / gs)
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


def csr_alg_bytes(pb):
    """Algorithmic bytes of one CSR step: every matrix entry (column index and
    weight) and every row pointer / destination index read once, every node
    value read once and every updated node written once."""
    nx, ny = pb.shape
    N = nx * ny
    sx, sy = pb.npml[0] + pb.npml[1], pb.npml[2] + pb.npml[3]
    npsi = 2 * nx * sy + 2 * sx * ny
    nnz_h = 2 * N * 3 + 2 * nx * sy // 2 + 2 * sx * ny // 2  # field rows + psi edges
    nnz_h += 3 * (nx * sy + sx * ny)                          # psi rows
    nnz_e = 5 * N + (nx * sy + sx * ny) + 3 * (nx * sy + sx * ny)
    rows = 3 * N + npsi
    nodes = 3 * N + npsi
    return 8 * (nnz_h + nnz_e) + 8 * rows + 4 * nodes * 2 + 4 * rows


def bench_batch(args, steps=500):
    from paper_2405_00814_amd import workloads as W
    from paper_2405_00814_amd.sim import Batch, Sim
    import torch
    probs = W.batch2d(count=256, steps=steps, seed=0)
    cells = sum(p.cells for p in probs)
    log("batch: %d problems, %.3e cells" % (len(probs), cells))
    b = Batch(probs)
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
                cells=cells, steps=steps, steps_per_pass=4, gcells_per_s=cells * steps / tb / 1e9,
                hbm_frac=ab * steps / tb / PEAK_HBM, pass_frac=ab * steps / 4 / tb / PEAK_HBM,
                plain_sequential_gcells_per_s=cells * steps / tp / 1e9,
                speedup_vs_plain=tp / tb, launches=lb, finite=bool(ok))


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
                forward_ms=tf, adjoint_ms=ta, adjoint_over_forward=ta / tf,
                checkpoint_interval=int(math.ceil(math.sqrt(pb.steps))),
                no_recompute_ms=tn, no_recompute_over_forward=tn / tf, no_recompute_same_bits=same,
                loss=loss, grad_finite=bool(np.isfinite(g).all()))


def cpu_baseline(target_s=15.0):
    """FP64 oracle on the host cores, on a bounded sample of the headline
    workload: the first 48 x planes (incl. the low CPML slab) of the 512^3
    scene, with as many steps as fit in about target_s seconds."""
    from oracle import oracle as O
    from paper_2405_00814_amd import workloads as W
    pb = W.yee3d(512, steps=1, seed=0)
    sub = (48, 512, 512)
    o = O.Oracle3D(sub, pb.dx, pb.dt, pb.eps_r[:48], None, None, (12, 0, 12, 12, 12, 12), pb.cpml)
    o.set_source((20, 256, 256), pb.source.kind, pb.source.params)
    o.set_probes([(30, 100, 100)])
    o.run(2)  # warm-up (thread start, first touch)
    t0 = time.perf_counter()
    o.run(4)
    t1 = time.perf_counter() - t0
    n = max(2, int(target_s / max(t1 / 4, 1e-3)))
    t0 = time.perf_counter()
    o.run(n)
    t = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    return dict(value=int(np.prod(sub)) * n / t / 1e9, unit="Gcell-updates/s", cores=cores,
                kind="oracle",
                sample="FP64 oracle, first 48 x-planes of the 512^3 scene (48x512x512 cells, "
                       "CPML on 5 faces), %d steps, %.1f s" % (n, t))


def copy_calibration(nbytes=1 << 30, reps=5):
    """A plain device copy of known size (torch's copy kernel): the reference
    point that scales rocprofv3's FETCH_SIZE / WRITE_SIZE readings to bytes."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps(dict(copy_bytes_read=nbytes, copy_bytes_written=nbytes, reps=reps, ms=ms,
                          GBps=2 * nbytes / (ms / 1e3) / 1e9)), flush=True)


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

    r = bench_3d(args)
    pb = r["pb"]
    two = r["dom_steps"] == 2
    src3 = os.path.join(ROOT, "paper_2405_00814_amd", "csrc", "k3dt.hip" if two else "k3dw.hip")
    traffic = traffic_record("yee3d_512_two" if two else "yee3d_512_interior", src3)
    dcells = r["prof"][r["dom"]]["cells"]
    roof = dict(bound="hbm", achieved=r["dom_achieved"] / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s",
                frac=r["dom_achieved"] / PEAK_HBM, traffic=traffic,
                kernel=("k3d_two launch (interior tiles, two steps per pass, z-slab CPML)" if two
                        else "k3d_march interior launch (z-slab CPML only)"),
                bytes_per_launch=r["dom_bytes"], bytes_per_cell_update=r["dom_bpc"],
                steps_per_launch=r["dom_steps"], cells_per_launch=dcells,
                cell_updates_per_launch=r["dom_steps"] * dcells,
                psi_per_launch=r["prof"][r["dom"]]["psi"], avg_launch_ms=r["dom_ms"],
                min_bytes_per_launch=r["dom_pass_bytes"],
                pass_frac=r["dom_pass_bytes"] / (r["dom_ms"] / 1e3) / PEAK_HBM,
                step=dict(launches_per_step=r["launches"] / args.steps,
                          bytes_per_step=r["bytes"], bytes_per_cell_update=r["bytes"] / pb.cells,
                          achieved=r["step_achieved"] / 1e9, frac=r["step_achieved"] / PEAK_HBM,
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
