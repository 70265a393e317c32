#!/usr/bin/env python3
"""Throughput of the reactive-mixture LBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sphere3d|flame_batch]

Default workload: 3D expanding spherical flame, 256^3 D3Q27 lattice, all faces open, 9
species / 19 reversible reactions (seeded synthetic mechanism), FP32 population
storage with FP64 arithmetic.  One step = the whole hot path (moments, temperature,
production rates, Stefan-Maxwell solve, collision of all M+1 sets, non-local
correction stencils, equilibrium ghosts, streaming).  Prints one JSON line.

--workload flame_batch: 256 independent quasi-1D flames of 512..8192 cells (seeded
lengths and equivalence ratios 0.5..3.0, FP32 storage) advanced as one batch lattice,
eagerly and replayed from a HIP graph, against the same 256 lattices stepped one by
one with their own launches (eager, and each replayed from its own graph).
"""
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

METRIC = "reactive MLUPS & % of HBM peak at stated error vs FP64; adjoint/forward cost"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_step_sphere3d_256.json")
# the step kernel's source and the host code that lays out its buffers (plane padding)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2101_01702_amd", "csrc", f) for f in ("lbm_device.hip", "lbm_api.cpp")]


def kernel_source_sha():
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from committed rocprofv3 counters, or None
    when they cover another kernel or the kernel source changed since."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("kernel_source_sha") != kernel_source_sha():
        return None
    return rec


def copy_ceiling_gbs(torch, dev, lbm=None, nbytes=4 << 30, reps=5):
    """Read+write bandwidth of a plain device copy: torch's copy (the runtime's copy
    kernel) and, with the library, its hand-written streaming copy of 16-byte loads and
    stores (lbm_stream_copy).  Returns (runtime copy, streaming kernel) in GB/s."""
    import ctypes as C
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    out = []
    for kind in ("runtime", "stream"):
        if kind == "stream" and lbm is None:
            out.append(None)
            continue
        def once():
            if kind == "runtime":
                b.copy_(a)
            else:
                st = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
                rc = lbm.load().lbm_stream_copy(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), nbytes, st)
                if rc != 0:
                    raise RuntimeError("lbm_stream_copy failed")
        once()
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(reps):
            once()
        torch.cuda.synchronize(dev)
        out.append(2.0 * nbytes / ((time.perf_counter() - t0) / reps) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return tuple(out)


def mix_ceiling_gbs(torch, dev, nbytes=4 << 30, reps=5):
    """Bandwidth of plain streaming kernels with other read:write mixes than a copy's
    1:1: an elementwise c = a + b (2:1, about the step kernel's own mix of counted reads
    and writes) over buffers of nbytes/2 each, and a sum over nbytes (read only).
    Returns (read 2 : write 1, read only) in GB/s of bytes moved."""
    a = torch.ones(nbytes // 8, dtype=torch.float32, device=dev)
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    r = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    out = []
    for moved, once in ((1.5 * nbytes, lambda: torch.add(a, b, out=c)), (1.0 * nbytes, lambda: r.sum())):
        once()
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(reps):
            once()
        torch.cuda.synchronize(dev)
        out.append(moved / ((time.perf_counter() - t0) / reps) / 1e9)
    del a, b, c, r
    torch.cuda.empty_cache()
    return tuple(out)


def host_cpu():
    """(CPU model, logical CPUs the host reports, threads the oracle may use: the box's
    share of 16)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    n = os.cpu_count() or 1
    return model, n, max(1, min(16, n))


def _oracle_rate(prob, threads, seconds):
    from oracle import oracle as orc
    sim = orc.OracleSim(prob).init()
    sim.step(1, threads)
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds or steps < 2:
        sim.step(1, threads)
        steps += 1
    dt = time.perf_counter() - t0
    return prob.N * steps / dt / 1e6, steps, dt


def cpu_baseline(prob=None, label="32^3 crop of the same spherical flame", seconds=8.0):
    """FP64 CPU oracle on a bounded sample of the workload, time-boxed: on all the
    threads of the machine's CPU share and on one thread."""
    from paper_2101_01702_amd import workloads as W
    model, nproc, cores = host_cpu()
    prob = prob or W.sphere3d(shape=(32, 32, 32))
    v_all, st_all, dt_all = _oracle_rate(prob, cores, seconds)
    v_one, st_one, dt_one = _oracle_rate(prob, 1, seconds)
    return {"value": round(v_all, 4), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{label} (M=9, R=19, FP64): {st_all} steps in {dt_all:.1f} s on {cores} threads, "
                      f"{st_one} steps in {dt_one:.1f} s on 1 thread",
            "single_thread_value": round(v_one, 4), "nproc": nproc, "cpu_model": model}


def error_vs_f64(lbm, W, storage, steps=100, prob=None, lattice="32^3 crop"):
    """Normwise field error of the benchmarked storage against FP64 storage on a 32^3
    crop (or on the given problem), with the velocity floor 1e-3 sqrt(zeta_ref)."""
    import numpy as np
    prob = prob or W.sphere3d(shape=(32, 32, 32))
    out = {}
    for st in (W.STORE_F64, storage):
        s = lbm.Solver(prob, storage=st).init()
        s.step(steps)
        out[st] = s.macros()
        s.close()
    a, b = out[storage], out[W.STORE_F64]
    zeta = prob.kappa * W.R_U * prob.T.min() / (1e-3 / (prob.Y[:, 0] / prob.mech.molar_mass).sum())
    errs = {}
    for k in ("rho", "T", "P"):
        errs[k] = float(np.abs(a[k] - b[k]).max() / np.abs(b[k]).max())
    errs["u"] = float(max(np.abs(a["u"][d] - b["u"][d]).max() / max(np.abs(b["u"][d]).max(), 1e-3 * math.sqrt(zeta))
                          for d in range(3)))
    errs["Y"] = float(max(np.abs(a["Y"][k] - b["Y"][k]).max() / max(np.abs(b["Y"][k]).max(), 1e-12)
                          for k in range(prob.M)))
    return {"max_rel": max(errs.values()), "fields": errs, "steps": steps, "lattice": lattice}


def burning_flame(torch, lbm, W, dev, storage, label, n, warm=200, steps=20):
    """A burning 3D lattice beside the specified (non-igniting) sphere: the circular
    flame of Sec. 5.2 extruded along z (n^3, open x and y faces, periodic z, a 2000 K
    cylinder of radius 32), timed over `steps` steps after `warm` steps of burning, and
    the storage's field error against FP64 storage on a 96 x 96 x 4 crop of the same
    flame after 500 steps."""
    prob = W.cylinder3d(n=n, storage=storage)
    s = lbm.Solver(prob, storage=storage, device=dev).init()
    s.step(warm)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize(dev)
    dt = time.perf_counter() - t0
    _, tot = s.diagnostics(1200.0)
    Tmax = float(s.macros(to_numpy=False)["T"].max())
    anomaly = s.status()
    s.close()
    del s
    torch.cuda.empty_cache()
    crop = W.cylinder3d(n=96, nz=4, radius=32.0)
    return {"workload": f"circular flame (Sec. 5.2 geometry) extruded along z, {n}^3, open x/y faces, periodic z, "
                        f"2000 K cylinder of radius 32, {label} population storage",
            "value": round(prob.N * steps / dt / 1e6, 2), "unit": "MLUPS", "ms_per_step": round(dt / steps * 1e3, 3),
            "after_steps": warm, "T_max": round(Tmax, 1), "burnt_cells": int(tot[1]), "anomaly_bits": anomaly,
            "error_vs_f64": error_vs_f64(lbm, W, storage, steps=500, prob=crop, lattice="96x96x4 crop of the burning flame")}


def circular_flame_2d(torch, lbm, W, dev, storage, label, n=1200, warm=200, steps=50, until=3000, every=250,
                      T_iso=1200.0, fit_from=1000):
    """The expanding circular flame of Sec. 5.2 on the paper's grid size, n x n x 1 (open
    x and y faces, a 2000 K disc of radius 32 in the premixture), timed over `steps`
    steps after `warm` steps of burning; then run on to `until` steps, with the mean
    radius of the T_iso isotherm (eq. rmean) every `every` steps, and, from step
    `fit_from` on (after the kernel's first contraction), the growth exponent of
    R = a t^alpha (Sec. 5.2) and the rate dR/dt of a straight line.  The centre is the
    centroid of the initial hot disc."""
    import numpy as np
    prob = W.cylinder3d(n=n, nz=1, storage=storage)
    hot = prob.T - prob.T.min()
    idx = np.arange(prob.N)
    centre = (float((idx % n * hot).sum() / hot.sum()), float((idx // n * hot).sum() / hot.sum()), 0.0)
    s = lbm.Solver(prob, storage=storage, device=dev).init()
    s.step(warm)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize(dev)
    dt = time.perf_counter() - t0
    _, tot = s.diagnostics(T_iso)
    Tmax = float(s.macros(to_numpy=False)["T"].max())
    done, ts, rs = warm + steps, [], []
    for target in range(every * ((done + every - 1) // every), until + 1, every):
        s.step(target - done)
        done = target
        ts.append(target)
        rs.append(round(s.mean_radius(T_iso, centre=centre), 3))
    anomaly = s.status()
    s.close()
    del s
    torch.cuda.empty_cache()
    fit = [(t, r) for t, r in zip(ts, rs) if t >= fit_from]
    _, alpha = lbm.growth_exponent([t for t, _ in fit], [r for _, r in fit])
    rate = float(np.polyfit([t for t, _ in fit], [r for _, r in fit], 1)[0])
    return {"workload": f"circular flame (Sec. 5.2), {n}x{n} (the paper's grid), open x/y faces, 2000 K disc of "
                        f"radius 32, {label} population storage",
            "value": round(prob.N * steps / dt / 1e6, 2), "unit": "MLUPS", "ms_per_step": round(dt / steps * 1e3, 3),
            "after_steps": warm, "T_max": round(Tmax, 1), "burnt_cells": int(tot[1]),
            "mean_radius": {"T_iso": T_iso, "steps": ts, "radius": rs}, "fit_from_step": fit_from,
            "growth_exponent": round(alpha, 4), "radius_rate_cells_per_step": round(rate, 7),
            "anomaly_bits": anomaly}


def error_vs_f64_full(lbm, W, storage, n, steps):
    """The same field error at full size: the benchmarked storage against FP64 storage
    on the n^3 flame after `steps` steps (both runs on the GPU), with the velocity floor
    1e-3 sqrt(zeta_ref) of error_vs_f64."""
    import numpy as np
    import torch
    out = {}
    zeta = None
    for st in (W.STORE_F64, storage):
        prob = W.sphere3d(n=n, storage=st)
        if zeta is None:   # the unburnt lattice RT, as in error_vs_f64
            zeta = prob.kappa * W.R_U * prob.T.min() / (1e-3 / (prob.Y[:, 0] / prob.mech.molar_mass).sum())
        s = lbm.Solver(prob, storage=st).init()
        del prob.rho, prob.u, prob.T, prob.Y
        s.step(steps)
        out[st] = s.macros()
        s.close()
        del s
        torch.cuda.empty_cache()
    a, b = out[storage], out[W.STORE_F64]
    zeta_floor = 1e-3 * math.sqrt(zeta)
    errs = {k: float(np.abs(a[k] - b[k]).max() / np.abs(b[k]).max()) for k in ("rho", "T", "P")}
    errs["u"] = float(max(np.abs(a["u"][d] - b["u"][d]).max() / max(np.abs(b["u"][d]).max(), zeta_floor)
                          for d in range(3)))
    errs["Y"] = float(max(np.abs(a["Y"][k] - b["Y"][k]).max() / max(np.abs(b["Y"][k]).max(), 1e-12)
                          for k in range(b["Y"].shape[0])))
    return {"max_rel": max(errs.values()), "fields": errs, "steps": steps, "lattice": f"{n}^3"}


def cpu_baseline_flame(prob):
    """FP64 CPU oracle on one flame of the batch (the shortest), time-boxed."""
    return cpu_baseline(prob, f"one flame of the batch ({prob.nx} cells)")


def adjoint_cost(torch, lbm, W, dev, storage, every=None):
    """Cost of the discrete adjoint on its workload (the 2048-cell quasi-1D flame, 4000
    steps, a snapshot every `every` steps; None: the spacing FlameFront takes by
    default, the smallest whose snapshots fit in half of the free device memory): the
    forward alone (steps replayed from a graph) against the whole gradient (forward
    with snapshots, then every segment recomputed and reversed step by step), and one
    adjoint step against one forward step."""
    from paper_2101_01702_amd import adjoint as A
    prob = W.adjoint_flame(storage=storage)
    steps = 4000
    sync = lambda: torch.cuda.synchronize(dev)
    s = lbm.Solver(prob, storage=storage, device=dev, adjoint=True).init()
    policy = "fixed"
    if every is None:
        free, _ = torch.cuda.mem_get_info(dev)
        every = A.snapshot_spacing(steps, s.state_size(), 0.5 * free)
        policy = f"the smallest that fits half of the {free / 2**30:.0f} GiB free"
    s.step_graph(steps)                      # records the graph
    s.init()
    sync()
    t0 = time.perf_counter()
    s.step_graph(steps)
    sync()
    fwd = time.perf_counter() - t0
    theta = torch.tensor(A.theta_of(prob.mech), dtype=torch.float64, requires_grad=True)
    T0 = torch.tensor(prob.T, dtype=torch.float64, requires_grad=True)
    sync()
    t0 = time.perf_counter()
    J = A.FlameFront.apply(s, theta, T0, steps, every)
    J.backward()
    sync()
    grad_wall = time.perf_counter() - t0
    # one adjoint step against one forward step, both eager, over 200 steps of the flame
    snap = s.state_save()
    lam = torch.ones(s.S, 27, s.N, dtype=torch.float64, device=dev)
    g = torch.zeros(prob.mech.R, 3, dtype=torch.float64, device=dev)
    sync()
    t0 = time.perf_counter()
    for _ in range(200):
        s.step(1)
    sync()
    f1 = (time.perf_counter() - t0) / 200
    t0 = time.perf_counter()
    for _ in range(200):
        s.adjoint_step(lam, state=snap, grad=g)
    sync()
    a1 = (time.perf_counter() - t0) / 200
    ok = bool(np.isfinite(theta.grad.numpy()).all() and np.isfinite(T0.grad.numpy()).all())
    anomaly = s.status()
    snap_bytes = s.state_size()
    s.close()
    return {"workload": f"quasi-1D flame of {prob.N} cells, 9 species, 19 reactions, {steps} steps, snapshot every "
                        f"{every}, {('f64', 'f32')[storage]} storage, FP64 adjoint",
            "snapshot_every": int(every), "snapshot_policy": policy,
            "snapshot_bytes": int(snap_bytes),
            "gradient_over_forward": round(grad_wall / fwd, 3), "forward_s": round(fwd, 4),
            "gradient_s": round(grad_wall, 4), "adjoint_step_ms": round(a1 * 1e3, 4),
            "forward_step_ms": round(f1 * 1e3, 4), "adjoint_step_over_forward_step": round(a1 / f1, 3),
            "parameters": int(3 * prob.mech.R), "finite": ok, "anomaly_bits": anomaly}


def bench_flame_batch(args, torch, lbm, W, dev):
    """The batch of 256 ragged flames: one lattice of segments, eager and graph
    replayed, against the 256 lattices stepped one by one."""
    prob = W.flame_batch(storage=W.STORE_F32)
    parts = W.split_batch(prob)
    M, N, K = prob.M, prob.N, args.steps
    sync = lambda: torch.cuda.synchronize(dev)
    solver = lbm.Solver(prob, storage=W.STORE_F32, device=dev).init()
    solver.step(args.warmup)
    sync()
    t0 = time.perf_counter()
    solver.step(K)
    sync()
    wall_eager = time.perf_counter() - t0
    solver.step_graph(K)            # records the graph, then replays it
    sync()
    t0 = time.perf_counter()
    solver.step_graph(K)
    sync()
    wall_graph = time.perf_counter() - t0
    kernel_ms = solver.step_timed(K)
    anomaly = solver.status()
    solver.close()
    del solver
    torch.cuda.empty_cache()

    sep = [lbm.Solver(p, storage=W.STORE_F32, device=dev).init() for p in parts]
    for s in sep:
        s.step(args.warmup)
    sync()
    t0 = time.perf_counter()
    for s in sep:
        s.step(K)
    sync()
    wall_sep = time.perf_counter() - t0
    for s in sep:                   # the same lattices with their steps replayed from graphs
        s.step_graph(K)
    sync()
    t0 = time.perf_counter()
    for s in sep:
        s.step_graph(K)
    sync()
    wall_sep_graph = time.perf_counter() - t0
    anomaly |= max(s.status() for s in sep)
    for s in sep:
        s.close()
    del sep
    torch.cuda.empty_cache()

    mlups = lambda wall: N * K / wall / 1e6
    alg_bytes_node = 2 * 27 * (M + 1) * 4
    step_ms = kernel_ms["step"] / K
    achieved = alg_bytes_node * N / (step_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(mlups(wall_graph), 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(wall_graph * 1e3 / K, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": f"batch of {len(parts)} quasi-1D flames, {N} cells (512..8192 each), 9 species, "
                               "19 reversible reactions, f32 population storage; FP64 temperature, thermo, rates and "
                               "Stefan-Maxwell solve, FP32 inter-species term",
                   "flames": len(parts), "cells": N, "species": M, "reactions": 19, "storage": "f32",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": "k_step", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "alg_bytes_per_node": alg_bytes_node},
        "kernel_ms_per_step": {k: round(v / K, 4) for k, v in kernel_ms.items()},
        "batch_eager_mlups": round(mlups(wall_eager), 2),
        "batch_graph_mlups": round(mlups(wall_graph), 2),
        "separate_lattices_mlups": round(mlups(wall_sep), 2),
        "separate_lattices_graph_mlups": round(mlups(wall_sep_graph), 2),
        "speedup_vs_separate": round(wall_sep / wall_graph, 2),
        "anomaly_bits": anomaly,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_flame(parts[int(min(range(len(parts)), key=lambda k: parts[k].nx))])
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256, help="lattice edge (256 = the benchmarked workload)")
    ap.add_argument("--workload", choices=("sphere3d", "flame_batch"), default="sphere3d")
    ap.add_argument("--storage", choices=("f32", "f64", "f16dev", "bf16dev"), default="f32",
                    help="population storage (f16dev/bf16dev: 16-bit deviations from the reference state)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error-check", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint cost measurement")
    ap.add_argument("--copy-only", action="store_true", help="run only the copy kernel (counter calibration)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint cost measurement (profiling the adjoint kernels)")
    ap.add_argument("--full-error-steps", type=int, default=0,
                    help="also measure the field error against FP64 storage at full size after this many steps")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the step has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2101_01702_amd import lbm
    from paper_2101_01702_amd import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_only:
        cc = copy_ceiling_gbs(torch, dev, lbm)
        mc = mix_ceiling_gbs(torch, dev)
        print(json.dumps({"copy_ceiling_GBps": {"runtime_copy": round(cc[0], 1), "stream_kernel": round(cc[1], 1),
                                                "read2_write1": round(mc[0], 1), "read_only": round(mc[1], 1)},
                          "bytes": 2 * (4 << 30)}))
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_cost(torch, lbm, W, dev, W.STORE_F32),
                          "adjoint_every_100": adjoint_cost(torch, lbm, W, dev, W.STORE_F32, every=100)}))
        return
    if args.workload == "flame_batch":
        bench_flame_batch(args, torch, lbm, W, dev)
        return

    storage = {"f32": W.STORE_F32, "f64": W.STORE_F64, "f16dev": W.STORE_F16_DEV,
               "bf16dev": W.STORE_BF16_DEV}[args.storage]
    word = {W.STORE_F64: 8, W.STORE_F32: 4}.get(storage, 2)
    prob = W.sphere3d(n=args.n, storage=storage)
    M = prob.M
    N = prob.N
    solver = lbm.Solver(prob, storage=storage, device=dev).init()
    del prob.rho, prob.u, prob.T, prob.Y
    torch.cuda.synchronize(dev)
    solver.step(args.warmup)
    if solver.status():
        raise RuntimeError("device anomaly during warm-up")
    torch.cuda.synchronize(dev)

    t0 = time.perf_counter()
    kernel_ms = solver.step_timed(args.steps)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    anomaly = solver.status()
    solver.close()
    del solver
    torch.cuda.empty_cache()

    mlups = N * args.steps / wall / 1e6
    ms_per_step = wall * 1e3 / args.steps
    # Algorithmic bytes per node of the step: every population of the M+1 sets read
    # once and written once.  The stream-and-collide kernel moves exactly these; the
    # stencil and ghost kernels move no population of the method (overhead).
    alg_bytes_node = 2 * 27 * (M + 1) * word
    kernel_alg_bytes = {"step": alg_bytes_node}
    dominant = max(kernel_ms, key=kernel_ms.get)
    dom_ms = kernel_ms[dominant] / args.steps
    dom_bytes = kernel_alg_bytes.get(dominant, 0)
    achieved = dom_bytes * N / (dom_ms * 1e-3) / 1e9
    rec = recorded_traffic(f"k_{dominant}")
    traffic = rec["traffic_bytes_per_launch"] if (rec and args.n == 256 and storage == W.STORE_F32) else None
    roofline = {"bound": "hbm", "kernel": f"k_{dominant}", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "alg_bytes_per_node": dom_bytes}

    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": f"spherical flame {args.n}^3 D3Q27, 9 species, 19 reversible reactions, "
                               f"{args.storage} population storage; FP64 temperature, thermo, rates and "
                               "Stefan-Maxwell solve, FP32 inter-species term",
                   "lattice": [args.n] * 3, "species": M, "reactions": 19, "storage": args.storage,
                   "state": "non-igniting: the 1500 K kernel of radius 12 cools over the timed steps",
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "kernel_ms_per_step": {k: round(v / args.steps, 4) for k, v in kernel_ms.items()},
        "whole_step_hbm_frac": round(alg_bytes_node * N / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "anomaly_bits": anomaly,
    }
    if not args.no_error_check:
        out["error_vs_f64"] = error_vs_f64(lbm, W, storage)
        out["burning_flame"] = burning_flame(torch, lbm, W, dev, storage, args.storage, args.n)
        out["circular_flame_2d"] = circular_flame_2d(torch, lbm, W, dev, storage, args.storage)
    if args.full_error_steps > 0 and storage != W.STORE_F64:
        out["error_vs_f64_full"] = error_vs_f64_full(lbm, W, storage, args.n, args.full_error_steps)
    cc_runtime, cc_stream = copy_ceiling_gbs(torch, dev, lbm)
    mc = mix_ceiling_gbs(torch, dev)
    out["copy_ceiling_GBps"] = {"runtime_copy": round(cc_runtime, 1), "stream_kernel": round(cc_stream, 1),
                                "read2_write1": round(mc[0], 1), "read_only": round(mc[1], 1)}
    if not args.no_adjoint:
        out["adjoint"] = adjoint_cost(torch, lbm, W, dev, W.STORE_F32)
        out["adjoint_every_100"] = adjoint_cost(torch, lbm, W, dev, W.STORE_F32, every=100)
        out["adjoint_forward_cost"] = out["adjoint"]["gradient_over_forward"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
