#!/usr/bin/env python3
"""Throughput of the partition/estimation hot path on one MI355X.

One step = one whole pass over a 110,000-atom synthetic assembly already
resident in HBM: atom binning and neighbourhood lists, the adaptive partition
and estimation (Section 2.2, Steps 1-3, h0 = 2 -> h_min = 0.25, tau = 1e-3,
D = 0.9, c = 1), corner classification, and the edge intersection points.

Printed: one JSON line.  ``value`` is cubes estimated per second (cubes
whose coefficient tensor was computed, summed over levels, divided by the
step time) for the FP32+guard path; the FP64 path, phi evaluations per
second, the dominant kernel's roofline position and the FP64 CPU oracle's
rate on a bounded sample ride along in the same line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

# MI355X published peaks (per GPU)
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of k_estimate_tiled from rocprofv3 FETCH_SIZE and
# WRITE_SIZE, each scaled by what the same counter reads for a plain copy of
# known size (FETCH x2.0, WRITE x1.0), mean of the level-2 and level-3
# launches on the 110,000-atom assembly (profiles/estimate_tiled_assembly110k_traffic.md);
# None when the kernel changed since the counters were taken
TRAFFIC_TILED = 12.16e9

# algorithmic work per unit
FLOP_PER_PAIR = 148      # rank-one update of a 4x4x4 tensor: 64 FMA + 20 MUL
FLOP_PER_PHI_PAIR = 14   # phi + grad per in-range (point, atom) pair, excl. exp


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_mode(ctx, tms, atoms_dev, w, precision, steps, warmup):
    import torch
    p = w.params(precision)
    cells = ctx.build_cells(atoms_dev, p)
    leaves, cphi, st = ctx.partition_estimate(cells)
    verts = ctx.extract(cells, leaves, cphi)
    # sized for the captured pass as well, which writes into these buffers
    cap_l, cap_v = ctx.graph_capacity(cells, margin=1.1)
    lb = torch.empty((cap_l, 20), dtype=torch.uint8, device=ctx.device)
    cb = torch.empty((cap_l, 8), dtype=torch.float64, device=ctx.device)
    vb = torch.empty((cap_v, 40), dtype=torch.uint8, device=ctx.device)

    def step():
        ctx.build_cells(atoms_dev, p, cells)
        nl, s = ctx.partition_into(cells, lb, cb)
        nv = ctx.extract_into(cells, lb, nl, cb, vb)
        return nl, nv, s

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ctx.get_timing(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        nl, nv, s = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = ctx.get_timing(reset=True)
    ctx.set_timing(False)
    sd = s.as_dict()
    ms = (t1 - t0) * 1e3 / steps
    per_step = {k: {"ms": v["ms"] / steps, "launches": v["launches"] / steps}
                for k, v in tm.items()}
    # the same pass replayed from a captured graph (build eager, rest one
    # graph) that writes its results into lb, cb, vb
    ctx.graph_capture(cells, margin=1.1, leaves=lb, cphi=cb, verts=vb)

    def gstep():
        ctx.build_cells(atoms_dev, p, cells)
        return ctx.graph_launch(cells, lb, cb, vb)

    for _ in range(warmup):
        gstep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        gnl, gnv, _ = gstep()
    torch.cuda.synchronize()
    gms = (time.perf_counter() - t0) * 1e3 / steps
    assert gnl == nl and gnv == nv
    ctx.free_cells(cells)
    return dict(ms_per_step=ms, stats=sd, n_leaves=nl, n_vertices=nv, timing=per_step,
                graph_ms_per_step=gms)


def run_adjoint(ctx, tms, steps, warmup):
    """Differentiation workload: forward pass (partition, corners, edge
    points) and the adjoint of the surface loss on a 20,000-atom globule."""
    import torch
    from paper_1611_03474_amd import workloads
    w = workloads.GLOBULE20K_ADJOINT
    atoms = torch.as_tensor(workloads.atoms(w), dtype=torch.float64, device="cuda:0")
    p = w.params(tms.PREC_FP32_GUARD)
    cells = ctx.build_cells(atoms, p)
    leaves, cphi, st = ctx.partition_estimate(cells)
    verts = ctx.extract(cells, leaves, cphi)
    _, phi = ctx.get_corners()
    t = tms.vertex_t(verts).clone()
    h = tms.vertex_edge_h(verts, w.h0)
    dphi = (2.0 * (phi - w.c)).contiguous()
    dt = (2.0 * (t - 0.5) * h * h).contiguous()
    g = torch.empty((atoms.shape[0], 4), dtype=torch.float64, device="cuda:0")
    for _ in range(warmup):
        ctx.backward(cells, dphi, dt, out=g)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ctx.get_timing(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.backward(cells, dphi, dt, out=g)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = ctx.get_timing(reset=True)
    ctx.set_timing(False)
    ctx.free_cells(cells)
    return {"workload": w.name, "atoms": int(atoms.shape[0]), "leaves": int(leaves.shape[0]),
            "corners": int(phi.shape[0]), "vertices": int(t.shape[0]),
            "backward_ms": (t1 - t0) * 1e3 / steps,
            "backward_device_ms": tm["backward"]["ms"] / steps,
            "atoms_per_s": atoms.shape[0] / ((t1 - t0) / steps)}


def run_batch(ctx, tms, confs, steps, warmup):
    """Batched refinement: every conformation of the batch in one pass
    (build, partition, extract), after the library's autotuner picked the
    launch shapes; beside it the same conformations one pass each, in
    FP32+guard and in FP64."""
    import numpy as np
    import torch
    from paper_1611_03474_amd import workloads
    w = workloads.BATCH256
    p = w.params(tms.PREC_FP32_GUARD)
    off = np.zeros(len(confs) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(c) for c in confs])
    a = torch.as_tensor(np.concatenate(confs, axis=0), dtype=torch.float64, device="cuda:0")
    singles = [torch.as_tensor(c, dtype=torch.float64, device="cuda:0") for c in confs]
    cells = ctx.build_cells_batch((a, off), p)
    tuning, tune_ms, tune_n = ctx.autotune(cells)
    leaves, cphi, st = ctx.partition_estimate(cells)
    verts = ctx.extract(cells, leaves, cphi)
    del leaves, cphi, verts
    # sized for the captured pass as well, which writes into these buffers
    cap_l, cap_v = ctx.graph_capacity(cells, margin=1.1)
    lb = torch.empty((cap_l, 20), dtype=torch.uint8, device="cuda:0")
    cb = torch.empty((cap_l, 8), dtype=torch.float64, device="cuda:0")
    vb = torch.empty((cap_v, 40), dtype=torch.uint8, device="cuda:0")

    def step():
        ctx.build_cells_batch((a, off), p, cells)
        nl, s_ = ctx.partition_into(cells, lb, cb)
        nv = ctx.extract_into(cells, lb, nl, cb, vb)
        return nl, nv, s_

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        nl, nv, s_ = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    sd = s_.as_dict()
    # one captured graph for the whole batched pass, writing into lb, cb, vb
    ctx.graph_capture(cells, margin=1.1, leaves=lb, cphi=cb, verts=vb)

    def gstep():
        ctx.build_cells_batch((a, off), p, cells)
        return ctx.graph_launch(cells, lb, cb, vb)

    for _ in range(warmup):
        gstep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        gnl, gnv, _ = gstep()
    torch.cuda.synchronize()
    gms = (time.perf_counter() - t0) * 1e3 / steps
    assert gnl == nl and gnv == nv
    ctx.free_cells(cells)

    def loop(prec):
        # the same conformations one pass each (the first sweep warms up)
        pp = w.params(prec)
        c1 = None
        dt = 0.0
        for sweep in range(2):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for c in singles:
                c1 = ctx.build_cells(c, pp, c1)
                n1, _ = ctx.partition_into(c1, lb, cb)
                ctx.extract_into(c1, lb, n1, cb, vb)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t1) * 1e3
        ctx.free_cells(c1)
        return dt

    loop32 = loop(tms.PREC_FP32_GUARD)
    loop64 = loop(tms.PREC_FP64)
    est = int(sum(sd["n_est"]))
    return {"workload": w.name, "conformations": len(confs), "atoms": int(off[-1]),
            "leaves": int(nl), "vertices": int(nv), "cubes_estimated": est,
            "ms_per_pass": ms, "cubes_per_s": est / (ms * 1e-3),
            "graph_ms_per_pass": gms, "graph_cubes_per_s": est / (gms * 1e-3),
            "tuning": tuning, "autotune_best_ms": tune_ms, "autotune_passes": tune_n,
            "loop_fp32g_ms": loop32, "loop_fp64_ms": loop64,
            "speedup_vs_loop_fp32g": loop32 / ms, "speedup_vs_loop_fp64": loop64 / ms}


def cpu_baseline(atoms, w, n_glob=4):
    """FP64 oracle on a bounded sample: the first n_glob globules of the
    assembly with their hydrogens (about n_glob/20 of the workload)."""
    import oracle
    from paper_1611_03474_amd import workloads
    sample = workloads.assembly_slice(atoms, n_glob)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    t0 = time.perf_counter()
    r = oracle.partition(sample, w.D, c=w.c, tau=w.tau, h0=w.h0, h_min=w.h_min, pad=w.pad,
                         eps_cut=w.eps_cut, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": r.cubes_estimated / dt, "unit": "cubes/s", "cores": threads,
            "kind": "oracle",
            "sample": "globules 0-%d of the assembly with their hydrogens (%d atoms, %d cubes "
                      "estimated, %.1f s wall)" % (n_glob - 1, len(sample), r.cubes_estimated, dt)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint workload")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--workload", default="assembly110k")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device-to-device copy first (counter scale for HBM traffic)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1611_03474_amd import tms, workloads

    w = workloads.ALL[args.workload]
    log("generating workload", w.name)
    t0 = time.perf_counter()
    atoms = workloads.atoms(w)
    log("  %d atoms in %.1f s" % (len(atoms), time.perf_counter() - t0))
    batch_confs = None
    if not args.no_batch:
        t0 = time.perf_counter()
        batch_confs = workloads.atoms(workloads.BATCH256)
        log("  batch of %d conformations (%d atoms) in %.1f s"
            % (len(batch_confs), sum(len(c) for c in batch_confs), time.perf_counter() - t0))
    atoms_dev = torch.as_tensor(atoms, dtype=torch.float64, device="cuda:0").contiguous()
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = tms.Context(0)

    log("FP32+guard run")
    f32 = run_mode(ctx, tms, atoms_dev, w, tms.PREC_FP32_GUARD, args.steps, args.warmup)
    log("  %.2f ms/step" % f32["ms_per_step"])
    f64 = None
    if not args.no_fp64:
        log("FP64 run")
        f64 = run_mode(ctx, tms, atoms_dev, w, tms.PREC_FP64, args.steps, args.warmup)
        log("  %.2f ms/step" % f64["ms_per_step"])

    def rates(r):
        st = r["stats"]
        return {"cubes_per_s": st["cubes_estimated"] / (r["ms_per_step"] * 1e-3),
                "phi_evals_per_s": st["n_corners"] / (r["timing"]["phi"]["ms"] * 1e-3)
                if r["timing"]["phi"]["ms"] > 0 else None}

    r32 = rates(f32)
    st = f32["stats"]
    # dominant kernel: the wave-per-chunk tensor estimate on the two deep
    # levels.  Its rank-one updates run in FP64 in both modes, so the FP64
    # vector peak applies; algorithmic work = in-range (cube, atom) pairs at
    # those levels x FLOP_PER_PAIR.
    tm = f32["timing"]
    deep_pairs = sum(st["n_pairs_lvl"][2:4])
    launches = tm["tiled"]["launches"]
    avg_launch_s = tm["tiled"]["ms"] * 1e-3 / max(launches, 1)
    work_per_launch = deep_pairs * FLOP_PER_PAIR / max(launches, 1)
    achieved = work_per_launch / avg_launch_s / 1e12
    roofline = {"bound": "alu", "kernel": "k_estimate_tiled (levels 2-3)",
                "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": TRAFFIC_TILED if w.name == "assembly110k" else None,
                "traffic_unit": "HBM bytes per launch",
                "work_per_unit": "%d flop per in-range (cube, atom) pair" % FLOP_PER_PAIR,
                "units_per_launch": deep_pairs / max(launches, 1),
                "launches_per_step": launches,
                "avg_launch_ms": avg_launch_s * 1e3}

    out = {
        "metric": "cubes estimated/sec and phi evals/sec at 100k atoms, FP32+guard vs FP64",
        "value": r32["cubes_per_s"],
        "unit": "cubes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "description": w.description, "atoms": int(len(atoms)),
                   "D": w.D, "c": w.c, "tau": w.tau, "h0": w.h0, "h_min": w.h_min,
                   "precision": "fp32+fp64 guard"},
        "phi_evals_per_s": r32["phi_evals_per_s"],
        "graph_ms_per_step": f32["graph_ms_per_step"],
        "graph_cubes_per_s": st["cubes_estimated"] / (f32["graph_ms_per_step"] * 1e-3),
        "cubes_estimated": st["cubes_estimated"],
        "per_level_estimated": st["n_est"][:4],
        "leaves": f32["n_leaves"], "surface_leaves": st["n_surface"],
        "unique_corners": st["n_corners"], "vertices": f32["n_vertices"],
        "pairs": st["n_pairs"], "bound_cubes": st["n_bound"],
        "guard_cubes": st["guard_cubes"], "guard_points": st["guard_points"],
        "guard_cube_fraction": st["guard_cubes"] / max(1, st["cubes_estimated"]),
        "device_ms_per_step": {k: round(v["ms"], 4) for k, v in tm.items()},
        "pairs_per_level": st["n_pairs_lvl"][:4],
        "roofline": roofline,
    }
    if f64 is not None:
        r64 = rates(f64)
        out["fp64"] = {"value": r64["cubes_per_s"], "ms_per_step": f64["ms_per_step"],
                       "graph_ms_per_step": f64["graph_ms_per_step"],
                       "phi_evals_per_s": r64["phi_evals_per_s"],
                       "device_ms_per_step": {k: round(v["ms"], 4)
                                              for k, v in f64["timing"].items()},
                       "same_leaf_count": f64["n_leaves"] == f32["n_leaves"]}
        out["speedup_fp32guard_vs_fp64"] = f64["ms_per_step"] / f32["ms_per_step"]
    if batch_confs is not None:
        log("batch run")
        out["batch"] = run_batch(ctx, tms, batch_confs, args.steps, args.warmup)
        log("  %.1f ms per batched pass, %.1f ms looped FP32+guard, %.1f ms looped FP64"
            % (out["batch"]["ms_per_pass"], out["batch"]["loop_fp32g_ms"],
               out["batch"]["loop_fp64_ms"]))
    if not args.no_adjoint:
        log("adjoint run")
        out["adjoint"] = run_adjoint(ctx, tms, args.steps, args.warmup)
        log("  %.2f ms per backward" % out["adjoint"]["backward_ms"])
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(atoms, w)
        log("  %s" % out["cpu_baseline"])
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
