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
TRAFFIC_TILED = 12.55e9

# algorithmic work per unit
FLOP_PER_PAIR = 148      # rank-one update of a 4x4x4 tensor: 64 FMA + 20 MUL
# phi at a corner, per in-range (point, atom) pair: 8 VALU lane-ops (3 sub,
# 3 FMA for the squared distance, 1 FMA for the scaled exponent, 1 add) plus
# one single-precision exponential, which issues at a quarter of the VALU
# rate (4 lane-op slots)
OPS_PER_PHI_PAIR = 8 + 4
# VALU lane-op issue peak: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
PEAK_VALU_TOPS = 39.3
# single-precision exponentials (v_exp_f32, quarter rate): 39.3 / 4 T/s
PEAK_TRANS_TOPS = PEAK_VALU_TOPS / 4
# FP64 flop slots the nested-SVD bound issues per hard cube: the
# SQ_INSTS_VALU_FLOPS_FP64 counter over five passes' k_bound launches (it
# counts per wavefront instruction, FMA as two), times 64 lanes, divided by
# the hard cubes of those passes (profiles/counters_assembly110k_fp32guard.md).
# Lanes masked off by divergence are included, so it is an upper bound on the
# flops the bound needs; the number of Jacobi sweeps and of inner problems
# varies per cube, so there is no fixed algorithmic count.
FLOP_PER_HARD_CUBE = 9256


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_steps(fn, steps):
    """Wall time of each of `steps` calls of fn (each ends synchronised);
    returns (list of ms, the last result)."""
    import torch
    out, r = [], None
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        out.append((time.perf_counter() - t0) * 1e3)
    return out, r


def spread(ms):
    import numpy as np
    a = np.asarray(ms)
    return {"mean": float(a.mean()), "median": float(np.median(a)), "min": float(a.min()),
            "max": float(a.max()), "p10": float(np.percentile(a, 10)),
            "p90": float(np.percentile(a, 90)), "n": int(len(a))}


def run_mode(ctx, tms, atoms_dev, w, precision, steps, warmup, with_mesh=False):
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
    step_ms, (nl, nv, s) = timed_steps(step, steps)
    tm = ctx.get_timing(reset=True)
    ctx.set_timing(False)
    sd = s.as_dict()
    per_step = {k: {"ms": v["ms"] / steps, "launches": v["launches"] / steps}
                for k, v in tm.items()}
    # algorithmic work of the corner values: the pairs phi sums over the
    # pass's unique corners (kept in ctx)
    cxyz, _ = ctx.get_corners()
    phi_pairs = ctx.debug_phi_pairs(cells, cxyz)
    del cxyz
    # stage-two points (Section 2.3) of the pass's leaves, outside the step
    ctx.set_timing(True)
    ctx.get_timing(reset=True)
    s2_ms, (s2rec, s2deg) = timed_steps(lambda: ctx.stage2_points(cells, lb[:nl], cb[:nl]), 3)
    s2tm = ctx.get_timing(reset=True)
    ctx.set_timing(False)
    stage2 = {"records": int(s2rec.shape[0]), "degenerate": s2deg,
              "ms_median": spread(s2_ms)["median"],
              "device_ms": s2tm["stage2"]["ms"] / 3,
              "leaves_per_s": nl / (spread(s2_ms)["median"] * 1e-3)}
    del s2rec
    # the same pass replayed from a captured graph (build eager, rest one
    # graph) that writes its results into lb, cb, vb
    ctx.graph_capture(cells, margin=1.1, leaves=lb, cphi=cb, verts=vb)

    def gstep():
        ctx.build_cells(atoms_dev, p, cells)
        return ctx.graph_launch(cells, lb, cb, vb)

    for _ in range(warmup):
        gstep()
    g_ms, (gnl, gnv, _) = timed_steps(gstep, steps)
    assert gnl == nl and gnv == nv
    # the Stage-2 mesh (host, Section 2.3) of the pass's leaves (the
    # replays wrote the same ones into lb, cb, vb) with open
    # faces closed, and its manifold checks (a), (b) (no intersection test at
    # this size), outside the step
    mesh = None
    if with_mesh:
        m_ms, m = timed_steps(lambda: ctx.mesh_build(cells, lb[:nl], cb[:nl], vb[:nv]), 1)
        t0 = time.perf_counter()
        rep = m.check(intersections=False)
        c_ms = (time.perf_counter() - t0) * 1e3
        # vertex density against h_min (Section 3.1 meshes at 1 and 2
        # vertices per square angstrom): coarser lattices of the same atoms
        dens = {}
        for h_min in (1.0, 0.5):
            pc = tms.make_params(D=w.D, c=w.c, tau=w.tau, h0=w.h0, h_min=h_min,
                                 precision=precision)
            cc = ctx.build_cells(atoms_dev, pc)
            lc, cpc, _ = ctx.partition_estimate(cc)
            vc = ctx.extract(cc, lc, cpc)
            mc = ctx.mesh_build(cc, lc, cpc, vc)
            ctx.free_cells(cc)
            rc = mc.check(intersections=False)
            dens[str(h_min)] = {k: rc[k] for k in ("density", "n_vertices", "n_triangles",
                                                   "added_cubes", "boundary_edges",
                                                   "nonmanifold_vertices")}
            del mc
        mesh = {"build_ms": m_ms[0], "check_ms": c_ms, "threads": os.cpu_count(),
                "by_h_min": dens,
                "surface_leaves_per_s": sd["n_surface"] / (m_ms[0] * 1e-3),
                **{k: rep[k] for k in ("n_vertices", "n_triangles", "n_loops", "n_fallback",
                                       "open_faces", "added_cubes", "boundary_edges",
                                       "nonmanifold_edges", "misoriented_edges",
                                       "nonmanifold_vertices", "components", "euler",
                                       "unused_vertices", "area", "volume", "density",
                                       "min_angle", "small_angles", "zero_area")}}
        del m
    ctx.free_cells(cells)
    return dict(ms_per_step=spread(step_ms)["mean"], step_ms=spread(step_ms), stats=sd,
                n_leaves=nl, n_vertices=nv, timing=per_step, phi_pairs=phi_pairs,
                stage2=stage2, mesh=mesh, graph_ms_per_step=spread(g_ms)["mean"],
                graph_step_ms=spread(g_ms))


def run_variants(ctx, tms, atoms_dev, w, steps, warmup):
    """The estimator variants (Section 2.2) on the benchmark's workload,
    FP32+guard: child tensors re-expanded from the parent (eq. childtensor)
    and the degree-2 series; partition with corner classification, cubes
    estimated per second."""
    import torch
    out = {}
    for name, kw in (("reexpand", dict(child_tensor=tms.CHILD_REEXPAND)),
                     ("degree2", dict(degree=2))):
        p = w.params(tms.PREC_FP32_GUARD)
        for k, v in kw.items():
            setattr(p, k, v)
        cells = ctx.build_cells(atoms_dev, p)
        leaves, cphi, st = ctx.partition_estimate(cells)
        lb = torch.empty((leaves.shape[0] + 1024, 20), dtype=torch.uint8, device=ctx.device)
        cb = torch.empty((leaves.shape[0] + 1024, 8), dtype=torch.float64, device=ctx.device)
        del leaves, cphi
        step = lambda: ctx.partition_into(cells, lb, cb)
        for _ in range(warmup):
            step()
        ms, (nl, s) = timed_steps(step, steps)
        sd = s.as_dict()
        est = int(sum(sd["n_est"]))
        med = spread(ms)["median"]
        out[name] = {"ms_median": med, "step_ms": spread(ms), "cubes_estimated": est,
                     "cubes_per_s": est / (med * 1e-3), "leaves": int(nl),
                     "surface_leaves": int(sd["n_surface"]), "pairs": int(sd["n_pairs"]),
                     "bound_cubes": int(sd["n_bound"])}
        ctx.free_cells(cells)
        del lb, cb
    return out


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
    b_ms, (nl, nv, s_) = timed_steps(step, steps)
    ms = spread(b_ms)["mean"]
    sd = s_.as_dict()
    # one captured graph for the whole batched pass, writing into lb, cb, vb
    ctx.graph_capture(cells, margin=1.1, leaves=lb, cphi=cb, verts=vb)

    def gstep():
        ctx.build_cells_batch((a, off), p, cells)
        return ctx.graph_launch(cells, lb, cb, vb)

    for _ in range(warmup):
        gstep()
    bg_ms, (gnl, gnv, _) = timed_steps(gstep, steps)
    gms = spread(bg_ms)["mean"]
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
            "ms_per_pass": ms, "pass_ms": spread(b_ms), "cubes_per_s": est / (ms * 1e-3),
            "graph_ms_per_pass": gms, "graph_pass_ms": spread(bg_ms),
            "graph_cubes_per_s": est / (gms * 1e-3),
            "tuning": tuning, "autotune_best_ms": tune_ms, "autotune_passes": tune_n,
            "loop_fp32g_ms": loop32, "loop_fp64_ms": loop64,
            "speedup_vs_loop_fp32g": loop32 / ms, "speedup_vs_loop_fp64": loop64 / ms}


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "cpus_usable": affinity,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(atoms, w, n_glob=4):
    """FP64 oracle on a bounded sample: the first n_glob globules of the
    assembly with their hydrogens (about n_glob/20 of the workload), on every
    thread the process may use; beside it one thread on a 1,000-atom globule
    (context for the paper's serial CPU)."""
    import oracle
    from paper_1611_03474_amd import synth, workloads
    sample = workloads.assembly_slice(atoms, n_glob)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    kw = dict(c=w.c, tau=w.tau, h0=w.h0, h_min=w.h_min, pad=w.pad, eps_cut=w.eps_cut)
    t0 = time.perf_counter()
    r = oracle.partition(sample, w.D, nthreads=threads, **kw)
    dt = time.perf_counter() - t0
    small = synth.globule(1000, 1006)
    t0 = time.perf_counter()
    r1 = oracle.partition(small, w.D, nthreads=1, **kw)
    dt1 = time.perf_counter() - t0
    return {"value": r.cubes_estimated / dt, "unit": "cubes/s", "cores": threads,
            "kind": "oracle",
            "sample": "globules 0-%d of the assembly with their hydrogens (%d atoms, %d cubes "
                      "estimated, %.1f s wall on %d threads)"
                      % (n_glob - 1, len(sample), r.cubes_estimated, dt, threads),
            "host": host_info(),
            "single_thread": {"sample": "1,000-atom globule (seed 1006), same parameters",
                              "atoms": len(small), "cubes_estimated": r1.cubes_estimated,
                              "s": dt1, "cubes_per_s": r1.cubes_estimated / dt1}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint workload")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--no-mesh", action="store_true", help="skip the Stage-2 mesh leg")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the estimator variants (re-expanded children, degree 2)")
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
    f32 = run_mode(ctx, tms, atoms_dev, w, tms.PREC_FP32_GUARD, args.steps, args.warmup,
                   with_mesh=not args.no_mesh)
    if f32["mesh"]:
        log("  mesh %s" % {k: f32["mesh"][k] for k in ("build_ms", "n_triangles", "added_cubes",
                                                      "boundary_edges", "nonmanifold_vertices")})
    log("  %.2f ms/step" % f32["ms_per_step"])
    f64 = None
    if not args.no_fp64:
        log("FP64 run")
        f64 = run_mode(ctx, tms, atoms_dev, w, tms.PREC_FP64, args.steps, args.warmup)
        log("  %.2f ms/step" % f64["ms_per_step"])

    def rates(r):
        st, tmr = r["stats"], r["timing"]
        # phi at the corners: the kernel plus, in FP32+guard, the
        # double-precision recompute of the guarded corners
        phi_ms = tmr["phi"]["ms"] + tmr["guard"]["ms"]
        return {"cubes_per_s": st["cubes_estimated"] / (r["ms_per_step"] * 1e-3),
                "phi_evals_per_s": st["n_corners"] / (phi_ms * 1e-3) if phi_ms > 0 else None,
                "phi_pairs_per_s": r["phi_pairs"] / (phi_ms * 1e-3) if phi_ms > 0 else None}

    r32 = rates(f32)
    st = f32["stats"]
    tm = f32["timing"]

    def launch_avg(slot):
        n = max(tm[slot]["launches"], 1)
        return tm[slot]["ms"] / n, n

    # dominant kernel: the wave-per-chunk tensor estimate on the two deep
    # levels.  Its rank-one updates run in FP64 in both modes, so the FP64
    # vector peak applies; algorithmic work = in-range (cube, atom) pairs at
    # those levels x FLOP_PER_PAIR.
    deep_pairs = sum(st["n_pairs_lvl"][2:4])
    t_ms, t_n = launch_avg("tiled")
    achieved = deep_pairs / t_n * FLOP_PER_PAIR / (t_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": "k_estimate_tiled (levels 2-3)",
                "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": TRAFFIC_TILED if w.name == "assembly110k" else None,
                "traffic_unit": "HBM bytes per launch",
                "work_per_unit": "%d flop per in-range (cube, atom) pair" % FLOP_PER_PAIR,
                "units_per_launch": deep_pairs / t_n, "launches_per_step": t_n,
                "avg_launch_ms": t_ms}
    # the other kernels with a large share of the pass
    p_ms, p_n = launch_avg("phi")
    phi_ach = f32["phi_pairs"] / p_n * OPS_PER_PHI_PAIR / (p_ms * 1e-3) / 1e12
    rooflines = [roofline, {
        "bound": "alu", "kernel": "k_phi_corners<FAST> (corner values)",
        "achieved": phi_ach, "peak": PEAK_VALU_TOPS, "unit": "T VALU lane-op/s",
        "frac": phi_ach / PEAK_VALU_TOPS, "traffic": None,
        "work_per_unit": "%d lane-ops per in-range (point, atom) pair (8 VALU + one "
                         "quarter-rate exponential)" % OPS_PER_PHI_PAIR,
        "units_per_launch": f32["phi_pairs"] / p_n, "avg_launch_ms": p_ms,
        # the same launches against the transcendental unit alone: one
        # single-precision exponential per in-range pair
        "exp_per_s": f32["phi_pairs"] / p_n / (p_ms * 1e-3),
        "exp_frac": f32["phi_pairs"] / p_n / (p_ms * 1e-3) / (PEAK_TRANS_TOPS * 1e12)}]
    b_ms, b_n = launch_avg("decide")
    if FLOP_PER_HARD_CUBE:
        b_ach = st["n_bound"] * FLOP_PER_HARD_CUBE / (tm["decide"]["ms"] * 1e-3) / 1e12
        rooflines.append({
            "bound": "alu", "kernel": "k_bound (nested-SVD bound of the hard cubes)",
            "achieved": b_ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": b_ach / PEAK_FP64_TFLOPS, "traffic": None,
            "work_per_unit": "%d FP64 flop slots issued per hard cube (from counters)"
                             % FLOP_PER_HARD_CUBE,
            "units_per_launch": st["n_bound"] / b_n, "avg_launch_ms": b_ms})

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
        "step_ms": f32["step_ms"],
        "phi_evals_per_s": r32["phi_evals_per_s"],
        "phi_pairs": f32["phi_pairs"], "phi_pairs_per_s": r32["phi_pairs_per_s"],
        "graph_ms_per_step": f32["graph_ms_per_step"], "graph_step_ms": f32["graph_step_ms"],
        "graph_cubes_per_s": st["cubes_estimated"] / (f32["graph_ms_per_step"] * 1e-3),
        "cubes_estimated": st["cubes_estimated"],
        "per_level_estimated": st["n_est"][:4],
        "leaves": f32["n_leaves"], "surface_leaves": st["n_surface"],
        "unique_corners": st["n_corners"], "vertices": f32["n_vertices"],
        "pairs": st["n_pairs"], "bound_cubes": st["n_bound"],
        "guard_points": st["guard_points"],
        "guard_point_fraction": st["guard_points"] / max(1, st["n_corners"]),
        "device_ms_per_step": {k: round(v["ms"], 4) for k, v in tm.items()},
        "pairs_per_level": st["n_pairs_lvl"][:4],
        "roofline": roofline,
        "rooflines": rooflines,
        "stage2": f32["stage2"],
        "mesh": f32["mesh"],
    }
    if f64 is not None:
        r64 = rates(f64)
        out["fp64"] = {"value": r64["cubes_per_s"], "ms_per_step": f64["ms_per_step"],
                       "step_ms": f64["step_ms"],
                       "graph_ms_per_step": f64["graph_ms_per_step"],
                       "phi_evals_per_s": r64["phi_evals_per_s"],
                       "phi_pairs_per_s": r64["phi_pairs_per_s"],
                       "device_ms_per_step": {k: round(v["ms"], 4)
                                              for k, v in f64["timing"].items()},
                       "same_leaf_count": f64["n_leaves"] == f32["n_leaves"]}
        out["speedup_fp32guard_vs_fp64"] = f64["ms_per_step"] / f32["ms_per_step"]
        # where single-precision exponentials enter: phi at the corners
        out["speedup_phi_fp32guard_vs_fp64"] = (
            f64["timing"]["phi"]["ms"] / (tm["phi"]["ms"] + tm["guard"]["ms"]))
    if batch_confs is not None:
        log("batch run")
        out["batch"] = run_batch(ctx, tms, batch_confs, args.steps, args.warmup)
        log("  %.1f ms per batched pass, %.1f ms looped FP32+guard, %.1f ms looped FP64"
            % (out["batch"]["ms_per_pass"], out["batch"]["loop_fp32g_ms"],
               out["batch"]["loop_fp64_ms"]))
    if not args.no_variants:
        log("estimator variants")
        out["variants"] = run_variants(ctx, tms, atoms_dev, w, args.steps, args.warmup)
        log("  %s" % {k: round(v["ms_median"], 2) for k, v in out["variants"].items()})
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
