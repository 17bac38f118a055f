"""Throughput benchmark of the immersed-boundary residual + update step.

Headline workload: the oscillating tube -- an open cylinder of radius 0.5 and
span 4 (65,536 triangles) translating transversely as y(t) = 0.2 cos(2 pi 0.2
t), M = 0.2, Re = 185, on a 384 x 256 x 64 grid (h = 1/16, periodic span),
SSP-RK3 with the compressible (IDW + image point) immersed-boundary family,
free-stream start.  A step re-poses the body, reclassifies every cell by ray
parity, rebuilds the IB lists and reconstruction records, and runs three
stages, each one launch of the fused residual + update over every cell whose
tiles near the body also fill the IB nodes they read: 3 * 384 * 256 * 64
cell-updates per step.  ``value`` is the mixed path's whole-job
cell-updates/s (FP32 reconstruction and fluxes on perturbation variables,
FP64 update) with the state resident in HBM; the FP64 path is timed the same
way.  Every stage launch of the timed region records HIP events at its
start and end on its own stream (the library's stage timer), which gives
the roofline entry of that kernel.

Unless --no-other-configs: the cylinder (C1), the supersonic wedge (C2) and
the low-Mach airfoil (C3), each with its throughput, its own stage-kernel
roofline, its surface forces and (C2, C3) its mixed-vs-FP64 error; the wedge
with WENO5 and with TVD-2 faces; the appendix A preprocessing of the
1200-triangle sphere in both IB frameworks; the wedge in both IB frameworks;
the wedge's oblique shock developed on a 512^2 grid, its angle and plateau
against the theta-beta-M relation and the Rankine-Hugoniot ratio.

Then the serving workload: the seeded stream of 2000 independent 2D solves
(grid side 64-512, cylinder / wedge / NACA 00tt, M 0.01-2, Re 40-1000, dual
time below M 0.1, 1500 residual evaluations each) arriving as a Poisson
process of 50 per second, served by the continuous-batching server in mixed
precision and in FP64 (p50 / p99 latency from arrival to completion), and
once with every request arriving at once (the server's capacity).

The CPU oracle is timed on bounded samples of the headline workload on all
host cores and on one core (cpu_baseline).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--serving-requests N] [--serving-rate R] [--no-other-configs]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-updates/s (full residual+IBM step) mixed vs FP64; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# FP32 vector peak without packed FP32 math (the kernels are compiled without it):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.  The packed peak,
# 157.3 TFLOP/s, is twice that.
FP32_PEAK_TFLOPS = 78.6

# Algorithmic work per cell-update of the fused stage kernel, counted from
# the formulas (each +, -, *, /, sqrt one flop; the derivation is listed
# with the kernels' rooflines in the design notes):
#   2D face: WENO5 68 flops x 8 reconstructions (4 variables x 2 sides),
#     LDFSS 118, central viscous flux 55 -> 717; 2 faces per cell;
#     per cell flux differences 31, primitive recovery 11, and the update:
#     SSP-RK3 20, or the dual-time point-implicit pseudo step 246 (local
#     pseudo step, the preconditioned and Jacobian matrices, the 4 x 4
#     system and its pivoted elimination);
#   3D face: WENO5 68 x 10, LDFSS 130, viscous 104 -> 914; 3 faces per cell;
#     per cell flux differences 42, recovery 17, SSP-RK3 update 25.
FLOPS_PER_CELL = {(2, "rk3"): 2 * (8 * 68 + 118 + 55) + 31 + 11 + 20,
                  (2, "dual"): 2 * (8 * 68 + 118 + 55) + 31 + 11 + 246,
                  (3, "rk3"): 3 * (10 * 68 + 130 + 104) + 42 + 17 + 25}
# HBM bytes per cell-update (algorithmic): stage input state read and output
# written (nv doubles each), the class byte; RK3 stages 2 and 3 also read
# Q^n (averaged over the three stages); a pseudo-iteration also reads the
# two history states.
BYTES_PER_CELL = {(2, "rk3"): (65 + 97 + 97) / 3.0, (2, "dual"): 129.0, (3, "rk3"): (81 + 121 + 121) / 3.0}

KERNEL_SOURCE = os.path.join(ROOT, "paper_1912_11908_amd", "csrc", "flow.hip")
COUNTERS = {
    ("C4", "mixed"): os.path.join(ROOT, "profiles", "step_ghost_kernel_3f_tube_384x256x64_hbm_counters.md"),
    ("C4", "fp64"): os.path.join(ROOT, "profiles", "step_dir_kernel_3d_tube_384x256x64_hbm_counters.md"),
    ("C2", "mixed"): os.path.join(ROOT, "profiles", "step_batch_kernel_2f_wedge_1024x512_hbm_counters.md"),
    ("C2", "fp64"): os.path.join(ROOT, "profiles", "step_batch_kernel_fp64_wedge_1024x512_hbm_counters.md"),
}
KERNEL_NAME = {
    (3, "rk3", "mixed"): "step_ghost_kernel_3f<RK3> (stage launch with inline IB fill)",
    (3, "rk3", "fp64"): "step_dir_kernel_3d<RK3> over every tile, after forcing_fill_kernel<3> and "
                        "ghost_fill_kernel<3> on the stage input (the stage time spans the three launches)",
    (2, "rk3", "mixed"): "step_batch_kernel_2f<RK3, true> (stage launch with inline IB fill)",
    (2, "rk3", "fp64"): "step_batch_kernel<2, double, RK3, true> (stage launch with inline IB fill)",
    (2, "dual", "mixed"): "step_batch_kernel_2f<DUAL, true> (pseudo-iteration with inline IB fill)",
    (2, "dual", "fp64"): "step_batch_kernel<2, double, DUAL, true> (pseudo-iteration with inline IB fill)",
}


def measured_traffic(key, precision):
    """HBM bytes per stage of workload `key` in `precision` from the
    committed counter summary, or None when there is none or the kernel
    source has changed since the counters were taken (the summary records
    the source's SHA-256)."""
    path = COUNTERS.get((key, precision))
    try:
        text = open(path).read()
        sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except (OSError, TypeError):
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("traffic_bytes_per_launch: ", "kernel_source_sha256: ")))
    if fields.get("kernel_source_sha256", "").strip() != sha or "traffic_bytes_per_launch" not in fields:
        return None
    return int(fields["traffic_bytes_per_launch"])


def roofline(case, precision, avg_ms, key=None):
    """Roofline entry of the stage kernel of `case` from its average launch
    duration: algorithmic flops and bytes per cell-update times the cells of
    one launch, over that duration, against the binding peak."""
    kind = (case.ndim, case.scheme)
    flops, nbytes = FLOPS_PER_CELL[kind], BYTES_PER_CELL[kind]
    ncell = case.ncells
    achieved_gbs = nbytes * ncell / (avg_ms * 1e-3) / 1e9
    achieved_tf = flops * ncell / (avg_ms * 1e-3) / 1e12
    fpeak = FP32_PEAK_TFLOPS if precision == "mixed" else FP64_PEAK_TFLOPS
    alu = {"bound": "alu", "achieved": round(achieved_tf, 3), "peak": fpeak, "unit": "TFLOP/s",
           "frac": round(achieved_tf / fpeak, 4)}
    hbm = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved_gbs / HBM_PEAK_GBS, 4)}
    alu_bound = flops / (fpeak * 1e12) >= nbytes / (HBM_PEAK_GBS * 1e9)
    roof, other = (alu, hbm) if alu_bound else (hbm, alu)
    roof["traffic"] = measured_traffic(key, precision) if key else None
    roof["kernel"] = KERNEL_NAME.get((case.ndim, case.scheme, precision))
    roof["kernel_avg_ms"] = round(avg_ms, 5)
    roof["traffic_unit"] = "HBM bytes per stage (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    roof["per_unit"] = {"flops_per_cell_update": flops, "bytes_per_cell_update": round(nbytes, 2),
                        "cells_per_launch": ncell}
    return roof, other


_T0 = time.perf_counter()


def log(msg):
    """Progress of the run on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precisions", default="mixed,fp64")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-rate", type=float, default=50.0)
    ap.add_argument("--no-serving-fp64", action="store_true", help="serve the stream in mixed precision only")
    ap.add_argument("--no-saturation", action="store_true", help="skip the all-at-once serving run")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="skip the cylinder, wedge and airfoil workloads and the side studies")
    ap.add_argument("--config-only", choices=("cylinder", "wedge", "airfoil", "tube", "supersonic", "shock",
                                              "preprocessing", "faces", "frameworks", "oblique"),
                    help="time only that one workload and print its line (for profiling); "
                         "supersonic: the moving / stationary cylinder pair of section 8.2.3; "
                         "shock: the shock-driven free cylinder of section 8.2.6; "
                         "preprocessing: the sphere-in-a-cube timing of appendix A; "
                         "faces: the wedge with WENO5 and with TVD-2 faces; "
                         "frameworks: the wedge with ray tracing / local normals and signed distance / surface normals; "
                         "oblique: the wedge's shock angle, developed on a 512^2 grid")
    ap.add_argument("--supersonic-t", type=float, default=10.0,
                    help="convective times t* of the supersonic cylinder pair")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="also run one plain device copy of 256 MiB (reference for HBM counters)")
    return ap.parse_args()


def serving(n, rate, precision="mixed"):
    """The seeded serving stream through the continuous-batching server."""
    import workloads as w
    from workloads.serving import request_stream
    from paper_1912_11908_amd.serving import Server, GpuBackend
    reqs = request_stream(n=n, rate=rate, steps=500)
    init = lambda c: w.freestream_prim(c.ndim, c.ni, c.nj, c.nk, c.p_inf)  # noqa: E731
    backend = GpuBackend(precision, init=init)
    st = Server(backend, mem_budget=64 << 30, max_active=128, tick_evals=30).run(reqs)
    out = st.summary()
    out.update({"workload": f"{n} seeded 2D solves, Poisson arrivals at {rate:g}/s, grid side "
                            f"64-512, 1500 residual evaluations each, {precision} precision",
                "precision": precision, "arrival_span_s": reqs[-1][0] if reqs else 0.0})
    return out


def _warm_graphs(s, case):
    """Build both whole-step graphs of a stationary solve (a chunk and a
    single step) before any timed call uses them."""
    if case.scheme == "rk3":
        s.advance(8)
        s.advance(1)
    else:
        s.advance(1)   # the first physical step runs eagerly (BDF1)
        s.advance(2)
        s.advance(1)


def run_case(case, precision, steps, warmup, timed_stages=True):
    """Whole steps of one workload from a free-stream start, state resident
    in HBM.  Moving bodies: `warmup` untimed steps, then `steps` timed ones
    with the stage timer on (HIP events at the start and end of every stage
    launch, on its stream).  Stationary bodies: the graphs of whole steps
    are built and `warmup` steps run untimed, `steps` timed steps replay the
    graphs, then 2 eager steps with the stage timer time the stage kernel."""
    import torch
    import workloads as w
    import paper_1912_11908_amd as P
    prim = w.freestream_prim(case.ndim, case.ni, case.nj, case.nk, case.p_inf, velocity=case.u_inf)
    s = P.Solver(case, precision, "cuda:0")
    s.init_prim(prim)
    s.classify()
    moving = bool(case.motion)
    if not moving:
        _warm_graphs(s, case)
    s.advance(warmup)
    torch.cuda.synchronize()
    s.check_status()
    per = case.evals_per_step
    if moving and timed_stages:
        s.set_stage_timing(steps * per)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    s.advance(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    s.check_status()
    stages = None
    if timed_stages:
        if not moving:
            k = 2
            s.set_stage_timing(k * per)
            s.advance(k)
        tot, n, lo, hi = s.stage_timing()
        s.set_stage_timing(0)
        stages = {"avg_ms": tot / n, "launches": n, "min_ms": lo, "max_ms": hi,
                  "where": "timed region" if moving else "2 eager steps after the timed region"}
        if moving:
            # the same launches without the next step's classification
            # running beside them (pipelining off for 4 steps)
            s.set_pipeline(False)
            s.set_stage_timing(4 * per)
            s.advance(4)
            tot, n, lo, hi = s.stage_timing()
            s.set_stage_timing(0)
            s.set_pipeline(True)
            stages["isolated_avg_ms"] = tot / n
            stages["isolated_note"] = ("4 steps after the timed region with the next step's classification "
                                       "not overlapped; in the timed region it runs beside the stages")
    torch.cuda.synchronize()
    done = {"cell_updates_per_s": case.ncells * per * steps / wall, "ms_per_step": wall * 1e3 / steps,
            "event_ms_per_step": ev_ms / steps, "steps": steps, "warmup": warmup}
    return s, done, stages


def surface_forces(s, lref, nrep=20):
    """Force coefficients of the final state (eq.9) and the device time of
    one evaluation (fill excluded)."""
    import torch
    t_end = s.info().time
    s.set_time(t_end)
    s.classify()
    s.fill(t_end)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nrep):
        F = s.forces()
    torch.cuda.synchronize()
    tf = (time.perf_counter() - t0) / nrep
    F = F.cpu().numpy()
    return {"C_x": float(2.0 * F[0] / lref), "C_y": float(2.0 * F[1] / lref), "ms_per_evaluation": tf * 1e3}


OTHER = [
    # key, label, case maker, precisions, timed steps, reference length or area
    ("cylinder", "C1", "cylinder 128x128, M=0.3, Re=40, RK3, 200 steps", "case_c1", ("fp64",), 200, 1.0),
    ("wedge", "C2", "supersonic wedge 1024x512, M=2, Re=1e4, RK3", "case_c2", ("mixed", "fp64"), 500, 1.0),
    ("airfoil", "C3", "NACA0012 2048x1024, M=0.001, Re=1000, dual time, 10 physical steps", "case_c3",
     ("mixed", "fp64"), 10, 1.0),
    ("tube", "C4", "oscillating tube 384x256x64, M=0.2, Re=185, RK3, moving", "case_c4", ("mixed", "fp64"), 50, 4.0),
]


def other_configs(only=None, exclude=("tube",)):
    """Throughput and stage-kernel roofline of the other fixed workloads."""
    import torch
    import workloads as w
    out = {}
    for key, tag, label, maker, precs, steps, lref in OTHER:
        if (only is None and key in exclude) or (only is not None and key != only):
            continue
        case = getattr(w, maker)()
        prims = {}
        for prec in precs:
            s, done, stages = run_case(case, prec, steps, 3)
            log(f"{tag} [{prec}]: {done['ms_per_step']:.3f} ms per step")
            roof, _ = roofline(case, prec, stages["avg_ms"], tag)
            done["stage_kernel"] = stages
            done["roofline"] = roof
            prims[prec] = s.to_prim()
            done["forces"] = surface_forces(s, lref)
            done["forces"]["facets"] = int(case.facet.shape[0])
            out[f"{tag} {label} [{prec}]"] = done
            del s
            torch.cuda.synchronize()
        if "mixed" in prims and "fp64" in prims:
            out[f"{tag} {label} [mixed]"]["mixed_vs_fp64_rel_l2"] = mixed_error(prims["mixed"], prims["fp64"],
                                                                              case.ndim, case.p_inf)
        del prims
    return out


def calibration_copy():
    """One plain device copy of 256 MiB (the reference of the HBM byte
    counters); returns the bytes it moves."""
    import torch
    src = torch.ones(32 << 20, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    return 2 * src.numel() * 8


def mixed_error(a, b, ndim, p_inf):
    """Relative L2 difference per primitive variable between the mixed and
    the FP64 state of the same run (device tensors).  Velocity components
    are measured against the free-stream scale (1 per cell) where their own
    norm is smaller; the pressure also as p - p_inf, against its own norm."""
    import torch
    names = ["rho"] + ["u", "v", "w"][:ndim] + ["p"]
    out = {}
    ncell = b[0].numel()
    for v, nm in enumerate(names):
        d = torch.linalg.vector_norm(a[v] - b[v]).item()
        ref = torch.linalg.vector_norm(b[v]).item()
        if nm in ("u", "v", "w"):
            ref = max(ref, ncell ** 0.5)
        out[nm] = d / ref
    pp = torch.linalg.vector_norm(b[ndim + 1] - p_inf).item()
    out["p_minus_p_inf"] = torch.linalg.vector_norm(a[ndim + 1] - b[ndim + 1]).item() / pp if pp > 0 else None
    return out


def supersonic_pair(t_end, mach=1.2, precision="mixed"):
    """Section 8.2.3 as a Galilean check: the cylinder moving at unit speed
    through still fluid and the same cylinder held in a unit stream, both
    from an impulsive start, eq.7 wall pressure; after t_end their surface
    pressure coefficients and drag, seen from the body, must agree up to the
    discretisation (the grid moves relative to one body, not the other)."""
    import numpy as np
    import torch
    import workloads as w
    from workloads.cases import case_supersonic_cylinder
    import paper_1912_11908_amd as P
    out = {}
    cp, cx = {}, {}
    for moving in (True, False):
        case = case_supersonic_cylinder(mach, moving=moving, t_end=t_end)
        prim = w.freestream_prim(2, case.ni, case.nj, 1, case.p_inf, velocity=case.u_inf)
        s = P.Solver(case, precision, "cuda:0")
        s.init_prim(prim)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance(case.steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s.check_status()
        t_now = s.info().time
        s.set_time(t_now)
        s.classify()
        s.fill(t_now)
        F, rows, missed = s.forces(facets=True)
        rows = rows.cpu().numpy()
        # seen from either body the fluid streams along -x, so the drag
        # points along -x in both problems
        cx["moving" if moving else "stationary"] = float(2.0 * F[0].item())
        cp["moving" if moving else "stationary"] = 2.0 * rows[:, 0]
        out["moving" if moving else "stationary"] = {
            "case": case.name, "cells": case.ncells, "steps": case.steps, "dt": case.dt,
            "ms_per_step": dt * 1e3 / case.steps,
            "cell_updates_per_s": case.ncells * 3 * case.steps / dt,
            "C_x": cx["moving" if moving else "stationary"], "facets_missed": int(missed.item())}
        del s
    d = cp["moving"] - cp["stationary"]
    out["galilean"] = {"t_star": t_end, "mach": mach, "precision": precision,
                       "Cp_max_abs_diff": float(np.abs(d).max()),
                       "Cp_rel_l2_diff": float(np.sqrt((d ** 2).sum() / (cp["stationary"] ** 2).sum())),
                       "Cp_stagnation": float(cp["stationary"].max()),
                       "C_D_moving": -cx["moving"], "C_D_stationary": -cx["stationary"]}
    return out


def preprocessing(reps=50):
    """Appendix A (Table A1) on the GPU: the IB preprocessing of a
    1200-triangle sphere in a 40^3 cube -- classification, tagging, list
    compaction, closest features, normals, P' and probe stencils (one
    ibm_classify call) -- for both frameworks the table compares: ray-parity
    classification with local normals, and signed-distance classification
    with surface normals (the standard HCIB/GC).  Timed with HIP events; the
    CPU baseline leg times the oracle's same work on the host cores."""
    import torch
    import workloads as w
    from workloads.cases import case_sphere_preprocessing
    import paper_1912_11908_amd as P
    out = {"workload": "sphere of 1200 triangles (D = 1) in a 40^3 cube [-1, 1]^3",
           "paper_table_A1_s": {"rtln": {"1 core": 4.296e-2, "8 cores": 5.3778e-3},
                                "sdsn": {"1 core": 1.6406e-1, "8 cores": 3.125e-2}}}
    for fw in ("rtln", "sdsn"):
        case = case_sphere_preprocessing(40, fw)
        s = P.Solver(case, "fp64", "cuda:0")
        s.init_prim(w.freestream_prim(3, case.ni, case.nj, case.nk, case.p_inf))
        s.classify()
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            s.classify()
        e1.record(st)
        torch.cuda.synchronize()
        gpu_s = e0.elapsed_time(e1) / 1e3 / reps
        cnt = s.counts()
        out[fw] = {"forcing_nodes": int(cnt[0]), "ghost_nodes": int(cnt[4]),
                   "gpu_s_per_preprocessing": gpu_s,
                   "cpu_baseline": cpu_baseline_preprocessing(case)}
        del s
    return out


def face_schemes(steps=500):
    """The supersonic wedge (1024 x 512, whole RK3 steps, graphs of eight
    steps) with fifth-order WENO faces and with second-order TVD faces
    (MUSCL, minmod; section 2), in both precisions."""
    import dataclasses
    import torch
    import workloads as w
    import paper_1912_11908_amd as P
    out = {"workload": "supersonic wedge 1024x512, M=2, Re=1e4, SSP-RK3", "steps": steps}
    for recon in ("weno5", "tvd2"):
        case = dataclasses.replace(w.case_c2(), reconstruction=recon)
        for prec in ("mixed", "fp64"):
            s = P.Solver(case, prec, "cuda:0")
            s.init_prim(w.freestream_prim(case.ndim, case.ni, case.nj, case.nk, case.p_inf))
            s.advance(16)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.advance(steps)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            s.check_status()
            out[f"{recon} [{prec}]"] = {"ms_per_step": dt * 1e3,
                                         "cell_updates_per_s": case.ncells * case.evals_per_step / dt}
            del s
    return out


def frameworks(steps=3000):
    """Section 7's contrast on the supersonic wedge (mixed precision, from a
    free-stream start): ray tracing with local normals against signed
    distance with surface normals.  On this convex body the classes agree
    (the bounding box makes signed distance exact); the surface normal at the
    three corners changes the reconstruction there.  Reported: the force
    coefficients of each (per unit span, length 1), and where and by how much
    their pressure fields differ."""
    import dataclasses
    import numpy as np
    import torch
    import workloads as w
    import paper_1912_11908_amd as P
    out = {"workload": f"supersonic wedge 1024x512, M=2, Re=1e4, {steps} RK3 steps, mixed", "steps": steps}
    base = w.case_c2()
    fields = {}
    for fw in ("rtln", "sdsn"):
        case = dataclasses.replace(base, ib_framework=fw)
        s = P.Solver(case, "mixed", "cuda:0")
        s.init_prim(w.freestream_prim(case.ndim, case.ni, case.nj, case.nk, case.p_inf))
        s.advance(steps)
        s.check_status()
        t_end = s.info().time
        fields[fw] = s.to_prim()[3, 0].cpu().numpy()
        s.classify()
        s.fill(t_end)
        F = s.forces().cpu().numpy()
        out[fw] = {"C_x": float(2.0 * F[0]), "C_y": float(2.0 * F[1]), "t": t_end}
        del s
    pinf = base.p_inf
    a, b = fields["rtln"], fields["sdsn"]
    d = np.abs(a - b) / pinf
    j, i = np.unravel_index(np.argmax(d), d.shape)
    xc = 0.5 * (base.xf[1:] + base.xf[:-1])
    yc = 0.5 * (base.yf[1:] + base.yf[:-1])
    corners = base.vert
    dist = float(np.min(np.hypot(corners[:, 0] - xc[i], corners[:, 1] - yc[j])))
    jj, ii = np.nonzero(d > 1e-3)
    far = np.min(np.hypot(corners[:, 0][None, :] - xc[ii][:, None], corners[:, 1][None, :] - yc[jj][:, None]),
                 axis=1) if len(ii) else np.zeros(1)
    out["pressure_difference"] = {
        "rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(a - pinf)),
        "max_over_p_inf": float(d.max()), "at": [float(xc[i]), float(yc[j])],
        "distance_to_nearest_corner": dist,
        "cells_differing_by_1e-3_p_inf": int(len(ii)),
        "farthest_such_cell_from_a_corner": float(far.max())}
    return out


def _beta_weak(mach, theta, gamma=1.4):
    """Weak root of the theta-beta-M relation of an attached oblique shock
    (bisection between the Mach angle and 64 degrees)."""
    def f(b):
        return math.tan(theta) - 2.0 / math.tan(b) * (mach ** 2 * math.sin(b) ** 2 - 1.0) / (
            mach ** 2 * (gamma + math.cos(2.0 * b)) + 2.0)
    lo, hi = math.asin(1.0 / mach) + 1e-12, math.radians(64.0)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (lo, mid) if f(lo) * f(mid) <= 0.0 else (mid, hi)
    return 0.5 * (lo + hi)


def oblique_shock(t_end=1.5):
    """The shock of the C2 wedge shape measured where the flow has reached
    it: the C2 run itself (2000 steps, t = 0.03) ends long before the shock
    is steady, so the 15 degree wedge at M = 2, Re = 1e4 is run on [-1, 1]^2
    at h = 1/256 (512^2 cells) from a uniform stream for t_end convective
    times.  At 0.2-0.5 from the apex: the shock angle (where the pressure,
    scanned down from the free stream, first reaches the mean of the free
    stream and the exact plateau) against the weak root of the
    theta-beta-M relation, and the plateau pressure ratio (median between
    30 and 70 % of the way from the wall to the shock) against the
    Rankine-Hugoniot ratio."""
    import numpy as np
    import torch
    import workloads as w
    from workloads.cases import Case, rk3_dt
    import paper_1912_11908_amd as P
    mach, theta, apex = 2.0, math.radians(15.0), (-0.5, 0.0)
    beta = _beta_weak(mach, theta)
    mn = mach * math.sin(beta)
    p21 = 1.0 + 2.0 * 1.4 / 2.4 * (mn ** 2 - 1.0)
    f = w.uniform_faces(512, -1.0, 1.0)
    v, s_ = w.wedge_polygon(15.0, 1.0, apex)
    bc = ("farfield", "extrap", "extrap", "extrap", "periodic", "periodic")
    case = Case("oblique-wedge", 2, f, f.copy(), np.array([-0.5, 0.5]), bc, v, s_, mach, 1.0e4,
                dt=rk3_dt(mach, 1.0e4, [f, f]))
    steps = int(round(t_end / case.dt))
    xc = 0.5 * (f[1:] + f[:-1])
    h = float(xc[1] - xc[0])
    out = {"workload": f"15 degree wedge, M = 2, Re = 1e4, 512^2 cells on [-1, 1]^2, {steps} RK3 steps "
                       f"(t = {t_end:g}) from a uniform stream",
           "beta_exact_deg": math.degrees(beta), "p2_over_p1_exact": p21}
    for prec in ("mixed", "fp64"):
        s = P.Solver(case, prec, "cuda:0")
        s.init_prim(w.freestream_prim(2, case.ni, case.nj, 1, case.p_inf))
        s.classify()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        s.check_status()
        p = s.to_prim().cpu().numpy()[3, 0] / case.p_inf
        mid = 0.5 * (p21 + 1.0)
        st = []
        for d0 in (0.2, 0.3, 0.4, 0.5):
            i = int(np.argmin(np.abs(xc - (apex[0] + d0))))
            d = float(xc[i] - apex[0])
            col = p[:, i]
            ywall = apex[1] + math.tan(theta) * d
            k = min(int(np.searchsorted(xc, apex[1] + 2.0 * math.tan(beta) * d)), case.nj - 2)
            while k > 0 and col[k] < mid and xc[k] > ywall:
                k -= 1
            ysh = xc[k] + (col[k] - mid) / (col[k] - col[k + 1]) * h
            sel = (xc > ywall + 0.3 * (ysh - ywall)) & (xc < ywall + 0.7 * (ysh - ywall))
            st.append({"distance_from_apex": round(d, 4),
                       "beta_deg": math.degrees(math.atan2(ysh - apex[1], d)),
                       "p2_over_p1": float(np.median(col[sel]))})
        out[prec] = {"stations": st, "ms_per_step": el * 1e3 / steps,
                     "max_beta_error_deg": max(abs(e["beta_deg"] - math.degrees(beta)) for e in st),
                     "max_p21_rel_error": max(abs(e["p2_over_p1"] / p21 - 1.0) for e in st)}
        del s
    return out


def cpu_baseline_preprocessing(case, reps=3):
    """CPU baseline leg of the appendix A timing: the oracle's classification
    and records of the same case, on this host's cores."""
    import oracle
    o = oracle.Oracle(case)
    o.classify()
    t0 = time.perf_counter()
    for _ in range(reps):
        o.classify()
    el = (time.perf_counter() - t0) / reps
    return {"value": el, "unit": "s per preprocessing", "kind": "oracle",
            "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
            "sample": f"{reps} full preprocessings of the same case"}


def shock_driven(t_end=2.0):
    """Section 8.2.6: a free cylinder driven by a Mach 1.5 shock (656^2
    cells, D / 164), eq.10 coupling; per precision the wall time per coupled
    step (force, host synchronisation, reclassification and the RK3 stages)
    and the body's trajectory at t* = 0.5, 1, 1.5, 2."""
    import torch
    from workloads.cases import case_shock_cylinder, shock_prim
    import paper_1912_11908_amd as P
    out = {}
    for prec in ("mixed", "fp64"):
        case = case_shock_cylinder(656, t_end=t_end)
        s = P.Solver(case, prec, "cuda:0")
        s.init_prim(shock_prim(case, 0.5))
        marks = [int(round(k * case.steps / 4)) for k in range(1, 5)]
        traj, done, wall = [], 0, 0.0
        for m in marks:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.advance(m - done)
            torch.cuda.synchronize()
            wall += time.perf_counter() - t0
            done = m
            x, u, a, fx = s.body_state()
            traj.append({"t_star": round(m * case.dt, 6), "x": float(x), "u": float(u), "C_x": float(2.0 * fx)})
        s.check_status()
        t_now = s.info().time
        s.set_time(t_now)
        s.classify()
        s.fill(t_now)
        F = s.forces().cpu().numpy()
        out[prec] = {"cells": case.ncells, "steps": case.steps, "ms_per_step": wall * 1e3 / case.steps,
                     "cell_updates_per_s": case.ncells * 3 * case.steps / wall, "trajectory": traj,
                     "lift_over_drag": float(abs(F[1]) / abs(F[0]))}
        del s
    return out


def cpu_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "host_cpus": os.cpu_count()}


def cpu_baseline(case):
    """The oracle as it stands on this host's cores, on bounded samples of
    the headline workload: two whole RK3 steps of the full grid on all
    threads (each re-poses and reclassifies the body, as the GPU step does),
    and one fill + residual evaluation of the full grid on one thread
    (classification and update excluded; one evaluation is one cell-update
    per cell)."""
    import numpy as np
    import oracle
    import workloads as w
    prim = w.freestream_prim(case.ndim, case.ni, case.nj, case.nk, case.p_inf)
    threads = oracle.threads()
    o = oracle.Oracle(case)
    q = o.prim_to_state(prim)
    steps = 2
    t0 = time.perf_counter()
    o.run(q, steps)
    el = time.perf_counter() - t0
    assert np.all(np.isfinite(o.interior(q)))
    cu = steps * case.evals_per_step * case.ncells
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        o.fill(q, o.t)
        o.bc(q)
        o.residual(q)
        el1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(threads)
    out = {"value": cu / el, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{steps} RK3 steps of the full {case.ni}x{case.nj}x{case.nk} oscillating tube, "
                     f"each reclassifying the body ({cu:.3g} cell-updates, {el:.1f} s wall, {threads} threads)",
           "one_core": {"value": case.ncells / el1, "unit": "cell-updates/s", "cores": 1,
                        "sample": f"one IB fill + residual evaluation of the full grid ({case.ncells} "
                                  f"cell-updates, {el1:.1f} s wall; classification and update excluded)"}}
    out.update(cpu_info())
    out.update(oracle.compiler())
    return out


def main():
    args = _parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import workloads as w

    if args.config_only == "oblique":
        print(json.dumps({"oblique_shock": oblique_shock()}), flush=True)
        return
    if args.config_only == "frameworks":
        print(json.dumps({"frameworks": frameworks()}), flush=True)
        return
    if args.config_only == "faces":
        print(json.dumps({"faces": face_schemes()}), flush=True)
        return
    if args.config_only == "preprocessing":
        print(json.dumps({"preprocessing": preprocessing()}), flush=True)
        return
    if args.config_only == "shock":
        print(json.dumps({"shock_driven": shock_driven()}), flush=True)
        return
    if args.config_only == "supersonic":
        print(json.dumps({"supersonic_pair": supersonic_pair(args.supersonic_t)}), flush=True)
        return
    if args.config_only:
        line = {"other_configs": other_configs(args.config_only)}
        if args.calibration_copy:
            line["calibration_copy_bytes"] = calibration_copy()
        print(json.dumps(line), flush=True)
        return

    case = w.case_c4(steps=args.steps)
    ncell = case.ncells
    res, prims = {}, {}
    for prec in [p for p in args.precisions.split(",") if p]:
        s, done, stages = run_case(case, prec, args.steps, args.warmup)
        log(f"oscillating tube [{prec}]: {done['ms_per_step']:.3f} ms per step")
        roof, other = roofline(case, prec, stages["avg_ms"], "C4")
        iso, _ = roofline(case, prec, stages["isolated_avg_ms"], "C4")
        done["stage_kernel"] = stages
        done["roofline_isolated"] = {k: iso[k] for k in ("bound", "achieved", "peak", "unit", "frac", "kernel_avg_ms")}
        res[prec] = (done, roof, other)
        prims[prec] = s.to_prim()
        done["forces"] = surface_forces(s, 4.0)
        done["forces"]["facets"] = int(case.facet.shape[0])
        del s
        torch.cuda.synchronize()
    head = "mixed" if "mixed" in res else "fp64"
    r, roof, other = res[head]
    out = {
        "metric": METRIC, "value": r["cell_updates_per_s"], "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": "oscillating tube 384x256x64 (65,536 triangles, y = 0.2 cos(2 pi 0.2 t)), "
                               "M=0.2, Re=185, SSP-RK3, IDW/image-point IB, reclassified every step",
                   "cells": ncell, "cell_updates_per_step": case.evals_per_step * ncell, "precision": head},
        "roofline": roof, "roofline_other": other,
        "roofline_isolated": r["roofline_isolated"],
        "stage_kernel": r["stage_kernel"], "forces": r["forces"],
    }
    if "fp64" in res and "mixed" in res:
        f, froof, fother = res["fp64"]
        out["fp64"] = {"value": f["cell_updates_per_s"], "ms_per_step": f["ms_per_step"],
                       "stage_kernel": f["stage_kernel"], "roofline": froof,
                       "roofline_isolated": f["roofline_isolated"], "forces": f["forces"]}
        out["mixed_speedup_vs_fp64"] = f["ms_per_step"] / r["ms_per_step"]
        out["mixed_vs_fp64_rel_l2"] = mixed_error(prims["mixed"], prims["fp64"], case.ndim, case.p_inf)
    del prims
    if not args.no_other_configs:
        out["other_configs"] = other_configs()
        out["faces"] = face_schemes(200)
        log("face schemes done")
        out["appendix_a"] = preprocessing()
        log("appendix A preprocessing done")
        out["frameworks"] = frameworks()
        log("IB frameworks done")
        out["oblique_shock"] = oblique_shock()
        log("oblique shock done")
    if args.calibration_copy:
        out["calibration_copy_bytes"] = calibration_copy()
    if args.serving_requests > 0:
        sv = serving(args.serving_requests, args.serving_rate, "mixed")
        log(f"serving [mixed]: p50 {sv['p50_s']:.4f} s, p99 {sv['p99_s']:.4f} s")
        out["latency_p50_s"] = sv["p50_s"]
        out["latency_p99_s"] = sv["p99_s"]
        out["serving"] = {"mixed": sv}
        if not args.no_serving_fp64:
            out["serving"]["fp64"] = serving(args.serving_requests, args.serving_rate, "fp64")
            log("serving [fp64] done")
        if not args.no_saturation:
            sat = serving(args.serving_requests, 1.0e5, "mixed")
            log("serving at saturation done")
            sat["note"] = "every request arrives within the first 0.03 s: throughput is the server's capacity"
            out["serving"]["saturated_mixed"] = sat
            out["serving_capacity_cell_updates_per_s"] = sat["cell_updates_per_s"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w.case_c4())
        log("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
