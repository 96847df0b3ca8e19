#!/usr/bin/env python3
"""Throughput benchmark of the MI355X nodal DG Euler solver.

One "step" is one full LSERK(5,4) step of the hot path: five fused stage
kernels (volume term, face gather with Lax-Friedrichs flux and boundary
states, LIFT, Runge-Kutta update, and in the last one the next step's CFL
bound) over the whole mesh.  The default workload is the roofline
configuration: the isentropic vortex on a seeded, jittered periodic square
of 999,698 triangles at P=5 (84M DOF), CFL 0.5, 200 steps, FP32; the only
configuration whose working set exceeds the caches, so its HBM fraction is a
real one.

Prints one JSON line: value = RK-stage DOF-updates/s (4 Np K x 5 stages x
steps / wall time, inputs resident in HBM), the FP64-plain path's rate on the
same workload, the dominant kernel's HBM roofline (algorithmic bytes over its
average launch time measured with HIP events inside the timed region, against
8 TB/s and against a device copy measured in the same run), the serving leg
(64 seeded requests, continuous batching: p50/p99 latency and aggregate
throughput) and the FP64 CPU oracle timed on this host's cores, all and one,
on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RK-stage DOF-updates/s (FP32/batched vs FP64 plain) + p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "cylinder": "Subsonic flow past a unit circle, Mach 0.38, AoA 0: annulus r in [1,20], "
                "20,000 triangles (200x50, graded, seeded jitter), cubic curved wall elements, "
                "P=4 (Np=15), slip wall + characteristic far field, CFL 0.5",
    "roofline": "Isentropic vortex on a seeded, jittered periodic square, 999,698 straight "
                "triangles (2x707x707), P=5 (Np=21, 84M DOF), CFL 0.5",
    "vortex": "Isentropic vortex on the periodic square [0,10]^2, 512 jittered, permuted "
              "triangles, P=2 (Np=6), CFL 0.5",
    "airfoil": "Transonic flow, Mach 0.8, AoA 1.25 deg, 4-digit 12% airfoil, far field R=30, "
               "120,000 triangles, cubic curved wall, P=3 (Np=10), Persson-Peraire sensor + "
               "LDG artificial viscosity, CFL 0.5, start from the freestream damped to rest at the wall",
    "tet3d": "3D Euler entropy wave (rho = 1 + 0.2 sin 2 pi x, velocity (1, 0.5, 0.25), p = 1) on a "
             "seeded, jittered periodic box of 16x16x17 cubes split into 26,112 straight tetrahedra "
             "(the paper's timing mesh has 25,956 cells), P=4 (Np=35, 5 fields), LF flux, CFL 0.5, "
             "200 steps; the time table at P=2,3,4 in FP64 and FP32",
}

# The paper's run times for 200 steps on 25,956 tetrahedra (Table time_table;
# one Tesla M2050 and a 4-core Xeon E5620): context, not the target.
PAPER_TIME_TABLE_S = {"P4": {"cpu_4core": 278.92, "gpu_fp64": 54.16, "gpu_fp32": 15.27},
                      "P3": {"cpu_4core": 92.88, "gpu_fp64": 21.34, "gpu_fp32": 7.96},
                      "P2": {"cpu_4core": 34.01, "gpu_fp64": 8.40, "gpu_fp32": 3.52}}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(precision="fp32", av=False, workload=None):
    """Hash of the sources of the stage's kernels for this precision (with
    artificial viscosity the sensor and gradient kernels too; the 3D
    workload's in their own file)."""
    h = hashlib.sha256()
    files = ("kernels.hip", "common.hpp") if precision == "fp64" else ("stage_mfma.hip", "common.hpp")
    if av and precision != "fp64":
        files += ("kernels.hip",)
    if workload == "tet3d":
        files = ("tet3d.hip", "common.hpp")
    for f in files:
        with open(os.path.join(ROOT, "paper_1208_4772_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_stage_bytes(case, s):
    """HBM bytes one fused stage launch must move (averaged over the 5 stages):
    state in + out and the Runge-Kutta register R (read in 4 of 5 stages,
    written in all), the neighbours' face traces once per interior face side,
    geometric factors (13 values for a straight element, 4 Np + 9 Nfp for a
    curved one) and 12 bytes of connectivity per element."""
    import numpy as np
    K, Np, Nfp = case.K, case.Np, case.P + 1
    m = case.mesh
    interior_sides = int((m.bc == 0).sum())
    if m.node_displacement is not None:
        curved = K
    elif m.curve is not None:
        curved = int((m.bc == 1).any(axis=1).sum())
    else:
        curved = 0
    state = K * 4 * Np * s * (3 + 4 / 5)
    traces = interior_sides * Nfp * 4 * s
    geom = (K - curved) * 13 * s + curved * (4 * Np + 9 * Nfp) * s
    conn = 12 * K
    total = state + traces + geom + conn
    if case.av:
        # the viscous terms add two launches per stage.  Sensor: density and
        # the element's viscosity ceiling in, viscosity out (the first stage
        # of a step also reads the rest of the state and the face Fscale for
        # the time-step bound).  Gradient: state, viscosity, per-node metrics
        # and face geometry (4 Np + 9 Nfp values) and 16 bytes of
        # connectivity in, the neighbours' state traces and viscosity,
        # sigma grad U (8 Np values) out.  Stage: sigma grad U and the
        # viscosity in, the neighbours' traces of it (8 values per face
        # node) and their viscosity.
        sensor = K * (Np * s + 2 * s) + K * (3 * Np + 3 * Nfp) * s / 5
        grad = (K * ((4 * Np + 1 + 8 * Np + 4 * Np + 9 * Nfp) * s + 16)
                + interior_sides * (Nfp * 4 * s + s))
        stage_av = K * (8 * Np * s + s) + interior_sides * (Nfp * 8 * s + s)
        total += sensor + grad + stage_av
    return total, dict(curved=curved, interior_sides=interior_sides)


def stage_kernel_label(case, precision, waves, form="nodal"):
    """The launch(es) one Runge-Kutta stage consists of: the stage kernel, and
    with artificial viscosity the sensor and gradient launches before it
    (their time is in the per-stage average, so their bytes are in the
    algorithmic figure; a step's first stage runs the sensor that also
    reduces the time-step bound, k_sensor, in place of k_sensor_elem)."""
    av = "true" if case.av else "false"
    if form == "weak":
        if precision != "fp64" and getattr(case.mesh, "node_displacement", None) is None:
            return f"k_stage_weak_mfma<{case.P}>"   # FP32, every element straight
        return f"k_stage_weak<{'double' if precision == 'fp64' else 'float'},{case.P}>"
    if precision == "fp64":
        k = f"k_stage<double,{case.P},{av}>"
    else:
        k = (f"k_stage_mfma<{case.P},{'true' if precision == 'bf16x3' else 'false'},"
             f"{waves or 4},{av}>")
    if case.av:
        return f"k_sensor_elem<{case.P}> + k_avgrad<{case.P}> + {k}"
    return k


def load_traffic(workload, precision, launch_bytes, av=False):
    """HBM traffic per launch (per stage, with artificial viscosity) from
    committed rocprofv3 counter runs, if they were taken on the current
    kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_stage_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_hash") != kernel_source_hash(precision, av, workload):
        return None
    return t.get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case, budget_s=12.0):
    """The FP64 oracle on this host's cores: one warm rhs to size the sample,
    then as many full steps of the same mesh as fit the budget, with every
    thread OpenMP gives it and again with one thread (the paper's 4-core and
    1-core CPU runs)."""
    from oracle import oracle as orc
    from oracle.refelem import ref
    R = ref(case.P)
    import meshgen
    oc = meshgen.make_case(case.name, R.r, R.s)
    o = orc.Oracle.for_case(oc)
    dofs = oc.dofs()
    nthreads = orc.max_threads()

    def timed(threads, budget):
        orc.set_threads(threads)
        t0 = time.perf_counter()
        o.rhs(oc.U0)
        t1 = time.perf_counter() - t0
        if 5.5 * t1 > budget:
            # one step exceeds the budget: time single stages (rhs evaluations)
            stages = max(1, int(budget / t1))
            t0 = time.perf_counter()
            for _ in range(stages):
                o.rhs(oc.U0)
            el = time.perf_counter() - t0
            return dofs * stages / el, f"{stages} rhs evaluations (RK stages), {el:.1f} s"
        steps = max(1, int(budget / (5.5 * t1)))
        t0 = time.perf_counter()
        o.run(oc.U0, steps)
        el = time.perf_counter() - t0
        return dofs * 5 * steps / el, f"{steps} full LSERK steps (of {case.steps}), {el:.1f} s"

    v_all, s_all = timed(nthreads, budget_s)
    v_one, s_one = timed(1, budget_s / 2)
    orc.set_threads(nthreads)
    return dict(value=v_all, unit="DOF-updates/s", cores=nthreads, kind="oracle",
                sample=f"the same {oc.K}-element P={oc.P} mesh, FP64: {s_all}",
                one_thread=dict(value=v_one, sample=s_one),
                cpu_model=cpu_model(), host_cpus=os.cpu_count())


def tet3d_stage_bytes(grid, P, s):
    """HBM bytes one 3D stage launch must move (averaged over the 5 stages):
    state in and out and the Runge-Kutta register (read in 4 of 5 stages,
    written in all), the neighbours' face traces once per interior face
    side, 25 geometric factors per element, and 16 bytes of connectivity
    (four neighbour ids with their face and orientation codes) per element.
    The kernel reads a face node map instead (4 Nfp ints per element); that
    excess is the kernel's, so it is not counted here."""
    K, Np, Nfp = grid.K, (P + 1) * (P + 2) * (P + 3) // 6, (P + 1) * (P + 2) // 2
    interior_sides = int((grid.bc == 0).sum())
    state = K * 5 * Np * s * (3 + 4 / 5)
    traces = interior_sides * Nfp * 5 * s
    return state + traces + K * 25 * s + 16 * K


def bench_tet3d(args, dev):
    """The 3D workload: 200 LSERK steps on the 26,112-tetrahedron box at
    P = 4 (the timed line) and the time table at P = 2, 3, 4 in FP64 and
    FP32, beside the paper's run times (context) and the oracle on this
    host's cores."""
    import numpy as np
    import torch

    from meshgen.tets import affine_node_coordinates, cube_tets, entropy_wave3
    from paper_1208_4772_amd import dg3
    steps = 200 if args.steps is None else args.steps
    grid = cube_tets((16, 16, 17), 1.0, 0.1, 3, periodic=True)
    log(f"workload tet3d: K={grid.K} steps={steps} warmup={args.warmup}")

    def timed(P, precision, nsteps, warmup):
        sol = dg3.Solver3D.from_mesh(grid, P, precision=precision, cfl=0.5)
        r, s_, t = dg3.reference_nodes3(P)
        U0 = sol.state(entropy_wave3(affine_node_coordinates(grid, r, s_, t), along=(1, 0, 0)))
        U = U0.clone()
        if warmup:
            sol.run(U, warmup)
        U.copy_(U0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = sol.run(U, nsteps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ok = bool(torch.isfinite(U).all().item())
        out = (wall, st, ok, sol.dofs(), U.double().cpu().numpy())
        sol.close()
        return out

    table = {}
    final = {}
    main_line = None
    for P in (4, 3, 2):
        row = {}
        for precision in ("fp32", "fp64"):
            wall, st, ok, dofs, Uf = timed(P, precision, steps, args.warmup)
            if not ok or st.status != 0:
                raise SystemExit(f"tet3d P={P} {precision}: state became non-finite")
            row[precision] = dict(seconds=round(wall, 5), dof_updates_per_s=dofs * 5 * steps / wall,
                                  device_s=round(st.wall_s, 5), t=st.t)
            final[(P, precision)] = Uf
            log(f"tet3d P={P} {precision}: {wall * 1e3:.2f} ms for {steps} steps -> "
                f"{dofs * 5 * steps / wall:.4e} DOF-updates/s")
            if P == 4 and precision == "fp32":
                main_line = (wall, st, dofs)
        d = final[(P, "fp32")] - final[(P, "fp64")]
        row["fp32_vs_fp64_rel_l2"] = float(np.linalg.norm(d) / np.linalg.norm(final[(P, "fp64")]))
        row["fp32_vs_fp64_max_abs"] = float(np.abs(d).max())
        row["fp64_over_fp32_time"] = round(row["fp64"]["seconds"] / row["fp32"]["seconds"], 3)
        table[f"P{P}"] = row
    wall, st, dofs = main_line
    value = dofs * 5 * steps / wall
    # device events bracket the steps: 5 stage launches and the dt kernel per
    # step (and the first step's bound kernel), so this average slightly
    # overstates the stage kernel's own duration
    avg_s = st.wall_s / (5 * steps)
    launch_bytes = tet3d_stage_bytes(grid, 4, 4)
    achieved = launch_bytes / avg_s / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "DOF-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOADS["tet3d"], "K": grid.K, "P": 4, "dof": dofs, "precision": "fp32"},
        "roofline": dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                         frac=round(achieved / HBM_PEAK_GBS, 4),
                         traffic=load_traffic("tet3d", "fp32", launch_bytes), kernel="k_stage3_mfma<4>",
                         avg_launch_us=round(avg_s * 1e6, 3), launches=5 * steps,
                         algorithmic_bytes_per_launch=int(launch_bytes),
                         note="average over the stage launches of the timed region (a step's last "
                              "stage also reduces the next step's bound), the per-step dt kernel included"),
        "time_table_200_steps": table,
        "paper_time_table_s": PAPER_TIME_TABLE_S,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_tet3d(grid, min(args.cpu_budget, 20.0))
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


def cpu_baseline_tet3d(grid, budget_s):
    """The FP64 3D oracle at P = 4 on the same mesh: rhs evaluations (one RK
    stage each) for about budget_s seconds.  Its contractions are NumPy
    einsums, which run on one thread."""
    from meshgen.tets import entropy_wave3
    from oracle import tet3d as T
    o = T.Oracle3D(T.TetMesh(grid.EToV, grid.X, grid.period), 4)
    U = entropy_wave3(o.xyz, along=(1, 0, 0))
    t0 = time.perf_counter()
    o.rhs(U)
    t1 = time.perf_counter() - t0
    n = max(1, int(budget_s / t1))
    t0 = time.perf_counter()
    for _ in range(n):
        o.rhs(U)
    el = time.perf_counter() - t0
    dofs = grid.K * 5 * o.R.Np
    return dict(value=dofs * n / el, unit="DOF-updates/s", cores=1, kind="oracle",
                sample=f"{n} rhs evaluations (RK stages) of the {grid.K}-tetrahedron P=4 mesh, FP64, "
                       f"{el:.1f} s; 200 steps at this rate: {1000 * el / n:.0f} s",
                cpu_model=cpu_model(), host_cpus=os.cpu_count())


def copy_peak(dev, gib=1.0, reps=10):
    """Device-to-device copy of `gib` GiB: the practical HBM rate (read plus
    write bytes per second) and the time of one copy in ms."""
    import torch
    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * 4 * n / (ms * 1e-3) / 1e9, ms


def serving_leg(budget_gib, precision="fp32"):
    """The serving configuration: 64 requests (seed 64) arriving as a Poisson
    process of mean gap 50 ms, cylinders and airfoils of 2k-60k elements,
    P in 1..5, Mach 0.3-0.85, 500-3000 steps, admitted by HBM footprint into
    16 slots, continuous batching in 50-step chunks.  Latency is arrival to
    completion; a request that stops on the state check counts at the time
    it stopped in the percentiles."""
    from paper_1208_4772_amd import serving
    t0 = time.perf_counter()
    reqs = serving.make_requests(64, 0.05, 64)
    build_s = time.perf_counter() - t0
    srv = serving.Server(int(budget_gib * 2 ** 30), 16, precision, 50)
    # workgroup shapes per kind of solve in the mix, before the clock starts
    shapes = srv.tune(reqs)
    rep = srv.run(reqs)
    out = rep.summary()
    out["build_s"] = round(build_s, 1)
    out["workgroup_waves"] = {f"P{P}{'_av' if av else ''}": w for (P, av), w in shapes.items()}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed LSERK steps (default: the workload's)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="roofline", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3", "fp64"])
    ap.add_argument("--form", default="nodal", choices=["nodal", "weak"],
                    help="discretisation: the nodal strong form or the over-integrated weak form")
    ap.add_argument("--riemann", default="lf", choices=["lf", "hllc"], help="numerical flux")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-plain comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the occupancy-limit launch shape instead of timing the candidates")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--serving-budget-gib", type=float, default=1.0)
    ap.add_argument("--copy-probe", type=float, default=0.0, metavar="GIB",
                    help="only run a device-to-device copy of this many GiB (HBM peak probe and "
                         "the known-size kernel that scales the traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver has no "
              f"multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import meshgen
    from paper_1208_4772_amd import dg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe > 0:
        gbs, ms = copy_peak(dev, args.copy_probe)
        n = int(args.copy_probe * (1 << 30)) // 4
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n,
                          "avg_ms": ms, "achieved_GBs": gbs}), flush=True)
        return
    if args.workload == "tet3d":
        bench_tet3d(args, dev)
        return
    P = {"cylinder": 4, "roofline": 5, "vortex": 2, "airfoil": 3}[args.workload]
    r, s = dg.reference_nodes(P)
    # the airfoil starts from the wall-damped freestream: from the impulsive
    # start this mesh reaches rho, p <= 0 within 2000 steps (in FP64 too)
    case = meshgen.make_case(args.workload, r, s,
                             **({"start": "damped"} if args.workload == "airfoil" else {}))
    steps = case.steps if args.steps is None else args.steps
    log(f"workload {args.workload}: K={case.K} P={case.P} Np={case.Np} DOF={case.dofs()} "
        f"steps={steps} warmup={args.warmup}")

    tuned = {}
    final = {}

    def timed_run(precision, nsteps, warmup):
        sol = dg.Solver.from_case(case, precision, device="cuda:0", form=args.form, riemann=args.riemann)
        U0 = sol.state(case.U0)
        U = U0.clone()
        if not args.no_autotune:
            tuned[precision] = sol.autotune(U)
        if warmup:
            sol.run(U, warmup)
        U.copy_(U0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = sol.run(U, nsteps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ok = bool(torch.isfinite(U).all().item())
        final[precision] = U.double().cpu().numpy()
        sol.close()
        return wall, st, ok

    # the timed run: replayed step graphs.  dg_run brackets its steps with a
    # HIP event pair on the launch stream; inside that region the GPU runs
    # the five stage launches of every step (plus one CFL launch before the
    # first step), so region time / stage launches is the stage kernel's
    # average launch duration, inter-launch gaps included.
    wall, st, ok = timed_run(args.precision, steps, args.warmup)
    if not ok or st.status != 0:
        raise SystemExit("state became non-finite in the timed run")
    dofs = case.dofs()
    value = dofs * 5 * steps / wall
    avg_s = st.wall_s / (5 * steps)
    log(f"{args.precision}: {wall * 1e3:.2f} ms for {steps} steps -> {value:.4e} DOF-updates/s "
        f"(device events {st.wall_s * 1e3:.2f} ms, {avg_s * 1e6:.2f} us per stage launch)")

    sbytes = 8 if args.precision == "fp64" else 4
    launch_bytes, geo_info = algorithmic_stage_bytes(case, sbytes)
    achieved = launch_bytes / avg_s / 1e9
    # counter traffic is committed for the default discretisation only
    traffic = (load_traffic(args.workload, args.precision, launch_bytes, case.av)
               if args.form == "nodal" and args.riemann == "lf" else None)
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    kernel=stage_kernel_label(case, args.precision, tuned.get(args.precision, (0, 0.0))[0],
                                              args.form),
                    avg_launch_us=round(avg_s * 1e6, 3),
                    launches=5 * steps,
                    waves_per_block=tuned.get(args.precision, (0, 0.0))[0] or None,
                    algorithmic_bytes_per_launch=int(launch_bytes))

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "K": case.K, "P": case.P,
                   "dof": dofs, "precision": args.precision,
                   "curved_elements": geo_info["curved"]},
    }
    if args.form != "nodal" or args.riemann != "lf":
        # the byte model is the nodal one (the weak form moves the same state,
        # register and traces; its straight-element geometry is smaller)
        out["config"].update(form=args.form, riemann=args.riemann)
    out["roofline"] = roofline
    if not args.no_fp64 and args.precision != "fp64":
        w64, st64, ok64 = timed_run("fp64", steps, args.warmup)
        out["fp64_plain"] = dict(value=dofs * 5 * steps / w64, ms_per_step=w64 * 1e3 / steps,
                                 finite=ok64)
        out["fp32_over_fp64_plain"] = round(value / out["fp64_plain"]["value"], 3)
        log(f"fp64 plain: {w64 * 1e3:.2f} ms -> {out['fp64_plain']['value']:.4e} DOF-updates/s")
        # the timed run's final state against the FP64 run's (which matches
        # the FP64 oracle to 1e-12): the reduced-precision error at that time
        from paper_1208_4772_amd import accuracy
        geo = accuracy.Geometry(case)
        acc = dict(vs="fp64_plain", step=steps, t=st.t,
                   **accuracy.state_errors(final[args.precision], final["fp64"]),
                   entropy_error=geo.entropy_error(final[args.precision], case.freestream),
                   entropy_error_fp64=geo.entropy_error(final["fp64"], case.freestream))
        loads = geo.wall_loads(final[args.precision], case.freestream)
        if loads is not None:
            acc["wall"] = loads
            acc["wall_fp64"] = geo.wall_loads(final["fp64"], case.freestream)
        out["accuracy"] = acc
        log(f"accuracy vs fp64 plain: {acc}")
    gbs, _ = copy_peak(dev)
    roofline["copy_peak_GBs"] = round(gbs, 1)
    roofline["frac_of_copy_peak"] = round(achieved / gbs, 4)
    log(f"device copy: {gbs:.0f} GB/s; stage kernel at {achieved / gbs:.3f} of it")
    if not args.no_serving:
        out["serving"] = serving_leg(args.serving_budget_gib, args.precision)
        # the batched aggregate beside the single-mesh rate of this run
        out["serving"]["aggregate_over_single_mesh"] = round(
            out["serving"]["aggregate_dof_updates_per_s"] / value, 4)
        log(f"serving: {out['serving']}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_budget)
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
